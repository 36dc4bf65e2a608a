// Molecular-dynamics modes (gfx950): R-index keys, partial radix sort of
// fixed index segments, particle reordering, CPC2000-style coding.
//
// The paper's modes for MD snapshots (Sec. 5.2, Sec. 6): best_speed = SZ-LV
// on every field; best_tradeoff = SZ-LV after a partial radix sort of the
// R-index that skips the k least significant digits (Table 5: segment 16384,
// k = 6); best_compression = CPC2000 coding of the sorted coordinate keys
// plus SZ-LV of the velocities in the same order; CPC2000 itself codes the
// velocities' integers with its variable-length code too (Sec. 2, Sec. 5.2).
// The R-index interleaves the bits of the coordinates turned into integers by
// the error bound (Sec. 2, CPC2000 steps 1-2); here the integers are the
// compressor's lattice indices, B bits each, x highest in each 3-bit digit.
// Velocity-based keys interleave vx, vy, vz the same way; six-field keys
// take the D = min(B, 10) leading bits of all six fields, xx highest in each
// 6-bit digit (Sec. 5.3, Table 6).
//
//   md_bits     key and value widths, segment count (one thread)
//   md_keys     lattice indices of the key fields -> interleaved key
//   md_sort     one workgroup per segment: stable LSD radix sort by key >> digit k
//   md_gather   apply the permutation to every field
//   md_vals     lattice indices of a reordered velocity field (CPC2000)
//   cpc_count   per segment: deltas (keys) or offsets from the minimum
//               (velocities), Rice parameter, coded size
//   cpc_offsets segment word offsets, stream header
//   cpc_pack    per segment: first key or minimum, parameter, Rice codes
//   cpc_decode  one workgroup per segment, one thread per 64 keys (entry
//               points stored in the stream): keys back
//   cpc_coords  keys -> coordinates
//   cpv_decode  the same for a velocity stream (one pass: no prefix sums)
//   md_assemble container header and sub-stream copies
//   md_parse    container header -> sub-stream descriptors (decompression)
//   md_status   first error of the call into the status word
#include <type_traits>

#include "sznb_internal.h"

namespace sznb {

constexpr uint32_t kEscQ = 32;   // quotients from 32 on are escaped
constexpr uint32_t kCpcLdsWords = 16384;  // decoder: a segment's code words staged in LDS (64 KiB)
constexpr int kMT = 1024;
constexpr int kMW = kMT / kWave;
constexpr int kKey6Bits = 10;    // bits per field of a six-field key

// 21-bit value spread to every third bit (bit j -> bit 3j)
__device__ inline uint64_t spread3(uint64_t x) {
  x &= 0x1fffffull;
  x = (x | (x << 32)) & 0x1f00000000ffffull;
  x = (x | (x << 16)) & 0x1f0000ff0000ffull;
  x = (x | (x << 8)) & 0x100f00f00f00f00full;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}
__device__ inline uint32_t compact3(uint64_t x) {
  x &= 0x1249249249249249ull;
  x = (x ^ (x >> 2)) & 0x10c30c30c30c30c3ull;
  x = (x ^ (x >> 4)) & 0x100f00f00f00f00full;
  x = (x ^ (x >> 8)) & 0x1f0000ff0000ffull;
  x = (x ^ (x >> 16)) & 0x1f00000000ffffull;
  x = (x ^ (x >> 32)) & 0x1fffffull;
  return (uint32_t)x;
}
// 10-bit value spread to every sixth bit (bit j -> bit 6j)
__device__ inline uint64_t spread6(uint32_t x) {
  uint64_t r = 0;
#pragma unroll
  for (int j = 0; j < kKey6Bits; j++) r |= (uint64_t)((x >> j) & 1u) << (6 * j);
  return r;
}

__device__ inline int32_t md_lattice(float v, const FState *s) {
  double t = __dmul_rn(__dsub_rn((double)v, (double)s->mn), s->inv);
  return (int32_t)floor(__dadd_rn(t, 0.5));
}
__device__ inline uint32_t bitlen64(uint64_t v) { return v ? 64u - (uint32_t)__clzll((long long)v) : 0u; }

// Key layout of the call: nk = 3 (coordinates or velocities; B = the widest
// lattice span, at most 21) or 6 (all fields; D = min(widest, 10) bits of
// each, the low bits of wider fields dropped), the velocity widths for
// CPC2000, the segment count.  The first error of any field stops the call.
__global__ void md_bits(MdStates ks, int nk, MdStates vs, int nv, MdCtl *ctl, uint64_t n, uint32_t seg,
                        uint32_t kind, uint32_t keysrc, uint32_t k_ignored) {
  if (threadIdx.x || blockIdx.x) return;
  int32_t st = 0;
  uint32_t w[6], wmax = 1;
  for (int c = 0; c < nk; c++) {
    if (!st && ks.s[c]->status) st = ks.s[c]->status;
    w[c] = max(bitlen64((uint64_t)ks.s[c]->P), 1u);
    wmax = max(wmax, w[c]);
  }
  for (int c = 0; c < nv; c++) {
    if (!st && vs.s[c]->status) st = vs.s[c]->status;
    ctl->vbits[c] = max(bitlen64((uint64_t)vs.s[c]->P), 1u);
  }
  if (nk != 6) {
    if (!st && wmax > 21) st = SZNB_EEBTOOSMALL;
    ctl->B = wmax;
    ctl->keybits = 3 * wmax;
    ctl->digit = 3;
    for (int c = 0; c < 6; c++) ctl->shift[c] = 0;
  } else {
    const uint32_t D = min(wmax, (uint32_t)kKey6Bits);
    ctl->B = D;
    ctl->keybits = 6 * D;
    ctl->digit = 6;
    for (int c = 0; c < 6; c++) ctl->shift[c] = w[c] > D ? w[c] - D : 0u;
  }
  ctl->nk = (uint32_t)nk;
  ctl->seg = seg;
  ctl->nseg = (uint32_t)((n + seg - 1) / seg);
  ctl->kind = kind;
  ctl->keysrc = keysrc;
  ctl->k = k_ignored;
  ctl->status = (uint32_t)st;
}

__global__ void md_keys(MdPtrs kf, MdStates ks, uint64_t n, const MdCtl *ctl, uint64_t *key, uint32_t *idx) {
  if (ctl->status) return;
  const uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x, stride = (uint64_t)gridDim.x * blockDim.x;
  if (ctl->nk == 3) {
    for (uint64_t i = i0; i < n; i += stride) {
      const uint64_t px = (uint64_t)(uint32_t)md_lattice(kf.f[0][i], ks.s[0]);
      const uint64_t py = (uint64_t)(uint32_t)md_lattice(kf.f[1][i], ks.s[1]);
      const uint64_t pz = (uint64_t)(uint32_t)md_lattice(kf.f[2][i], ks.s[2]);
      key[i] = (spread3(px) << 2) | (spread3(py) << 1) | spread3(pz);
      idx[i] = (uint32_t)i;
    }
  } else {
    uint32_t sh[6];
    for (int c = 0; c < 6; c++) sh[c] = ctl->shift[c];
    for (uint64_t i = i0; i < n; i += stride) {
      uint64_t k = 0;
#pragma unroll
      for (int c = 0; c < 6; c++)
        k |= spread6((uint32_t)md_lattice(kf.f[c][i], ks.s[c]) >> sh[c]) << (5 - c);
      key[i] = k;
      idx[i] = (uint32_t)i;
    }
  }
}

__device__ inline uint64_t md_lanemask_lt() {
  const uint32_t l = lane_id();
  return l ? (~0ull >> (64 - l)) : 0ull;
}

// Stable sort of one segment's (key, idx) pairs from (kin, iin) into (kout,
// iout) by key >> (digit k), LSD on 8-bit digits; each of the 16 waves owns a
// contiguous slice of the current order and keeps it.  When the sorted bits
// and the 14-bit position in the segment fit in 64 bits, every pass stays in
// LDS (dynamic, 8 bytes per element): the packed values are scattered there
// and read back in the next pass's order, and the keys and indices are
// gathered by position at the end.  Otherwise each pass ping-pongs between
// the two buffers (the input's are overwritten).
__global__ __launch_bounds__(kMT) void md_sort(uint64_t *kin, uint32_t *iin, uint64_t *kout, uint32_t *iout,
                                               uint64_t n, uint32_t k_ignored, const MdCtl *ctl) {
  extern __shared__ __align__(16) uint64_t s_v[];
  __shared__ uint32_t s_cnt[256 * kMW];
  __shared__ uint32_t s_tot[kMW];
  if (ctl->status) return;
  const uint32_t seg = blockIdx.x, S = ctl->seg;
  const uint64_t base = (uint64_t)seg * S;
  if (base >= n) return;
  const uint32_t m = (uint32_t)min((uint64_t)S, n - base);
  const int t = threadIdx.x, w = t / kWave;
  const uint32_t shift0 = ctl->digit * k_ignored;
  const uint32_t bits = ctl->keybits > shift0 ? ctl->keybits - shift0 : 0;
  const uint32_t passes = (bits + 7) / 8;
  uint64_t *ka = kin + base, *kb = kout + base;
  uint32_t *ia = iin + base, *ib = iout + base;
  const uint32_t segw = (m + kMW - 1) / kMW;
  const uint32_t beg = min(m, segw * w), end = min(m, beg + segw);
  constexpr int kPL = kMdSegMax / kMT;  // chunks of 64 per wave
  // one pass over the digit at bit sh of the values get(c) (chunk c of the
  // wave's slice): counts, the exclusive scan over (digit, wave),
  // digit-major, then put(c, pos) for every element
  const auto pass = [&](auto get, uint32_t sh, auto put) {
    for (uint32_t i = t; i < 256u * kMW; i += kMT) s_cnt[i] = 0;
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kPL; c++)
      if (beg + (uint32_t)c * kWave + lane_id() < end) atomicAdd(&s_cnt[((get(c) >> sh) & 255u) * kMW + w], 1u);
    __syncthreads();
    uint32_t loc = 0;
    for (int j = 0; j < 4; j++) loc += s_cnt[4 * t + j];
    const uint32_t inc = wave_incl_scan(loc);
    if (lane_id() == kWave - 1) s_tot[w] = inc;
    __syncthreads();
    uint32_t run = inc - loc;
    for (int j = 0; j < w; j++) run += s_tot[j];
    for (int j = 0; j < 4; j++) { const uint32_t x = s_cnt[4 * t + j]; s_cnt[4 * t + j] = run; run += x; }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kPL; c++) {
      const uint32_t i = beg + (uint32_t)c * kWave + lane_id();
      const bool valid = i < end;
      const uint32_t dg = valid ? (uint32_t)((get(c) >> sh) & 255u) : 0u;
      uint64_t mk = __ballot(valid);
      for (int bt = 0; bt < 8; bt++) {
        const uint64_t bb = __ballot(valid && ((dg >> bt) & 1u));
        mk &= ((dg >> bt) & 1u) ? bb : ~bb;
      }
      const uint32_t rank = __popcll(mk & md_lanemask_lt()), cnt = __popcll(mk);
      uint32_t pos = 0;
      if (valid) pos = s_cnt[dg * kMW + w] + rank;
      __builtin_amdgcn_wave_barrier();
      if (valid) {
        put(c, pos);
        if (rank == cnt - 1) s_cnt[dg * kMW + w] += cnt;
      }
      __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
  };
  if (bits + 14u <= 64u) {
    uint64_t v[kPL];
#pragma unroll
    for (int c = 0; c < kPL; c++) {
      const uint32_t i = beg + (uint32_t)c * kWave + lane_id();
      v[c] = i < end ? (((ka[i] >> shift0) << 14) | i) : 0ull;
    }
    for (uint32_t ps = 0; ps < passes; ps++) {
      pass([&](int c) { return v[c]; }, 14 + 8 * ps, [&](int c, uint32_t pos) { s_v[pos] = v[c]; });
#pragma unroll
      for (int c = 0; c < kPL; c++) {
        const uint32_t i = beg + (uint32_t)c * kWave + lane_id();
        if (i < end) v[c] = s_v[i];
      }
    }
    // element v & 16383 of the input takes position i; every gather load
    // is issued before the first store (a store could alias a later load,
    // which would otherwise wait for it)
    uint64_t kv[kPL];
    uint32_t iv[kPL];
#pragma unroll
    for (int c = 0; c < kPL; c++) {
      const uint32_t i = beg + (uint32_t)c * kWave + lane_id();
      const uint32_t src = i < end ? (uint32_t)(v[c] & 16383u) : 0u;
      kv[c] = ka[src];
      iv[c] = ia[src];
    }
#pragma unroll
    for (int c = 0; c < kPL; c++) {
      const uint32_t i = beg + (uint32_t)c * kWave + lane_id();
      if (i < end) { kb[i] = kv[c]; ib[i] = iv[c]; }
    }
    return;
  }
  // keys too wide to pack with the position: the elements are read where
  // they are used (from L2: the segment's 192 KiB stay there)
  for (uint32_t ps = 0; ps < passes; ps++) {
    const auto at = [&](int c) { return beg + (uint32_t)c * kWave + lane_id(); };
    pass([&](int c) { return ka[at(c)]; }, shift0 + 8 * ps, [&](int c, uint32_t pos) {
      kb[pos] = ka[at(c)];
      ib[pos] = ia[at(c)];
    });
    uint64_t *tk = ka; ka = kb; kb = tk;
    uint32_t *ti = ia; ia = ib; ib = ti;
  }
  // the result to (kout, iout): after an even number of passes it is back
  // in the input buffers
  if (!(passes & 1u)) {
    for (uint32_t i = t; i < m; i += kMT) { kb[i] = ka[i]; ib[i] = ia[i]; }
  }
}

__global__ void md_gather(const float *src, float *dst, const uint32_t *perm, uint64_t n, const MdCtl *ctl) {
  if (ctl->status) return;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    dst[i] = src[perm[i]];
}

// lattice indices of a velocity field in the sorted order
__global__ void md_vals(const float *v, const uint32_t *perm, const FState *s, uint64_t n, const MdCtl *ctl,
                        uint64_t *out) {
  if (ctl->status) return;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    out[i] = (uint64_t)(uint32_t)md_lattice(v[perm[i]], s);
}

// identity order (best_speed keeps the stored order)
__global__ void md_iota(uint32_t *perm, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    perm[i] = (uint32_t)i;
}

// ------------------------------------------------------------- CPC2000

// Rice cost of a value with parameter r
__device__ inline uint64_t rice_cost(uint64_t d, uint32_t r, uint32_t vb) {
  const uint64_t q = d >> r;
  return q >= kEscQ ? (uint64_t)(kEscQ + vb) : q + 1 + r;
}

// Per segment: kOffset = false (sorted keys): the deltas of keys 1..m-1;
// kOffset = true (velocity values): every value minus the segment minimum.
// Rice parameter r = argmin_r sum cost (ties to the smaller r) and the
// segment's coded bits (first key or minimum, 6-bit parameter, codes).
template <bool kOffset>
__global__ __launch_bounds__(kMT) void cpc_count(const uint64_t *val, uint64_t n, const MdCtl *ctl,
                                                 const uint32_t *vbp, uint32_t *seg_r, uint32_t *seg_bits,
                                                 uint64_t *seg_min) {
  __shared__ unsigned long long s_sum[kMW], s_best;
  __shared__ uint32_t s_cost[64 * kMW], s_num[kMW];
  __shared__ bool s_ok;
  if (ctl->status) return;
  const uint32_t seg = blockIdx.x, S = ctl->seg;
  const uint64_t base = (uint64_t)seg * S;
  if (base >= n) return;
  const uint32_t m = (uint32_t)min((uint64_t)S, n - base);
  const uint32_t vb = *vbp;
  const int t = threadIdx.x, w = t / kWave;
  // this thread's codes, read once (at most kMdSegMax / kMT of them)
  constexpr int kPer = kMdSegMax / kMT;
  const uint32_t first = kOffset ? 0u : 1u;
  uint64_t dl[kPer];
  uint64_t vmin = 0;
  if (kOffset) {
    uint64_t mn = ~0ull;
#pragma unroll
    for (int j = 0; j < kPer; j++) {
      const uint32_t i = t + (uint32_t)j * kMT;
      dl[j] = i < m ? val[base + i] : ~0ull;
      mn = min(mn, dl[j]);
    }
    mn = wave_min_u64(mn);
    if (lane_id() == 0) s_sum[w] = mn;
    __syncthreads();
    vmin = s_sum[0];
    for (int j = 1; j < kMW; j++) vmin = min(vmin, (uint64_t)s_sum[j]);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kPer; j++) dl[j] -= vmin;
  } else {
#pragma unroll
    for (int j = 0; j < kPer; j++) {
      const uint32_t i = 1 + t + (uint32_t)j * kMT;
      dl[j] = i < m ? val[base + i] - val[base + i - 1] : 0u;
    }
  }
  const auto coded = [&](int j) { return first + t + (uint32_t)j * kMT < m; };
  // the parameters' costs C(r) (sums of rice_cost) for r in [lo, lo + nr),
  // each wave's into s_cost[(r - lo) * kMW + w]
  const auto costs = [&](uint32_t lo, uint32_t nr) {
    for (uint32_t r = lo; r < lo + nr; r++) {
      uint32_t c = 0;
#pragma unroll
      for (int j = 0; j < kPer; j++)
        if (coded(j)) c += (uint32_t)rice_cost(dl[j], r, vb);
      c = wave_sum(c);
      if (lane_id() == 0) s_cost[(r - lo) * kMW + w] = c;
    }
  };
  // wave 0: the smallest (C(r), r) of the nr parameters from lo, as C << 6 | r
  const auto best_of = [&](uint32_t lo, uint32_t nr) {
    const uint32_t i = lane_id();
    uint64_t tot = 0;
    if (i < nr)
      for (int j = 0; j < kMW; j++) tot += s_cost[i * kMW + j];
    return wave_min_u64(i < nr ? (tot << 6) | (lo + i) : ~0ull);
  };
  // Eight parameters around the codes' mean bit length, then proof that
  // no other parameter does better: every code costs at least 1 + r bits, so
  // for r above the window C(r) >= (number of codes)(1 + r); below the
  // window a code costs at least min(32 + vb, (d >> (lo - 1)) + 1) bits.
  // Without the proof every parameter is costed.  Either way the cheapest
  // parameter is taken, the smaller on a tie.
  uint64_t su = 0;
  uint32_t cn = 0;
#pragma unroll
  for (int j = 0; j < kPer; j++)
    if (coded(j)) { su += bitlen64(dl[j]); cn++; }
  su = wave_sum(su);
  cn = wave_sum(cn);
  if (lane_id() == 0) { s_sum[w] = su; s_num[w] = cn; }
  __syncthreads();
  uint64_t sum_all = 0, num_all = 0;
  for (int j = 0; j < kMW; j++) { sum_all += s_sum[j]; num_all += s_num[j]; }
  const uint32_t mb = (uint32_t)(num_all ? sum_all / num_all : 0ull);
  const uint32_t lo = min(mb > 4u ? mb - 4u : 0u, vb), nr = min(vb - lo + 1u, 8u);
  costs(lo, nr);
  if (lo > 0) {
    uint32_t c = 0;
#pragma unroll
    for (int j = 0; j < kPer; j++)
      if (coded(j)) c += (uint32_t)min((uint64_t)kEscQ + vb, (dl[j] >> (lo - 1)) + 1u);
    c = wave_sum(c);
    if (lane_id() == 0) s_cost[8 * kMW + w] = c;
  }
  __syncthreads();
  if (w == 0) {
    const uint64_t best = best_of(lo, nr);
    uint64_t low = 0;
    for (int j = 0; j < kMW; j++) low += s_cost[8 * kMW + j];
    const bool ok_hi = lo + nr > vb || num_all * (2u + (lo + nr - 1u)) >= (best >> 6);
    const bool ok_lo = lo == 0 || low > (best >> 6);
    if (lane_id() == 0) { s_best = best; s_ok = ok_hi && ok_lo; }
  }
  __syncthreads();
  uint64_t best = s_best;
  if (!s_ok) {
    costs(0, vb + 1);
    __syncthreads();
    if (w == 0) best = best_of(0, vb + 1);
  }
  if (t == 0) {
    seg_r[seg] = (uint32_t)(best & 63u);
    seg_bits[seg] = (uint32_t)(vb + 6 + (m > first ? (best >> 6) : 0ull));
    if (kOffset) seg_min[seg] = vmin;
  }
}

// entry points of all segments (one per 64 values)
__host__ __device__ inline uint64_t cpc_entries(uint64_t n, uint32_t seg) {
  const uint64_t nseg = (n + seg - 1) / seg;
  return nseg ? (nseg - 1) * (seg / kMdSub) + (n - (nseg - 1) * seg + kMdSub - 1) / kMdSub : 0;
}

__device__ inline void put32(uint8_t *p, uint64_t o, uint32_t v) { *reinterpret_cast<uint32_t *>(p + o) = v; }
__device__ inline void put64(uint8_t *p, uint64_t o, uint64_t v) {
  put32(p, o, (uint32_t)v);
  put32(p, o + 4, (uint32_t)(v >> 32));
}

// Stream headers, then u32 seg_bits[nseg] (padded to 8 bytes), then the
// entry points (for every segment and every 64 values of it, u32 bit offset
// from the segment start of that value's code; padded to 8 bytes), then the
// segments' words.
// Coordinates (104 bytes): "SZCP" u16 2 u8 B u8 0 u64 n u32 nseg u32 seg
//   u32 keybits f32 (mn, mx) x3, f64 eb_abs x3, f64 step x3, padding.
// Velocities (56 bytes): "SZCV" u16 1 u8 vbits u8 0 u64 n u32 nseg u32 seg
//   u32 vbits f32 mn f32 mx f64 eb_abs f64 step, padding.
template <bool kOffset>
__global__ void cpc_offsets(const uint32_t *seg_bits, uint32_t nseg_max, uint64_t n, const MdCtl *ctl, MdStates fs,
                            int vfield, uint8_t *cs, uint32_t *seg_woff, uint64_t *len_out) {
  if (blockIdx.x || ctl->status) return;
  const uint32_t nseg = min(ctl->nseg, nseg_max), S = ctl->seg, l = threadIdx.x;
  const uint32_t hb = kOffset ? kCvHdr : kCpHdr;
  // word offsets of the segments (a wave scan, 64 segments at a time) and
  // the segments' bit counts into the stream
  uint32_t o = 0;
  for (uint32_t s0 = 0; s0 < nseg; s0 += kWave) {
    const uint32_t s = s0 + l;
    const uint32_t sbits = s < nseg ? seg_bits[s] : 0u, wds = (sbits + 31) / 32;
    const uint32_t inc = wave_incl_scan(wds);
    if (s < nseg) {
      seg_woff[s] = o + inc - wds;
      put32(cs, hb + 4ull * s, sbits);
    }
    o += (uint32_t)__builtin_amdgcn_readlane((int)inc, kWave - 1);
  }
  if (l) return;
  const uint64_t tab = hb + align8((uint64_t)4 * nseg) + align8(4ull * cpc_entries(n, S));
  *len_out = tab + 4ull * o;
  for (uint32_t i = 0; i < hb; i += 4) put32(cs, i, 0u);
  put32(cs, 8, (uint32_t)n);
  put32(cs, 12, (uint32_t)(n >> 32));
  put32(cs, 16, nseg);
  put32(cs, 20, S);
  if (kOffset) {
    const uint32_t vb = ctl->vbits[vfield];
    const FState *s = fs.s[0];
    put32(cs, 0, 0x56435A53u);  // "SZCV"
    put32(cs, 4, 1u | (vb << 16));
    put32(cs, 24, vb);
    *reinterpret_cast<float *>(cs + 28) = s->mn;
    *reinterpret_cast<float *>(cs + 32) = s->mx;
    put64(cs, 36, (uint64_t)__double_as_longlong(s->eb_abs));
    put64(cs, 44, (uint64_t)__double_as_longlong(s->step));
  } else {
    put32(cs, 0, 0x50435A53u);  // "SZCP"
    put32(cs, 4, 2u | (ctl->B << 16));
    put32(cs, 24, ctl->keybits);
    for (int c = 0; c < 3; c++) {
      *reinterpret_cast<float *>(cs + 28 + 8 * c) = fs.s[c]->mn;
      *reinterpret_cast<float *>(cs + 32 + 8 * c) = fs.s[c]->mx;
      put64(cs, 52 + 8 * c, (uint64_t)__double_as_longlong(fs.s[c]->eb_abs));
      put64(cs, 76 + 8 * c, (uint64_t)__double_as_longlong(fs.s[c]->step));
    }
  }
  if (nseg & 1u) put32(cs, hb + 4ull * nseg, 0u);
  const uint64_t ne = cpc_entries(n, S);
  if (ne & 1u) put32(cs, hb + align8(4ull * nseg) + 4ull * ne, 0u);
}

// bit writer over global words: whole words are stored, words that may be
// shared with a neighbour thread are OR-ed (the region is zeroed first)
struct WBits {
  uint32_t *w;
  uint64_t pos;   // next bit
  uint64_t acc;   // pending bits, MSB-aligned
  uint32_t na;
  uint64_t first_word, last_word;
};
__device__ inline void wb_flush_word(WBits &b, uint64_t wi, uint32_t word) {
  if (wi == b.first_word || wi == b.last_word) atomicOr(&b.w[wi], word);
  else b.w[wi] = word;
}
__device__ inline void wb_put(WBits &b, uint64_t v, uint32_t nb) {  // nb <= 32
  if (!nb) return;
  b.acc |= (v & ((nb == 64) ? ~0ull : ((1ull << nb) - 1))) << (64u - b.na - nb);
  b.na += nb;
  if (b.na >= 32u) {
    wb_flush_word(b, b.pos >> 5, (uint32_t)(b.acc >> 32));
    b.pos += 32;
    b.acc <<= 32;
    b.na -= 32u;
  }
}
__device__ inline void wb_put_wide(WBits &b, uint64_t v, uint32_t nb) {  // nb <= 64
  if (nb > 32u) { wb_put(b, v >> 32, nb - 32u); wb_put(b, v, 32u); }
  else wb_put(b, v, nb);
}
__device__ inline void wb_rice(WBits &b, uint64_t d, uint32_t r, uint32_t vb) {
  const uint64_t q = d >> r;
  if (q >= kEscQ) {
    wb_put(b, 0xffffffffull, kEscQ);
    wb_put_wide(b, d, vb);
  } else {
    // q ones then a zero, then the r low bits
    wb_put(b, ((1ull << (q + 1)) - 2ull), (uint32_t)q + 1);
    wb_put_wide(b, d & ((1ull << r) - 1), r);
  }
}

template <bool kOffset>
__global__ __launch_bounds__(kMT) void cpc_pack(const uint64_t *val, uint64_t n, const MdCtl *ctl,
                                                const uint32_t *vbp, const uint32_t *seg_r,
                                                const uint32_t *seg_bits, const uint32_t *seg_woff,
                                                const uint64_t *seg_min, uint8_t *cs) {
  __shared__ unsigned long long s_tot[kMW];
  if (ctl->status) return;
  const uint32_t seg = blockIdx.x, S = ctl->seg;
  const uint64_t base = (uint64_t)seg * S;
  if (base >= n) return;
  const uint32_t m = (uint32_t)min((uint64_t)S, n - base);
  const uint32_t vb = *vbp, r = seg_r[seg];
  const uint64_t vmin = kOffset ? seg_min[seg] : 0;
  const int t = threadIdx.x, w = t / kWave;
  const uint64_t etab = (kOffset ? kCvHdr : kCpHdr) + align8((uint64_t)4 * ctl->nseg);
  const uint64_t tab = etab + align8(4ull * cpc_entries(n, S));
  uint32_t *words = reinterpret_cast<uint32_t *>(cs + tab) + seg_woff[seg];
  uint32_t *ent = reinterpret_cast<uint32_t *>(cs + etab) + (uint64_t)seg * (S / kMdSub);
  const uint32_t nw = (seg_bits[seg] + 31) / 32;
  for (uint32_t i = t; i < nw; i += kMT) words[i] = 0u;
  __syncthreads();
  auto code_of = [&](uint32_t i) -> uint64_t {  // value i's coded quantity (i >= 1 for keys)
    return kOffset ? val[base + i] - vmin : val[base + i] - val[base + i - 1];
  };
  // thread t codes values i in [lo, hi); bit offsets by a workgroup scan
  const uint32_t per = (m + kMT - 1) / kMT;
  const uint32_t lo = min(m, t * per), hi = min(m, lo + per);
  // this thread's coded quantities, read once (at most kMdSegMax / kMT)
  constexpr int kPer = kMdSegMax / kMT;
  uint64_t cq[kPer];
#pragma unroll
  for (int j = 0; j < kPer; j++) {
    const uint32_t i = lo + (uint32_t)j;
    cq[j] = i < hi && (kOffset || i > 0) ? code_of(i) : 0ull;
  }
  unsigned long long mine = 0;
#pragma unroll
  for (int j = 0; j < kPer; j++) {
    const uint32_t i = lo + (uint32_t)j;
    if (i < hi && (kOffset || i > 0)) mine += rice_cost(cq[j], r, vb);
  }
  if (lo == 0 && hi > 0) mine += vb + 6;
  const unsigned long long inc = wave_incl_scan(mine);
  if (lane_id() == kWave - 1) s_tot[w] = inc;
  __syncthreads();
  unsigned long long pre = inc - mine;
  for (int j = 0; j < w; j++) pre += s_tot[j];
  if (hi > lo) {
    WBits b;
    b.w = words;
    b.pos = pre & ~31ull;
    b.na = (uint32_t)(pre & 31u);
    b.acc = 0;
    b.first_word = pre >> 5;
    b.last_word = (pre + mine - 1) >> 5;
#pragma unroll
    for (int j = 0; j < kPer; j++) {
      const uint32_t i = lo + (uint32_t)j;
      if (i >= hi) break;
      if (i == 0) {
        if (!kOffset) ent[0] = 0u;  // a key segment starts with its first key raw
        wb_put_wide(b, kOffset ? vmin : val[base], vb);
        wb_put(b, r, 6);
        if (!kOffset) continue;
      }
      if ((i & (kMdSub - 1)) == 0) ent[i / kMdSub] = (uint32_t)(b.pos + b.na);
      wb_rice(b, cq[j], r, vb);
    }
    if (b.na) wb_flush_word(b, b.pos >> 5, (uint32_t)(b.acc >> 32));
  }
}

// Per-lane bit reader over one segment's words (LDS or global, chosen once
// per segment): a 64-bit window holding the bits from pos on (more than 32
// of them after every refill) and the next word, read one refill ahead so
// that a refill never waits for its load; words past the segment read as
// zero and a read that would pass nbits marks the segment corrupt.
template <bool kL>
struct SegReader {
  const uint32_t *lw;
  gptr<const uint32_t> gw;
  uint64_t nw, nbits, pos, buf, wi;
  uint32_t nv;
  bool *bad;
  uint32_t pend;  // word wi
  __device__ uint32_t word(uint64_t i) const { return i >= nw ? 0u : (kL ? lw[i] : gw[i]); }
  __device__ void seek(uint64_t p) {
    pos = p;
    wi = p >> 5;
    const uint32_t sh = (uint32_t)(p & 31u);
    const uint64_t w0 = word(wi), w1 = word(wi + 1);
    buf = ((w0 << 32) | w1) << sh;
    nv = 64u - sh;
    wi += 2;
    pend = word(wi);
  }
  __device__ void skip(uint32_t nb) {  // nb <= 32
    buf = nb ? buf << nb : buf;
    nv -= nb;
    pos += nb;
    if (nv <= 32u) {
      buf |= (uint64_t)pend << (32u - nv);
      nv += 32u;
      wi++;
      pend = word(wi);
    }
  }
  __device__ uint64_t take(uint32_t nb) {  // nb <= 32
    if (!nb) return 0;
    if (pos + nb > nbits) { *bad = true; return 0; }
    const uint64_t v = buf >> (64u - nb);
    skip(nb);
    return v;
  }
  __device__ uint64_t take_wide(uint32_t nb) {
    if (nb > 32u) { const uint64_t hi = take(nb - 32u); return (hi << 32) | take(32u); }
    return take(nb);
  }
  // one Rice code: unary quotient (the ones before the first zero, at most
  // kEscQ), then r low bits or the escaped raw value
  __device__ uint64_t rice(uint32_t r, uint32_t vb) {
    const uint32_t ones = ~(uint32_t)(buf >> 32);
    const uint32_t q = ones ? (uint32_t)__clz(ones) : kEscQ;
    if (q + r < 32u) {  // the whole code lies in the window's upper 32 bits
      const uint32_t nb = q + 1u + r;
      if (pos + nb > nbits) { *bad = true; return 0; }
      const uint64_t v = ((uint64_t)q << r) | (((buf << (q + 1u)) >> 1) >> (63u - r));
      skip(nb);
      return v;
    }
    const uint32_t ub = q < kEscQ ? q + 1u : kEscQ;
    if (pos + ub > nbits) { *bad = true; return 0; }
    skip(ub);
    if (q == kEscQ) return take_wide(vb);
    return ((uint64_t)q << r) | take_wide(r);
  }
  // The Rice codes of values i0 .. i1-1, f(v) for each.  A code that fits in
  // the window's upper 32 bits (nearly all) is taken without a bound check:
  // the caller compares the end position with the next entry point, and
  // words past the segment read as zero.
  template <class Fn>
  __device__ void codes(uint32_t i0, uint32_t i1, uint32_t r, uint32_t vb, Fn f) {
    for (uint32_t i = i0; i < i1; i++) {
      const uint32_t ones = ~(uint32_t)(buf >> 32);
      const uint32_t q = ones ? (uint32_t)__clz(ones) : kEscQ;
      uint64_t v;
      if (q + r < 32u) {
        const uint32_t nb = q + 1u + r;
        v = ((uint64_t)q << r) | (((buf << (q + 1u)) >> 1) >> (63u - r));
        buf <<= nb;
        nv -= nb;
        pos += nb;
        if (nv <= 32u) {
          buf |= (uint64_t)pend << (32u - nv);
          nv += 32u;
          wi++;
          pend = word(wi);
        }
      } else {
        v = rice(r, vb);
      }
      f(v);
    }
  }
};

// stages a segment's words in LDS (coalesced over the workgroup, four loads
// per thread in flight before they are stored)
__device__ inline void stage_words(uint32_t *s_seg, gptr<const uint32_t> gw, uint64_t nw) {
  const uint32_t t = threadIdx.x, nt = blockDim.x;
  for (uint32_t i0 = 0; i0 < nw; i0 += 4u * nt) {
    uint32_t a[4];
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const uint32_t i = i0 + (uint32_t)u * nt + t;
      a[u] = i < nw ? gw[i] : 0u;
    }
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const uint32_t i = i0 + (uint32_t)u * nt + t;
      if (i < nw) s_seg[i] = a[u];
    }
  }
}

__device__ inline bool seg_size_ok(uint32_t S) { return S >= 1024u && S <= kMdSegMax && !(S & (S - 1)); }

// One workgroup per segment, one thread per 64 keys (kCpcThreads threads):
// each thread starts at its entry point and writes the running sums of its
// deltas to kout; the workgroup scans the threads' totals into kbase (one
// entry per 64 keys: key i is kout[i] + kbase[i / 64]).  Every read is
// checked against the segment's bit count and the stream length, and every
// thread must end exactly at the next thread's entry point; a stream that
// fails a check sets ECORRUPT.  The stream is sub-stream 0 of the container
// (offset and length from md_parse); the grid covers the smallest segment
// size.
__global__ __launch_bounds__(kCpcThreads) void cpc_decode(const uint8_t *in, const MdCtl *ctl, uint64_t n,
                                                          uint64_t *kout, uint64_t *kbase, int *status) {
  __shared__ uint32_t s_seg[kCpcLdsWords];
  __shared__ unsigned long long s_wtot[kCpcThreads / kWave];
  if (ctl->status || ctl->kind < 2) return;
  const uint8_t *cs = in + ctl->sub_off[0];
  const uint64_t cs_len = ctl->sub_len[0];
  const uint32_t seg = blockIdx.x, t = threadIdx.x, w = t / kWave;
  if (cs_len < kCpHdr) { if (seg == 0 && t == 0) atomicCAS(status, 0, SZNB_ECORRUPT); return; }
  const uint32_t nseg = *reinterpret_cast<const uint32_t *>(cs + 16);
  const uint32_t S = *reinterpret_cast<const uint32_t *>(cs + 20);
  const uint32_t kb = *reinterpret_cast<const uint32_t *>(cs + 24);
  const uint64_t nhdr = (uint64_t)*reinterpret_cast<const uint32_t *>(cs + 8) |
                        ((uint64_t)*reinterpret_cast<const uint32_t *>(cs + 12) << 32);
  if (*reinterpret_cast<const uint32_t *>(cs) != 0x50435A53u || (*reinterpret_cast<const uint32_t *>(cs + 4) & 0xffffu) != 2u ||
      nhdr != n || !seg_size_ok(S) || S != ctl->seg || nseg != (n + S - 1) / S || kb > 63 || kb == 0 ||
      kCpHdr + align8(4ull * nseg) + align8(4ull * cpc_entries(n, S)) > cs_len) {
    if (seg == 0 && t == 0) atomicCAS(status, 0, SZNB_ECORRUPT);
    return;
  }
  const uint64_t etab = kCpHdr + align8(4ull * nseg);
  const uint64_t tab = etab + align8(4ull * cpc_entries(n, S));
  if (seg >= nseg) return;
  const gptr<const uint32_t> sb = G(reinterpret_cast<const uint32_t *>(cs + kCpHdr));
  uint64_t woff = 0;  // every wave sums the earlier segments' words
  for (uint32_t s2 = lane_id(); s2 < seg; s2 += kWave) woff += (sb[s2] + 31) / 32;
  woff = wave_sum(woff);
  const uint64_t nbits = sb[seg];
  const uint64_t avail = (cs_len - tab) / 4;
  bool bad = woff + (nbits + 31) / 32 > avail;
  const gptr<const uint32_t> gw = G(reinterpret_cast<const uint32_t *>(cs + tab) + woff);
  const gptr<const uint32_t> ent = G(reinterpret_cast<const uint32_t *>(cs + etab)) + (uint64_t)seg * (S / kMdSub);
  const uint64_t base = (uint64_t)seg * S;
  const uint32_t m = (uint32_t)min((uint64_t)S, n - base);
  const uint32_t k0 = t * kMdSub, k1 = min(m, k0 + kMdSub);  // this thread's keys
  const bool active = k0 < m;
  const uint64_t nw = (nbits + 31) / 32;
  const bool in_lds = !bad && nw <= kCpcLdsWords;
  if (in_lds) stage_words(s_seg, gw, nw);
  __syncthreads();
  // The bit reader refills from LDS or from global memory, decided once per
  // segment: a refill that could take either path made the compiler wait
  // for every vector-memory operation in flight (the key stores) at each
  // refill.
  const auto run = [&](auto lds) {
    constexpr bool kL = decltype(lds)::value;
    SegReader<kL> R{s_seg, gw, nw, nbits, 0, 0, 0, 0, &bad};
    // the Rice parameter follows the first key
    uint32_t r = 0;
    if (!bad) {
      R.seek(kb);
      r = (uint32_t)R.take(6);
      if (r > kb) bad = true;
    }
    const uint64_t start = active ? ent[t] : 0;
    const uint64_t stop = (k1 < m) ? ent[t + 1] : nbits;
    if (active && (start > stop || stop > nbits || (t == 0 && start != 0))) bad = true;
    // the segment's first key is stored raw (before the Rice parameter)
    const auto first = [&]() -> uint64_t {
      const uint64_t k = R.take_wide(kb);
      (void)R.take(6);
      return k;
    };
    // one pass: the running sums of the deltas (global stores: flat stores
    // in flight would hold up every LDS refill of the bit reader)
    uint64_t sum = 0;
    if (active && !bad) {
      R.seek(start);
      gptr<uint64_t> gk = G(kout) + base + k0;
      if (k0 == 0) *gk++ = sum = first();
      R.codes(k0 == 0 ? 1u : k0, k1, r, kb, [&](uint64_t v) {
        sum += v;
        *gk++ = sum;
      });
      if (R.pos != stop) bad = true;
    }
    // exclusive scan of the threads' totals over the workgroup
    const unsigned long long inc = wave_incl_scan((unsigned long long)sum);
    if (lane_id() == kWave - 1) s_wtot[w] = inc;
    if (__syncthreads_or(bad)) {
      if (t == 0) atomicCAS(status, 0, SZNB_ECORRUPT);
      return;
    }
    uint64_t pre = inc - sum;
    for (uint32_t j = 0; j < w; j++) pre += s_wtot[j];
    if (active) G(kbase)[base / kMdSub + t] = pre;
  };
  if (in_lds) run(std::true_type{}); else run(std::false_type{});
}

// The decoded keys back to coordinates (key i = kout[i] + kbase[i / 64]),
// x~ = fl32(fma(p, step, mn)) of each coordinate's lattice index (the bits of the key at its place in every
// 3-bit digit), after cpc_decode, over the whole grid.  Nothing is written
// for a container that failed a check.
__global__ void cpc_coords(const uint8_t *in, const MdCtl *ctl, uint64_t n, const uint64_t *key,
                           const uint64_t *kbase, float *ox, float *oy, float *oz, const int *status) {
  if (ctl->status || ctl->kind < 2 || *status || ctl->sub_len[0] < kCpHdr) return;
  const uint8_t *cs = in + ctl->sub_off[0];
  float mn[3];
  double step[3];
  for (int c = 0; c < 3; c++) {
    mn[c] = *reinterpret_cast<const float *>(cs + 28 + 8 * c);
    const uint64_t lo = *reinterpret_cast<const uint32_t *>(cs + 76 + 8 * c);
    const uint64_t hi = *reinterpret_cast<const uint32_t *>(cs + 80 + 8 * c);
    step[c] = __longlong_as_double((long long)(lo | (hi << 32)));
  }
  const gptr<const uint64_t> gk = G(key), gb = G(kbase);
  const gptr<float> gx = G(ox), gy = G(oy), gz = G(oz);
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t k = gk[i] + gb[i / kMdSub];
    gx[i] = (float)fma((double)(int32_t)compact3(k >> 2), step[0], (double)mn[0]);
    gy[i] = (float)fma((double)(int32_t)compact3(k >> 1), step[1], (double)mn[1]);
    gz[i] = (float)fma((double)(int32_t)compact3(k), step[2], (double)mn[2]);
  }
}

// CPC2000 velocity stream (sub-stream 1 + j of the container): one
// workgroup per segment, one thread per 64 values, one pass (each value is
// the minimum plus its code; no prefix).  The same checks as the key decoder.
__global__ __launch_bounds__(kCpcThreads) void cpv_decode(const uint8_t *in, const MdCtl *ctl, int j, uint64_t n,
                                                          float *out, int *status) {
  __shared__ uint32_t s_seg[kCpcLdsWords];
  if (ctl->status || ctl->kind != 3) return;
  const uint8_t *cs = in + ctl->sub_off[1 + j];
  const uint64_t cs_len = ctl->sub_len[1 + j];
  const uint32_t seg = blockIdx.x, t = threadIdx.x;
  if (cs_len < kCvHdr) { if (seg == 0 && t == 0) atomicCAS(status, 0, SZNB_ECORRUPT); return; }
  const uint32_t nseg = *reinterpret_cast<const uint32_t *>(cs + 16);
  const uint32_t S = *reinterpret_cast<const uint32_t *>(cs + 20);
  const uint32_t vb = *reinterpret_cast<const uint32_t *>(cs + 24);
  const uint32_t h1 = *reinterpret_cast<const uint32_t *>(cs + 4);
  const uint64_t nhdr = (uint64_t)*reinterpret_cast<const uint32_t *>(cs + 8) |
                        ((uint64_t)*reinterpret_cast<const uint32_t *>(cs + 12) << 32);
  if (*reinterpret_cast<const uint32_t *>(cs) != 0x56435A53u || (h1 & 0xffffu) != 1u || (h1 >> 16) != vb ||
      nhdr != n || !seg_size_ok(S) || S != ctl->seg || nseg != (n + S - 1) / S || vb > 31 || vb == 0 ||
      kCvHdr + align8(4ull * nseg) + align8(4ull * cpc_entries(n, S)) > cs_len) {
    if (seg == 0 && t == 0) atomicCAS(status, 0, SZNB_ECORRUPT);
    return;
  }
  if (seg >= nseg) return;
  const uint64_t etab = kCvHdr + align8(4ull * nseg);
  const uint64_t tab = etab + align8(4ull * cpc_entries(n, S));
  const float mn = *reinterpret_cast<const float *>(cs + 28);
  const double step = __longlong_as_double((long long)((uint64_t)*reinterpret_cast<const uint32_t *>(cs + 44) |
                                                       ((uint64_t)*reinterpret_cast<const uint32_t *>(cs + 48) << 32)));
  const gptr<const uint32_t> sb = G(reinterpret_cast<const uint32_t *>(cs + kCvHdr));
  uint64_t woff = 0;
  for (uint32_t s2 = lane_id(); s2 < seg; s2 += kWave) woff += (sb[s2] + 31) / 32;
  woff = wave_sum(woff);
  const uint64_t nbits = sb[seg];
  bool bad = woff + (nbits + 31) / 32 > (cs_len - tab) / 4;
  const gptr<const uint32_t> gw = G(reinterpret_cast<const uint32_t *>(cs + tab) + woff);
  const gptr<const uint32_t> ent = G(reinterpret_cast<const uint32_t *>(cs + etab)) + (uint64_t)seg * (S / kMdSub);
  const uint64_t base = (uint64_t)seg * S;
  const uint32_t m = (uint32_t)min((uint64_t)S, n - base);
  const uint32_t v0 = t * kMdSub, v1 = min(m, v0 + kMdSub);
  const bool active = v0 < m;
  const uint64_t nw = (nbits + 31) / 32;
  const bool in_lds = !bad && nw <= kCpcLdsWords;
  if (in_lds) stage_words(s_seg, gw, nw);
  __syncthreads();
  const auto run = [&](auto lds) {
    constexpr bool kL = decltype(lds)::value;
    SegReader<kL> R{s_seg, gw, nw, nbits, 0, 0, 0, 0, &bad};
    uint64_t vmin = 0;
    uint32_t r = 0;
    if (!bad) {
      R.seek(0);
      vmin = R.take_wide(vb);
      r = (uint32_t)R.take(6);
      if (r > vb) bad = true;
    }
    const uint64_t start = active ? ent[t] : 0;
    const uint64_t stop = (v1 < m) ? ent[t + 1] : nbits;
    if (active && (start > stop || stop > nbits || (t == 0 && start != vb + 6u))) bad = true;
    if (__syncthreads_or(bad)) {
      if (t == 0) atomicCAS(status, 0, SZNB_ECORRUPT);
      return;
    }
    if (active) {
      R.seek(start);
      gptr<float> go = G(out) + base + v0;
      R.codes(v0, v1, r, vb, [&](uint64_t v) {
        *go++ = (float)fma((double)(int32_t)(uint32_t)(vmin + v), step, (double)mn);
      });
      if (R.pos != stop) bad = true;
    }
    if (__syncthreads_or(bad) && t == 0) atomicCAS(status, 0, SZNB_ECORRUPT);
  };
  if (in_lds) run(std::true_type{}); else run(std::false_type{});
}

// Container (96-byte header): "SZMD" u16 1 u8 kind u8 nf u64 n u32 seg
// u32 k_ignored u64 total u64 offsets[6] u32 key fields; sub-streams 8-byte
// aligned.
__global__ void md_assemble(uint8_t *out, uint64_t out_cap, uint64_t *out_len, MdSubs subs, int nsub, int nf,
                            uint64_t n, const MdCtl *ctl, int *status) {
  // every workgroup computes the same offsets
  uint64_t offs[6] = {0, 0, 0, 0, 0, 0}, o = kMdHdr;
  uint64_t lens[6] = {0, 0, 0, 0, 0, 0};
  const bool bad = ctl->status != 0;
  for (int i = 0; i < nsub; i++) {
    lens[i] = bad ? 0 : *subs.len[i];
    offs[i] = o;
    o += align8(lens[i]);
  }
  const uint64_t total = o;
  const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  if (bad || total > out_cap) {
    if (tid == 0) {
      if (out_len) *out_len = 0;
      atomicCAS(status, 0, bad ? (int)ctl->status : SZNB_ENOSPC);
    }
    return;
  }
  for (int i = 0; i < nsub; i++) {
    if (lens[i] == 0) {
      if (tid == 0) atomicCAS(status, 0, SZNB_ENOSPC);
      continue;
    }
    const uint64_t padded = align8(lens[i]);
    for (uint64_t j = tid; j < padded; j += stride) out[offs[i] + j] = j < lens[i] ? subs.p[i][j] : 0;
  }
  if (tid == 0) {
    uint32_t *h = reinterpret_cast<uint32_t *>(out);
    for (int i = 0; i < (int)kMdHdr / 4; i++) h[i] = 0u;
    h[0] = 0x444D5A53u;  // "SZMD"
    h[1] = 1u | (ctl->kind << 16) | ((uint32_t)nf << 24);
    h[2] = (uint32_t)n; h[3] = (uint32_t)(n >> 32);
    h[4] = ctl->seg;
    h[5] = ctl->k;
    h[6] = (uint32_t)total; h[7] = (uint32_t)(total >> 32);
    for (int i = 0; i < 6; i++) { h[8 + 2 * i] = (uint32_t)offs[i]; h[9 + 2 * i] = (uint32_t)(offs[i] >> 32); }
    h[20] = ctl->keysrc;
    if (out_len) *out_len = total;
  }
}

// Decompression: checks the container header and points the descriptors
// at the sub-streams: the SZ-LV decoder's descriptor of output f gets its
// stream (skip = 0) or nothing (skip = 1: output f comes from a CPC stream);
// the CPC decoders read offsets and lengths from ctl.
__global__ void md_parse(const uint8_t *in, uint64_t in_len, int nf, uint64_t n, MdCtl *ctl, DField *D,
                         int *status) {
  if (threadIdx.x || blockIdx.x) return;
  int bad = in_len < kMdHdr;
  uint32_t h[kMdHdr / 4];
  for (int i = 0; i < (int)kMdHdr / 4; i++) h[i] = bad ? 0u : *reinterpret_cast<const uint32_t *>(in + 4 * i);
  const uint32_t kind = (h[1] >> 16) & 255u, hnf = h[1] >> 24, S = h[4], k = h[5], keysrc = h[20];
  const uint64_t hn = (uint64_t)h[2] | ((uint64_t)h[3] << 32), total = (uint64_t)h[6] | ((uint64_t)h[7] << 32);
  if (h[0] != 0x444D5A53u || (h[1] & 0xffffu) != 1u || kind > 3 || hnf != (uint32_t)nf || hn != n ||
      total > in_len || keysrc > 2 || !seg_size_ok(S))
    bad = 1;
  const int nsub = kind >= 2 ? nf - 2 : nf;
  for (int i = 0; i < nsub && !bad; i++) {
    const uint64_t off = (uint64_t)h[8 + 2 * i] | ((uint64_t)h[9 + 2 * i] << 32);
    const uint64_t end = i + 1 < nsub ? ((uint64_t)h[10 + 2 * i] | ((uint64_t)h[11 + 2 * i] << 32)) : total;
    if (off < kMdHdr || end < off || end > total || (off & 7u)) bad = 1;
    ctl->sub_off[i] = off;
    ctl->sub_len[i] = end - off;
  }
  ctl->kind = kind;
  ctl->seg = S;
  ctl->nsub = (uint32_t)nsub;
  ctl->status = bad ? (uint32_t)SZNB_ECORRUPT : 0u;
  if (bad) atomicCAS(status, 0, SZNB_ECORRUPT);
  for (int f = 0; f < nf; f++) {
    const int first_sz = kind == 2 ? 3 : kind == 3 ? nf : 0;  // outputs decoded by SZ-LV: f >= first_sz
    const bool sz = !bad && f >= first_sz;
    const int sub = kind == 2 ? f - 2 : f;
    D[f].skip = sz ? 0u : 1u;
    D[f].in = sz ? in + ctl->sub_off[sub] : in;
    D[f].in_len = sz ? ctl->sub_len[sub] : 0;
  }
}

// first non-zero status of the call into *out
__global__ void md_status(MdStatus ss, int ns, int32_t *out) {
  if (threadIdx.x || blockIdx.x) return;
  int32_t v = 0;
  for (int i = 0; i < ns && !v; i++) v = *ss.s[i];
  *out = v;
}

template __global__ void cpc_count<false>(const uint64_t *, uint64_t, const MdCtl *, const uint32_t *, uint32_t *,
                                          uint32_t *, uint64_t *);
template __global__ void cpc_count<true>(const uint64_t *, uint64_t, const MdCtl *, const uint32_t *, uint32_t *,
                                         uint32_t *, uint64_t *);
template __global__ void cpc_offsets<false>(const uint32_t *, uint32_t, uint64_t, const MdCtl *, MdStates, int,
                                            uint8_t *, uint32_t *, uint64_t *);
template __global__ void cpc_offsets<true>(const uint32_t *, uint32_t, uint64_t, const MdCtl *, MdStates, int,
                                           uint8_t *, uint32_t *, uint64_t *);
template __global__ void cpc_pack<false>(const uint64_t *, uint64_t, const MdCtl *, const uint32_t *,
                                         const uint32_t *, const uint32_t *, const uint32_t *, const uint64_t *,
                                         uint8_t *);
template __global__ void cpc_pack<true>(const uint64_t *, uint64_t, const MdCtl *, const uint32_t *,
                                        const uint32_t *, const uint32_t *, const uint32_t *, const uint64_t *,
                                        uint8_t *);

}  // namespace sznb
