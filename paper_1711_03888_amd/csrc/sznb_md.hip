// Molecular-dynamics modes (gfx950): R-index keys, partial radix sort of
// fixed index segments, particle reordering, CPC2000-style key coding.
//
// The paper's modes for MD snapshots (Sec. 5.2, Sec. 6): best_speed = SZ-LV
// on every field; best_tradeoff = SZ-LV after a partial radix sort of the
// R-index that skips the k least significant 3-bit digits (Table 5: segment
// 16384, k = 6); best_compression = CPC2000 coding of the sorted coordinate
// keys plus SZ-LV of the velocities in the same order.  The R-index
// interleaves the bits of the coordinates turned into integers by the error
// bound (Sec. 2, CPC2000 step 1-2); here the integers are the compressor's
// lattice indices, B bits each, x highest in each 3-bit digit.
//
//   md_keys     lattice indices of x, y, z -> 3B-bit interleaved key
//   md_sort     one workgroup per segment: stable LSD radix sort by key >> 3k
//   md_gather   apply the permutation to every field
//   cpc_count   per segment: key deltas, Rice parameter, coded size
//   cpc_offsets segment word offsets, coordinate stream header
//   cpc_pack    per segment: first key, parameter, Rice-coded deltas
//   cpc_decode  one wave per segment, one lane per 256 keys (entry points
//               stored in the stream): keys back, then lattice values
//   md_assemble container header and sub-stream copies
#include <type_traits>

#include "sznb_internal.h"

namespace sznb {

constexpr uint32_t kSeg = 16384;
constexpr uint32_t kSub = 256;   // keys per decoder entry point (kSeg / kSub = 64 lanes)
constexpr uint32_t kEscQ = 32;   // quotients from 32 on are escaped
constexpr uint32_t kCpcLdsWords = 16384;  // decoder: a segment's code words staged in LDS (64 KiB)
constexpr int kMT = 1024;
constexpr int kMW = kMT / kWave;

struct MdCtl {
  uint32_t B, keybits, nseg, status;
  uint64_t coord_bytes;          // CPC coordinate stream length
  uint64_t total;                // container length
};

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

__device__ inline int32_t md_lattice(float v, const FState *s) {
  double t = __dmul_rn(__dsub_rn((double)v, (double)s->mn), s->inv);
  return (int32_t)floor(__dadd_rn(t, 0.5));
}

// key bits per coordinate: the widest lattice span of the three
__global__ void md_bits(const FState *s0, const FState *s1, const FState *s2, MdCtl *ctl, uint64_t n) {
  if (threadIdx.x || blockIdx.x) return;
  const FState *s[3] = {s0, s1, s2};
  uint32_t B = 1, st = 0;
  for (int c = 0; c < 3; c++) {
    if (s[c]->status) st = (uint32_t)s[c]->status;
    uint64_t P = (uint64_t)s[c]->P, b = 0;
    while (P >> b) b++;
    if (b > B) B = (uint32_t)b;
  }
  if (!st && B > 21) st = (uint32_t)SZNB_EEBTOOSMALL;
  ctl->B = B;
  ctl->keybits = 3 * B;
  ctl->nseg = (uint32_t)((n + kSeg - 1) / kSeg);
  ctl->status = st;
}

__global__ void md_keys(const float *x, const float *y, const float *z, uint64_t n, const FState *s0,
                        const FState *s1, const FState *s2, const MdCtl *ctl, uint64_t *key, uint32_t *idx) {
  if (ctl->status) return;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t px = (uint64_t)(uint32_t)md_lattice(x[i], s0);
    const uint64_t py = (uint64_t)(uint32_t)md_lattice(y[i], s1);
    const uint64_t pz = (uint64_t)(uint32_t)md_lattice(z[i], s2);
    key[i] = (spread3(px) << 2) | (spread3(py) << 1) | spread3(pz);
    idx[i] = (uint32_t)i;
  }
}

__device__ inline uint64_t md_lanemask_lt() {
  const uint32_t l = lane_id();
  return l ? (~0ull >> (64 - l)) : 0ull;
}

// Stable sort of one segment's (key, idx) pairs by (key >> shift0), LSD on
// 8-bit digits, ping-pong between (k0, i0) and (k1, i1); each of the 16
// waves owns a contiguous slice and keeps its order.
__global__ __launch_bounds__(kMT) void md_sort(uint64_t *k0, uint32_t *i0, uint64_t *k1, uint32_t *i1, uint64_t n,
                                               uint32_t k_ignored, const MdCtl *ctl) {
  __shared__ uint32_t s_cnt[256 * kMW];
  __shared__ uint32_t s_tot[kMW];
  if (ctl->status) return;
  const uint32_t seg = blockIdx.x;
  const uint64_t base = (uint64_t)seg * kSeg;
  if (base >= n) return;
  const uint32_t m = (uint32_t)min((uint64_t)kSeg, n - base);
  const int t = threadIdx.x, w = t / kWave;
  const uint32_t shift0 = 3 * k_ignored;
  const uint32_t bits = ctl->keybits > shift0 ? ctl->keybits - shift0 : 0;
  const uint32_t passes = (bits + 7) / 8;
  uint64_t *ka = k0 + base, *kb = k1 + base;
  uint32_t *ia = i0 + base, *ib = i1 + base;
  const uint32_t segw = (m + kMW - 1) / kMW;
  const uint32_t beg = min(m, segw * w), end = min(m, beg + segw);
  // the wave's keys and indices of a pass are read once, in one round trip
  constexpr int kPL = kSeg / kMT;  // chunks of 64 per wave
  for (uint32_t ps = 0; ps < passes; ps++) {
    const uint32_t sh = shift0 + 8 * ps;
    uint64_t kv[kPL];
    uint32_t iv[kPL];
#pragma unroll
    for (int c = 0; c < kPL; c++) {
      const uint32_t i = beg + (uint32_t)c * kWave + lane_id();
      kv[c] = i < end ? ka[i] : 0ull;
      iv[c] = i < end ? ia[i] : 0u;
    }
    for (uint32_t i = t; i < 256u * kMW; i += kMT) s_cnt[i] = 0;
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kPL; c++)
      if (beg + (uint32_t)c * kWave + lane_id() < end) atomicAdd(&s_cnt[((kv[c] >> sh) & 255u) * kMW + w], 1u);
    __syncthreads();
    // exclusive scan over (digit, wave), digit-major
    uint32_t loc = 0;
    for (int j = 0; j < 4; j++) loc += s_cnt[4 * t + j];
    const uint32_t inc = wave_incl_scan(loc);
    if (lane_id() == kWave - 1) s_tot[w] = inc;
    __syncthreads();
    uint32_t run = inc - loc;
    for (int j = 0; j < w; j++) run += s_tot[j];
    for (int j = 0; j < 4; j++) { const uint32_t v = s_cnt[4 * t + j]; s_cnt[4 * t + j] = run; run += v; }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kPL; c++) {
      const uint32_t i = beg + (uint32_t)c * kWave + lane_id();
      const bool valid = i < end;
      const uint32_t dg = (uint32_t)((kv[c] >> sh) & 255u);
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
        kb[pos] = kv[c];
        ib[pos] = iv[c];
        if (rank == cnt - 1) s_cnt[dg * kMW + w] += cnt;
      }
      __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    uint64_t *tk = ka; ka = kb; kb = tk;
    uint32_t *ti = ia; ia = ib; ib = ti;
  }
  // leave the result in (k0, i0)
  if (passes & 1u) {
    for (uint32_t i = t; i < m; i += kMT) { kb[i] = ka[i]; ib[i] = ia[i]; }
  }
}

__global__ void md_gather(const float *src, float *dst, const uint32_t *perm, uint64_t n, const MdCtl *ctl) {
  if (ctl->status) return;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    dst[i] = src[perm[i]];
}

// ------------------------------------------------------------- CPC2000

// Rice cost of a delta with parameter r
__device__ inline uint64_t rice_cost(uint64_t d, uint32_t r, uint32_t keybits) {
  const uint64_t q = d >> r;
  return q >= kEscQ ? (uint64_t)(kEscQ + keybits) : q + 1 + r;
}

// per segment: parameter r = argmin_r sum cost (ties to the smaller r) and
// the segment's coded bits (first key, 6-bit parameter, deltas)
__global__ __launch_bounds__(kMT) void cpc_count(const uint64_t *key, uint64_t n, const MdCtl *ctl,
                                                 uint32_t *seg_r, uint32_t *seg_bits) {
  __shared__ unsigned long long s_sum[kMW];
  __shared__ unsigned long long s_best;
  __shared__ uint32_t s_r;
  if (ctl->status) return;
  const uint32_t seg = blockIdx.x;
  const uint64_t base = (uint64_t)seg * kSeg;
  if (base >= n) return;
  const uint32_t m = (uint32_t)min((uint64_t)kSeg, n - base);
  const uint32_t kb = ctl->keybits;
  const int t = threadIdx.x, w = t / kWave;
  if (t == 0) { s_best = ~0ull; s_r = 0; }
  // this thread's deltas, read once (kSeg / kMT of them)
  constexpr int kPer = kSeg / kMT;
  uint64_t dl[kPer];
#pragma unroll
  for (int j = 0; j < kPer; j++) {
    const uint32_t i = 1 + t + (uint32_t)j * kMT;
    dl[j] = i < m ? key[base + i] - key[base + i - 1] : 0u;
  }
  for (uint32_t r = 0; r <= kb; r++) {
    unsigned long long c = 0;
#pragma unroll
    for (int j = 0; j < kPer; j++)
      if (1 + t + (uint32_t)j * kMT < m) c += rice_cost(dl[j], r, kb);
    c = wave_sum(c);
    if (lane_id() == 0) s_sum[w] = c;
    __syncthreads();
    if (t == 0) {
      unsigned long long tot = 0;
      for (int j = 0; j < kMW; j++) tot += s_sum[j];
      if (tot < s_best) { s_best = tot; s_r = r; }
    }
    __syncthreads();
  }
  if (t == 0) {
    seg_r[seg] = s_r;
    seg_bits[seg] = (uint32_t)(kb + 6 + (m > 1 ? s_best : 0ull));
  }
}

// Coordinate stream header (104 bytes):
//   "SZCP" u16 2 u8 B u8 0 u64 n u32 nseg u32 seg u32 keybits
//   f32 (mn, mx) x3, f64 eb_abs x3, f64 step x3, padding to 104
// then u32 seg_bits[nseg] (padded to 8 bytes), then the entry points: for
// every segment and every 256 keys of it, u32 bit offset (from the segment
// start) of that key's code (padded to 8 bytes), then the segments' words.
constexpr uint32_t kCpHdr = 104;
__host__ __device__ inline uint64_t cpc_entries(uint64_t n) {  // entry points of all segments
  const uint64_t nseg = (n + kSeg - 1) / kSeg;
  return nseg ? (nseg - 1) * (kSeg / kSub) + (n - (nseg - 1) * kSeg + kSub - 1) / kSub : 0;
}

__global__ void cpc_offsets(const uint32_t *seg_bits, uint32_t nseg_max, uint64_t n, MdCtl *ctl, const FState *s0,
                            const FState *s1, const FState *s2, uint8_t *cs, uint32_t *seg_woff) {
  if (threadIdx.x || blockIdx.x) return;
  if (ctl->status) return;
  const uint32_t nseg = ctl->nseg;
  uint32_t o = 0;
  for (uint32_t s = 0; s < nseg && s < nseg_max; s++) {
    seg_woff[s] = o;
    o += (seg_bits[s] + 31) / 32;
  }
  const uint64_t tab = align8((uint64_t)4 * nseg) + align8(4ull * cpc_entries(n));
  ctl->coord_bytes = kCpHdr + tab + 4ull * o;
  for (uint32_t i = 0; i < kCpHdr; i += 4) *reinterpret_cast<uint32_t *>(cs + i) = 0u;
  *reinterpret_cast<uint32_t *>(cs + 0) = 0x50435A53u;  // "SZCP"
  *reinterpret_cast<uint32_t *>(cs + 4) = 2u | (ctl->B << 16);
  *reinterpret_cast<uint32_t *>(cs + 8) = (uint32_t)n;
  *reinterpret_cast<uint32_t *>(cs + 12) = (uint32_t)(n >> 32);
  *reinterpret_cast<uint32_t *>(cs + 16) = nseg;
  *reinterpret_cast<uint32_t *>(cs + 20) = kSeg;
  *reinterpret_cast<uint32_t *>(cs + 24) = ctl->keybits;
  const FState *s[3] = {s0, s1, s2};
  for (int c = 0; c < 3; c++) {
    *reinterpret_cast<float *>(cs + 28 + 8 * c) = s[c]->mn;
    *reinterpret_cast<float *>(cs + 32 + 8 * c) = s[c]->mx;
    const uint64_t eb = (uint64_t)__double_as_longlong(s[c]->eb_abs);
    const uint64_t stp = (uint64_t)__double_as_longlong(s[c]->step);
    *reinterpret_cast<uint32_t *>(cs + 52 + 8 * c) = (uint32_t)eb;
    *reinterpret_cast<uint32_t *>(cs + 56 + 8 * c) = (uint32_t)(eb >> 32);
    *reinterpret_cast<uint32_t *>(cs + 76 + 8 * c) = (uint32_t)stp;
    *reinterpret_cast<uint32_t *>(cs + 80 + 8 * c) = (uint32_t)(stp >> 32);
  }
  for (uint32_t s2i = 0; s2i < nseg; s2i++) *reinterpret_cast<uint32_t *>(cs + kCpHdr + 4ull * s2i) = seg_bits[s2i];
  if (nseg & 1u) *reinterpret_cast<uint32_t *>(cs + kCpHdr + 4ull * nseg) = 0u;
  const uint64_t ne = cpc_entries(n);
  if (ne & 1u) *reinterpret_cast<uint32_t *>(cs + kCpHdr + align8(4ull * nseg) + 4ull * ne) = 0u;
}

// bit writer over LDS-free global words: whole words are stored, words that
// may be shared with a neighbour thread are OR-ed (the region is zeroed first)
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

__global__ __launch_bounds__(kMT) void cpc_pack(const uint64_t *key, uint64_t n, const MdCtl *ctl, const uint32_t *seg_r,
                                                const uint32_t *seg_bits, const uint32_t *seg_woff, uint8_t *cs) {
  __shared__ unsigned long long s_tot[kMW];
  if (ctl->status) return;
  const uint32_t seg = blockIdx.x;
  const uint64_t base = (uint64_t)seg * kSeg;
  if (base >= n) return;
  const uint32_t m = (uint32_t)min((uint64_t)kSeg, n - base);
  const uint32_t kb = ctl->keybits, r = seg_r[seg];
  const int t = threadIdx.x, w = t / kWave;
  const uint64_t etab = kCpHdr + align8((uint64_t)4 * ctl->nseg);
  const uint64_t tab = etab + align8(4ull * cpc_entries(n));
  uint32_t *words = reinterpret_cast<uint32_t *>(cs + tab) + seg_woff[seg];
  uint32_t *ent = reinterpret_cast<uint32_t *>(cs + etab) + (uint64_t)seg * (kSeg / kSub);
  const uint32_t nw = (seg_bits[seg] + 31) / 32;
  for (uint32_t i = t; i < nw; i += kMT) words[i] = 0u;
  __syncthreads();
  // thread t codes deltas i in [lo, hi); bit offsets by a workgroup scan
  const uint32_t per = (m + kMT - 1) / kMT;
  const uint32_t lo = min(m, t * per), hi = min(m, lo + per);
  unsigned long long mine = 0;
  for (uint32_t i = max(lo, 1u); i < hi; i++) mine += rice_cost(key[base + i] - key[base + i - 1], r, kb);
  if (lo == 0 && hi > 0) mine += kb + 6;
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
    for (uint32_t i = lo; i < hi; i++) {
      if ((i & (kSub - 1)) == 0) ent[i / kSub] = (uint32_t)(b.pos + b.na);
      if (i == 0) {
        wb_put_wide(b, key[base], kb);
        wb_put(b, r, 6);
        continue;
      }
      const uint64_t d = key[base + i] - key[base + i - 1];
      const uint64_t q = d >> r;
      if (q >= kEscQ) {
        wb_put(b, 0xffffffffull, kEscQ);
        wb_put_wide(b, d, kb);
      } else {
        // q ones then a zero, in pieces of at most 32 bits
        uint32_t ones = (uint32_t)q;
        while (ones >= 32u) { wb_put(b, 0xffffffffull, 32u); ones -= 32u; }
        wb_put(b, ((1ull << (ones + 1)) - 2ull), ones + 1);
        wb_put_wide(b, d & ((r == 64) ? ~0ull : ((1ull << r) - 1)), r);
      }
    }
    if (b.na) wb_flush_word(b, b.pos >> 5, (uint32_t)(b.acc >> 32));
  }
}

// One wave per segment, one lane per 256 keys: each lane starts at its entry
// point, sums its deltas (pass 1), the wave scans the sums, and each lane
// decodes again writing keys and coordinates (pass 2).  Every read is checked
// against the segment's bit count and the stream length, and every lane must
// end exactly at the next lane's entry point; a stream that fails a check
// sets ECORRUPT.
__global__ __launch_bounds__(kWave) void cpc_decode(const uint8_t *cs, uint64_t cs_len, uint64_t n, float *ox,
                                                    float *oy, float *oz, int *status) {
  const uint32_t seg = blockIdx.x, lane = threadIdx.x;
  if (cs_len < kCpHdr) { if (seg == 0 && lane == 0) atomicCAS(status, 0, SZNB_ECORRUPT); return; }
  const uint32_t nseg = *reinterpret_cast<const uint32_t *>(cs + 16);
  const uint32_t kb = *reinterpret_cast<const uint32_t *>(cs + 24);
  const uint64_t nhdr = (uint64_t)*reinterpret_cast<const uint32_t *>(cs + 8) |
                        ((uint64_t)*reinterpret_cast<const uint32_t *>(cs + 12) << 32);
  const uint64_t etab = kCpHdr + align8(4ull * nseg);
  const uint64_t tab = etab + align8(4ull * cpc_entries(n));
  if (*reinterpret_cast<const uint32_t *>(cs) != 0x50435A53u || (*reinterpret_cast<const uint32_t *>(cs + 4) & 0xffffu) != 2u ||
      nhdr != n || nseg != (n + kSeg - 1) / kSeg || kb > 63 || kb == 0 || tab > cs_len) {
    if (seg == 0 && lane == 0) atomicCAS(status, 0, SZNB_ECORRUPT);
    return;
  }
  if (seg >= nseg) return;
  float mn[3];
  double step[3];
  for (int c = 0; c < 3; c++) {
    mn[c] = *reinterpret_cast<const float *>(cs + 28 + 8 * c);
    const uint64_t lo = *reinterpret_cast<const uint32_t *>(cs + 76 + 8 * c);
    const uint64_t hi = *reinterpret_cast<const uint32_t *>(cs + 80 + 8 * c);
    step[c] = __longlong_as_double((long long)(lo | (hi << 32)));
  }
  const gptr<const uint32_t> sb = G(reinterpret_cast<const uint32_t *>(cs + kCpHdr));
  uint64_t woff = 0;
  for (uint32_t s = lane; s < seg; s += kWave) woff += (sb[s] + 31) / 32;
  woff = wave_sum(woff);
  const uint64_t nbits = sb[seg];
  const uint64_t avail = (cs_len - tab) / 4;
  bool bad = woff + (nbits + 31) / 32 > avail;
  const uint32_t *wp = reinterpret_cast<const uint32_t *>(cs + tab) + woff;
  const gptr<const uint32_t> ent = G(reinterpret_cast<const uint32_t *>(cs + etab)) + (uint64_t)seg * (kSeg / kSub);
  const uint64_t base = (uint64_t)seg * kSeg;
  const uint32_t m = (uint32_t)min((uint64_t)kSeg, n - base);
  const uint32_t k0 = lane * kSub, k1 = min(m, k0 + kSub);  // this lane's keys
  const bool active = k0 < m;
  // Bit reader of this lane: a 64-bit window holding the bits from pos on
  // (more than 32 of them after every refill), words past the segment read
  // as zero; a read that would pass nbits marks the segment corrupt.
  const gptr<const uint32_t> gw = G(wp);
  const uint64_t nw = (nbits + 31) / 32;
  // the segment's words are staged in LDS when they fit (coalesced, sixteen
  // loads per lane in flight before they are stored; both passes then
  // refill from LDS)
  __shared__ uint32_t s_seg[kCpcLdsWords];
  const bool in_lds = !bad && nw <= kCpcLdsWords;
  if (in_lds)
    for (uint32_t i0 = 0; i0 < nw; i0 += 16u * kWave) {
      uint32_t a[16];
#pragma unroll
      for (int u = 0; u < 16; u++) {
        const uint32_t i = i0 + (uint32_t)u * kWave + lane;
        a[u] = i < nw ? gw[i] : 0u;
      }
#pragma unroll
      for (int u = 0; u < 16; u++) {
        const uint32_t i = i0 + (uint32_t)u * kWave + lane;
        if (i < nw) s_seg[i] = a[u];
      }
    }
  __syncthreads();
  // The bit reader refills from LDS or from global memory, decided once per
  // segment: a refill that could take either path made the compiler wait
  // for every vector-memory operation in flight (pass 2's stores) at each
  // refill.
  const auto run = [&](auto lds) {
    constexpr bool kL = decltype(lds)::value;
    auto word = [&](uint64_t i) -> uint32_t { return i >= nw ? 0u : (kL ? s_seg[i] : gw[i]); };
    uint64_t pos = 0, buf = 0, wi = 0;
    uint32_t nv = 0;
    auto seek = [&](uint64_t p) {
      pos = p;
      wi = p >> 5;
      const uint32_t sh = (uint32_t)(p & 31u);
      const uint64_t w0 = word(wi), w1 = word(wi + 1);
      buf = ((w0 << 32) | w1) << sh;
      nv = 64u - sh;
      wi += 2;
    };
    auto skip = [&](uint32_t nb) {  // nb <= 32
      buf = nb ? buf << nb : buf;
      nv -= nb;
      pos += nb;
      if (nv <= 32u) {
        buf |= (uint64_t)word(wi) << (32u - nv);
        nv += 32u;
        wi++;
      }
    };
    auto take = [&](uint32_t nb) -> uint64_t {  // nb <= 32
      if (!nb) return 0;
      if (pos + nb > nbits) { bad = true; return 0; }
      const uint64_t v = buf >> (64u - nb);
      skip(nb);
      return v;
    };
    auto take_wide = [&](uint32_t nb) -> uint64_t {
      if (nb > 32u) { const uint64_t hi = take(nb - 32u); return (hi << 32) | take(32u); }
      return take(nb);
    };
    // the Rice parameter follows the first key
    uint32_t r = 0;
    if (!bad) {
      seek(kb);
      r = (uint32_t)take(6);
      if (r > kb) bad = true;
    }
    const uint64_t start = active ? ent[lane] : 0;
    const uint64_t stop = (k1 < m) ? ent[lane + 1] : nbits;
    if (active && (start > stop || stop > nbits || (lane == 0 && start != 0))) bad = true;
    auto next = [&](uint32_t i) -> uint64_t {  // delta of key i (the raw key for i = 0)
      if (i == 0) { const uint64_t k = take_wide(kb); (void)take(6); return k; }
      // unary quotient: the ones before the first zero, at most kEscQ (= 32)
      const uint32_t ones = ~(uint32_t)(buf >> 32);
      const uint32_t q = ones ? (uint32_t)__clz(ones) : kEscQ;
      const uint32_t ub = q < kEscQ ? q + 1u : kEscQ;
      if (pos + ub > nbits) { bad = true; return 0; }
      skip(ub);
      if (q == kEscQ) return take_wide(kb);
      return ((uint64_t)q << r) | take_wide(r);
    };
    // pass 1: sum of this lane's deltas
    uint64_t sum = 0;
    if (active && !bad) {
      seek(start);
      for (uint32_t i = k0; i < k1 && !bad; i++) sum += next(i);
      if (pos != stop) bad = true;
    }
    // exclusive prefix of the lane sums
    uint64_t inc = sum;
    for (int d = 1; d < kWave; d <<= 1) {
      const uint64_t o = __shfl_up(inc, d, kWave);
      if ((int)lane >= d) inc += o;
    }
    const bool any_bad = __ballot(bad) != 0;
    if (any_bad) {
      if (lane == 0) atomicCAS(status, 0, SZNB_ECORRUPT);
      return;
    }
    // pass 2: keys and coordinates (global stores: flat stores in flight
    // would hold up every LDS refill of the bit reader)
    if (!active) return;
    uint64_t k = inc - sum;
    seek(start);
    const gptr<float> gx = G(ox), gy = G(oy), gz = G(oz);
    for (uint32_t i = k0; i < k1; i++) {
      k += next(i);
      const uint32_t px = compact3(k >> 2), py = compact3(k >> 1), pz = compact3(k);
      gx[base + i] = (float)fma((double)(int32_t)px, step[0], (double)mn[0]);
      gy[base + i] = (float)fma((double)(int32_t)py, step[1], (double)mn[1]);
      gz[base + i] = (float)fma((double)(int32_t)pz, step[2], (double)mn[2]);
    }
  };
  if (in_lds) run(std::true_type{}); else run(std::false_type{});
}

// Container (96-byte header): "SZMD" u16 1 u8 mode u8 nf u64 n u32 seg
// u32 k_ignored u64 total u64 offsets[6]; sub-streams 8-byte aligned.
constexpr uint32_t kMdHdr = 96;

__global__ void md_assemble(uint8_t *out, uint64_t out_cap, uint64_t *out_len, const uint8_t *const *subs,
                            const uint64_t *sub_len_dev, int nsub, int md_mode, int nf, uint64_t n, uint32_t k_ignored,
                            const MdCtl *ctl, int *status) {
  // every workgroup computes the same offsets
  uint64_t offs[6] = {0, 0, 0, 0, 0, 0}, o = kMdHdr;
  uint64_t lens[6] = {0, 0, 0, 0, 0, 0};
  const bool bad = ctl->status != 0;
  for (int i = 0; i < nsub; i++) {
    lens[i] = (md_mode == 2 && i == 0) ? ctl->coord_bytes : sub_len_dev[i];
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
    for (uint64_t j = tid; j < padded; j += stride) out[offs[i] + j] = j < lens[i] ? subs[i][j] : 0;
  }
  if (tid == 0) {
    uint32_t *h = reinterpret_cast<uint32_t *>(out);
    for (int i = 0; i < (int)kMdHdr / 4; i++) h[i] = 0u;
    h[0] = 0x444D5A53u;  // "SZMD"
    h[1] = 1u | ((uint32_t)md_mode << 16) | ((uint32_t)nf << 24);
    h[2] = (uint32_t)n; h[3] = (uint32_t)(n >> 32);
    h[4] = kSeg;
    h[5] = k_ignored;
    h[6] = (uint32_t)total; h[7] = (uint32_t)(total >> 32);
    for (int i = 0; i < 6; i++) { h[8 + 2 * i] = (uint32_t)offs[i]; h[9 + 2 * i] = (uint32_t)(offs[i] >> 32); }
    if (out_len) *out_len = total;
  }
}

}  // namespace sznb
