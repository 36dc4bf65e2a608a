// Compression kernels of the sznb library (gfx950, wave64).
//
// Pipeline over a table of fields (one field or a batch share the code):
//   k_init    clear per-call state (look-back words, tickets, counters)
//   k_range   per-block exact min / max / non-finite flag      (reads 4 B/value)
//   k_params  per-field range R, bound, lattice step, header    (Problem Statement)
//   k_quant   lattice quantization, LV/LCF/QCF residuals, per-block best-fit
//             trial, one code histogram per predictor          (reads 4 B/value)
//   k_huff    canonical Huffman code per (field, predictor)     (Sec. 2 / 5.2)
//   k_books   codebook sections and payload offset of each stream
//   k_pack    codewords, block bit counts, decoupled look-back scan of block
//             sizes, MSB-first bit packing, escapes             (reads 4 B/value,
//             writes the payload)
#include "sznb_internal.h"

namespace sznb {


// ------------------------------------------------------------------ init

// Grid (kInitParts, min(nf, 65535)): workgroup (x, y) clears part x of the
// histograms of fields y, y + gridDim.y, ...; part 0 also resets their
// state; every workgroup clears its share of the look-back words.
constexpr int kInitParts = 16;
__global__ void k_init(const CField *__restrict__ F, int nf, GCtl *gc, uint64_t *lbflag_all,
                       uint64_t total_blocks) {
  const uint64_t wg = (uint64_t)blockIdx.y * gridDim.x + blockIdx.x;
  const uint64_t tid = wg * blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * gridDim.y * blockDim.x;
  if (tid == 0) gc->ticket = 0;
  if (tid < kHuffSlots) gc->hdone[tid] = 0;
  for (uint64_t g = tid; g < total_blocks; g += stride) lbflag_all[g] = 0;
  for (int f = blockIdx.y; f < nf; f += gridDim.y) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      FState *s = F[f].st;
      s->status = 0;
      s->is_const = 0;
      s->blocks_done = 0;
      s->fallbacks = 0;
      s->payload_words = 0;
      s->off_payload = 0;
      for (int k = 0; k < 3; k++) { s->nsym[k] = 0; s->maxlen[k] = 0; }
    }
    // code histograms start from zero on every call
    uint4 *h = reinterpret_cast<uint4 *>(F[f].hist);
    const uint64_t n4 = (uint64_t)F[f].nhist * kNSyms / 4;
    const uint64_t part = (n4 + kInitParts - 1) / kInitParts;
    const uint64_t lo = part * blockIdx.x, hi = min(n4, lo + part);
    for (uint64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) h[i] = make_uint4(0u, 0u, 0u, 0u);
  }
}

// ----------------------------------------------------------------- range

__global__ __launch_bounds__(kThreads) void k_range(const CField *__restrict__ F, int nf,
                                                    const uint64_t *__restrict__ fb0, uint64_t total) {
  __shared__ uint32_t s_mn[kThreads / kWave], s_mx[kThreads / kWave], s_bad[kThreads / kWave];
  const int t = threadIdx.x, w = t / kWave;
  for (uint64_t g = blockIdx.x; g < total; g += gridDim.x) {
    const int f = find_field(fb0, nf, g);
    const CField &c = F[f];
    const uint64_t b = g - c.gblock0;
    const uint64_t i0 = b << c.log2S;
    const uint32_t len = (uint32_t)min((uint64_t)c.S, c.n - i0);
    const gptr<const float> x = G(c.x) + i0;
    uint32_t mn = 0xffffffffu, mx = 0u, bad = 0u;
    for (uint32_t j = 4u * t; j < len; j += 4u * kThreads) {
      float v[4];
      if (j + 4 <= len) {
        const f32x4 q = *reinterpret_cast<gptr<const f32x4>>(x + j);
        v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
      } else {
        for (int e = 0; e < 4; e++) v[e] = j + e < len ? x[j + e] : x[j];
      }
#pragma unroll
      for (int e = 0; e < 4; e++) {
        if (!isfinite(v[e])) { bad = 1u; continue; }
        uint32_t k = float_key(v[e]);
        mn = min(mn, k);
        mx = max(mx, k);
      }
    }
    mn = wave_min_u32(mn);
    mx = wave_max_u32(mx);
    bad = wave_max_u32(bad);
    if ((t & (kWave - 1)) == 0) { s_mn[w] = mn; s_mx[w] = mx; s_bad[w] = bad; }
    __syncthreads();
    if (t == 0) {
      for (int i = 1; i < kThreads / kWave; i++) {
        mn = min(mn, s_mn[i]);
        mx = max(mx, s_mx[i]);
        bad |= s_bad[i];
      }
      const gptr<uint32_t> bs = G(c.blkstat) + 3 * b;
      bs[0] = mn;
      bs[1] = mx;
      bs[2] = bad;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- params

__device__ inline void put32(uint8_t *o, uint64_t off, uint32_t v) { *reinterpret_cast<uint32_t *>(o + off) = v; }
__device__ inline void put64(uint8_t *o, uint64_t off, uint64_t v) {
  put32(o, off, (uint32_t)v);
  put32(o, off + 4, (uint32_t)(v >> 32));
}
__device__ inline void putf64(uint8_t *o, uint64_t off, double v) { put64(o, off, (uint64_t)__double_as_longlong(v)); }

// One workgroup per field: reduce the block extrema, derive the bound and the
// lattice step, write the fixed part of the header.
//   R = max - min; eb_abs = eb_rel * R when relative (Problem Statement).
//   step = 2 (eb_abs - g), g = 2 ulp_f32(max |x|): the float32 rounding of the
//   reconstructed value then never carries the error past eb_abs.
__global__ __launch_bounds__(kThreads) void k_params(const CField *__restrict__ F) {
  __shared__ uint32_t s_mn[kThreads], s_mx[kThreads], s_bad[kThreads];
  const CField &c = F[blockIdx.x];
  FState *st = c.st;
  const int t = threadIdx.x;
  uint32_t mn = 0xffffffffu, mx = 0u, bad = 0u;
  const gptr<const uint32_t> bs = G(static_cast<const uint32_t *>(c.blkstat));
#pragma unroll 8
  for (uint32_t b = t; b < c.nblocks; b += kThreads) {
    mn = min(mn, bs[3 * b]);
    mx = max(mx, bs[3 * b + 1]);
    bad |= bs[3 * b + 2];
  }
  s_mn[t] = mn; s_mx[t] = mx; s_bad[t] = bad;
  __syncthreads();
  for (int h = kThreads / 2; h > 0; h >>= 1) {
    if (t < h) {
      s_mn[t] = min(s_mn[t], s_mn[t + h]);
      s_mx[t] = max(s_mx[t], s_mx[t + h]);
      s_bad[t] |= s_bad[t + h];
    }
    __syncthreads();
  }
  __shared__ int s_ok;
  uint8_t *o = c.out;
  if (t == 0) {
    int status = 0;
    uint32_t is_const = 0;
    float fmn = 0.0f, fmx = 0.0f;
    double R = 0.0, eb_abs = 0.0, step = 0.0, inv = 0.0;
    int64_t P = 0;
    if (c.n == 0) {
      is_const = 1;
    } else if (s_bad[0]) {
      status = SZNB_ENONFINITE;
    } else {
      fmn = key_float(s_mn[0]);
      fmx = key_float(s_mx[0]);
      if (fmn == 0.0f) fmn = 0.0f;
      if (fmx == 0.0f) fmx = 0.0f;
      R = __dsub_rn((double)fmx, (double)fmn);
      eb_abs = c.eb_rel ? __dmul_rn(c.eb, R) : c.eb;
      if (R == 0.0) {
        is_const = 1;
      } else {
        float am = fabsf(fmn) > fabsf(fmx) ? fabsf(fmn) : fabsf(fmx);
        double ebp = __dsub_rn(eb_abs, guard_of(am));
        if (!(ebp > 0.0)) {
          status = SZNB_EEBTOOSMALL;
        } else {
          step = __dmul_rn(2.0, ebp);
          inv = __ddiv_rn(1.0, step);
          double tt = __dmul_rn(__dsub_rn((double)fmx, (double)fmn), inv);
          double Pd = floor(__dadd_rn(tt, 0.5));
          if (Pd > (double)kPMax) status = SZNB_EEBTOOSMALL;
          else P = (int64_t)Pd;
        }
      }
    }
    st->status = status;
    st->is_const = is_const;
    st->mn = fmn; st->mx = fmx; st->R = R; st->eb_abs = eb_abs; st->step = step; st->inv = inv; st->P = P;
    s_ok = status == 0 && !is_const;
    if (status != 0) {
      if (c.out_len) *c.out_len = 0;
    } else {
      // header words 0..127
      for (int i = 0; i < kHdr; i += 4) put32(o, i, 0u);
      put32(o, H_MAGIC, kMagic);
      put32(o, H_VERSION, (uint32_t)1 | ((uint32_t)c.policy << 16) |
                              ((uint32_t)((is_const ? 1u : 0u) | (c.eb_rel << 1)) << 24));
      put64(o, H_N, c.n);
      put32(o, H_S, c.S);
      put32(o, H_MN, __float_as_uint(fmn));
      put32(o, H_MX, __float_as_uint(fmx));
      putf64(o, H_EBABS, eb_abs);
      if (is_const) {
        put64(o, H_TOTAL, kHdr);
        if (c.out_len) *c.out_len = kHdr;
      } else {
        put32(o, H_NB, c.nblocks);
        putf64(o, H_STEP, step);
        put64(o, H_OFF_PRED, c.sec.pred);
        put64(o, H_OFF_PFIRST, c.sec.pfirst);
        put64(o, H_OFF_CWORDS, c.sec.cwords);
        put64(o, H_OFF_NESC, c.sec.nesc);
        put64(o, H_OFF_BOOKS, c.sec.books);
      }
    }
  }
  __syncthreads();
  if (s_ok) {
    // zero the alignment padding after each fixed-size table
    const uint64_t nb = c.nblocks;
    if (t < 8) {
      if (c.policy >= 2 && c.sec.pred + nb + t < c.sec.pfirst) o[c.sec.pred + nb + t] = 0;
      if (c.sec.pfirst + 4 * nb + t < c.sec.cwords) o[c.sec.pfirst + 4 * nb + t] = 0;
      if (c.sec.cwords + 2 * nb + t < c.sec.nesc) o[c.sec.cwords + 2 * nb + t] = 0;
      if (c.sec.nesc + 2 * nb + t < c.sec.books) o[c.sec.nesc + 2 * nb + t] = 0;
    }
  }
}

// --------------------------------------------------- quantize and select

__device__ inline int32_t lattice_of(float x, float mn, double inv) {
  double t = __dmul_rn(__dsub_rn((double)x, (double)mn), inv);
  return (int32_t)floor(__dadd_rn(t, 0.5));
}

// This thread's E contiguous values of a block (16-byte loads when the run
// is whole; the tail of a ragged block reads as mn).
template <int E>
__device__ inline void load_raw(gptr<const float> x_block, uint32_t len, float mn, float (&v)[E]) {
  const int t = threadIdx.x;
  const gptr<const float> x = x_block + (uint64_t)t * E;
  if ((uint32_t)(t + 1) * E <= len) {
#pragma unroll
    for (int e = 0; e < E; e += 4) {
      const f32x4 q = *reinterpret_cast<gptr<const f32x4>>(x + e);
      v[e] = q.x; v[e + 1] = q.y; v[e + 2] = q.z; v[e + 3] = q.w;
    }
  } else {
#pragma unroll
    for (int e = 0; e < E; e++) v[e] = ((uint32_t)t * E + e < len) ? x[e] : mn;
  }
}

// Lattice index of this thread's values relative to the block anchor
// (d_j = p_j - p_0), and the three values that precede the thread's run
// (zero before the block start).
template <int E>
__device__ inline void block_d_from_raw(const float (&v)[E], float mn, double inv, int32_t (&d)[E], int32_t (&pv)[3],
                                        int32_t *s_tail, int32_t &p0_out, int32_t *s_p0) {
  const int t = threadIdx.x;
  int32_t p[E];
#pragma unroll
  for (int e = 0; e < E; e++) p[e] = lattice_of(v[e], mn, inv);
  // the anchor and every thread's last three lattice values, one barrier
  if (t == 0) *s_p0 = p[0];
  s_tail[3 * t + 0] = p[E - 1];
  s_tail[3 * t + 1] = p[E - 2];
  s_tail[3 * t + 2] = p[E - 3];
  __syncthreads();
  const int32_t p0 = *s_p0;
#pragma unroll
  for (int e = 0; e < E; e++) d[e] = (int32_t)((uint32_t)p[e] - (uint32_t)p0);
  if (t == 0) { pv[0] = pv[1] = pv[2] = 0; }
  else {
#pragma unroll
    for (int i = 0; i < 3; i++) pv[i] = (int32_t)((uint32_t)s_tail[3 * (t - 1) + i] - (uint32_t)p0);
  }
  p0_out = p0;
}

template <int E>
__device__ inline void load_block_d(const CField &c, float mn, double inv, uint64_t i0, uint32_t len,
                                    int32_t (&d)[E], int32_t (&pv)[3], int32_t *s_tail, int32_t &p0_out,
                                    int32_t *s_p0) {
  float v[E];
  load_raw<E>(G(c.x) + i0, len, mn, v);
  block_d_from_raw<E>(v, mn, inv, d, pv, s_tail, p0_out, s_p0);
}

// residual of predictor k at element e given the run d[] and its three
// predecessors pv = (d_{-1}, d_{-2}, d_{-3})
template <int E>
__device__ inline int32_t residual_at(const int32_t (&d)[E], const int32_t (&pv)[3], int e, int k) {
  auto D = [&](int i) -> uint32_t { return (uint32_t)(i >= 0 ? d[i] : pv[-i - 1]); };
  uint32_t a0 = D(e) - D(e - 1);
  if (k == 0) return (int32_t)a0;
  uint32_t a1 = D(e - 1) - D(e - 2);
  uint32_t b0 = a0 - a1;
  if (k == 1) return (int32_t)b0;
  uint32_t a2 = D(e - 2) - D(e - 3);
  return (int32_t)(b0 - (a1 - a2));
}

// Residual classes of the best-fit estimate: zigzag z < 4 is its own class;
// a larger z of bit length b is class 4 + 2(b-3) + (bit b-2 of z) with b-2
// extra bits; an escape (|r| >= 32768) is class 32 with 32 extra bits.
// Class-counter slots of the trial, per predictor: class 0 at slot 0, class
// c >= 1 at slot c + 2 (slots 1 and 2 stay empty).  For a residual r with
// zigzag code z < 65535, the float z + 0.5 (exact) has unbiased exponent
// bitlen(z) - 1 and, below it, bit bitlen(z) - 2 of z as its first mantissa
// bit, so (bits(z + 0.5) >> 22) - 252 is that slot; z = 0 lands on slot 0.
// An escape (z >= 65535, class 32) takes slot 34.
constexpr int kClsSlots = kNClass + 2;
constexpr int kClsCopies = 8, kClsStride = 108;  // class-counter copies of the trial
__device__ inline uint32_t class_slot_biased(int32_t r) {  // slot + 252
  const uint32_t z = ((uint32_t)r << 1) ^ (uint32_t)(r >> 31);
  const uint32_t u = __float_as_uint((float)z + 0.5f) >> 22;
  return z >= 65535u ? 34u + 252u : u;
}
// extra bits of a class: bitlen(z) - 2 for c >= 4, 32 for an escape
__device__ inline uint32_t class_extra(uint32_t c) { return c == 32u ? 32u : (c < 4u ? 0u : (c - 2u) >> 1); }

// Exhaustive trial of one block: the two-part size estimate of LV, LCF and
// QCF residuals (classes of res_class, 2^-16 bit units), argmin with ties to
// the lowest predictor.  Leaves the costs in s_cost and the choice in
// *s_pred; all threads of the workgroup take part.
template <int E>
__device__ inline void block_trial(const int32_t (&d)[E], const int32_t (&pv)[3], uint32_t len,
                                   const uint32_t *__restrict__ logt, uint32_t *s_cls,
                                   unsigned long long *s_cost, int *s_pred) {
  const int t = threadIdx.x;
  // kClsCopies copies of the 3 x 35 slots, lane l of a wave on copy l mod 8:
  // a slot hit by a whole wave costs 8 serialised updates, not 64 (the
  // copies' strides put one slot of all copies on distinct banks)
  for (int i = t; i < kClsCopies * kClsStride; i += kThreads) s_cls[i] = 0;
  if (t < 3) s_cost[t] = 0;
  __syncthreads();
  // per predictor, the address of slot 0 minus 252 slots
  uint32_t *my = s_cls + (t & (kClsCopies - 1)) * kClsStride;
#pragma unroll
  for (int e = 0; e < E; e++) {
    if ((uint32_t)t * E + e < len) {
#pragma unroll
      for (int k = 0; k < 3; k++) {
        const uint32_t slot = class_slot_biased(residual_at<E>(d, pv, e, k)) - 252u;
        atomicAdd(&my[k * kClsSlots + slot], 1u);
      }
    }
  }
  __syncthreads();
  if (t < 3 * kNClass) {
    const uint32_t k = (uint32_t)t / kNClass, c = (uint32_t)t % kNClass;
    const uint32_t slot = k * kClsSlots + (c ? c + 2u : 0u);
    uint32_t n_c = 0;
    for (int j = 0; j < kClsCopies; j++) n_c += s_cls[j * kClsStride + slot];
    if (n_c)
      atomicAdd(&s_cost[k], (unsigned long long)n_c * (unsigned long long)(logt[len] - logt[n_c]) +
                                65536ull * (unsigned long long)n_c * class_extra(c));
  }
  __syncthreads();
  if (t == 0) {
    int best = 0;
    unsigned long long bc = 0;
    for (int k = 0; k < 3; k++) {
      const unsigned long long ck = s_cost[k];
      if (k == 0 || ck < bc) { bc = ck; best = k; }
    }
    *s_pred = best;
  }
  __syncthreads();
}

// Selector features of one block, read on every 4th position of the block
// (exact integer sums and counts of the lattice values p and of their LV /
// LCF residuals Dp, D2p over the sample J = {j : j = 0 mod 4}, m = |J|):
//   0 sum p / (m P')   1 (max p - min p) / P'   2 F(sum|Dp|) - F(m)
//   3 F(sum|D2p|) - F(m)   4 F(max|Dp|)   5 F(max|D2p|)   6 #(Dp=0)/m
//   7 #(D2p=0)/m   8 #(|Dp|<=1)/m   9 #(|D2p|<=1)/m
//   10 #(Dp_j Dp_{j-1} < 0)/m   11 F(sum bitlen|Dp|) - F(m)
//   12 F(sum bitlen|D2p|) - F(m)   13 #(|Dp|>=32768)/m   14 F(P')   15 1
// with P' = max(P, 1), F = flog_u64 and every ratio one fp64 division
// rounded to float.  Threads 0..15 (wave 0) leave the 16 features in s_feat,
// bfloat16-rounded if kRound, with no barrier after.
constexpr int kFeatStride = 4;
// Per-wave partials of the features, one 16-word record per wave, every
// word combined over the waves by a 32-bit sum or maximum: the 64-bit sums
// as (low 24 bits, signed rest) pairs, the signed extrema as unsigned maxima
// of order-preserving images.
enum : int { FR_SD = 0, FR_S1 = 2, FR_S2 = 4, FR_DMX = 6, FR_DMN = 7, FR_M1 = 8, FR_M2 = 9, FR_ZZ = 10,
             FR_OO = 11, FR_SE = 12, FR_B1 = 13, FR_B2 = 14, FR_WORDS = 16 };
struct alignas(16) FeatRed {
  uint32_t w[kThreads / kWave][FR_WORDS];
};

template <int E, bool kRound>
__device__ inline void block_features(const int32_t (&d)[E], const int32_t (&pv)[3], int32_t p0, uint32_t len,
                                      int64_t P, FeatRed *r, float *s_feat) {
  const int t = threadIdx.x, w = t / kWave;
  const uint32_t lane = lane_id();
  long long sd = 0;
  unsigned long long s1 = 0, s2 = 0;
  int32_t dmx = INT32_MIN, dmn = INT32_MAX;
  uint32_t m1 = 0, m2 = 0, zz = 0, oo = 0, se = 0, b1 = 0, b2 = 0;
#pragma unroll
  for (int e = 0; e < E; e += kFeatStride) {
    // Dp at e - 1 and at e, D2p at e (values before the block read as zero)
    const int32_t dm1 = e >= 1 ? d[e - 1] : pv[0];
    const int32_t dm2 = e >= 2 ? d[e - 2] : (e == 1 ? pv[0] : pv[1]);
    const int32_t prev = (int32_t)((uint32_t)dm1 - (uint32_t)dm2);
    const int32_t r1 = (int32_t)((uint32_t)d[e] - (uint32_t)dm1);
    const int32_t r2 = (int32_t)((uint32_t)r1 - (uint32_t)prev);
    if ((uint32_t)t * E + e < len) {
      const uint32_t a1 = (uint32_t)(r1 < 0 ? -r1 : r1), a2 = (uint32_t)(r2 < 0 ? -r2 : r2);
      sd += d[e];
      dmx = max(dmx, d[e]);
      dmn = min(dmn, d[e]);
      s1 += a1;
      s2 += a2;
      m1 = max(m1, a1);
      m2 = max(m2, a2);
      zz += (a1 == 0u ? 1u : 0u) + (a2 == 0u ? 0x10000u : 0u);
      oo += (a1 <= 1u ? 1u : 0u) + (a2 <= 1u ? 0x10000u : 0u);
      se += (((r1 > 0 && prev < 0) || (r1 < 0 && prev > 0)) ? 1u : 0u) + (a1 >= (uint32_t)kRadius ? 0x10000u : 0u);
      b1 += 32u - __clz(a1);
      b2 += 32u - __clz(a2);
    }
  }
  // wave totals with DPP lane moves (the two bit-length sums share a word;
  // the paired counts stay below 2^16 over the whole block)
  static_assert(E / kFeatStride * 32 * kWave < 65536, "bit-length sums share a word");
  static_assert(E / kFeatStride * kThreads < 65536, "paired counts share a word");
  const auto add = [](uint32_t a, uint32_t b) { return a + b; };
  const auto umax = [](uint32_t a, uint32_t b) { return a > b ? a : b; };
  uint32_t rec[FR_WORDS];
  rec[FR_SD] = wave_reduce_dpp((uint32_t)sd & 0xffffffu, add);
  rec[FR_SD + 1] = wave_reduce_dpp((uint32_t)(sd >> 24), add);
  rec[FR_S1] = wave_reduce_dpp((uint32_t)s1 & 0xffffffu, add);
  rec[FR_S1 + 1] = wave_reduce_dpp((uint32_t)(s1 >> 24), add);
  rec[FR_S2] = wave_reduce_dpp((uint32_t)s2 & 0xffffffu, add);
  rec[FR_S2 + 1] = wave_reduce_dpp((uint32_t)(s2 >> 24), add);
  rec[FR_DMX] = wave_reduce_dpp((uint32_t)dmx ^ 0x80000000u, umax);
  rec[FR_DMN] = wave_reduce_dpp(~((uint32_t)dmn ^ 0x80000000u), umax);
  rec[FR_M1] = wave_reduce_dpp(m1, umax);
  rec[FR_M2] = wave_reduce_dpp(m2, umax);
  rec[FR_ZZ] = wave_reduce_dpp(zz, add);
  rec[FR_OO] = wave_reduce_dpp(oo, add);
  rec[FR_SE] = wave_reduce_dpp(se, add);
  const uint32_t bb = wave_reduce_dpp(b1 | (b2 << 16), add);
  rec[FR_B1] = bb & 0xffffu;
  rec[FR_B2] = bb >> 16;
  rec[15] = 0;
  if (lane == 0) {
    uint4 *o = reinterpret_cast<uint4 *>(r->w[w]);
#pragma unroll
    for (int q = 0; q < FR_WORDS / 4; q++) o[q] = make_uint4(rec[4 * q], rec[4 * q + 1], rec[4 * q + 2], rec[4 * q + 3]);
  }
  __syncthreads();
  if (w != 0) return;
  // wave 0: lane l reads wave (l mod 4)'s record; two quad moves leave the
  // block totals in every lane
  {
    const uint4 *in = reinterpret_cast<const uint4 *>(r->w[lane & 3u]);
#pragma unroll
    for (int q = 0; q < FR_WORDS / 4; q++) {
      const uint4 v = in[q];
      rec[4 * q] = v.x; rec[4 * q + 1] = v.y; rec[4 * q + 2] = v.z; rec[4 * q + 3] = v.w;
    }
  }
#pragma unroll
  for (int k = 0; k < FR_WORDS - 1; k++) {
    const bool mx = k >= FR_DMX && k <= FR_M2;
    uint32_t x = rec[k];
    uint32_t y = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0xb1, 0xf, 0xf, false);  // quad_perm 1,0,3,2
    x = mx ? (x > y ? x : y) : x + y;
    y = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x4e, 0xf, 0xf, false);  // quad_perm 2,3,0,1
    rec[k] = mx ? (x > y ? x : y) : x + y;
  }
  const auto wide = [&](int k) { return (long long)(int32_t)rec[k + 1] * 16777216ll + (long long)rec[k]; };
  // lane k < 16 finishes feature k: a numerator and a denominator, then one
  // of four formulas, all chosen by selects
  const uint64_t Pp = P > 0 ? (uint64_t)P : 1u;
  const uint32_t m = (len + kFeatStride - 1) / kFeatStride;  // sampled positions
  const int k = (int)lane;
  const int64_t span = (int64_t)(int32_t)(rec[FR_DMX] ^ 0x80000000u) - (int64_t)(int32_t)(~rec[FR_DMN] ^ 0x80000000u);
  uint64_t a = (uint64_t)(wide(FR_SD) + (long long)m * (long long)p0);
  a = k == 1 ? (uint64_t)span : a;
  a = k == 2 ? (uint64_t)wide(FR_S1) : a;
  a = k == 3 ? (uint64_t)wide(FR_S2) : a;
  a = k == 4 ? rec[FR_M1] : a;
  a = k == 5 ? rec[FR_M2] : a;
  a = k == 6 ? rec[FR_ZZ] & 0xffffu : a;
  a = k == 7 ? rec[FR_ZZ] >> 16 : a;
  a = k == 8 ? rec[FR_OO] & 0xffffu : a;
  a = k == 9 ? rec[FR_OO] >> 16 : a;
  a = k == 10 ? rec[FR_SE] & 0xffffu : a;
  a = k == 11 ? rec[FR_B1] : a;
  a = k == 12 ? rec[FR_B2] : a;
  a = k == 13 ? rec[FR_SE] >> 16 : a;
  a = k == 14 ? Pp : a;
  const uint64_t den = k == 0 ? (uint64_t)m * Pp : k == 1 ? Pp : (uint64_t)m;
  // kind: 0 a / den, 1 F(a) - F(m), 2 F(a), 3 one
  constexpr uint32_t kKinds = (1u << 4) | (1u << 6) | (2u << 8) | (2u << 10) | (1u << 22) | (1u << 24) |
                              (2u << 28) | (3u << 30);
  const uint32_t kind = (kKinds >> (2 * (k & 15))) & 3u;
  const float q = __double2float_rn(__ddiv_rn((double)a, (double)den));
  const float fa = flog_u64(a);
  const float fv = kind == 0 ? q : kind == 1 ? fa - flog_u64(m) : kind == 2 ? fa : 1.0f;
  if (k < kNFeat) s_feat[k] = kRound ? bf16_round(fv) : fv;
}

// Adds v (<= 64) to 16-bit counter idx16 of the LDS window.  The add that
// takes a counter from below 0x8000 to 0x8000 or more takes 0x8000 back out
// and hands it to the counter's global histogram bin.  A block adds at most
// S <= 0x4000 counts to one counter and ends at a barrier, so every counter
// starts a block below 0x8000, crosses 0x8000 at most once in it, and never
// exceeds 0xC000 - 1 + 64: it never carries into the neighbour sharing its
// word, and no add reads a neighbour's transient value.
__device__ inline void gadd(gptr<uint32_t> p, uint32_t v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void win_add(uint32_t *s_win, uint32_t idx16, uint32_t v, gptr<uint32_t> gbin) {
  const uint32_t sh = (idx16 & 1u) << 4;
  const uint32_t c = (atomicAdd(&s_win[idx16 >> 1], v << sh) >> sh) & 0xffffu;
  if (c < 0x8000u && c + v >= 0x8000u) {
    atomicSub(&s_win[idx16 >> 1], 0x8000u << sh);
    gadd(gbin, 0x8000u);
  }
}

// Each workgroup takes one contiguous run of blocks and counts codes in LDS
// windows of 16-bit counters (qwin_of).  When it leaves a field it stores
// the window words to its own slab: the visit (workgroup w, field f) owns
// slab visit_base[w] + f - ffirst[w].  k_hmerge then adds the slabs of each
// field into its histogram.  (Device-scope atomics are executed beyond the
// XCD's L2, at the memory side, and are slow; only codes outside the window
// and counter wraps take that path.)
template <int E, bool kLearn>
__global__ __launch_bounds__(kThreads, kLearn ? 4 : 5) void k_quant(const CField *__restrict__ F, int nf,
                                                    const uint64_t *__restrict__ fb0, uint64_t total,
                                                    const uint32_t *__restrict__ logt, uint32_t nslots,
                                                    const uint32_t *__restrict__ qmeta, uint32_t *__restrict__ slabs,
                                                    const float *__restrict__ sel) {
  constexpr int S = E * kThreads;
  extern __shared__ uint32_t s_win[];
  // the selector's parameters, staged once per workgroup (learned policy)
  __shared__ __align__(16) float s_mlp[kLearn ? kMlpLds : 4];
  if (kLearn) {
    for (int i = threadIdx.x; i < kMlpParams; i += kThreads) s_mlp[mlp_lds_slot(i)] = sel[i];
    __syncthreads();
  }
  __shared__ int32_t s_tail[3 * kThreads];
  __shared__ uint32_t s_cls[kClsCopies * kClsStride];
  __shared__ unsigned long long s_cost[3];
  __shared__ int32_t s_p0;
  __shared__ int s_pred, s_fb;
  __shared__ FeatRed s_red;
  __shared__ __align__(16) float s_feat[kNFeat];
  __shared__ __align__(16) float s_h[kLearn ? 32 : 4];
  const int t = threadIdx.x;
  int cur = -1;

  auto flush = [&](int f) {
    __syncthreads();
    if (f >= 0) {
      const uint32_t *visit_base = qmeta, *ffirst = qmeta + gridDim.x + 1;
      uint32_t *slab = slabs + (uint64_t)(visit_base[blockIdx.x] + (uint32_t)f - ffirst[blockIdx.x]) * kWinWords;
      for (uint32_t i = t; i < (uint32_t)kWinWords; i += kThreads) slab[i] = s_win[i];
    }
    for (uint32_t i = t; i < (uint32_t)kWinWords; i += kThreads) s_win[i] = 0;
    __syncthreads();
  };

  const uint64_t g_begin = (uint64_t)blockIdx.x * total / gridDim.x;
  const uint64_t g_end = ((uint64_t)blockIdx.x + 1) * total / gridDim.x;
  // The values of block g + 1 are loaded while block g's histogram is
  // counted.  The load is issued once block g's predictor is chosen: waits
  // for vector memory are in issue order, and the trial's table reads would
  // otherwise wait for it.  A workgroup's blocks are consecutive, so the
  // field of the next block comes from a cursor that only moves forward.
  int fcur = g_begin < g_end ? find_field(fb0, nf, g_begin) : 0;
  uint64_t fend = fcur + 1 < nf ? fb0[fcur + 1] : total;
  int fn = fcur;  // field of the block in vn
  auto fetch = [&](uint64_t g, float (&v)[E]) {
    while (g >= fend) {
      fcur++;
      fend = fcur + 1 < nf ? fb0[fcur + 1] : total;
    }
    const CField &c = F[fcur];
    const uint64_t i0 = (g - c.gblock0) * S;
    load_raw<E>(G(c.x) + i0, (uint32_t)min((uint64_t)S, c.n - i0), K(static_cast<const FState *>(c.st))->mn, v);
    fn = fcur;
  };
  float vn[E];
  if (g_begin < g_end) fetch(g_begin, vn);
  for (uint64_t g = g_begin; g < g_end; g++) {
    float v[E];
#pragma unroll
    for (int e = 0; e < E; e++) v[e] = vn[e];
    const int f = fn;
    const CField &c = F[f];
    // per-field parameters through the scalar cache
    const cptr<FState> st = K(static_cast<const FState *>(c.st));
    if ((st->status != 0) | (st->is_const != 0)) {
      if (g + 1 < g_end) fetch(g + 1, vn);
      continue;
    }
    if (f != cur) { flush(cur); cur = f; }
    const uint64_t b = g - c.gblock0;
    const uint64_t i0 = b * S;
    const uint32_t len = (uint32_t)min((uint64_t)S, c.n - i0);
    int32_t d[E], pv[3], p0;
    block_d_from_raw<E>(v, st->mn, st->inv, d, pv, s_tail, p0, &s_p0);

    int pred = (int)c.policy;
    if (c.policy >= 2) {
      bool trial = true;
      if (kLearn && c.policy == 3) {
        block_features<E, true>(d, pv, p0, len, st->P, &s_red, s_feat);
        if (t < kWave) {  // wave 0 wrote the features
          float margin, z[3];
          const int top = mlp_select_wave(s_mlp, s_feat, s_h, margin, z);
          if (t == 0) {
            s_pred = top;
            s_fb = !(margin >= c.tau);
          }
        }
        __syncthreads();
        trial = s_fb != 0;
        if (trial && t == 0) atomicAdd(&c.st->fallbacks, 1u);
      }
      if (trial) block_trial<E>(d, pv, len, logt, s_cls, s_cost, &s_pred);
      pred = s_pred;
      if (t == 0) G(c.out)[c.sec.pred + b] = (uint8_t)pred;
    }
    if (t == 0) reinterpret_cast<gptr<int32_t>>(G(c.out) + c.sec.pfirst)[b] = p0;
    if (g + 1 < g_end) fetch(g + 1, vn);

    // code histogram of the chosen predictor
    const int slot = c.policy >= 2 ? pred : 0;
    const QWin qw = qwin_of(nslots, (uint32_t)slot);
    const gptr<uint32_t> gh = G(c.hist) + (uint64_t)slot * kNSyms;
#pragma unroll
    for (int e = 0; e < E; e++) {
      const bool valid = (uint32_t)t * E + e < len;
      int32_t r = residual_at<E>(d, pv, e, pred);
      uint32_t q = (r > -kRadius && r < kRadius) ? (uint32_t)(r + kRadius) : 0u;
      // the zero residual is aggregated per wave (it dominates smooth fields)
      const uint64_t zmask = __ballot(valid && q == (uint32_t)kRadius);
      if ((t & (kWave - 1)) == 0 && zmask)
        win_add(s_win, qw.off + qw.size / 2, (uint32_t)__popcll(zmask), &gh[kRadius]);
      if (valid && q != (uint32_t)kRadius) {
        if (q - qw.base < qw.size) win_add(s_win, qw.off + (q - qw.base), 1u, &gh[q]);
        else gadd(gh + q, 1u);
      }
    }
    __syncthreads();
  }
  flush(cur);
}

// Window part of each (field, predictor) code histogram: adds the 16-bit
// counters of the slabs of every workgroup that visited the field (see
// k_quant) to the wrap carries and out-of-window counts already there.
// Grid: (largest window / 256, nslots, nf).
__global__ __launch_bounds__(256) void k_hmerge(const CField *__restrict__ F, uint32_t nslots, uint32_t QG,
                                                const uint32_t *__restrict__ qmeta,
                                                const uint32_t *__restrict__ slabs) {
  const int f = blockIdx.z;
  const uint32_t slot = blockIdx.y;
  const CField &c = F[f];
  if (slot >= c.nhist || c.st->status != 0 || c.st->is_const) return;
  const QWin qw = qwin_of(nslots, slot);
  const uint32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= qw.size) return;
  const uint32_t *visit_base = qmeta, *ffirst = qmeta + QG + 1, *wf0 = qmeta + 2 * QG + 1;
  const uint32_t *wf1 = wf0 + gridDim.z;
  const uint32_t k = qw.off + i, sh = (k & 1u) << 4;
  // the visits of field f are workgroups w0..w1 in turn: w0's last visit,
  // then one visit each, so their slabs are consecutive from w0's
  const uint32_t w0 = wf0[f], w1 = min(wf1[f], QG - 1);
  uint32_t v = 0;
  if (w0 <= w1) {
    const uint32_t nv = w1 - w0 + 1;
    const gptr<const uint32_t> sp =
        G(slabs) + (uint64_t)(visit_base[w0] + (uint32_t)f - ffirst[w0]) * kWinWords + (k >> 1);
    uint32_t j = 0;
    for (; j + 16 <= nv; j += 16) {  // sixteen slabs per round trip
      uint32_t a[16];
#pragma unroll
      for (int u = 0; u < 16; u++) a[u] = sp[(uint64_t)(j + u) * kWinWords];
#pragma unroll
      for (int u = 0; u < 16; u++) v += (a[u] >> sh) & 0xffffu;
    }
    for (; j < nv; j++) v += (sp[(uint64_t)j * kWinWords] >> sh) & 0xffffu;
  }
  G(c.hist)[(uint64_t)slot * kNSyms + qw.base + i] += v;
}

// Training data of the selector: features, the three trial costs and the
// trial's choice of every block (global block order of the field table).
template <int E>
__global__ __launch_bounds__(kThreads) void k_features(const CField *__restrict__ F, int nf,
                                                       const uint64_t *__restrict__ fb0, uint64_t total,
                                                       const uint32_t *__restrict__ logt, float *feat,
                                                       uint64_t *cost, uint8_t *label) {
  constexpr int S = E * kThreads;
  __shared__ int32_t s_tail[3 * kThreads];
  __shared__ uint32_t s_cls[kClsCopies * kClsStride];
  __shared__ unsigned long long s_cost[3];
  __shared__ int32_t s_p0;
  __shared__ int s_pred;
  __shared__ FeatRed s_red;
  __shared__ float s_feat[kNFeat];
  const int t = threadIdx.x;
  for (uint64_t g = blockIdx.x; g < total; g += gridDim.x) {
    const int f = find_field(fb0, nf, g);
    const CField &c = F[f];
    const cptr<FState> st = K(static_cast<const FState *>(c.st));
    if (st->status != 0 || st->is_const) {
      if (t < kNFeat) feat[g * kNFeat + t] = 0.0f;
      if (t < 3) cost[g * 3 + t] = 0;
      if (t == 0) label[g] = 0;
      continue;
    }
    const uint64_t b = g - c.gblock0;
    const uint64_t i0 = b * S;
    const uint32_t len = (uint32_t)min((uint64_t)S, c.n - i0);
    int32_t d[E], pv[3], p0;
    load_block_d<E>(c, st->mn, st->inv, i0, len, d, pv, s_tail, p0, &s_p0);
    block_features<E, false>(d, pv, p0, len, st->P, &s_red, s_feat);
    block_trial<E>(d, pv, len, logt, s_cls, s_cost, &s_pred);
    if (t < kNFeat) feat[g * kNFeat + t] = s_feat[t];
    if (t < 3) cost[g * 3 + t] = s_cost[t];
    if (t == 0) label[g] = (uint8_t)s_pred;
    __syncthreads();
  }
}

// --------------------------------------------------------------- Huffman
//
// One workgroup of 1024 threads builds the code of one (field, predictor)
// histogram.  Leaves are sorted by (weight, symbol) with a stable radix sort;
// the two-queue Huffman merge (leaf taken first on equal weight, merged nodes
// first-in first-out) runs in batches: with s the sum of the two lightest
// nodes, every node of weight <= s precedes every node created from now on,
// so the first 2j of them (j = floor(count/2)) pair up in order at once.  A
// batch therefore reproduces exactly the sequential merge order.  Depths are
// assigned batch by batch from the root; lengths above 24 halve every weight
// ((w+1)/2) and rebuild; codes are canonical (RFC 1951, Sec. 3.2.2).

constexpr int kHT = 1024;
constexpr int kHW = kHT / kWave;
constexpr int kStage = 6144;  // largest merge batch ordered in LDS (and leaf sort in LDS)
constexpr int kHLds = 8192;   // merge queues (sorted leaves, merged nodes) in LDS up to this many leaves

struct HScratch {
  uint16_t *a_sym; uint32_t *a_f;        // present symbols in symbol order
  uint16_t *l_sym[2]; uint32_t *l_f[2];  // sort ping-pong
  uint32_t *iw;                          // merged-node weights
  uint32_t *parent;                      // 2n node parents
  uint32_t *seqw, *seqid;                // merged order of one batch
  uint32_t *batch_end;                   // merged-node count after each batch
  uint8_t *depth;                        // 2n node depths
  uint8_t *len_of;                       // 65536 lengths by symbol
  uint16_t *c_sym;                       // canonical order
};
__host__ __device__ inline uint64_t hscratch_bytes() {
  const uint64_t N = kNSyms;
  return align8(2 * N) + align8(4 * N) + 2 * align8(2 * N) + 2 * align8(4 * N) + align8(4 * N) +
         align8(8 * N) + 2 * align8(8 * N) + align8(4 * N) + align8(2 * N) + align8(N) + align8(2 * N) + 256;
}
__device__ inline HScratch hscratch_at(uint8_t *base) {
  const uint64_t N = kNSyms;
  HScratch h;
  uint8_t *p = base;
  h.a_sym = (uint16_t *)p; p += align8(2 * N);
  h.a_f = (uint32_t *)p; p += align8(4 * N);
  h.l_sym[0] = (uint16_t *)p; p += align8(2 * N);
  h.l_sym[1] = (uint16_t *)p; p += align8(2 * N);
  h.l_f[0] = (uint32_t *)p; p += align8(4 * N);
  h.l_f[1] = (uint32_t *)p; p += align8(4 * N);
  h.iw = (uint32_t *)p; p += align8(4 * N);
  h.parent = (uint32_t *)p; p += align8(8 * N);
  h.seqw = (uint32_t *)p; p += align8(8 * N);
  h.seqid = (uint32_t *)p; p += align8(8 * N);
  h.batch_end = (uint32_t *)p; p += align8(4 * N);
  h.depth = (uint8_t *)p; p += align8(2 * N);
  h.len_of = (uint8_t *)p; p += align8(N);
  h.c_sym = (uint16_t *)p;
  return h;
}

__device__ inline uint64_t lanemask_lt() {
  const uint32_t l = lane_id();
  return l ? (~0ull >> (64 - l)) : 0ull;
}

// Stable counting sort of n (key, sym) pairs by digit (key >> shift) & mask,
// nbits <= 8.  Wave w sorts segment w; order inside a segment and across
// segments is kept.  keys_out may be null (then only syms move).
__device__ void wg_split(const uint32_t *keys, const uint16_t *syms, uint32_t *keys_out, uint16_t *syms_out,
                         const uint8_t *digit_of_sym, uint32_t n, int shift, int nbits, uint32_t *s_cnt,
                         uint32_t *s_tot) {
  const int t = threadIdx.x, w = t / kWave;
  const uint32_t nd = 1u << nbits, mask = nd - 1;
  const uint32_t seg = (n + kHW - 1) / kHW;
  const uint32_t beg = min(n, seg * w), end = min(n, beg + seg);
  for (uint32_t i = t; i < nd * kHW; i += kHT) s_cnt[i] = 0;
  __syncthreads();
  auto dig = [&](uint32_t i) -> uint32_t {
    return digit_of_sym ? digit_of_sym[syms[i]] : (keys[i] >> shift) & mask;
  };
  for (uint32_t i = beg + lane_id(); i < end; i += kWave) atomicAdd(&s_cnt[dig(i) * kHW + w], 1u);
  __syncthreads();
  // exclusive scan over (digit, wave) in digit-major order
  const uint32_t per = (nd * kHW + kHT - 1) / kHT;
  uint32_t loc = 0;
  for (uint32_t j = 0; j < per; j++) {
    uint32_t i = t * per + j;
    if (i < nd * kHW) loc += s_cnt[i];
  }
  uint32_t inc = wave_incl_scan(loc);
  if (lane_id() == kWave - 1) s_tot[w] = inc;
  __syncthreads();
  uint32_t wpre = 0;
  for (int i = 0; i < w; i++) wpre += s_tot[i];
  uint32_t run = wpre + inc - loc;
  for (uint32_t j = 0; j < per; j++) {
    uint32_t i = t * per + j;
    if (i < nd * kHW) { uint32_t v = s_cnt[i]; s_cnt[i] = run; run += v; }
  }
  __syncthreads();
  for (uint32_t base = beg; base < end; base += kWave) {
    const uint32_t i = base + lane_id();
    const bool valid = i < end;
    const uint32_t dg = valid ? dig(i) : 0u;
    uint64_t m = __ballot(valid);
    for (int bt = 0; bt < nbits; bt++) {
      const uint64_t bb = __ballot(valid && ((dg >> bt) & 1u));
      m &= ((dg >> bt) & 1u) ? bb : ~bb;
    }
    const uint32_t rank = __popcll(m & lanemask_lt());
    const uint32_t cnt = __popcll(m);
    uint32_t pos = 0;
    if (valid) pos = s_cnt[dg * kHW + w] + rank;
    __builtin_amdgcn_wave_barrier();
    if (valid) {
      if (keys_out) keys_out[pos] = keys[i];
      syms_out[pos] = syms[i];
      if (rank == cnt - 1) s_cnt[dg * kHW + w] += cnt;
    }
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
}

// number of elements of a[0..n) that are <= v (a sorted)
__device__ inline uint32_t count_le(const uint32_t *a, uint32_t n, uint32_t v) {
  uint32_t lo = 0, hi = n;
  while (lo < hi) { uint32_t mid = (lo + hi) >> 1; if (a[mid] <= v) lo = mid + 1; else hi = mid; }
  return lo;
}
__device__ inline uint32_t count_lt(const uint32_t *a, uint32_t n, uint32_t v) {
  uint32_t lo = 0, hi = n;
  while (lo < hi) { uint32_t mid = (lo + hi) >> 1; if (a[mid] < v) lo = mid + 1; else hi = mid; }
  return lo;
}

// With nvar > 1 the grid is (3 nf) x nvar and variant v of a pair starts
// from v halvings of the weights (halving h times gives ceil(w / 2^h)); the
// last variant keeps halving until the lengths fit.  The first variant whose
// lengths fit is the one the sequential procedure stops at; the last
// variant of the pair to finish builds the canonical code from its lengths.
__global__ __launch_bounds__(kHT) void k_huff(const CField *__restrict__ F, int nf, uint8_t *scratch,
                                              uint64_t slot_bytes, uint32_t nvar, GCtl *gc) {
  __shared__ uint32_t s_cnt[256 * kHW];
  __shared__ uint32_t s_tot[kHW];
  __shared__ uint32_t s_red[kHW];
  __shared__ uint32_t s_n, s_maxf, s_maxlen, s_niter, s_lp, s_ip, s_ni, s_aL, s_wsum, s_c1[2], s_c2[2];
  __shared__ uint32_t s_last, s_win, s_aL2[2];
  // one merge batch: the weights of both queues' candidates, then its order
  __shared__ uint32_t s_stage[kStage], s_seqw[kStage], s_seqid[kStage];
  // the two queues of the merge, when the leaves fit: every batch reads
  // their heads, samples and runs
  __shared__ uint32_t s_lw[kHLds], s_iw[kHLds];
  __shared__ uint32_t s_blc[32], s_first[32], s_base[32];
  const int t = threadIdx.x, w = t / kWave;
  HScratch H = hscratch_at(scratch + (uint64_t)blockIdx.x * slot_bytes);
  const uint32_t var = nvar > 1 ? blockIdx.x % nvar : 0u;
  const int pair0 = nvar > 1 ? (int)(blockIdx.x / nvar) : (int)blockIdx.x;
  const int pstep = nvar > 1 ? 3 * nf : (int)gridDim.x;

  for (int pair = pair0; pair < 3 * nf; pair += pstep) {
    const int f = pair / 3, slot = pair % 3;
    const CField &c = F[f];
    FState *st = c.st;
    if ((uint32_t)slot >= c.nhist || st->status != 0 || st->is_const) continue;
    const int k = slot_pred((int)c.policy, slot);
    uint32_t *hist = c.hist + (uint64_t)slot * kNSyms;

    // 1. present symbols in symbol order: wave w reads symbols
    // [4096 w, 4096 w + 4096) in rows of 64, eight rows per round trip,
    // counts them, then writes them after the counts of the waves before it
    {
      constexpr int SPW = kNSyms / kHW, RB = 8;
      const gptr<const uint32_t> hw = G(static_cast<const uint32_t *>(hist)) + (uint32_t)w * SPW + lane_id();
      uint32_t cnt = 0, mf = 0;
#pragma unroll 1
      for (int r = 0; r < SPW / kWave; r += RB) {
        uint32_t v[RB];
        const gptr<const uint32_t> hr = hw + r * kWave;
#pragma unroll
        for (int i = 0; i < RB; i++) v[i] = hr[i * kWave];
#pragma unroll
        for (int i = 0; i < RB; i++) { cnt += v[i] != 0u; mf = max(mf, v[i]); }
      }
      cnt = wave_sum(cnt);
      mf = wave_max_u32(mf);
      if (lane_id() == 0) { s_tot[w] = cnt; s_red[w] = mf; }
      __syncthreads();
      uint32_t o = 0;
      for (int i = 0; i < w; i++) o += s_tot[i];
      const uint64_t lt = lanemask_lt();
#pragma unroll 1
      for (int r = 0; r < SPW / kWave; r += RB) {
        uint32_t v[RB];
        const gptr<const uint32_t> hr = hw + r * kWave;
#pragma unroll
        for (int i = 0; i < RB; i++) v[i] = hr[i * kWave];
#pragma unroll
        for (int i = 0; i < RB; i++) {
          const uint64_t m = __ballot(v[i] != 0u);
          if (v[i]) {
            const uint32_t pos = o + (uint32_t)__popcll(m & lt);
            H.a_sym[pos] = (uint16_t)((uint32_t)w * SPW + (uint32_t)(r + i) * kWave + lane_id());
            H.a_f[pos] = v[i];
          }
          o += (uint32_t)__popcll(m);
        }
      }
      if (t == 0) {
        uint32_t nn = 0, m2 = 0;
        for (int i = 0; i < kHW; i++) { nn += s_tot[i]; m2 = max(m2, s_red[i]); }
        s_n = nn; s_maxf = m2;
      }
      __syncthreads();
    }
    const uint32_t n = s_n;
    if (n == 0) continue;
    if (var) {
      for (uint32_t i = t; i < n; i += kHT)
        H.a_f[i] = (uint32_t)(((uint64_t)H.a_f[i] + (1ull << var) - 1) >> var);
      __syncthreads();
    }

    bool built = false;
    for (;;) {
      uint32_t maxlen = 1;
      if (n == 1) {
        if (t == 0) { H.depth[0] = 1; H.l_sym[0][0] = H.a_sym[0]; }
        __syncthreads();
      } else {
        // 2. leaves sorted by (weight, symbol): stable LSD radix on the
        // weight, in LDS when the leaves fit (the merge buffers are free
        // until step 3), and the sorted run stored to l_f[0], l_sym[0]
        const bool in_lds = n <= (uint32_t)kStage;
        uint16_t *sy0 = reinterpret_cast<uint16_t *>(s_seqid), *sy1 = sy0 + kStage;
        {
          uint32_t mf = 0;  // weights may have been halved since step 1
          for (uint32_t i = t; i < n; i += kHT) {
            const uint32_t f = H.a_f[i];
            mf = max(mf, f);
            if (in_lds) { s_stage[i] = f; sy0[i] = H.a_sym[i]; }
          }
          mf = wave_max_u32(mf);
          if (lane_id() == 0) s_red[w] = mf;
          __syncthreads();
          if (t == 0) {
            uint32_t m2 = 0;
            for (int i = 0; i < kHW; i++) m2 = max(m2, s_red[i]);
            s_maxf = m2;
          }
          __syncthreads();
        }
        int passes = 0;
        {
          uint32_t mf = s_maxf;
          while (mf) { passes++; mf >>= 8; }
          if (passes == 0) passes = 1;
        }
        const uint32_t *Lw;
        const uint16_t *Ls;
        if (in_lds) {
          uint32_t *kin = s_stage, *kout = s_seqw;
          uint16_t *sin = sy0, *sout = sy1;
          for (int ps = 0; ps < passes; ps++) {
            wg_split(kin, sin, kout, sout, nullptr, n, 8 * ps, 8, s_cnt, s_tot);
            uint32_t *tk = kin; kin = kout; kout = tk;
            uint16_t *ts = sin; sin = sout; sout = ts;
          }
          for (uint32_t i = t; i < n; i += kHT) { s_lw[i] = kin[i]; H.l_sym[0][i] = sin[i]; }
          __syncthreads();
          Lw = s_lw;
          Ls = H.l_sym[0];
        } else {
          const uint32_t *kin = H.a_f;
          const uint16_t *sin = H.a_sym;
          int pp = 0;
          for (int ps = 0; ps < passes; ps++) {
            wg_split(kin, sin, H.l_f[pp], H.l_sym[pp], nullptr, n, 8 * ps, 8, s_cnt, s_tot);
            kin = H.l_f[pp];
            sin = H.l_sym[pp];
            pp ^= 1;
          }
          Lw = kin;
          Ls = sin;
          if (n <= (uint32_t)kHLds) {
            for (uint32_t i = t; i < n; i += kHT) s_lw[i] = kin[i];
            __syncthreads();
            Lw = s_lw;
          }
        }
        uint32_t *const IW = n <= (uint32_t)kHLds ? s_iw : H.iw;

        // 3. batched two-queue merge.  Per batch: the weight s of the next
        // merged node from the heads of both queues; the counts cL, cI of
        // leaves and merged nodes of weight <= s (two rounds of samples of
        // each sorted queue, half of the workgroup per queue); the merged
        // order of those nodes by rank search, in LDS when the batch fits.
        if (t == 0) { s_lp = 0; s_ip = 0; s_ni = 0; s_niter = 0; s_aL2[0] = 0; s_aL2[1] = 0; }
        __syncthreads();
        if (n <= (uint32_t)kHLds) {
          // Both queues in LDS: every thread finds the batch itself (the
          // weight of the next merged node from the queues' heads, and the
          // counts of nodes of weight <= it by binary search), so a batch
          // takes two barriers: after the merged order, after the new nodes.
          uint32_t lp = 0, ip = 0, ni = 0, niter = 0;
          for (;;) {
            if ((n - lp) + (ni - ip) <= 1) break;
            const uint32_t x0 = lp < n ? s_lw[lp] : ~0u, x1 = lp + 1 < n ? s_lw[lp + 1] : ~0u;
            const uint32_t y0 = ip < ni ? s_iw[ip] : ~0u, y1 = ip + 1 < ni ? s_iw[ip + 1] : ~0u;
            const uint32_t wsum = min(x0, y0) + (x0 <= y0 ? min(x1, y0) : min(x0, y1));
            const uint32_t cL = count_le(s_lw + lp, n - lp, wsum), cI = count_le(s_iw + ip, ni - ip, wsum);
            const uint32_t j = (cL + cI) / 2;
            const bool staged = 2 * j <= (uint32_t)kStage;
            const uint32_t par = niter & 1u;
            if (t == 0) s_aL2[par ^ 1u] = 0;  // the next batch's count (last read before this batch)
            uint32_t aL = 0;
            for (uint32_t e = t; e < cL + cI; e += kHT) {
              uint32_t wv, id, pos;
              if (e < cL) {
                wv = s_lw[lp + e];
                pos = e + count_lt(s_iw + ip, cI, wv);
                id = lp + e;
                aL += pos < 2 * j;
              } else {
                const uint32_t kk = e - cL;
                wv = s_iw[ip + kk];
                pos = kk + count_le(s_lw + lp, cL, wv);
                id = n + ip + kk;
              }
              if (pos < 2 * j) {
                if (staged) { s_seqw[pos] = wv; s_seqid[pos] = id; }
                else { H.seqw[pos] = wv; H.seqid[pos] = id; }
              }
            }
            aL = wave_sum(aL);
            if (lane_id() == 0 && aL) atomicAdd(&s_aL2[par], aL);
            __syncthreads();
            const uint32_t aLt = s_aL2[par];
            for (uint32_t i = t; i < j; i += kHT) {
              const uint32_t w0 = staged ? s_seqw[2 * i] : H.seqw[2 * i];
              const uint32_t w1 = staged ? s_seqw[2 * i + 1] : H.seqw[2 * i + 1];
              const uint32_t i0 = staged ? s_seqid[2 * i] : H.seqid[2 * i];
              const uint32_t i1 = staged ? s_seqid[2 * i + 1] : H.seqid[2 * i + 1];
              s_iw[ni + i] = w0 + w1;
              H.parent[i0] = n + ni + i;
              H.parent[i1] = n + ni + i;
            }
            if (t == 0) H.batch_end[niter] = ni + j;
            __syncthreads();
            lp += aLt;
            ip += 2 * j - aLt;
            ni += j;
            niter++;
          }
          if (t == 0) { s_ni = ni; s_niter = niter; }
          __syncthreads();
        }
        for (; n > (uint32_t)kHLds;) {
          const uint32_t lp = s_lp, ip = s_ip, ni = s_ni;
          if ((n - lp) + (ni - ip) <= 1) break;
          if (t == 0) {
            const uint32_t x0 = lp < n ? Lw[lp] : ~0u, x1 = lp + 1 < n ? Lw[lp + 1] : ~0u;
            const uint32_t y0 = ip < ni ? IW[ip] : ~0u, y1 = ip + 1 < ni ? IW[ip + 1] : ~0u;
            s_wsum = min(x0, y0) + (x0 <= y0 ? min(x1, y0) : min(x0, y1));
            s_c1[0] = 0; s_c1[1] = 0; s_c2[0] = 0; s_c2[1] = 0;
          }
          __syncthreads();
          const uint32_t wsum = s_wsum;
          const uint32_t q = (uint32_t)t / (kHT / 2), tq = (uint32_t)t % (kHT / 2);
          const uint32_t *qa = q ? IW + ip : Lw + lp;
          const uint32_t qlen = q ? ni - ip : n - lp;
          const uint32_t stp = (qlen + kHT / 2 - 1) / (kHT / 2);
          {
            const bool le = (uint64_t)tq * stp < qlen && qa[tq * stp] <= wsum;
            const uint32_t c = (uint32_t)__popcll(__ballot(le));
            if (lane_id() == 0 && c) atomicAdd(&s_c1[q], c);
          }
          __syncthreads();
          const uint32_t c1 = s_c1[q];
          {
            // the count lies in ((c1 - 1) stp, c1 stp]
            const uint32_t o = (c1 - 1) * stp + 1 + tq;
            const bool le = c1 && tq + 1 < stp && o < qlen && qa[o] <= wsum;
            const uint32_t c = (uint32_t)__popcll(__ballot(le));
            if (lane_id() == 0 && c) atomicAdd(&s_c2[q], c);
          }
          __syncthreads();
          const uint32_t cL = s_c1[0] ? (s_c1[0] - 1) * ((n - lp + kHT / 2 - 1) / (kHT / 2)) + 1 + s_c2[0] : 0u;
          const uint32_t cI = s_c1[1] ? (s_c1[1] - 1) * ((ni - ip + kHT / 2 - 1) / (kHT / 2)) + 1 + s_c2[1] : 0u;
          const uint32_t j = (cL + cI) / 2;
          const bool staged = cL + cI <= (uint32_t)kStage;
          if (t == 0) s_aL = 0;
          if (staged) {
            for (uint32_t e = t; e < cL + cI; e += kHT) s_stage[e] = e < cL ? Lw[lp + e] : IW[ip + e - cL];
          }
          __syncthreads();
          uint32_t aL = 0;
          for (uint32_t e = t; e < cL + cI; e += kHT) {
            uint32_t wv, id, pos;
            if (e < cL) {
              wv = staged ? s_stage[e] : Lw[lp + e];
              pos = e + (staged ? count_lt(s_stage + cL, cI, wv) : count_lt(IW + ip, cI, wv));
              id = lp + e;
              aL += pos < 2 * j;
            } else {
              const uint32_t kk = e - cL;
              wv = staged ? s_stage[e] : IW[ip + kk];
              pos = kk + (staged ? count_le(s_stage, cL, wv) : count_le(Lw + lp, cL, wv));
              id = n + ip + kk;
            }
            if (pos < 2 * j) {
              if (staged) { s_seqw[pos] = wv; s_seqid[pos] = id; }
              else { H.seqw[pos] = wv; H.seqid[pos] = id; }
            }
          }
          aL = wave_sum(aL);
          if (lane_id() == 0 && aL) atomicAdd(&s_aL, aL);
          __syncthreads();
          for (uint32_t i = t; i < j; i += kHT) {
            const uint32_t w0 = staged ? s_seqw[2 * i] : H.seqw[2 * i];
            const uint32_t w1 = staged ? s_seqw[2 * i + 1] : H.seqw[2 * i + 1];
            const uint32_t i0 = staged ? s_seqid[2 * i] : H.seqid[2 * i];
            const uint32_t i1 = staged ? s_seqid[2 * i + 1] : H.seqid[2 * i + 1];
            IW[ni + i] = w0 + w1;
            H.parent[i0] = n + ni + i;
            H.parent[i1] = n + ni + i;
          }
          __syncthreads();
          if (t == 0) {
            s_lp = lp + s_aL;
            s_ip = ip + 2 * j - s_aL;
            s_ni = ni + j;
            H.batch_end[s_niter] = ni + j;
            s_niter = s_niter + 1;
          }
          __syncthreads();
        }
        // 4. depths from the root down, batch by batch
        const uint32_t ni = s_ni, niter = s_niter;
        const uint32_t root = n + ni - 1;
        for (int it = (int)niter - 1; it >= 0; it--) {
          const uint32_t lo = it ? H.batch_end[it - 1] : 0u, hi = H.batch_end[it];
          for (uint32_t i = lo + t; i < hi; i += kHT) {
            const uint32_t v = n + i;
            H.depth[v] = v == root ? 0 : (uint8_t)(H.depth[H.parent[v]] + 1);
          }
          __syncthreads();
        }
        uint32_t ml = 0;
        for (uint32_t i = t; i < n; i += kHT) {
          uint8_t dd = (uint8_t)(H.depth[H.parent[i]] + 1);
          H.depth[i] = dd;
          ml = max(ml, (uint32_t)dd);
        }
        ml = wave_max_u32(ml);
        if (lane_id() == 0) s_red[w] = ml;
        __syncthreads();
        if (t == 0) {
          uint32_t m2 = 0;
          for (int i = 0; i < kHW; i++) m2 = max(m2, s_red[i]);
          s_maxlen = m2;
        }
        __syncthreads();
        maxlen = s_maxlen;
        if (maxlen > (uint32_t)kLMax) {
          if (var + 1 < nvar) break;  // a later variant has halved further
          for (uint32_t i = t; i < n; i += kHT) H.a_f[i] = (H.a_f[i] + 1) >> 1;
          __syncthreads();
          continue;
        }
        // lengths by symbol (leaves are in sorted order in Ls)
        for (uint32_t i = t; i < n; i += kHT) H.len_of[Ls[i]] = H.depth[i];
        __syncthreads();
      }
      if (n == 1) {
        if (t == 0) H.len_of[H.a_sym[0]] = 1;
        __syncthreads();
      }
      built = true;
      break;
    }
    // hand-over between the variants of the pair: each publishes whether
    // its lengths fit; the last to finish takes the first that fits
    uint64_t win = blockIdx.x;
    if (nvar > 1) {
      // every thread's code lengths reach device scope before the count
      __threadfence();
      __syncthreads();
      if (t == 0) {
        __hip_atomic_store(&gc->hres[blockIdx.x], built ? 1u : 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        s_last = atomicAdd(&gc->hdone[pair], 1u) == nvar - 1;
      }
      __syncthreads();
      if (!s_last) continue;
      __threadfence();
      if (t == 0) {
        uint32_t u = 0;
        while (u + 1 < nvar &&
               !__hip_atomic_load(&gc->hres[pair * nvar + u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
          u++;
        s_win = pair * nvar + u;
        gc->hdone[pair] = 0;
      }
      __syncthreads();
      win = s_win;
    }
    const uint8_t *len_of = hscratch_at(scratch + win * slot_bytes).len_of;
    {
      // 5. canonical order = symbols stably sorted by length
      wg_split(nullptr, H.a_sym, nullptr, H.c_sym, len_of, n, 0, 5, s_cnt, s_tot);
      if (t < 32) s_blc[t] = 0;
      __syncthreads();
      for (uint32_t i = t; i < n; i += kHT) atomicAdd(&s_blc[len_of[H.a_sym[i]]], 1u);
      __syncthreads();
      if (t == 0) {
        uint32_t code = 0, idx = 0, ml = 0;
        for (int l = 1; l <= kLMax; l++) {
          s_first[l] = code;
          s_base[l] = idx;
          code = (code + s_blc[l]) << 1;
          idx += s_blc[l];
          if (s_blc[l]) ml = (uint32_t)l;
        }
        s_maxlen = ml;
      }
      __syncthreads();
      // 6. encoder table and staged codebook
      uint32_t *enc = c.enc + (uint64_t)slot * kNSyms;
      uint32_t *book = c.book + (uint64_t)slot * kBookWords;
      uint16_t *bsym = reinterpret_cast<uint16_t *>(book + 32);
      for (uint32_t i = t; i < n; i += kHT) {
        const uint16_t sym = H.c_sym[i];
        const uint32_t l = len_of[sym];
        const uint32_t code = s_first[l] + (i - s_base[l]);
        enc[sym] = code | (l << 24);
        bsym[i] = sym;
      }
      if (t < 32) book[t] = (t >= 1 && t <= kLMax) ? s_blc[t] : 0u;
      if (t == 0) { st->nsym[k] = n; st->maxlen[k] = s_maxlen; }
      __syncthreads();
    }
  }
}

// ----------------------------------------------------------------- books

// One workgroup per field: copy the staged codebooks into the stream, zero
// their padding, and fix the payload offset.
__global__ __launch_bounds__(kThreads) void k_books(const CField *__restrict__ F) {
  const CField &c = F[blockIdx.x];
  FState *st = c.st;
  if (st->status != 0 || st->is_const) return;
  const int t = threadIdx.x;
  uint8_t *o = c.out;
  uint64_t off = c.sec.books;
  for (int k = 0; k < 3; k++) {
    const uint32_t ns = st->nsym[k], ml = st->maxlen[k];
    if (!ns) continue;
    int slot = c.policy >= 2 ? k : 0;
    const uint32_t *book = c.book + (uint64_t)slot * kBookWords;
    const uint16_t *bsym = reinterpret_cast<const uint16_t *>(book + 32);
    uint32_t *blc = reinterpret_cast<uint32_t *>(o + off);
    for (uint32_t l = t; l < ml; l += kThreads) blc[l] = book[l + 1];
    uint16_t *sy = reinterpret_cast<uint16_t *>(o + off + 4ull * ml);
    for (uint32_t i = t; i < ns; i += kThreads) sy[i] = bsym[i];
    const uint64_t end = off + 4ull * ml + 2ull * ns, nxt = align8(end);
    if (t < 8 && end + t < nxt) o[end + t] = 0;
    off = nxt;
  }
  if (t == 0) {
    st->off_payload = off;
    for (int k = 0; k < 3; k++) put32(o, H_NSYM + 4 * k, st->nsym[k]);
    put32(o, H_MAXLEN, st->maxlen[0] | (st->maxlen[1] << 8) | (st->maxlen[2] << 16));
    put64(o, H_OFF_PAYLOAD, off);
  }
}

// ------------------------------------------------------------------ pack

constexpr uint64_t kFlagAgg = 1ull << 62, kFlagPre = 2ull << 62, kValMask = (1ull << 62) - 1;

constexpr int kEncWin = 2048;  // pack kernel: codewords held in LDS
constexpr uint32_t kEncBase = 32768u - kEncWin / 2;
template <int E>
__global__ __launch_bounds__(kThreads, 4) void k_pack(const CField *__restrict__ F, int nf,
                                                   const uint64_t *__restrict__ fb0, uint64_t total, GCtl *gc) {
  constexpr int S = E * kThreads;
  constexpr int CWMAX = S * kLMax / 32 + 16;  // code words plus the skip table
  __shared__ uint32_t s_words[CWMAX];
  __shared__ int32_t s_tail[3 * kThreads];
  __shared__ int32_t s_p0;
  __shared__ uint32_t s_g;
  __shared__ unsigned long long s_wtot[kThreads / kWave];
  __shared__ unsigned long long s_prefix;
  // codewords of the codes around 32768 of the last (field, predictor)
  // coded here, for fields long enough that a workgroup's successive tickets
  // mostly fall in one field: most lookups then stay in LDS
  __shared__ uint32_t s_enc[kEncWin];
  const int t = threadIdx.x, w = t / kWave;
  int cur = -1;

  for (;;) {
    if (t == 0) s_g = atomicAdd(&gc->ticket, 1u);
    __syncthreads();
    const uint64_t g = s_g;
    __syncthreads();
    if (g >= total) break;
    const int f = find_field(fb0, nf, g);
    const CField &c = F[f];
    const gptr<FState> st = G(c.st);
    // The status is read through the scalar cache, so that no vector-memory
    // wait precedes the block's loads.  A field is skipped only for a status
    // set before this kernel: every block of a field that runs out of space
    // here still publishes its look-back value (later blocks of the field
    // wait for it); it only stores nothing.
    const cptr<FState> sk = K(static_cast<const FState *>(c.st));
    const int32_t status = sk->status;
    if ((status != 0 && status != SZNB_ENOSPC) | (sk->is_const != 0)) continue;
    const uint64_t b = g - c.gblock0;
    const uint64_t i0 = b * S;
    const uint32_t len = (uint32_t)min((uint64_t)S, c.n - i0);
    const gptr<uint8_t> out = G(c.out);
    const int pred = c.policy >= 2 ? (int)out[c.sec.pred + b] : (int)c.policy;
    int32_t d[E], pv[3], p0;
    load_block_d<E>(c, st->mn, st->inv, i0, len, d, pv, s_tail, p0, &s_p0);
    const int slot = c.policy >= 2 ? pred : 0;
    const gptr<const uint32_t> enc = G(c.enc) + (uint64_t)slot * kNSyms;
    const bool win = c.nblocks >= 2ull * gridDim.x;
    if (win && f * 3 + slot != cur) {
      // the previous block's lookups are behind this block's first barriers
      for (uint32_t i = t; i < (uint32_t)kEncWin; i += kThreads) s_enc[i] = enc[kEncBase + i];
      __syncthreads();
      cur = f * 3 + slot;
    }

    uint32_t cw[E];
    int32_t rr[E];
    uint32_t bits = 0, nesc = 0;
#pragma unroll
    for (int e = 0; e < E; e++) {
      const bool valid = (uint32_t)t * E + e < len;
      int32_t r = residual_at<E>(d, pv, e, pred);
      uint32_t q = (r > -kRadius && r < kRadius) ? (uint32_t)(r + kRadius) : 0u;
      rr[e] = r;
      cw[e] = !valid ? 0u : (win && q - kEncBase < (uint32_t)kEncWin ? s_enc[q - kEncBase] : enc[q]);
      bits += cw[e] >> 24;
      nesc += (valid && q == 0u) ? 1u : 0u;
    }
    // block exclusive scan of (bits, escapes)
    const unsigned long long mine = (unsigned long long)bits | ((unsigned long long)nesc << 32);
    const unsigned long long inc = wave_incl_scan(mine);
    if (lane_id() == kWave - 1) s_wtot[w] = inc;
    __syncthreads();
    unsigned long long pre = 0, tot = 0;
    for (int i = 0; i < kThreads / kWave; i++) {
      if (i < w) pre += s_wtot[i];
      tot += s_wtot[i];
    }
    const unsigned long long ex = pre + inc - mine;
    const uint32_t bit0 = (uint32_t)ex, esc0 = (uint32_t)(ex >> 32);
    const uint32_t tbits = (uint32_t)tot, tesc = (uint32_t)(tot >> 32);
    const uint32_t cwn = (tbits + 31) / 32;
    const uint32_t R = n_ranges(cwn), swd = skip_width(st->maxlen[pred]);
    const uint32_t skw = skip_words(cwn, st->maxlen[pred]);
    const uint64_t words = (uint64_t)skw + cwn + tesc;

    // the block's own size is published at once (an inclusive prefix for
    // the field's first block); the look-back itself runs after the packing
    // below, so the other waves pack while wave 0 resolves it
    if (t == 0) st_relaxed_u64(&G(c.lbflag)[b], (b == 0 ? kFlagPre : kFlagAgg) | words);
    for (uint32_t i = t; i < skw + cwn; i += kThreads) s_words[i] = 0u;
    __syncthreads();
    // skip table entries of the range starts inside this thread's bits
    if (bits && R > 1) {
      const uint32_t w0 = (bit0 + 31) >> 5;
      uint32_t lr = (w0 * R + cwn - 1) / cwn;
      if (lr < 1) lr = 1;
      for (; lr < R; lr++) {
        const uint32_t st0 = range_start(lr, cwn, R);
        if (st0 >= bit0 + bits) break;
        uint32_t o = bit0, T = bit0 + bits;
#pragma unroll
        for (int e = 0; e < E; e++) {
          if (o >= st0 && T == bit0 + bits) T = o;
          o += cw[e] >> 24;
        }
        const uint32_t v = T - st0, pos = (lr - 1) * swd;
        const uint32_t wi = pos >> 5, sh = pos & 31u;
        if (sh + swd <= 32u) {
          atomicOr(&s_words[wi], v << (32u - sh - swd));
        } else {
          const uint32_t over = sh + swd - 32u;
          atomicOr(&s_words[wi], v >> over);
          atomicOr(&s_words[wi + 1], v << (32u - over));
        }
      }
    }
    // MSB-first packing: whole words of this thread's run are stored, the
    // first and last word (possibly shared with a neighbour) are OR-ed in
    {
      uint32_t *s_code = s_words + skw;
      uint32_t wi = bit0 >> 5;
      const uint32_t wfirst = wi;
      uint32_t na = bit0 & 31u;
      uint64_t acc = 0;
#pragma unroll
      for (int e = 0; e < E; e++) {
        const uint32_t l = cw[e] >> 24;
        if (l) {
          acc |= (uint64_t)(cw[e] & 0xffffffu) << (64u - na - l);
          na += l;
          if (na >= 32u) {
            const uint32_t word = (uint32_t)(acc >> 32);
            if (wi == wfirst) atomicOr(&s_code[wi], word); else s_code[wi] = word;
            wi++;
            acc <<= 32;
            na -= 32u;
          }
        }
      }
      if (bits && na) atomicOr(&s_code[wi], (uint32_t)(acc >> 32));
    }
    // decoupled look-back over the field's earlier blocks, 64 at a time by
    // wave 0: sum the aggregates back to the nearest published prefix
    if (w == 0) {
      const uint32_t lane = lane_id();
      uint64_t P = 0;
      if (b > 0) {
        int64_t base = (int64_t)b - 1;
        for (;;) {
          const int64_t j = base - (int64_t)lane;
          const uint64_t v = j >= 0 ? ld_relaxed_u64(&G(c.lbflag)[j]) : kFlagPre;
          const uint64_t pre = __ballot((v >> 62) == 2);
          const uint64_t zero = __ballot(v == 0);
          if (pre) {
            const uint32_t pl = (uint32_t)__builtin_ctzll(pre);
            const uint64_t upto = pl == 63 ? ~0ull : ((2ull << pl) - 1);
            if (zero & upto) { __builtin_amdgcn_s_sleep(1); continue; }
            P += wave_sum((unsigned long long)(lane <= pl ? (v & kValMask) : 0ull));
            break;
          }
          if (zero) { __builtin_amdgcn_s_sleep(1); continue; }
          P += wave_sum((unsigned long long)(v & kValMask));
          base -= kWave;
        }
        if (lane == 0) st_relaxed_u64(&G(c.lbflag)[b], kFlagPre | (P + words));
      }
      if (lane == 0) s_prefix = P;
    }
    __syncthreads();
    const uint64_t P = s_prefix;
    const uint64_t wbase = st->off_payload / 4 + P;
    const bool fits = (wbase + words) * 4 <= c.out_cap;
    const gptr<uint32_t> ow = reinterpret_cast<gptr<uint32_t>>(out);
    if (fits) {
      for (uint32_t i = t; i < skw + cwn; i += kThreads) ow[wbase + i] = s_words[i];
      if (nesc) {
        uint32_t ei = skw + esc0;
#pragma unroll
        for (int e = 0; e < E; e++) {
          const bool valid = (uint32_t)t * E + e < len;
          if (valid && !(rr[e] > -kRadius && rr[e] < kRadius)) ow[wbase + cwn + ei++] = (uint32_t)rr[e];
        }
      }
    } else if (t == 0) {
      st->status = SZNB_ENOSPC;
    }
    if (t == 0) {
      reinterpret_cast<gptr<uint16_t>>(out + c.sec.cwords)[b] = (uint16_t)cwn;
      reinterpret_cast<gptr<uint16_t>>(out + c.sec.nesc)[b] = (uint16_t)tesc;
      if (b + 1 == c.nblocks) st->payload_words = P + words;
    }
    __syncthreads();
  }
}

// ----------------------------------------------------------------- final

// After the pack kernel: payload size, total size and output length.
__global__ void k_final(const CField *__restrict__ F, int nf) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  const CField &c = F[f];
  FState *st = c.st;
  if (st->is_const || (st->status != 0 && st->status != SZNB_ENOSPC)) return;
  const uint64_t pw = st->payload_words;
  const uint64_t tb = st->off_payload + 4 * pw;
  if (st->status != 0 || tb > c.out_cap) {
    st->status = SZNB_ENOSPC;
    if (c.out_len) *c.out_len = 0;
  } else {
    put64(c.out, H_PWORDS, pw);
    put64(c.out, H_TOTAL, tb);
    if (c.out_len) *c.out_len = tb;
  }
}

// explicit instantiations (block sizes 1K..16K)
#define SZNB_INST(E)                                                                                        \
  template __global__ void k_quant<E, false>(const CField *, int, const uint64_t *, uint64_t,              \
                                             const uint32_t *, uint32_t, const uint32_t *, uint32_t *,      \
                                             const float *);                                                \
  template __global__ void k_quant<E, true>(const CField *, int, const uint64_t *, uint64_t,               \
                                            const uint32_t *, uint32_t, const uint32_t *, uint32_t *,       \
                                            const float *);                                                 \
  template __global__ void k_features<E>(const CField *, int, const uint64_t *, uint64_t, const uint32_t *,  \
                                         float *, uint64_t *, uint8_t *);                                    \
  template __global__ void k_pack<E>(const CField *, int, const uint64_t *, uint64_t, GCtl *);
SZNB_INST(4)
SZNB_INST(8)
SZNB_INST(16)
SZNB_INST(32)
SZNB_INST(64)

}  // namespace sznb

namespace sznb {
uint64_t hscratch_bytes_host() { return hscratch_bytes(); }
}  // namespace sznb
