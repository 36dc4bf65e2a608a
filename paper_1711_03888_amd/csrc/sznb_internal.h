// Internal definitions of the sznb HIP library (device structs, stream
// layout constants, wave-level primitives).  gfx950 only: wave64.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sznb.h"

namespace sznb {

constexpr int kRadius = 32768;       // 65536 quantization intervals, code 0 = escape
constexpr int kNSyms = 65536;
constexpr int kLMax = 24;            // Huffman code lengths are limited to 24 bits
constexpr int64_t kPMax = 1 << 27;   // largest lattice span accepted
constexpr int kHdr = 128;
constexpr int kLutBits = 12;         // first-level decode table
constexpr int kNClass = 33;          // residual classes of the block-cost estimate
constexpr int kThreads = 256;        // workgroup size of the per-block kernels
constexpr int kWave = 64;
// LDS windows of the code histograms around code 32768: 16-bit counters,
// kWinWords 32-bit words per quantization workgroup.  One predictor slot
// takes all 12288 counters; three slots take 8192 (LV) + 2048 + 2048.
constexpr int kWinWords = 6144;
struct QWin {
  uint32_t base, size, off;  // first code, number of codes, first counter
};
__host__ __device__ inline QWin qwin_of(uint32_t nslots, uint32_t slot) {
  QWin w;
  if (nslots <= 1) { w.size = 2 * kWinWords; w.off = 0; }
  else if (slot == 0) { w.size = 8192; w.off = 0; }
  else { w.size = 2048; w.off = 8192 + 2048 * (slot - 1); }
  w.base = 32768u - w.size / 2;
  return w;
}

// header byte offsets
enum : int {
  H_MAGIC = 0, H_VERSION = 4, H_POLICY = 6, H_FLAGS = 7, H_N = 8, H_S = 16, H_NB = 20,
  H_MN = 24, H_MX = 28, H_EBABS = 32, H_STEP = 40, H_NSYM = 48, H_MAXLEN = 60,
  H_PWORDS = 64, H_TOTAL = 72, H_OFF_PRED = 80, H_OFF_PFIRST = 88, H_OFF_CWORDS = 96,
  H_OFF_NESC = 104, H_OFF_BOOKS = 112, H_OFF_PAYLOAD = 120
};
constexpr uint32_t kMagic = 0x424E5A53u;  // "SZNB"

__host__ __device__ inline uint64_t align8(uint64_t x) { return (x + 7) & ~uint64_t(7); }

// Global-memory view of a pointer.  Kernels reach their buffers through
// pointers held in descriptor tables; such a pointer could as well address
// LDS, so the compiler accesses it with flat instructions, and a flat load
// in flight counts on the LDS wait counter too: every wait for an LDS read
// would also wait for it.  Through the global address space the loads and
// stores are global_* and LDS waits stay short.
template <class T>
using gptr = T __attribute__((address_space(1))) *;
template <class T>
__device__ __forceinline__ gptr<T> G(T *p) {
  return (gptr<T>)p;
}
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
// Read-only view through the scalar data cache (constant address space),
// for per-field parameters that nothing writes while the reading kernel
// runs.  Uniform loads through it are scalar loads, counted apart from
// vector memory, so waiting for them does not wait for data loads in flight.
template <class T> using cptr = const T __attribute__((address_space(4))) *;
template <class T> __device__ __forceinline__ cptr<T> K(const T *p) { return (cptr<T>)p; }

// Section offsets that depend only on the block count and the policy.
struct Sections {
  uint64_t pred, pfirst, cwords, nesc, books;
};
__host__ __device__ inline Sections sections_of(uint64_t nb, int policy) {
  Sections s;
  uint64_t o = kHdr;
  s.pred = 0;
  if (policy >= 2) { s.pred = o; o = align8(o + nb); }
  s.pfirst = o; o = align8(o + 4 * nb);
  s.cwords = o; o = align8(o + 2 * nb);
  s.nesc = o; o = align8(o + 2 * nb);
  s.books = o;
  return s;
}
__host__ __device__ inline uint64_t book_bytes(uint32_t nsym, uint32_t maxlen) {
  return nsym ? align8(4ull * maxlen + 2ull * nsym) : 0;
}

// ---------------------------------------------------------------- compress

// per-field state written by the device
struct alignas(64) FState {
  int32_t status;
  uint32_t is_const;
  float mn, mx;
  double R, eb_abs, step, inv;
  int64_t P;
  uint32_t nsym[3];
  uint32_t maxlen[3];
  uint64_t off_payload;
  uint64_t payload_words;
  uint32_t blocks_done;
  uint32_t fallbacks;     // learned policy: blocks decided by the exhaustive trial
};

// per-field descriptor written by the host
struct alignas(16) CField {
  const float *x;
  uint64_t n;
  double eb;
  uint8_t *out;
  uint64_t out_cap;
  uint64_t *out_len;      // device word receiving the stream length
  uint32_t policy, eb_rel, S, log2S;
  uint32_t nblocks, nhist;
  uint64_t gblock0;       // first global block index of this field
  Sections sec;
  FState *st;
  uint32_t *blkstat;      // 3 words per block: min key, max key, non-finite flag
  uint32_t *hist;         // nhist x 65536 code counts
  uint32_t *enc;          // nhist x 65536 codewords: code | len << 24
  uint32_t *book;         // nhist x (32 bl_count words + 32768 words of u16 symbols)
  uint64_t *lbflag;       // decoupled look-back words, one per block
  const float *sel;       // learned policy: selector parameters (weights bfloat16-rounded)
  float tau;              // learned policy: smallest logit margin trusted
  uint32_t pad_sel;
};
constexpr int kBookWords = 32 + kNSyms / 2;

constexpr int kHuffSlots = 64;  // Huffman workgroups (and scratch slots), at most
struct alignas(64) GCtl {
  uint32_t ticket;        // block tickets of the pack kernel
  uint32_t pad[15];
  uint32_t hdone[kHuffSlots];  // Huffman variants finished, per (field, predictor) pair
  uint32_t hres[kHuffSlots];   // per Huffman workgroup: its code lengths fit
};

// Skip table of a block: its code words are cut into R word-aligned ranges
// (range l starts at bit 32 floor(l cw / R), R = min(64, max(1, cw / 8)));
// for each range after the first the stream stores, in w = bitlen(maxlen-1)
// bits MSB first ahead of the code words, the distance from the range start
// to the first codeword starting at or after it.
__host__ __device__ inline uint32_t n_ranges(uint32_t cw) {
  const uint32_t r = cw / 8;
  return r < 1 ? 1u : (r > 64 ? 64u : r);
}
__host__ __device__ inline uint32_t skip_width(uint32_t maxlen) {
  uint32_t w = 0;
  while ((1u << w) < maxlen) w++;
  return w;
}
__host__ __device__ inline uint32_t skip_words(uint32_t cw, uint32_t maxlen) {
  return ((n_ranges(cw) - 1) * skip_width(maxlen) + 31) / 32;
}
__host__ __device__ inline uint32_t range_start(uint32_t l, uint32_t cw, uint32_t R) {
  return 32u * ((l * cw) / R);  // l <= 64 and cw <= 2^14 * 24 / 32: no overflow
}

// predictor that histogram slot s of a field codes
__host__ __device__ inline int slot_pred(int policy, int s) { return policy >= 2 ? s : policy; }

// ------------------------------------------------------------- decompress

struct alignas(64) DState {
  int32_t status;
  uint32_t is_const;
  uint32_t policy, S, nblocks;
  uint32_t multi;         // bit k: predictor k's code decodes two or three small symbols per lookup often
  uint64_t n;
  float mn;
  uint32_t pad2;
  double step;
  uint64_t off_pred, off_pfirst, off_cwords, off_nesc, off_payload, payload_words;
  uint32_t nsym[3], maxlen[3];
  uint64_t book_off[3];
  uint32_t grp_count[3];  // blocks per predictor
  uint32_t grp_start[3];  // first entry of each predictor's run in `desc`
};

struct alignas(16) DField {
  const uint8_t *in;
  uint64_t in_len;
  float *out;
  uint64_t n;             // expected field size
  uint32_t nblocks_max;
  uint32_t skip;          // set on the device: this descriptor decodes nothing
  DState *st;
  u32x4 *desc;            // per block, grouped by predictor: {block id, payload
                          // word offset, codewords | escapes << 16, first value}
  uint32_t *lut;          // 3 x (4096 first-code entries + 4096 small-symbol entries)
  uint32_t *slow;         // 3 x (32 first + 32 base + 64 limit words)
  uint16_t *syms;         // 3 x 65536 canonical symbols
};
constexpr int kSlowWords = 128;
// block sizes of the stream format: powers of two from 2^10 to 2^14 values
constexpr uint32_t kMinBlock = 1024, kMaxBlock = 16384;
// largest decode grid (workgroups); the decoder's piece tables are sized for it
constexpr uint32_t kMaxDecodeGrid = 8192;

// decode-table entry: sym | len << 16; flags.  A long entry (a prefix of
// codes longer than the table's bits) holds the shortest length under the
// prefix; with kLutOne every code under the prefix has that length and bits
// 0-15 hold the canonical index of the prefix's first code.
constexpr uint32_t kLutOne = 1u << 21;
constexpr uint32_t kLutLong = 1u << 22;
constexpr uint32_t kLutInvalid = 1u << 23;

// ------------------------------------------------------------ MD modes

constexpr uint32_t kMdSegMax = 16384;  // largest reorder / CPC segment
constexpr uint32_t kMdSub = 64;        // values per CPC decoder entry point
constexpr int kCpcThreads = (int)(kMdSegMax / kMdSub);  // CPC decoders: one thread per entry point of a segment
constexpr uint32_t kMdHdr = 96;        // container header bytes
constexpr uint32_t kCpHdr = 104;       // CPC coordinate stream header bytes
constexpr uint32_t kCvHdr = 56;        // CPC velocity stream header bytes

// Keying and stream state of one MD call, in the workspace.
struct MdCtl {
  uint32_t B, keybits, nseg, status;  // bits per key field, key bits, segments, first error
  uint32_t seg, digit, nk, kind;      // segment size, bits per radix digit, key fields, mode kind
  uint32_t shift[6];                  // six-field keys: low bits dropped from each field
  uint32_t vbits[3];                  // CPC2000: bits of each velocity lattice span
  uint32_t keysrc;
  uint64_t coord_bytes;               // CPC coordinate stream length
  uint64_t vel_bytes[3];              // CPC velocity stream lengths
  uint64_t sub_off[6], sub_len[6];    // decompression: sub-streams of the container
  uint32_t nsub, k;
};
struct MdPtrs {
  const float *f[6];
};
struct MdStates {
  const FState *s[6];
};
struct MdSubs {
  const uint8_t *p[6];
  const uint64_t *len[6];   // device words holding each sub-stream's length
};
struct MdStatus {
  const int32_t *s[8];
};

// ------------------------------------------------------ learned selector

// Network 16 -> 32 -> 32 -> 3 (ReLU); flat parameters W1[32][16], b1[32],
// W2[32][32], b2[32], W3[3][32], b3[3].
constexpr int kNFeat = 16;
constexpr int kMlpParams = 1699;
constexpr int kW1 = 0, kB1 = 512, kW2 = 544, kB2 = 1568, kW3 = 1600, kB3 = 1696;

// bfloat16 rounding to nearest, ties to even (finite values)
__host__ __device__ inline float bf16_round(float x) {
  uint32_t u;
  __builtin_memcpy(&u, &x, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  u &= 0xffff0000u;
  float r;
  __builtin_memcpy(&r, &u, 4);
  return r;
}

// bit length of v plus the 8 bits after its leading one, over 256
__device__ inline float flog_u64(uint64_t v) {
  if (!v) return 0.0f;
  const int b = 64 - __clzll((long long)v);
  const uint64_t frac = b - 1 >= 8 ? (v >> (b - 9)) & 255u : (v << (9 - b)) & 255u;
  return (float)b + (float)frac * (1.0f / 256.0f);
}

// Copy of the parameters in LDS for the wave inference below: each weight
// matrix output-major with its rows padded to 20 (W1) and 36 (W2, W3)
// words, so that one 128-bit read gives a lane four consecutive weights of
// its output and the lanes of a read fall on distinct banks.
constexpr int kR1 = 20, kR2 = 36;
constexpr int kL1 = 0, kLB1 = kL1 + 32 * kR1, kL2 = kLB1 + 32, kLB2 = kL2 + 32 * kR2, kL3 = kLB2 + 32,
              kLB3 = kL3 + 3 * kR2, kMlpLds = kLB3 + 4;
static_assert(kL2 % 4 == 0 && kL3 % 4 == 0, "rows start on 16-byte boundaries");
__device__ inline int mlp_lds_slot(int i) {
  if (i < kB1) return kL1 + (i / 16) * kR1 + i % 16;
  if (i < kW2) return kLB1 + (i - kB1);
  if (i < kB2) return kL2 + ((i - kW2) / 32) * kR2 + (i - kW2) % 32;
  if (i < kW3) return kLB2 + (i - kB2);
  if (i < kB3) return kL3 + ((i - kW3) / 32) * kR2 + (i - kW3) % 32;
  return kLB3 + (i - kB3);
}

// Orders the LDS accesses of one wave around it (a wave's LDS operations
// are executed in issue order; this keeps the compiler from moving them).
__device__ inline void wave_lds_order() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Inference on one block's features by one whole wave (lanes j and j + 32
// both compute neuron j).  wl: the LDS copy above, bfloat16-rounded weights
// and float32 biases; xb: the 16 features, already bfloat16-rounded, in LDS;
// s_h: 32 floats of LDS that only this wave uses (the hidden layers pass
// through it).  Each neuron starts from its bias and adds w_k x_k for k
// ascending, one fused multiply-add each; hidden outputs are ReLU'd and
// bfloat16-rounded.  Returns the argmax (ties to the lowest index) and the
// margin to the runner-up, uniform over the wave.  xb, wl and s_h are
// 16-byte aligned.
__device__ inline int mlp_select_wave(const float *__restrict__ wl, const float *xb, float *s_h, float &margin,
                                      float (&z_out)[3]) {
  const uint32_t lane = __lane_id();
  const int j = (int)(lane & 31u);
  const f32x4 *x4 = reinterpret_cast<const f32x4 *>(xb);
  const f32x4 *h4 = reinterpret_cast<const f32x4 *>(s_h);
  // sixteen terms per step: the reads of a step are issued together, steps
  // are kept apart so that no more than 32 registers hold operands
  const auto dot = [](float acc, const f32x4 *w, const f32x4 *x, int nq) {
#pragma unroll
    for (int q0 = 0; q0 < nq; q0 += 4) {
      if (q0) wave_lds_order();
#pragma unroll
      for (int q = q0; q < q0 + 4; q++) {
        const f32x4 a = w[q], b = x[q];
        acc = __builtin_fmaf(a.x, b.x, acc);
        acc = __builtin_fmaf(a.y, b.y, acc);
        acc = __builtin_fmaf(a.z, b.z, acc);
        acc = __builtin_fmaf(a.w, b.w, acc);
      }
    }
    return acc;
  };
  wave_lds_order();
  float acc = dot(wl[kLB1 + j], reinterpret_cast<const f32x4 *>(wl + kL1 + kR1 * j), x4, 4);
  const float h1 = bf16_round(acc > 0.0f ? acc : 0.0f);
  if (lane < 32u) s_h[j] = h1;
  wave_lds_order();
  acc = dot(wl[kLB2 + j], reinterpret_cast<const f32x4 *>(wl + kL2 + kR2 * j), h4, 8);
  const float h2 = bf16_round(acc > 0.0f ? acc : 0.0f);
  wave_lds_order();
  if (lane < 32u) s_h[j] = h2;
  wave_lds_order();
  const int jj = j < 3 ? j : 0;
  acc = dot(wl[kLB3 + jj], reinterpret_cast<const f32x4 *>(wl + kL3 + kR2 * jj), h4, 8);
  float z[3];
#pragma unroll
  for (int k = 0; k < 3; k++) z[k] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(acc), k));
  int top = 0;
  if (z[1] > z[top]) top = 1;
  if (z[2] > z[top]) top = 2;
  float second = -__builtin_inff();
#pragma unroll
  for (int k = 0; k < 3; k++)
    if (k != top && z[k] > second) second = z[k];
  margin = z[top] - second;
#pragma unroll
  for (int k = 0; k < 3; k++) z_out[k] = z[k];
  return top;
}

// ------------------------------------------------------------ primitives

__device__ inline uint32_t lane_id() { return __lane_id(); }

__device__ inline uint32_t float_key(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline float key_float(uint32_t k) {
  uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
  return __uint_as_float(u);
}

template <typename T>
__device__ inline T wave_incl_scan(T v) {
  const uint32_t l = lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    T o = __shfl_up(v, d, kWave);
    if (l >= (uint32_t)d) v += o;
  }
  return v;
}
// Inclusive wave64 prefix sum with DPP lane moves (GFX9: row_shr inside
// 16-lane rows, then row_bcast:15 and row_bcast:31 across rows); no LDS.
__device__ inline uint32_t wave_scan_dpp(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);  // row_shr:1
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);  // row_shr:2
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);  // row_shr:4
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);  // row_shr:8
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);  // row_bcast:15
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return x;
}

// Wave64 total under op with the same lane moves (op's identity must be 0,
// which the moves shift in); read from lane 63, uniform over the wave.
template <class Op>
__device__ inline uint32_t wave_reduce_dpp(uint32_t x, Op op) {
  x = op(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false));
  x = op(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false));
  x = op(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false));
  x = op(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false));
  x = op(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false));
  x = op(x, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false));
  return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int d = kWave / 2; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}
__device__ inline uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
  for (int d = kWave / 2; d >= 1; d >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, d, kWave));
  return v;
}
__device__ inline uint64_t wave_min_u64(uint64_t v) {
#pragma unroll
  for (int d = kWave / 2; d >= 1; d >>= 1) {
    const uint64_t o = __shfl_xor(v, d, kWave);
    v = o < v ? o : v;
  }
  return v;
}
__device__ inline uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
  for (int d = kWave / 2; d >= 1; d >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, d, kWave));
  return v;
}

// field of global block g (fblock0 holds nf+1 prefix entries)
__device__ inline int find_field(const uint64_t *fblock0, int nf, uint64_t g) {
  int lo = 0, hi = nf - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (fblock0[mid] <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Coherent (agent-scope) relaxed accesses.  Acquire/release would add cache
// write-back and invalidation to every access; the look-back words carry all
// the information their readers need, so none is required.
__device__ inline uint64_t ld_relaxed_u64(gptr<const uint64_t> p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_relaxed_u64(gptr<uint64_t> p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// 2 ulp of a float32 magnitude, exact, as a double
__device__ inline double guard_of(float am) {
  uint32_t e = (__float_as_uint(am) >> 23) & 0xffu;
  int ex = e == 0 ? -149 : (int)e - 150;
  return 2.0 * ldexp(1.0, ex);
}

}  // namespace sznb
