// Host side of the sznb C ABI: argument checks, workspace layout, launches.
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <cstdio>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "sznb_internal.h"

namespace sznb {

// kernels (defined in sznb_compress.hip / sznb_decompress.hip)
__global__ void k_init(const CField *, int, GCtl *, uint64_t *, uint64_t);
__global__ void k_range(const CField *, int, const uint64_t *, uint64_t);
__global__ void k_params(const CField *);
template <int E, bool kLearn>
__global__ void k_quant(const CField *, int, const uint64_t *, uint64_t, const uint32_t *, uint32_t,
                        const uint32_t *, uint32_t *, const float *);
__global__ void k_hmerge(const CField *, uint32_t, uint32_t, const uint32_t *, const uint32_t *);
__global__ void k_huff(const CField *, int, uint8_t *, uint64_t, uint32_t, GCtl *);
__global__ void k_books(const CField *);
template <int E> __global__ void k_pack(const CField *, int, const uint64_t *, uint64_t, GCtl *);
__global__ void k_final(const CField *, int);
uint64_t hscratch_bytes_host();

__global__ void d_prep(const DField *);
__global__ void d_heads(const DField *, int, uint32_t *);
__global__ void d_tables(const DField *);
__global__ void d_tasks(const DField *, int, uint32_t, uint32_t, uint32_t *, uint32_t *);
__global__ void d_const(const DField *, int, const uint32_t *);
__global__ void d_decode(const DField *, int, uint32_t *, uint32_t, uint32_t, uint32_t);

template <int E>
__global__ void k_features(const CField *, int, const uint64_t *, uint64_t, const uint32_t *, float *, uint64_t *,
                           uint8_t *);
__global__ void mlp_fwd_bwd(const float *, const float *, const uint8_t *, uint32_t, float *);
__global__ void mlp_grad(const float *, const float *, uint32_t, float *);
__global__ void mlp_loss(const float *, uint32_t, float *);
__global__ void mlp_adam(float *, float *, float *, const float *, uint32_t, float, float, float, float);
__global__ void mlp_infer(const float *, const float *, uint64_t, float *, uint8_t *, float *);
__global__ void md_bits(MdStates, int, MdStates, int, MdCtl *, uint64_t, uint32_t, uint32_t, uint32_t, uint32_t);
__global__ void md_keys(MdPtrs, MdStates, uint64_t, const MdCtl *, uint64_t *, uint32_t *);
__global__ void md_sort(uint64_t *, uint32_t *, uint64_t *, uint32_t *, uint64_t, uint32_t, const MdCtl *);
__global__ void md_gather(const float *, float *, const uint32_t *, uint64_t, const MdCtl *);
__global__ void md_vals(const float *, const uint32_t *, const FState *, uint64_t, const MdCtl *, uint64_t *);
__global__ void md_iota(uint32_t *, uint64_t);
template <bool kOffset>
__global__ void cpc_count(const uint64_t *, uint64_t, const MdCtl *, const uint32_t *, uint32_t *, uint32_t *,
                          uint64_t *);
template <bool kOffset>
__global__ void cpc_offsets(const uint32_t *, uint32_t, uint64_t, const MdCtl *, MdStates, int, uint8_t *, uint32_t *,
                            uint64_t *);
template <bool kOffset>
__global__ void cpc_pack(const uint64_t *, uint64_t, const MdCtl *, const uint32_t *, const uint32_t *,
                         const uint32_t *, const uint32_t *, const uint64_t *, uint8_t *);
__global__ void cpc_decode(const uint8_t *, const MdCtl *, uint64_t, uint64_t *, uint64_t *, int *);
__global__ void cpc_coords(const uint8_t *, const MdCtl *, uint64_t, const uint64_t *, const uint64_t *, float *,
                           float *, float *, const int *);
__global__ void cpv_decode(const uint8_t *, const MdCtl *, int, uint64_t, float *, int *);
__global__ void md_assemble(uint8_t *, uint64_t, uint64_t *, MdSubs, int, int, uint64_t, const MdCtl *, int *);
__global__ void md_parse(const uint8_t *, uint64_t, int, uint64_t, MdCtl *, DField *, int *);
__global__ void md_status(MdStatus, int, int32_t *);

constexpr uint64_t kStateStride = 256;

// ------------------------------------------------------------ profiling
// When enabled, every launch is bracketed by HIP events recorded on the
// caller's stream; sznb_profile_summary() aggregates them per kernel.
struct ProfRec {
  const char *name;
  hipEvent_t a, b;
};
static std::vector<ProfRec> g_prof;
static std::vector<hipEvent_t> g_evpool;
static size_t g_evnext = 0;
static bool g_prof_on = false;
static std::string g_prof_only;  // comma-separated kernel names to bracket; empty: every kernel

static bool prof_wanted(const char *name) {
  if (g_prof_only.empty()) return true;
  const size_t n = std::strlen(name);
  for (size_t p = 0; p <= g_prof_only.size();) {
    size_t q = g_prof_only.find(',', p);
    if (q == std::string::npos) q = g_prof_only.size();
    if (q - p == n && g_prof_only.compare(p, n, name) == 0) return true;
    p = q + 1;
  }
  return false;
}

static hipEvent_t prof_event() {
  if (g_evnext == g_evpool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    g_evpool.push_back(e);
  }
  return g_evpool[g_evnext++];
}
struct ProfScope {
  hipEvent_t b = nullptr;
  const char *name;
  hipStream_t s;
  ProfScope(const char *n, hipStream_t st) : name(n), s(st) {
    if (!g_prof_on || !prof_wanted(n)) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    hipEvent_t a = prof_event();
    b = prof_event();
    if (!a || !b) { b = nullptr; return; }
    (void)hipEventRecord(a, s);
    g_prof.push_back({name, a, b});
  }
  ~ProfScope() {
    if (b) (void)hipEventRecord(b, s);
  }
};
#define SZNB_LAUNCH(name, kernel, grid, block, lds, stream, ...)        \
  do {                                                                  \
    ProfScope _ps(name, stream);                                        \
    hipLaunchKernelGGL(kernel, grid, block, lds, stream, __VA_ARGS__); \
  } while (0)
static_assert(sizeof(FState) <= kStateStride, "FState too large");
static_assert(sizeof(DState) <= kStateStride, "DState too large");

__device__ uint32_t g_logt[16385];

// Workspace of the allocation-free decompression entry point: a fixed array
// in device memory, one copy per GPU for the life of the process.  Host code
// reaches it only through the address hipGetSymbolAddress gives per device
// (DevInfo::scratch), never through its name.
constexpr uint64_t kScratchBytes = 8ull << 20;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

struct DevInfo {
  int ok = 0;
  int cus = 0;
  size_t lds_per_block = 0;
  float *sel = nullptr;   // learned selector parameters on this device
  float tau = 0.0f;
  uint8_t *scratch = nullptr;  // this device's copy of `scratch`
};
static DevInfo g_dev[64];
static std::mutex g_mu;

static int dev_init(DevInfo **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return SZNB_EDEVICE;
  std::lock_guard<std::mutex> lk(g_mu);
  DevInfo &d = g_dev[dev];
  if (!d.ok) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return SZNB_EDEVICE;
    d.cus = p.multiProcessorCount;
    d.lds_per_block = p.sharedMemPerBlock;
    // LOG[m] = round(2^16 log2 m): the fixed-point log of the block-cost estimate
    std::vector<uint32_t> t(16385, 0u);
    for (int m = 1; m <= 16384; m++) t[m] = (uint32_t)std::floor(65536.0 * std::log2((double)m) + 0.5);
    if (hipMemcpyToSymbol(HIP_SYMBOL(g_logt), t.data(), t.size() * sizeof(uint32_t)) != hipSuccess) return SZNB_EDEVICE;
    if (hipGetSymbolAddress(reinterpret_cast<void **>(&d.scratch), HIP_SYMBOL(scratch)) != hipSuccess || !d.scratch)
      return SZNB_EDEVICE;
    if (hipDeviceSynchronize() != hipSuccess) return SZNB_EDEVICE;
    d.ok = 1;
  }
  *out = &d;
  return SZNB_OK;
}

static inline uint64_t al256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

// ------------------------------------------------------ descriptor uploads
// Host-built descriptors reach the workspace through pinned staging slots:
// a copy from pinned memory is queued and the call returns without waiting;
// a slot is refilled only after the event recorded behind its last copy.
// Uploads larger than a slot (or with staging unavailable or not wanted)
// are copied from the caller's memory and waited for.
struct Upload {
  void *dst;
  const void *src;
  size_t bytes;
};
constexpr int kStageSlots = 16;
constexpr size_t kStageSlotBytes = 1u << 20;
struct Staging {
  uint8_t *buf = nullptr;
  bool failed = false;
  hipEvent_t ev[kStageSlots] = {};
  bool used[kStageSlots] = {};
  int next = 0;
};
static Staging g_stage[64];

static int upload(const std::vector<Upload> &ups, hipStream_t s, bool may_stage) {
  size_t tot = 0;
  for (const Upload &u : ups) tot += al256(u.bytes);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return SZNB_EDEVICE;
  if (may_stage && tot <= kStageSlotBytes) {
    std::lock_guard<std::mutex> lk(g_mu);
    Staging &g = g_stage[dev];
    if (!g.buf && !g.failed) {
      bool ok = hipHostMalloc(reinterpret_cast<void **>(&g.buf), kStageSlots * kStageSlotBytes, hipHostMallocDefault) ==
                hipSuccess;
      for (int i = 0; ok && i < kStageSlots; i++)
        ok = hipEventCreateWithFlags(&g.ev[i], hipEventDisableTiming) == hipSuccess;
      if (!ok) g.failed = true;
    }
    if (g.buf && !g.failed) {
      const int slot = g.next;
      g.next = (g.next + 1) % kStageSlots;
      if (g.used[slot] && hipEventSynchronize(g.ev[slot]) != hipSuccess) return SZNB_EDEVICE;
      uint8_t *p0 = g.buf + (size_t)slot * kStageSlotBytes, *p = p0;
      // destinations laid out as the slot packs them take one copy
      bool packed = true;
      for (size_t i = 0; i + 1 < ups.size(); i++)
        packed = packed && static_cast<uint8_t *>(ups[i + 1].dst) == static_cast<uint8_t *>(ups[i].dst) +
                                                                       al256(ups[i].bytes);
      for (const Upload &u : ups) {
        std::memcpy(p, u.src, u.bytes);
        if (!packed && hipMemcpyAsync(u.dst, p, u.bytes, hipMemcpyHostToDevice, s) != hipSuccess) return SZNB_EDEVICE;
        p += al256(u.bytes);
      }
      if (packed && !ups.empty()) {
        const size_t span = (size_t)(p - p0) - al256(ups.back().bytes) + ups.back().bytes;
        if (hipMemcpyAsync(ups[0].dst, p0, span, hipMemcpyHostToDevice, s) != hipSuccess) return SZNB_EDEVICE;
      }
      if (hipEventRecord(g.ev[slot], s) != hipSuccess) return SZNB_EDEVICE;
      g.used[slot] = true;
      return SZNB_OK;
    }
  }
  for (const Upload &u : ups)
    if (hipMemcpyAsync(u.dst, u.src, u.bytes, hipMemcpyHostToDevice, s) != hipSuccess) return SZNB_EDEVICE;
  // pageable source buffers must stay valid until the copies are consumed
  return hipStreamSynchronize(s) == hipSuccess ? SZNB_OK : SZNB_EDEVICE;
}

// Header read-backs land in a pinned buffer per device (a copy into pageable
// memory would hold the host until the stream drains), held under the
// device's own lock from the copy until the values are read.
constexpr size_t kReadbackBytes = 1u << 16;
struct Readback {
  uint32_t *buf = nullptr;
  bool failed = false;
  std::mutex mu;
};
static Readback g_rb[64];

static int block_log2_of(uint32_t mode) {
  uint32_t b = (mode >> 8) & 15u;
  return b == 0 ? 12 : (int)b;
}
static bool mode_ok(uint32_t mode) {
  if (mode & ~(uint32_t)(3u | 16u | (15u << 8))) return false;
  int bl = block_log2_of(mode);
  return bl >= 10 && bl <= 14;
}

// ----------------------------------------------------------- compress plan

constexpr uint64_t kMaxQuantWG = 4096;  // workgroups of the quantization kernel, at most

struct CLayout {
  uint64_t gctl, states, fields, fb0, blkstat, lbflag, perfield_base, hscratch, qmeta, slabs, total;
  std::vector<uint64_t> hist, enc, book, nblocks, gblock0, nhist;
  uint64_t total_blocks;
  int nslots;         // Huffman workgroups, at most 64
  int hvar;           // Huffman variants per (field, predictor) pair
  uint32_t qslots;    // histogram windows per quantization workgroup
  uint64_t qmax;      // quantization workgroups the slabs are sized for
};

static CLayout compress_layout(int nf, const uint64_t *n, const uint32_t *mode) {
  CLayout L;
  uint64_t o = 0;
  L.total_blocks = 0;
  L.nblocks.resize(nf); L.gblock0.resize(nf); L.nhist.resize(nf);
  int npairs = 0;
  for (int f = 0; f < nf; f++) {
    const uint64_t S = 1ull << block_log2_of(mode[f]);
    L.nblocks[f] = (n[f] + S - 1) / S;
    L.gblock0[f] = L.total_blocks;
    L.total_blocks += L.nblocks[f];
    L.nhist[f] = (mode[f] & 3u) >= 2 ? 3 : 1;
    npairs += (int)L.nhist[f];
  }
  // quantization plan: per workgroup its first visit and first field, per
  // field its first and last workgroup; one histogram slab per visit
  L.qslots = 1;
  for (int f = 0; f < nf; f++) L.qslots = std::max<uint32_t>(L.qslots, (uint32_t)L.nhist[f]);
  L.qmax = std::max<uint64_t>(1, std::min<uint64_t>(kMaxQuantWG, L.total_blocks));
  L.gctl = o; o = al256(o + sizeof(GCtl));
  L.states = o; o = al256(o + kStateStride * nf);
  // the host-built descriptors back to back (one copy uploads them)
  L.fields = o; o = al256(o + sizeof(CField) * nf);
  L.fb0 = o; o = al256(o + 8ull * (nf + 1));
  L.qmeta = o; o = al256(o + 4ull * (2 * L.qmax + 1 + 2ull * nf));
  L.blkstat = o; o = al256(o + 12ull * L.total_blocks);
  L.lbflag = o; o = al256(o + 8ull * L.total_blocks);
  L.hist.resize(nf); L.enc.resize(nf); L.book.resize(nf);
  for (int f = 0; f < nf; f++) {
    L.hist[f] = o; o = al256(o + 4ull * kNSyms * L.nhist[f]);
    L.enc[f] = o; o = al256(o + 4ull * kNSyms * L.nhist[f]);
    L.book[f] = o; o = al256(o + 4ull * kBookWords * L.nhist[f]);
  }
  // Huffman workgroups: with few fields, several per (field, predictor)
  // pair, each starting from another number of weight halvings
  L.hvar = 3 * nf <= kHuffSlots / 2 ? std::min(4, kHuffSlots / (3 * nf)) : 1;
  L.nslots = L.hvar > 1 ? 3 * nf * L.hvar : std::min(std::max(npairs, 1), kHuffSlots);
  L.hscratch = o; o = al256(o + hscratch_bytes_host() * (uint64_t)L.nslots);
  L.slabs = o; o = al256(o + 4ull * kWinWords * (L.qmax + (uint64_t)nf));
  L.total = o;
  return L;
}

// The quantization plan of a grid of G workgroups over the field table:
// workgroup w takes blocks [w T / G, (w + 1) T / G).
static void quant_plan(const CLayout &L, int nf, uint32_t G, std::vector<uint32_t> &meta) {
  const uint64_t T = L.total_blocks;
  meta.assign(2 * (size_t)G + 1 + 2 * (size_t)nf, 0u);
  uint32_t *visit_base = meta.data(), *ffirst = visit_base + G + 1, *wf0 = ffirst + G, *wf1 = wf0 + nf;
  auto field_of = [&](uint64_t g) {  // largest f with gblock0[f] <= g (fields without blocks skipped)
    int lo = 0, hi = nf - 1;
    while (lo < hi) {
      int mid = (lo + hi + 1) >> 1;
      if (L.gblock0[mid] <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
  };
  for (int f = 0; f < nf; f++) { wf0[f] = 1; wf1[f] = 0; }
  for (uint32_t w = 0; w < G; w++) {
    const uint64_t gb = (uint64_t)w * T / G, ge = ((uint64_t)w + 1) * T / G;
    uint32_t f0 = 0, f1 = 0;
    if (ge > gb) {
      f0 = (uint32_t)field_of(gb);
      f1 = (uint32_t)field_of(ge - 1);
      for (uint32_t f = f0; f <= f1; f++) {
        if (wf0[f] > wf1[f]) wf0[f] = w;
        wf1[f] = w;
      }
    }
    ffirst[w] = f0;
    visit_base[w + 1] = visit_base[w] + (ge > gb ? f1 - f0 + 1 : 0);
  }
}

static uint64_t compress_bound_impl(uint64_t n, uint32_t mode) {
  const uint64_t S = 1ull << block_log2_of(mode);
  const uint64_t nb = (n + S - 1) / S;
  Sections s = sections_of(nb, (int)(mode & 3u));
  const uint64_t books = 3 * align8(4ull * kLMax + 2ull * kNSyms);
  const uint64_t cwmax = S * kLMax / 32;
  return s.books + books + 4ull * nb * (cwmax + S);
}

static uint64_t compress_min_cap_impl(uint64_t n, uint32_t mode) {
  const uint64_t S = 1ull << block_log2_of(mode);
  const uint64_t nb = (n + S - 1) / S;
  Sections s = sections_of(nb, (int)(mode & 3u));
  return s.books + 3 * align8(4ull * kLMax + 2ull * kNSyms);
}

struct Launch {
  int cus;
  bool learned;   // some field uses the learned policy
  uint32_t gq;    // quantization workgroups (the plan in the workspace is for this count)
  const float *sel;  // selector parameters of the learned policy (device)
  int E;
  uint64_t total_blocks;
  int nf;
  int nslots;
  uint8_t *ws;
  CLayout L;
};

template <int E>
static void launch_quant_pack(bool quant, const Launch &P, hipStream_t s, int grid) {
  const CField *F = reinterpret_cast<const CField *>(P.ws + P.L.fields);
  const uint64_t *fb0 = reinterpret_cast<const uint64_t *>(P.ws + P.L.fb0);
  if (quant) {
    uint32_t *logt = nullptr;
    (void)hipGetSymbolAddress(reinterpret_cast<void **>(&logt), HIP_SYMBOL(g_logt));
    const size_t smem = (size_t)kWinWords * sizeof(uint32_t);
    auto kern = P.learned ? k_quant<E, true> : k_quant<E, false>;
    SZNB_LAUNCH("k_quant", kern, dim3(P.gq), dim3(kThreads), smem, s, F, P.nf, fb0, P.total_blocks, logt,
                P.L.qslots, reinterpret_cast<const uint32_t *>(P.ws + P.L.qmeta),
                reinterpret_cast<uint32_t *>(P.ws + P.L.slabs), P.sel);
    SZNB_LAUNCH("k_hmerge", k_hmerge, dim3(qwin_of(P.L.qslots, 0).size / 256, P.L.qslots, P.nf), dim3(256), 0, s, F,
                P.L.qslots, P.gq,
                reinterpret_cast<const uint32_t *>(P.ws + P.L.qmeta),
                reinterpret_cast<const uint32_t *>(P.ws + P.L.slabs));
  } else {
    SZNB_LAUNCH("k_pack", k_pack<E>, dim3(grid), dim3(kThreads), 0, s, F, P.nf, fb0, P.total_blocks,
                reinterpret_cast<GCtl *>(P.ws + P.L.gctl));
  }
}

static void launch_E(bool quant, const Launch &P, hipStream_t s, int grid) {
  switch (P.E) {
    case 4: launch_quant_pack<4>(quant, P, s, grid); break;
    case 8: launch_quant_pack<8>(quant, P, s, grid); break;
    case 16: launch_quant_pack<16>(quant, P, s, grid); break;
    case 32: launch_quant_pack<32>(quant, P, s, grid); break;
    default: launch_quant_pack<64>(quant, P, s, grid); break;
  }
}

// workgroups per CU of the persistent per-block kernels (tunable)
static int g_wg_per_cu = 8;

// Workgroups of the quantization kernel: as many as stay resident together
// (each takes a contiguous run of blocks), at most the tunable width per CU,
// a multiple of the XCD count.
template <int E>
static int quant_occupancy(bool learned, size_t smem) {
  int occ = 0;
  auto kern = learned ? k_quant<E, true> : k_quant<E, false>;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, kThreads, smem) != hipSuccess || occ < 1) occ = 1;
  return occ;
}
static uint32_t quant_grid(int E, bool learned, const CLayout &L, int cus) {
  const size_t smem = (size_t)kWinWords * sizeof(uint32_t);
  int occ = 1;
  switch (E) {
    case 4: occ = quant_occupancy<4>(learned, smem); break;
    case 8: occ = quant_occupancy<8>(learned, smem); break;
    case 16: occ = quant_occupancy<16>(learned, smem); break;
    case 32: occ = quant_occupancy<32>(learned, smem); break;
    default: occ = quant_occupancy<64>(learned, smem); break;
  }
  occ = std::min(occ, g_wg_per_cu);
  uint64_t g = std::min<uint64_t>({(uint64_t)cus * (uint64_t)occ, L.total_blocks, L.qmax});
  if (g > 8) g &= ~uint64_t(7);
  return (uint32_t)std::max<uint64_t>(g, 1);
}

static int compress_run(const Launch &P, hipStream_t s, DevInfo *dv, bool params_only = false) {
  const CField *F = reinterpret_cast<const CField *>(P.ws + P.L.fields);
  const uint64_t *fb0 = reinterpret_cast<const uint64_t *>(P.ws + P.L.fb0);
  GCtl *gc = reinterpret_cast<GCtl *>(P.ws + P.L.gctl);
  uint64_t *lb = reinterpret_cast<uint64_t *>(P.ws + P.L.lbflag);
  const uint64_t tb = P.total_blocks;
  SZNB_LAUNCH("k_init", k_init, dim3(16, (unsigned)std::min(P.nf, 65535)), dim3(kThreads), 0, s, F, P.nf, gc, lb, tb);
  int gper = (int)std::min<uint64_t>((uint64_t)dv->cus * g_wg_per_cu, std::max<uint64_t>(tb, 1));
  if (gper > 8) gper &= ~7;  // multiple of the XCD count keeps a block on one XCD across passes
  if (tb) SZNB_LAUNCH("k_range", k_range, dim3(gper), dim3(kThreads), 0, s, F, P.nf, fb0, tb);
  SZNB_LAUNCH("k_params", k_params, dim3(P.nf), dim3(kThreads), 0, s, F);
  if (params_only) return hipGetLastError() == hipSuccess ? SZNB_OK : SZNB_EDEVICE;
  if (tb) launch_E(true, P, s, gper);
  SZNB_LAUNCH("k_huff", k_huff, dim3(P.L.nslots), dim3(1024), 0, s, F, P.nf, P.ws + P.L.hscratch, hscratch_bytes_host(),
              (uint32_t)P.L.hvar, gc);
  SZNB_LAUNCH("k_books", k_books, dim3(P.nf), dim3(kThreads), 0, s, F);
  // the pack kernel takes its blocks by ticket: one resident generation of
  // workgroups (four per CU) so that none pays its start-up twice
  if (tb) launch_E(false, P, s, (int)std::min<uint64_t>((uint64_t)dv->cus * 4, std::max<uint64_t>(tb, 1)));
  SZNB_LAUNCH("k_final", k_final, dim3((P.nf + 63) / 64), dim3(64), 0, s, F, P.nf);
  return hipGetLastError() == hipSuccess ? SZNB_OK : SZNB_EDEVICE;
}

// Validates a field table, writes its descriptors and quantization plan
// into the workspace (waits for the upload) and fills the launch record.
static int compress_prepare(int nf, const float *const *fields, const uint64_t *n, const double *eb,
                            const uint32_t *mode, void *const *outs, const uint64_t *caps, uint64_t *d_lens,
                            bool lens_is_array, void *d_ws, uint64_t ws_bytes, hipStream_t stream, Launch &P,
                            DevInfo *&dv) {
  if (nf <= 0 || !d_ws) return SZNB_EINVAL;
  int rc = dev_init(&dv);
  if (rc) return rc;
  uint32_t s0 = 0;
  for (int f = 0; f < nf; f++) {
    if (!mode_ok(mode[f]) || !(eb[f] > 0.0) || !std::isfinite(eb[f]) || n[f] >= SZNB_MAX_N) return SZNB_EINVAL;
    if (n[f] && (!fields[f] || (reinterpret_cast<uintptr_t>(fields[f]) & 15u))) return SZNB_EINVAL;
    if (!outs[f] || (reinterpret_cast<uintptr_t>(outs[f]) & 7u)) return SZNB_EINVAL;
    if (caps[f] < compress_min_cap_impl(n[f], mode[f])) return SZNB_ENOSPC;
    const uint32_t bl = (uint32_t)block_log2_of(mode[f]);
    if (f == 0) s0 = bl; else if (bl != s0) return SZNB_EINVAL;
  }
  CLayout L = compress_layout(nf, n, mode);
  if (ws_bytes < L.total) return SZNB_ENOSPC;
  uint8_t *ws = static_cast<uint8_t *>(d_ws);
  std::vector<CField> hf(nf);
  std::vector<uint64_t> fb0(nf + 1);
  for (int f = 0; f < nf; f++) {
    CField &c = hf[f];
    std::memset(&c, 0, sizeof c);
    const int bl = block_log2_of(mode[f]);
    c.x = fields[f];
    c.n = n[f];
    c.eb = eb[f];
    c.out = static_cast<uint8_t *>(outs[f]);
    c.out_cap = caps[f];
    c.out_len = d_lens ? (lens_is_array ? d_lens + f : d_lens) : nullptr;
    c.policy = mode[f] & 3u;
    c.eb_rel = (mode[f] >> 4) & 1u;
    c.S = 1u << bl;
    c.log2S = (uint32_t)bl;
    c.nblocks = (uint32_t)L.nblocks[f];
    c.nhist = (uint32_t)L.nhist[f];
    c.gblock0 = L.gblock0[f];
    c.sec = sections_of(L.nblocks[f], (int)c.policy);
    c.st = reinterpret_cast<FState *>(ws + L.states + kStateStride * f);
    c.blkstat = reinterpret_cast<uint32_t *>(ws + L.blkstat) + 3 * L.gblock0[f];
    c.hist = reinterpret_cast<uint32_t *>(ws + L.hist[f]);
    c.enc = reinterpret_cast<uint32_t *>(ws + L.enc[f]);
    c.book = reinterpret_cast<uint32_t *>(ws + L.book[f]);
    c.lbflag = reinterpret_cast<uint64_t *>(ws + L.lbflag) + L.gblock0[f];
    if (c.policy == 3) {
      if (!dv->sel) return SZNB_EINVAL;  // no selector loaded on this device
      c.sel = dv->sel;
      c.tau = dv->tau;
    }
    fb0[f] = L.gblock0[f];
  }
  fb0[nf] = L.total_blocks;
  bool learned = false;
  for (int f = 0; f < nf; f++) learned |= (mode[f] & 3u) == 3u;
  const uint32_t gq = quant_grid((int)((1u << s0) / kThreads), learned, L, dv->cus);
  std::vector<uint32_t> qmeta;
  quant_plan(L, nf, gq, qmeta);
  rc = upload({{ws + L.fields, hf.data(), sizeof(CField) * nf},
               {ws + L.fb0, fb0.data(), 8ull * (nf + 1)},
               {ws + L.qmeta, qmeta.data(), 4 * qmeta.size()}},
              stream, true);
  if (rc) return rc;
  P.cus = dv->cus;
  P.learned = learned;
  P.gq = gq;
  P.sel = dv->sel;
  P.E = (int)((1u << s0) / kThreads);
  P.total_blocks = L.total_blocks;
  P.nf = nf;
  P.nslots = L.nslots;
  P.ws = ws;
  P.L = L;
  return SZNB_OK;
}

static int compress_impl(int nf, const float *const *fields, const uint64_t *n, const double *eb,
                         const uint32_t *mode, void *const *outs, const uint64_t *caps, uint64_t *d_lens,
                         bool lens_is_array, void *d_ws, uint64_t ws_bytes, hipStream_t stream,
                         bool params_only = false) {
  Launch P;
  DevInfo *dv = nullptr;
  int rc = compress_prepare(nf, fields, n, eb, mode, outs, caps, d_lens, lens_is_array, d_ws, ws_bytes, stream, P, dv);
  if (rc) return rc;
  return compress_run(P, stream, dv, params_only);
}

// ------------------------------------------------- plans and HIP graphs

}  // namespace sznb

struct sznb_plan_s {
  sznb::Launch P;                 // compression plan
  sznb::DevInfo *dv = nullptr;
  void *dplan = nullptr;          // decompression plan (a DLaunch) instead, when set
  int device = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace sznb {

static int plan_create(int nf, const float *const *fields, const uint64_t *n, const double *eb, const uint32_t *mode,
                       void *const *outs, const uint64_t *caps, uint64_t *d_lens, void *d_ws, uint64_t ws_bytes,
                       hipStream_t stream, sznb_plan *out) {
  if (!out) return SZNB_EINVAL;
  *out = nullptr;
  sznb_plan p = new (std::nothrow) sznb_plan_s;
  if (!p) return SZNB_EDEVICE;
  int rc = compress_prepare(nf, fields, n, eb, mode, outs, caps, d_lens, true, d_ws, ws_bytes, stream, p->P, p->dv);
  if (rc == SZNB_OK && hipGetDevice(&p->device) != hipSuccess) rc = SZNB_EDEVICE;
  if (rc) { delete p; return rc; }
  *out = p;
  return SZNB_OK;
}

static int dplan_run(void *dplan, hipStream_t stream);

static int plan_body(sznb_plan p, hipStream_t stream) {
  return p->dplan ? dplan_run(p->dplan, stream) : compress_run(p->P, stream, p->dv);
}

static int plan_graph(sznb_plan p, hipStream_t stream) {
  if (!p) return SZNB_EINVAL;
  if (p->exec) return SZNB_OK;
  if (hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return SZNB_EDEVICE;
  const int rc = plan_body(p, stream);
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(stream, &g);
  if (rc || ec != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    return rc ? rc : SZNB_EDEVICE;
  }
  if (hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g);
    p->exec = nullptr;
    return SZNB_EDEVICE;
  }
  p->graph = g;
  return SZNB_OK;
}

static int plan_run(sznb_plan p, hipStream_t stream) {
  if (!p) return SZNB_EINVAL;
  if (p->exec) return hipGraphLaunch(p->exec, stream) == hipSuccess ? SZNB_OK : SZNB_EDEVICE;
  return plan_body(p, stream);
}

static void dplan_free(void *dplan);

static void plan_destroy(sznb_plan p) {
  if (!p) return;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->dplan) dplan_free(p->dplan);
  delete p;
}

// ------------------------------------------------------------- autotuner
//
// Times the compression of a field table for every block size 2^10..2^14
// and every persistent-grid width of 2, 4, 8, 16 workgroups per CU (kernel
// time, HIP events, best of three after a warm-up), keeps the candidates
// whose streams are within 1 % of the smallest, and picks the fastest.
// Results are cached in a text file, one line per key:
//   <arch>|<log2 total values>|<fields>|<policy bits> <block log2> <wg per CU> <ms>

static std::string tune_key(int nf, const uint64_t *n, uint32_t policy_mode) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  hipDeviceProp_t p;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&p, dev) == hipSuccess) arch = p.gcnArchName;
  for (char &ch : arch) if (ch == ' ' || ch == '|') ch = '_';
  uint64_t tot = 0;
  for (int f = 0; f < nf; f++) tot += n[f];
  int cls = 0;
  while ((tot >> cls) > 1) cls++;
  int fcls = 0;
  while ((1 << fcls) < nf) fcls++;
  char buf[256];
  std::snprintf(buf, sizeof buf, "%s|%d|%d|%u", arch.c_str(), cls, fcls, policy_mode & 0x13u);
  return buf;
}

static int autotune_impl(int nf, const float *const *fields, const uint64_t *n, const double *eb,
                         uint32_t policy_mode, const char *cache_path, uint32_t *best_mode, int *best_wg,
                         hipStream_t stream) {
  if (nf <= 0 || !best_mode || !best_wg || (policy_mode & ~0x13u)) return SZNB_EINVAL;
  DevInfo *dv;
  int rc = dev_init(&dv);
  if (rc) return rc;
  const std::string key = tune_key(nf, n, policy_mode);
  if (cache_path) {
    if (FILE *fp = std::fopen(cache_path, "r")) {
      char k[256];
      int bl = 0, wg = 0;
      double ms = 0;
      bool hit = false;
      while (std::fscanf(fp, "%255s %d %d %lf", k, &bl, &wg, &ms) == 4) {
        if (key == k && bl >= 10 && bl <= 14 && wg >= 1 && wg <= 16) {
          *best_mode = policy_mode | ((uint32_t)bl << 8);
          *best_wg = wg;
          hit = true;
        }
      }
      std::fclose(fp);
      if (hit) return SZNB_OK;
    }
  }
  // buffers for the largest candidate
  std::vector<uint64_t> caps(nf, 0);
  uint64_t wsb = 0;
  for (int bl = 10; bl <= 14; bl++) {
    std::vector<uint32_t> m(nf, policy_mode | ((uint32_t)bl << 8));
    wsb = std::max<uint64_t>(wsb, compress_layout(nf, n, m.data()).total);
    for (int f = 0; f < nf; f++) caps[f] = std::max<uint64_t>(caps[f], compress_bound_impl(n[f], m[f]));
  }
  std::vector<void *> outs(nf, nullptr);
  void *ws = nullptr;
  uint64_t *lens = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  bool ok = hipMalloc(&ws, wsb) == hipSuccess && hipMalloc(reinterpret_cast<void **>(&lens), 8ull * nf) == hipSuccess &&
            hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
  for (int f = 0; ok && f < nf; f++) ok = hipMalloc(&outs[f], caps[f]) == hipSuccess;
  struct Cand { int bl, wg; float ms; uint64_t bytes; };
  std::vector<Cand> cands;
  const int saved_wg = g_wg_per_cu;
  rc = ok ? SZNB_OK : SZNB_EDEVICE;
  for (int bl = 10; rc == SZNB_OK && bl <= 14; bl++) {
    std::vector<uint32_t> m(nf, policy_mode | ((uint32_t)bl << 8));
    Launch P;
    DevInfo *d2 = nullptr;
    rc = compress_prepare(nf, fields, n, eb, m.data(), outs.data(), caps.data(), lens, true, ws, wsb, stream, P, d2);
    for (int wg : {2, 4, 8, 16}) {
      if (rc) break;
      g_wg_per_cu = wg;
      float best = 1e30f;
      for (int rep = 0; rep < 4 && rc == SZNB_OK; rep++) {
        (void)hipEventRecord(e0, stream);
        rc = compress_run(P, stream, d2);
        (void)hipEventRecord(e1, stream);
        if (hipEventSynchronize(e1) != hipSuccess) rc = SZNB_EDEVICE;
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (rep) best = std::min(best, ms);
      }
      std::vector<uint64_t> hl(nf);
      if (rc == SZNB_OK && hipMemcpy(hl.data(), lens, 8ull * nf, hipMemcpyDeviceToHost) != hipSuccess) rc = SZNB_EDEVICE;
      uint64_t bytes = 0;
      for (uint64_t v : hl) bytes += v;
      if (rc == SZNB_OK) cands.push_back({bl, wg, best, bytes});
    }
  }
  g_wg_per_cu = saved_wg;
  for (void *p : outs) if (p) (void)hipFree(p);
  if (ws) (void)hipFree(ws);
  if (lens) (void)hipFree(lens);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (rc) return rc;
  uint64_t smallest = ~0ull;
  for (const Cand &c : cands) smallest = std::min(smallest, c.bytes);
  const Cand *pick = nullptr;
  for (const Cand &c : cands)
    if ((double)c.bytes <= 1.01 * (double)smallest && (!pick || c.ms < pick->ms)) pick = &c;
  if (!pick) return SZNB_EDEVICE;
  *best_mode = policy_mode | ((uint32_t)pick->bl << 8);
  *best_wg = pick->wg;
  if (cache_path) {
    if (FILE *fp = std::fopen(cache_path, "a")) {
      std::fprintf(fp, "%s %d %d %.4f\n", key.c_str(), pick->bl, pick->wg, pick->ms);
      std::fclose(fp);
    }
  }
  return SZNB_OK;
}

template <int E>
static int launch_features(const Launch &P, hipStream_t s, int grid, float *feat, uint64_t *cost, uint8_t *label) {
  const CField *F = reinterpret_cast<const CField *>(P.ws + P.L.fields);
  const uint64_t *fb0 = reinterpret_cast<const uint64_t *>(P.ws + P.L.fb0);
  uint32_t *logt = nullptr;
  if (hipGetSymbolAddress(reinterpret_cast<void **>(&logt), HIP_SYMBOL(g_logt)) != hipSuccess) return SZNB_EDEVICE;
  SZNB_LAUNCH("k_features", k_features<E>, dim3(grid), dim3(kThreads), 0, s, F, P.nf, fb0, P.total_blocks, logt, feat,
              cost, label);
  return hipGetLastError() == hipSuccess ? SZNB_OK : SZNB_EDEVICE;
}

// features, trial costs and trial choice of every block of a field table
static int features_impl(int nf, const float *const *fields, const uint64_t *n, const double *eb,
                         const uint32_t *mode, float *feat, uint64_t *cost, uint8_t *label, void *d_ws,
                         uint64_t ws_bytes, hipStream_t stream) {
  if (nf <= 0 || !feat || !cost || !label) return SZNB_EINVAL;
  // stream headers of the parameter pass go to the end of the workspace
  std::vector<uint64_t> caps(nf);
  std::vector<void *> outs(nf);
  CLayout L = compress_layout(nf, n, mode);
  uint64_t o = L.total;
  for (int f = 0; f < nf; f++) {
    if (!mode_ok(mode[f])) return SZNB_EINVAL;
    caps[f] = compress_min_cap_impl(n[f], mode[f]);
    outs[f] = static_cast<uint8_t *>(d_ws) + o;
    o = al256(o + caps[f]);
  }
  if (ws_bytes < o) return SZNB_ENOSPC;
  int rc = compress_impl(nf, fields, n, eb, mode, outs.data(), caps.data(), nullptr, false, d_ws, L.total, stream,
                         true);
  if (rc) return rc;
  DevInfo *dv;
  if ((rc = dev_init(&dv))) return rc;
  Launch P;
  P.cus = dv->cus;
  P.learned = false;
  P.gq = 1;
  P.sel = nullptr;
  P.E = (int)((1u << block_log2_of(mode[0])) / kThreads);
  P.total_blocks = L.total_blocks;
  P.nf = nf;
  P.nslots = L.nslots;
  P.ws = static_cast<uint8_t *>(d_ws);
  P.L = L;
  if (!L.total_blocks) return SZNB_OK;
  int grid = (int)std::min<uint64_t>((uint64_t)dv->cus * 8, L.total_blocks);
  switch (P.E) {
    case 4: return launch_features<4>(P, stream, grid, feat, cost, label);
    case 8: return launch_features<8>(P, stream, grid, feat, cost, label);
    case 16: return launch_features<16>(P, stream, grid, feat, cost, label);
    case 32: return launch_features<32>(P, stream, grid, feat, cost, label);
    default: return launch_features<64>(P, stream, grid, feat, cost, label);
  }
}

static uint64_t features_ws_bytes(int nf, const uint64_t *n, const uint32_t *mode) {
  uint64_t o = compress_layout(nf, n, mode).total;
  for (int f = 0; f < nf; f++) o = al256(o + compress_min_cap_impl(n[f], mode[f]));
  return o;
}

static int set_selector_impl(const float *h_params, float tau) {
  if (!h_params || std::isnan(tau)) return SZNB_EINVAL;
  DevInfo *dv;
  int rc = dev_init(&dv);
  if (rc) return rc;
  std::vector<float> w(h_params, h_params + kMlpParams);
  for (int i = 0; i < kMlpParams; i++) {
    const bool bias = (i >= kB1 && i < kW2) || (i >= kB2 && i < kW3) || i >= kB3;
    if (!std::isfinite(w[i])) return SZNB_EINVAL;
    if (!bias) w[i] = bf16_round(w[i]);
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!dv->sel && hipMalloc(reinterpret_cast<void **>(&dv->sel), sizeof(float) * kMlpParams) != hipSuccess) {
    dv->sel = nullptr;
    return SZNB_EDEVICE;
  }
  if (hipMemcpy(dv->sel, w.data(), sizeof(float) * kMlpParams, hipMemcpyHostToDevice) != hipSuccess)
    return SZNB_EDEVICE;
  dv->tau = tau;
  return SZNB_OK;
}

// ---------------------------------------------------------- decompress

struct DLayout {
  uint64_t gctl, states, fields, tbase, heads, total;
  std::vector<uint64_t> desc, lut, slow, syms, nbmax;
};

static DLayout decompress_layout(int nf, const uint64_t *n) {
  DLayout L;
  uint64_t o = 0;
  L.gctl = o; o = al256(o + sizeof(GCtl));
  L.states = o; o = al256(o + kStateStride * nf);
  L.fields = o; o = al256(o + sizeof(DField) * nf);
  // group offsets, piece tables and counters
  L.tbase = o; o = al256(o + 4ull * (6ull * nf + 3 + 3ull * (3ull * nf + kMaxDecodeGrid)));
  L.heads = o; o = al256(o + 16ull * nf);
  L.desc.resize(nf); L.lut.resize(nf); L.slow.resize(nf); L.syms.resize(nf); L.nbmax.resize(nf);
  for (int f = 0; f < nf; f++) {
    L.nbmax[f] = (n[f] + 1023) / 1024;
    L.desc[f] = o; o = al256(o + 16ull * L.nbmax[f]);
    L.lut[f] = o; o = al256(o + 4ull * 3 * (2u << kLutBits));  // per predictor: first-code table, small-symbol table
    L.slow[f] = o; o = al256(o + 4ull * 3 * kSlowWords);
    L.syms[f] = o; o = al256(o + 2ull * 3 * kNSyms);
  }
  L.total = o;
  return L;
}

// Everything a decompression launch needs beyond the workspace.
struct DLaunch {
  int nf = 0;
  uint8_t *ws = nullptr;
  DLayout L;
  uint32_t smax = 1024, symcap = 0, dw = 1, lut_words = 1u << kLutBits;
  size_t lds = 0;
  int grid = 1;
};

// Writes the stream descriptors, reads block size and codebook sizes of
// every header (one gather kernel, one copy back) and chooses the decoder's
// LDS layout: most resident waves per CU under the LDS of a CU, with the
// tables once per workgroup and one code region per wave (1 KiB stays free
// for the kernel's static LDS and alignment).
// With `assumed` (largest block size, largest codebook size) the headers are
// not read back: the launch is laid out for those sizes, the descriptors'
// stream pointers are left to a kernel (MD containers: md_parse) and the
// call does not wait for the GPU.
// The header checks and the decode tables (the first two kernels of every
// decompression).
static void launch_front(const DField *D, int nf, hipStream_t stream) {
  SZNB_LAUNCH("d_prep", d_prep, dim3(nf), dim3(1024), 0, stream, D);
  SZNB_LAUNCH("d_tables", d_tables, dim3(3 * nf), dim3(kThreads), 0, stream, D);
}

// With `front`, a call that reads the headers back also enqueues the first
// two kernels before it waits, and sets *front.
static int decompress_prepare(int nf, const void *const *streams, const uint64_t *lens, float *const *outs,
                              const uint64_t *n, void *d_ws, uint64_t ws_bytes, hipStream_t stream, DLaunch &P,
                              const uint32_t *assumed = nullptr, bool *front = nullptr) {
  if (nf <= 0 || !d_ws) return SZNB_EINVAL;
  DevInfo *dv;
  int rc = dev_init(&dv);
  if (rc) return rc;
  DLayout L = decompress_layout(nf, n);
  if (ws_bytes < L.total) return SZNB_ENOSPC;
  uint8_t *ws = static_cast<uint8_t *>(d_ws);
  std::vector<DField> hf(nf);
  for (int f = 0; f < nf; f++) {
    if (!assumed && (!streams[f] || lens[f] < kHdr || (reinterpret_cast<uintptr_t>(streams[f]) & 7u)))
      return SZNB_EINVAL;
    if (n[f] && (!outs[f] || (reinterpret_cast<uintptr_t>(outs[f]) & 15u))) return SZNB_EINVAL;
    if (n[f] >= SZNB_MAX_N) return SZNB_EINVAL;
    DField &d = hf[f];
    std::memset(&d, 0, sizeof d);
    d.in = assumed ? nullptr : static_cast<const uint8_t *>(streams[f]);
    d.in_len = assumed ? 0 : lens[f];
    d.skip = assumed ? 1u : 0u;
    d.out = outs[f];
    d.n = n[f];
    d.nblocks_max = (uint32_t)L.nbmax[f];
    d.st = reinterpret_cast<DState *>(ws + L.states + kStateStride * f);
    d.desc = reinterpret_cast<u32x4 *>(ws + L.desc[f]);
    d.lut = reinterpret_cast<uint32_t *>(ws + L.lut[f]);
    d.slow = reinterpret_cast<uint32_t *>(ws + L.slow[f]);
    d.syms = reinterpret_cast<uint16_t *>(ws + L.syms[f]);
  }
  uint32_t smax = 1024, nsym_max = 0;
  if (assumed) {
    rc = upload({{ws + L.fields, hf.data(), sizeof(DField) * nf}}, stream, true);
    if (rc) return rc;
    smax = assumed[0];
    nsym_max = assumed[1];
  } else {
    rc = upload({{ws + L.fields, hf.data(), sizeof(DField) * nf}}, stream, true);
    if (rc) return rc;
    const DField *D = reinterpret_cast<const DField *>(ws + L.fields);
    SZNB_LAUNCH("d_heads", d_heads, dim3((nf + 255) / 256), dim3(256), 0, stream, D, nf,
                reinterpret_cast<uint32_t *>(ws + L.heads));
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return SZNB_EDEVICE;
    Readback &rb = g_rb[dev];
    std::unique_lock<std::mutex> rlk(rb.mu, std::defer_lock);
    std::vector<uint32_t> hv;
    uint32_t *heads = nullptr;
    if (16ull * nf <= kReadbackBytes) {
      rlk.lock();
      if (!rb.buf && !rb.failed &&
          hipHostMalloc(reinterpret_cast<void **>(&rb.buf), kReadbackBytes, hipHostMallocDefault) != hipSuccess) {
        rb.buf = nullptr;
        rb.failed = true;
      }
      if (rb.buf) heads = rb.buf; else rlk.unlock();
    }
    if (!heads) {
      hv.resize(4ull * nf);
      heads = hv.data();
    }
    if (hipMemcpyAsync(heads, ws + L.heads, 16ull * nf, hipMemcpyDeviceToHost, stream) != hipSuccess)
      return SZNB_EDEVICE;
    hipEvent_t got;
    if (hipEventCreateWithFlags(&got, hipEventDisableTiming) != hipSuccess) return SZNB_EDEVICE;
    bool ok = hipEventRecord(got, stream) == hipSuccess;
    // header checks and decode tables need no launch layout: they run on
    // the device while the host waits for the header read-back (the launch
    // layout depends on the block and codebook sizes)
    if (ok && front) {
      launch_front(D, nf, stream);
      *front = true;
    }
    ok = ok && hipEventSynchronize(got) == hipSuccess;
    hipEventDestroy(got);
    if (!ok) return SZNB_EDEVICE;
    for (int f = 0; f < nf; f++) {
      const uint32_t S = heads[4 * f];
      if (S >= kMinBlock && S <= kMaxBlock && !(S & (S - 1)) && S > smax) smax = S;
      for (int k = 0; k < 3; k++) {
        const uint32_t ns = heads[4 * f + 1 + k];
        if (ns <= (uint32_t)kNSyms && ns > nsym_max) nsym_max = ns;
      }
    }
  }
  // the multi-symbol table pays when every codebook is small (short codes,
  // symbols near 32768); otherwise its LDS is better spent on waves
  const uint32_t lut_words = nsym_max <= 4096 ? (2u << kLutBits) : (1u << kLutBits);
  const size_t lds_cu = (dv->lds_per_block ? dv->lds_per_block : 65536) - 1024;
  const size_t tables = 4ull * lut_words + 4ull * 64 + 8ull * 32;
  const size_t per_wave = 2ull * smax;
  // canonical symbols in LDS (long codes resolve without a global read) or
  // in global memory (more waves per CU): the layout with more resident
  // waves wins, LDS symbols on a tie
  uint32_t symcap = 0, dw = 1, best = 0;
  for (uint32_t cap : {nsym_max, 0u}) {
    const size_t symb = (2ull * cap + 15) & ~15ull;
    for (uint32_t cand = 1; cand <= 16; cand++) {
      const size_t need = tables + symb + cand * per_wave;
      if (need > lds_cu) break;
      const uint32_t waves = cand * (uint32_t)(lds_cu / need);
      if (waves > best || (waves == best && cap == symcap)) { best = waves; dw = cand; symcap = cap; }
    }
  }
  const size_t symb = (2ull * symcap + 15) & ~15ull;
  const size_t lds = tables + symb + dw * per_wave;
  if (lds > 65536) {
    if (hipFuncSetAttribute(reinterpret_cast<const void *>(d_decode), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds) != hipSuccess)
      return SZNB_EDEVICE;
  }
  P.nf = nf;
  P.ws = ws;
  P.L = L;
  P.lut_words = lut_words;
  P.smax = smax;
  P.symcap = symcap;
  P.dw = dw;
  P.lds = lds;
  P.grid = (int)std::min<size_t>(kMaxDecodeGrid, (size_t)dv->cus * std::max<size_t>(1, lds_cu / lds));
  return SZNB_OK;
}

// Kernels only (capturable): streams whose block size exceeds the planned
// one are reported corrupt rather than decoded.  front_done: the first two
// kernels are already enqueued.
static int decompress_run(const DLaunch &P, hipStream_t stream, bool front_done = false) {
  const DField *D = reinterpret_cast<const DField *>(P.ws + P.L.fields);
  uint32_t *tbase = reinterpret_cast<uint32_t *>(P.ws + P.L.tbase);
  if (!front_done) launch_front(D, P.nf, stream);
  uint32_t *nconst = &reinterpret_cast<GCtl *>(P.ws + P.L.gctl)->pad[0];
  SZNB_LAUNCH("d_tasks", d_tasks, dim3(1), dim3(kThreads), 0, stream, D, P.nf, (uint32_t)P.grid, P.smax, tbase,
              nconst);
  SZNB_LAUNCH("d_const", d_const, dim3(256), dim3(kThreads), 0, stream, D, P.nf, nconst);
  SZNB_LAUNCH("d_decode", d_decode, dim3(P.grid), dim3(kWave * P.dw), P.lds, stream, D, P.nf, tbase, P.smax,
              P.symcap, P.lut_words);
  return hipGetLastError() == hipSuccess ? SZNB_OK : SZNB_EDEVICE;
}

static int decompress_impl(int nf, const void *const *streams, const uint64_t *lens, float *const *outs,
                           const uint64_t *n, void *d_ws, uint64_t ws_bytes, hipStream_t stream) {
  DLaunch P;
  bool front = false;
  int rc = decompress_prepare(nf, streams, lens, outs, n, d_ws, ws_bytes, stream, P, nullptr, &front);
  if (rc) return rc;
  return decompress_run(P, stream, front);
}

static int dplan_run(void *dplan, hipStream_t stream) {
  return decompress_run(*static_cast<DLaunch *>(dplan), stream);
}
static void dplan_free(void *dplan) { delete static_cast<DLaunch *>(dplan); }

static int dplan_create(int nf, const void *const *streams, const uint64_t *lens, float *const *outs,
                        const uint64_t *n, void *d_ws, uint64_t ws_bytes, hipStream_t stream, sznb_plan *out) {
  if (!out) return SZNB_EINVAL;
  *out = nullptr;
  DLaunch *dl = new (std::nothrow) DLaunch;
  sznb_plan p = new (std::nothrow) sznb_plan_s;
  if (!dl || !p) { delete dl; delete p; return SZNB_EDEVICE; }
  int rc = decompress_prepare(nf, streams, lens, outs, n, d_ws, ws_bytes, stream, *dl);
  if (rc == SZNB_OK && hipGetDevice(&p->device) != hipSuccess) rc = SZNB_EDEVICE;
  if (rc) { delete dl; delete p; return rc; }
  p->dplan = dl;
  *out = p;
  return SZNB_OK;
}

// ------------------------------------------------------------ MD modes

constexpr uint32_t kMdPrx = 6;  // Table 5: six ignored 3-bit digits
constexpr uint32_t kMdMode = SZNB_PRED_LV | SZNB_EB_REL;

// A decoded MD mode word (include/sznb.h).
struct MdMode {
  int kind = 0;          // 0 best_speed, 1 reorder + SZ-LV, 2 best_compression, 3 CPC2000
  uint32_t seg = kMdSegMax;
  uint32_t k = 0;        // ignored digits
  int keysrc = 0;        // 0 coordinates, 1 velocities, 2 all six fields
};
static int md_mode_of(int mode, int nf, MdMode &m) {
  const uint32_t u = (uint32_t)mode;
  m.kind = (int)(u & 255u);
  const uint32_t sl = (u >> 8) & 15u, kf = (u >> 12) & 15u;
  m.keysrc = (int)((u >> 16) & 3u);
  if (mode < 0 || (u >> 18) || m.kind > 3 || m.keysrc > 2 || (sl && (sl < 10 || sl > 14))) return SZNB_EINVAL;
  m.seg = 1u << (sl ? sl : 14);
  m.k = kf ? kf - 1 : (m.kind == 1 ? kMdPrx : 0u);
  if (m.kind == 0 && (sl || kf || m.keysrc)) return SZNB_EINVAL;
  if (m.keysrc && (nf != 6 || m.kind > 1)) return SZNB_EINVAL;
  if ((m.keysrc == 2 ? 6u : 3u) * m.k >= 64u) return SZNB_EINVAL;
  return SZNB_OK;
}

// MD workspace.  The call's status word sits where sznb_read_status(d_ws, 1)
// reads it.
struct MdLayout {
  uint64_t status, ctl, cstat, cws, hdr, keys0, keys1, idx0, idx1, perm, subs, sublen, segr, segb, segw, segm, coord,
      bws, total;
  uint64_t cws_bytes, hdr_cap, sub_cap, coord_cap, bws_bytes, nseg_max, perm_stride;
};

static uint64_t md_vel_cap(uint64_t n, uint64_t nseg) {  // worst case of a CPC velocity stream
  return kCvHdr + align8(4 * nseg) + align8(4 * (n / kMdSub + nseg)) + 8 * n + 8 * nseg + 64;
}

static MdLayout md_layout(int nf, uint64_t n) {
  MdLayout L;
  uint64_t o = 0;
  L.nseg_max = (n + 1023) / 1024;
  L.status = al256(sizeof(GCtl));
  o = L.status + kStateStride;
  L.ctl = o; o = al256(o + sizeof(MdCtl));
  L.cstat = o; o = al256(o + 64);
  std::vector<uint64_t> n6(6, n);
  std::vector<uint32_t> m6(6, kMdMode);
  L.cws_bytes = compress_layout(6, n6.data(), m6.data()).total;
  L.cws = o; o = al256(o + L.cws_bytes);
  L.hdr_cap = compress_min_cap_impl(n, kMdMode);
  L.hdr = o; o = al256(o + 6 * L.hdr_cap);
  L.keys0 = o; o = al256(o + 8 * n);
  L.keys1 = o; o = al256(o + 8 * n);
  L.idx0 = o; o = al256(o + 4 * n);
  L.idx1 = o; o = al256(o + 4 * n);
  L.perm_stride = al256(4 * n);
  L.perm = o; o = al256(o + L.perm_stride * nf);
  L.sub_cap = std::max(al256(compress_bound_impl(n, kMdMode)), al256(md_vel_cap(n, L.nseg_max)));
  L.subs = o; o = al256(o + L.sub_cap * nf);
  L.sublen = o; o = al256(o + 8 * 6);
  L.segr = o; o = al256(o + 4 * L.nseg_max);
  L.segb = o; o = al256(o + 4 * L.nseg_max);
  L.segw = o; o = al256(o + 4 * L.nseg_max);
  L.segm = o; o = al256(o + 8 * L.nseg_max);
  L.coord_cap = kCpHdr + align8(4 * L.nseg_max) + align8(4 * (n / kMdSub + L.nseg_max)) + 12 * n + 64 +
                8 * L.nseg_max;
  L.coord = o; o = al256(o + L.coord_cap);
  std::vector<uint64_t> nn(nf, n);
  std::vector<uint32_t> mm(nf, kMdMode);
  L.bws_bytes = std::max(compress_layout(nf, nn.data(), mm.data()).total, decompress_layout(nf, nn.data()).total);
  L.bws = o; o = al256(o + L.bws_bytes);
  L.total = o;
  return L;
}

// Enqueues the whole MD compression; returns without waiting.  The status
// of the call (first error of the keying, of any sub-stream, of the
// container) lands in the status word; the container length in *d_out_len.
static int md_compress_impl(int nf, const float *const *fields, uint64_t n, double eb_rel, int md_mode, void *d_out,
                            uint64_t out_cap, uint64_t *d_out_len, uint32_t *d_perm, void *d_ws, uint64_t ws_bytes,
                            hipStream_t s) {
  MdMode M;
  if ((nf != 3 && nf != 6) || md_mode_of(md_mode, nf, M) || n == 0 || n >= SZNB_MAX_N || !d_out || !d_ws)
    return SZNB_EINVAL;
  if (!(eb_rel > 0.0) || !std::isfinite(eb_rel)) return SZNB_EINVAL;
  for (int f = 0; f < nf; f++)
    if (!fields[f] || (reinterpret_cast<uintptr_t>(fields[f]) & 15u)) return SZNB_EINVAL;
  DevInfo *dv;
  int rc = dev_init(&dv);
  if (rc) return rc;
  MdLayout L = md_layout(nf, n);
  if (ws_bytes < L.total) return SZNB_ENOSPC;
  uint8_t *ws = static_cast<uint8_t *>(d_ws);
  MdCtl *ctl = reinterpret_cast<MdCtl *>(ws + L.ctl);
  int *cstat = reinterpret_cast<int *>(ws + L.cstat);
  if (hipMemsetAsync(ws + L.ctl, 0, L.cstat + 64 - L.ctl, s) != hipSuccess) return SZNB_EDEVICE;
  const int grid = dv->cus * 8;
  const unsigned nseg = (unsigned)((n + M.seg - 1) / M.seg);
  uint32_t *i0 = reinterpret_cast<uint32_t *>(ws + L.idx0), *i1 = reinterpret_cast<uint32_t *>(ws + L.idx1);
  uint64_t *k0 = reinterpret_cast<uint64_t *>(ws + L.keys0), *k1 = reinterpret_cast<uint64_t *>(ws + L.keys1);
  // the fields whose range and bound the keys and CPC2000 values need,
  // computed exactly as the compressor computes them
  std::vector<int> pf;
  if (M.kind >= 1) {
    if (M.keysrc != 1) for (int c = 0; c < 3; c++) pf.push_back(c);
    if (M.keysrc >= 1 || (M.kind == 3 && nf == 6)) for (int c = 3; c < 6; c++) pf.push_back(c);
  }
  const int np = (int)pf.size();
  auto state_of = [&](int f) -> const FState * {
    std::vector<uint64_t> nn(np, n);
    std::vector<uint32_t> mm(np, kMdMode);
    CLayout CL = compress_layout(np, nn.data(), mm.data());
    for (int i = 0; i < np; i++)
      if (pf[i] == f) return reinterpret_cast<const FState *>(ws + L.cws + CL.states + kStateStride * i);
    return nullptr;
  };
  MdStates ks{}, vs{};
  MdPtrs kf{};
  int nk = 0, nv = 0;
  if (np) {
    std::vector<const float *> pp(np);
    std::vector<uint64_t> nn(np, n);
    std::vector<double> ee(np, eb_rel);
    std::vector<uint32_t> mm(np, kMdMode);
    std::vector<void *> ho(np);
    std::vector<uint64_t> hc(np, L.hdr_cap);
    for (int i = 0; i < np; i++) { pp[i] = fields[pf[i]]; ho[i] = ws + L.hdr + i * L.hdr_cap; }
    rc = compress_impl(np, pp.data(), nn.data(), ee.data(), mm.data(), ho.data(), hc.data(), nullptr, false,
                       ws + L.cws, L.cws_bytes, s, true);
    if (rc) return rc;
    const int k0f = M.keysrc == 1 ? 3 : 0;
    nk = M.keysrc == 2 ? 6 : 3;
    for (int c = 0; c < nk; c++) { ks.s[c] = state_of(k0f + c); kf.f[c] = fields[k0f + c]; }
    if (M.kind == 3)
      for (int c = 3; c < nf; c++) vs.s[nv++] = state_of(c);
  }
  SZNB_LAUNCH("md_bits", md_bits, dim3(1), dim3(64), 0, s, ks, nk, vs, nv, ctl, n, M.seg, (uint32_t)M.kind,
              (uint32_t)M.keysrc, M.k);
  std::vector<const float *> szf;   // the SZ-LV inputs: the fields, or their reordered copies
  if (M.kind == 0) {
    for (int f = 0; f < nf; f++) szf.push_back(fields[f]);
    if (d_perm) SZNB_LAUNCH("md_iota", md_iota, dim3(grid), dim3(256), 0, s, d_perm, n);
  } else {
    SZNB_LAUNCH("md_keys", md_keys, dim3(grid), dim3(256), 0, s, kf, ks, n, ctl, k1, i1);
    // the sort's LDS-resident passes: 8 bytes per element of a segment
    const size_t sort_lds = 8ull * M.seg;
    if (hipFuncSetAttribute(reinterpret_cast<const void *>(md_sort), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)sort_lds) != hipSuccess)
      return SZNB_EDEVICE;
    SZNB_LAUNCH("md_sort", md_sort, dim3(nseg), dim3(1024), sort_lds, s, k1, i1, k0, i0, n, M.k, ctl);
    const int first = M.kind == 2 ? 3 : M.kind == 3 ? nf : 0;
    for (int f = first; f < nf; f++) {
      float *pfp = reinterpret_cast<float *>(ws + L.perm + L.perm_stride * f);
      SZNB_LAUNCH("md_gather", md_gather, dim3(grid), dim3(256), 0, s, fields[f], pfp, i0, n, ctl);
      szf.push_back(pfp);
    }
    uint32_t *sr = reinterpret_cast<uint32_t *>(ws + L.segr), *sbits = reinterpret_cast<uint32_t *>(ws + L.segb);
    uint32_t *sw = reinterpret_cast<uint32_t *>(ws + L.segw);
    uint64_t *sm = reinterpret_cast<uint64_t *>(ws + L.segm);
    if (M.kind >= 2) {
      uint8_t *cs = ws + L.coord;
      SZNB_LAUNCH("cpc_count", cpc_count<false>, dim3(nseg), dim3(1024), 0, s, k0, n, ctl, &ctl->keybits, sr, sbits,
                  sm);
      SZNB_LAUNCH("cpc_offsets", cpc_offsets<false>, dim3(1), dim3(64), 0, s, sbits, (uint32_t)L.nseg_max, n, ctl,
                  ks, 0, cs, sw, &ctl->coord_bytes);
      SZNB_LAUNCH("cpc_pack", cpc_pack<false>, dim3(nseg), dim3(1024), 0, s, k0, n, ctl, &ctl->keybits, sr, sbits,
                  sw, sm, cs);
    }
    if (M.kind == 3) {
      for (int j = 0; j < nv; j++) {
        uint8_t *vsb = ws + L.subs + (uint64_t)j * L.sub_cap;
        MdStates one{};
        one.s[0] = vs.s[j];
        SZNB_LAUNCH("md_vals", md_vals, dim3(grid), dim3(256), 0, s, fields[3 + j], i0, vs.s[j], n, ctl, k1);
        SZNB_LAUNCH("cpc_count", cpc_count<true>, dim3(nseg), dim3(1024), 0, s, k1, n, ctl, &ctl->vbits[j], sr,
                    sbits, sm);
        SZNB_LAUNCH("cpc_offsets", cpc_offsets<true>, dim3(1), dim3(64), 0, s, sbits, (uint32_t)L.nseg_max, n, ctl,
                    one, j, vsb, sw, &ctl->vel_bytes[j]);
        SZNB_LAUNCH("cpc_pack", cpc_pack<true>, dim3(nseg), dim3(1024), 0, s, k1, n, ctl, &ctl->vbits[j], sr, sbits,
                    sw, sm, vsb);
      }
    }
    if (d_perm && hipMemcpyAsync(d_perm, i0, 4 * n, hipMemcpyDeviceToDevice, s) != hipSuccess) return SZNB_EDEVICE;
  }
  // SZ-LV streams of the (reordered) fields
  const int nsz = (int)szf.size();
  const int szbase = M.kind == 3 ? nv : 0;  // CPC2000's velocity streams take the first sub-stream buffers
  MdSubs subs{};
  int nsub = 0;
  if (M.kind >= 2) { subs.p[nsub] = ws + L.coord; subs.len[nsub] = &ctl->coord_bytes; nsub++; }
  for (int j = 0; M.kind == 3 && j < nv; j++) {
    subs.p[nsub] = ws + L.subs + (uint64_t)j * L.sub_cap;
    subs.len[nsub] = &ctl->vel_bytes[j];
    nsub++;
  }
  uint64_t *sublen = reinterpret_cast<uint64_t *>(ws + L.sublen);
  MdStatus ss{};
  int nss = 0;
  ss.s[nss++] = reinterpret_cast<const int32_t *>(&ctl->status);
  if (nsz) {
    std::vector<uint64_t> nn(nsz, n), caps(nsz, L.sub_cap);
    std::vector<double> ee(nsz, eb_rel);
    std::vector<uint32_t> mm(nsz, kMdMode);
    std::vector<void *> outs(nsz);
    for (int i = 0; i < nsz; i++) outs[i] = ws + L.subs + (uint64_t)(szbase + i) * L.sub_cap;
    rc = compress_impl(nsz, szf.data(), nn.data(), ee.data(), mm.data(), outs.data(), caps.data(), sublen, true,
                       ws + L.bws, L.bws_bytes, s);
    if (rc) return rc;
    for (int i = 0; i < nsz; i++) {
      subs.p[nsub] = static_cast<const uint8_t *>(outs[i]);
      subs.len[nsub] = sublen + i;
      nsub++;
      ss.s[nss++] = reinterpret_cast<const int32_t *>(ws + L.bws + al256(sizeof(GCtl)) + kStateStride * i);
    }
  }
  SZNB_LAUNCH("md_assemble", md_assemble, dim3(grid), dim3(256), 0, s, static_cast<uint8_t *>(d_out), out_cap,
              d_out_len, subs, nsub, nf, n, ctl, cstat);
  // statuses: the keying, every SZ stream, then the container (whose ENOSPC
  // may only echo a failed sub-stream)
  ss.s[nss++] = cstat;
  SZNB_LAUNCH("md_status", md_status, dim3(1), dim3(64), 0, s, ss, nss, reinterpret_cast<int32_t *>(ws + L.status));
  return hipGetLastError() == hipSuccess ? SZNB_OK : SZNB_EDEVICE;
}

// Enqueues the whole MD decompression; returns without waiting (status as
// for compression).  The container header is read on the device: md_parse
// points the SZ-LV decoder's descriptors and the CPC decoders at the
// sub-streams, so the host needs nothing from the stream.
static int md_decompress_impl(const void *d_in, uint64_t in_len, int nf, uint64_t n, float *const *outs, void *d_ws,
                              uint64_t ws_bytes, hipStream_t s) {
  if ((nf != 3 && nf != 6) || !d_in || (reinterpret_cast<uintptr_t>(d_in) & 7u) || in_len < kMdHdr || n == 0 ||
      n >= SZNB_MAX_N || !d_ws)
    return SZNB_EINVAL;
  for (int f = 0; f < nf; f++)
    if (!outs[f] || (reinterpret_cast<uintptr_t>(outs[f]) & 15u)) return SZNB_EINVAL;
  DevInfo *dv;
  int rc = dev_init(&dv);
  if (rc) return rc;
  MdLayout L = md_layout(nf, n);
  if (ws_bytes < L.total) return SZNB_ENOSPC;
  uint8_t *ws = static_cast<uint8_t *>(d_ws);
  const uint8_t *in = static_cast<const uint8_t *>(d_in);
  MdCtl *ctl = reinterpret_cast<MdCtl *>(ws + L.ctl);
  int *cstat = reinterpret_cast<int *>(ws + L.cstat);
  if (hipMemsetAsync(ws + L.ctl, 0, L.cstat + 64 - L.ctl, s) != hipSuccess) return SZNB_EDEVICE;
  // SZ-LV sub-streams are 4096-value blocks; codebooks up to 8192 symbols
  // keep their symbols in LDS
  const uint32_t assumed[2] = {4096u, 8192u};
  std::vector<uint64_t> nn(nf, n);
  DLaunch P;
  rc = decompress_prepare(nf, nullptr, nullptr, outs, nn.data(), ws + L.bws, L.bws_bytes, s, P, assumed);
  if (rc) return rc;
  DField *D = reinterpret_cast<DField *>(P.ws + P.L.fields);
  SZNB_LAUNCH("md_parse", md_parse, dim3(1), dim3(64), 0, s, in, in_len, nf, n, ctl, D, cstat);
  rc = decompress_run(P, s);
  if (rc) return rc;
  const unsigned gmax = (unsigned)L.nseg_max;  // the smallest segment size's count: extra workgroups return
  // relative keys and the bases of every 64 keys (n / 64 + 1 entries at most)
  uint64_t *keys = reinterpret_cast<uint64_t *>(ws + L.keys0), *kbase = reinterpret_cast<uint64_t *>(ws + L.keys1);
  SZNB_LAUNCH("cpc_decode", cpc_decode, dim3(gmax), dim3(kCpcThreads), 0, s, in, ctl, n, keys, kbase, cstat);
  SZNB_LAUNCH("cpc_coords", cpc_coords, dim3(dv->cus * 8), dim3(256), 0, s, in, ctl, n, keys, kbase, outs[0],
              outs[1], outs[2], cstat);
  for (int j = 0; j + 3 < nf; j++)
    SZNB_LAUNCH("cpv_decode", cpv_decode, dim3(gmax), dim3(kCpcThreads), 0, s, in, ctl, j, n, outs[3 + j], cstat);
  MdStatus ss{};
  int nss = 0;
  ss.s[nss++] = cstat;
  for (int f = 0; f < nf; f++)
    ss.s[nss++] = reinterpret_cast<const int32_t *>(P.ws + P.L.states + kStateStride * f);
  SZNB_LAUNCH("md_status", md_status, dim3(1), dim3(64), 0, s, ss, nss, reinterpret_cast<int32_t *>(ws + L.status));
  return hipGetLastError() == hipSuccess ? SZNB_OK : SZNB_EDEVICE;
}

}  // namespace sznb

using namespace sznb;

extern "C" {

uint64_t sznb_compress_bound(uint64_t n, uint32_t mode) { return compress_bound_impl(n, mode); }

uint64_t sznb_compress_min_capacity(uint64_t n, uint32_t mode) { return compress_min_cap_impl(n, mode); }

uint64_t sznb_compress_workspace_bytes(int nf, const uint64_t *h_n, const uint32_t *h_mode) {
  if (nf <= 0) return 0;
  return compress_layout(nf, h_n, h_mode).total;
}

int sznb_compress(const float *d_field, uint64_t n, double eb, uint32_t mode, void *d_out, uint64_t out_cap,
                  uint64_t *d_out_len, void *d_ws, uint64_t ws_bytes, hipStream_t stream) {
  void *outs[1] = {d_out};
  return compress_impl(1, &d_field, &n, &eb, &mode, outs, &out_cap, d_out_len, false, d_ws, ws_bytes, stream);
}

int sznb_compress_batch(int nf, const float *const *h_fields, const uint64_t *h_n, const double *h_eb,
                        const uint32_t *h_mode, void *const *h_outs, const uint64_t *h_caps, uint64_t *d_lens,
                        void *d_ws, uint64_t ws_bytes, hipStream_t stream) {
  return compress_impl(nf, h_fields, h_n, h_eb, h_mode, h_outs, h_caps, d_lens, true, d_ws, ws_bytes, stream);
}

int sznb_stream_info(const void *h_hdr, uint64_t hdr_len, uint64_t *n, uint32_t *mode, double *eb_abs,
                     uint64_t *total_bytes) {
  if (!h_hdr || hdr_len < kHdr) return SZNB_EINVAL;
  const uint8_t *h = static_cast<const uint8_t *>(h_hdr);
  uint32_t magic;
  uint16_t ver;
  std::memcpy(&magic, h, 4);
  std::memcpy(&ver, h + 4, 2);
  if (magic != kMagic || ver != 1) return SZNB_ECORRUPT;
  uint32_t S;
  std::memcpy(&S, h + H_S, 4);
  int bl = 0;
  while ((1u << bl) < S && bl < 31) bl++;
  if (n) std::memcpy(n, h + H_N, 8);
  if (mode) *mode = (uint32_t)h[H_POLICY] | ((h[H_FLAGS] & 2u) ? SZNB_EB_REL : 0u) | SZNB_BLOCK_LOG2(bl);
  if (eb_abs) std::memcpy(eb_abs, h + H_EBABS, 8);
  if (total_bytes) std::memcpy(total_bytes, h + H_TOTAL, 8);
  return SZNB_OK;
}

uint64_t sznb_decompress_workspace_bytes(int nf, const uint64_t *h_n) {
  if (nf <= 0) return 0;
  return decompress_layout(nf, h_n).total;
}

int sznb_decompress(const void *d_stream, uint64_t stream_len, float *d_out, uint64_t n, void *d_ws,
                    uint64_t ws_bytes, hipStream_t stream) {
  float *outs[1] = {d_out};
  return decompress_impl(1, &d_stream, &stream_len, outs, &n, d_ws, ws_bytes, stream);
}

int sznb_decompress_noalloc(const void *d_stream, uint64_t stream_len, float *d_out, uint64_t n,
                            hipStream_t stream) {
  DevInfo *dv = nullptr;
  int rc = dev_init(&dv);
  if (rc) return rc;
  if (n > SZNB_NOALLOC_MAX_N || decompress_layout(1, &n).total > kScratchBytes) return SZNB_ENOSPC;
  float *outs[1] = {d_out};
  rc = decompress_impl(1, &d_stream, &stream_len, outs, &n, dv->scratch, kScratchBytes, stream);
  if (rc) return rc;
  int st = SZNB_OK;
  return sznb_read_status(dv->scratch, 1, &st, stream);
}

int sznb_decompress_batch(int nf, const void *const *h_streams, const uint64_t *h_lens, float *const *h_outs,
                          const uint64_t *h_n, void *d_ws, uint64_t ws_bytes, hipStream_t stream) {
  return decompress_impl(nf, h_streams, h_lens, h_outs, h_n, d_ws, ws_bytes, stream);
}

int sznb_read_status(const void *d_ws, int nf, int *h_status, hipStream_t stream) {
  if (!d_ws || nf <= 0 || !h_status) return SZNB_EINVAL;
  if (hipStreamSynchronize(stream) != hipSuccess) return SZNB_EDEVICE;
  const uint8_t *base = static_cast<const uint8_t *>(d_ws) + al256(sizeof(GCtl));
  int first = SZNB_OK;
  for (int f = 0; f < nf; f++) {
    int32_t v = 0;
    if (hipMemcpy(&v, base + kStateStride * f, 4, hipMemcpyDeviceToHost) != hipSuccess) return SZNB_EDEVICE;
    h_status[f] = v;
    if (v != SZNB_OK && first == SZNB_OK) first = v;
  }
  return first;
}

int sznb_compress_plan(int nf, const float *const *h_fields, const uint64_t *h_n, const double *h_eb,
                       const uint32_t *h_mode, void *const *h_outs, const uint64_t *h_caps, uint64_t *d_lens,
                       void *d_ws, uint64_t ws_bytes, hipStream_t stream, sznb_plan *plan_out) {
  return plan_create(nf, h_fields, h_n, h_eb, h_mode, h_outs, h_caps, d_lens, d_ws, ws_bytes, stream, plan_out);
}
int sznb_decompress_plan(int nf, const void *const *h_streams, const uint64_t *h_lens, float *const *h_outs,
                         const uint64_t *h_n, void *d_ws, uint64_t ws_bytes, hipStream_t stream, sznb_plan *plan_out) {
  return dplan_create(nf, h_streams, h_lens, h_outs, h_n, d_ws, ws_bytes, stream, plan_out);
}
int sznb_plan_capture(sznb_plan plan, hipStream_t stream) { return plan_graph(plan, stream); }
int sznb_plan_launch(sznb_plan plan, hipStream_t stream) { return plan_run(plan, stream); }
void sznb_plan_destroy(sznb_plan plan) { plan_destroy(plan); }

int sznb_set_workgroups_per_cu(int wg) {
  if (wg < 1 || wg > 16) return SZNB_EINVAL;
  g_wg_per_cu = wg;
  return SZNB_OK;
}
int sznb_get_workgroups_per_cu(void) { return g_wg_per_cu; }

int sznb_autotune(int nf, const float *const *h_fields, const uint64_t *h_n, const double *h_eb,
                  uint32_t policy_mode, const char *cache_path, uint32_t *h_best_mode, int *h_best_wg,
                  hipStream_t stream) {
  return autotune_impl(nf, h_fields, h_n, h_eb, policy_mode, cache_path, h_best_mode, h_best_wg, stream);
}

int sznb_set_selector(const float *h_params, float tau) { return set_selector_impl(h_params, tau); }

uint64_t sznb_features_workspace_bytes(int nf, const uint64_t *h_n, const uint32_t *h_mode) {
  return features_ws_bytes(nf, h_n, h_mode);
}

int sznb_block_features(int nf, const float *const *h_fields, const uint64_t *h_n, const double *h_eb,
                        const uint32_t *h_mode, float *d_feat, uint64_t *d_cost, uint8_t *d_label, void *d_ws,
                        uint64_t ws_bytes, hipStream_t stream) {
  return features_impl(nf, h_fields, h_n, h_eb, h_mode, d_feat, d_cost, d_label, d_ws, ws_bytes, stream);
}

int sznb_compress_fallbacks(const void *d_ws, int nf, uint32_t *h_out, hipStream_t stream) {
  if (!d_ws || nf <= 0 || !h_out) return SZNB_EINVAL;
  if (hipStreamSynchronize(stream) != hipSuccess) return SZNB_EDEVICE;
  const uint8_t *ws = static_cast<const uint8_t *>(d_ws);
  for (int f = 0; f < nf; f++) {
    const uint8_t *st = ws + al256(sizeof(GCtl)) + kStateStride * f + offsetof(FState, fallbacks);
    if (hipMemcpy(&h_out[f], st, 4, hipMemcpyDeviceToHost) != hipSuccess) return SZNB_EDEVICE;
  }
  return SZNB_OK;
}

uint64_t sznb_mlp_grad_workspace_bytes(uint32_t batch) { return 4ull * 132 * batch; }

int sznb_mlp_grad(const float *d_params, const float *d_feat, const uint8_t *d_label, uint32_t batch, float *d_grad,
                  float *d_loss, void *d_ws, uint64_t ws_bytes, hipStream_t stream) {
  if (!d_params || !d_feat || !d_label || !d_grad || !d_loss || !d_ws || batch == 0) return SZNB_EINVAL;
  if (ws_bytes < sznb_mlp_grad_workspace_bytes(batch)) return SZNB_ENOSPC;
  float *buf = static_cast<float *>(d_ws);
  SZNB_LAUNCH("mlp_fwd_bwd", mlp_fwd_bwd, dim3((batch + 255) / 256), dim3(256), 0, stream, d_params, d_feat, d_label,
              batch, buf);
  SZNB_LAUNCH("mlp_grad", mlp_grad, dim3((kMlpParams + 255) / 256), dim3(256), 0, stream, d_feat, buf, batch, d_grad);
  SZNB_LAUNCH("mlp_loss", mlp_loss, dim3(1), dim3(256), 0, stream, buf, batch, d_loss);
  return hipGetLastError() == hipSuccess ? SZNB_OK : SZNB_EDEVICE;
}

int sznb_mlp_adam(float *d_params, float *d_m, float *d_v, const float *d_grad, uint32_t step, float lr, float beta1,
                  float beta2, float eps, hipStream_t stream) {
  if (!d_params || !d_m || !d_v || !d_grad || step == 0) return SZNB_EINVAL;
  SZNB_LAUNCH("mlp_adam", mlp_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, stream, d_params, d_m, d_v, d_grad,
              step, lr, beta1, beta2, eps);
  return hipGetLastError() == hipSuccess ? SZNB_OK : SZNB_EDEVICE;
}

int sznb_mlp_infer(const float *d_params, const float *d_feat, uint64_t nb, float *d_logits, uint8_t *d_choice,
                   float *d_margin, hipStream_t stream) {
  if (!d_params || !d_feat || !d_logits || !d_choice || !d_margin) return SZNB_EINVAL;
  if (!nb) return SZNB_OK;
  DevInfo *dv;
  int rc = dev_init(&dv);
  if (rc) return rc;
  const uint64_t grid = std::min<uint64_t>((nb + 3) / 4, (uint64_t)dv->cus * 8);
  SZNB_LAUNCH("mlp_infer", mlp_infer, dim3((unsigned)grid), dim3(256), 0, stream, d_params, d_feat, nb, d_logits,
              d_choice, d_margin);
  return hipGetLastError() == hipSuccess ? SZNB_OK : SZNB_EDEVICE;
}

uint64_t sznb_md_workspace_bytes(int nf, uint64_t n) { return md_layout(nf, n).total; }

uint64_t sznb_md_bound(int nf, uint64_t n) {
  const MdLayout L = md_layout(nf, n);
  return kMdHdr + (uint64_t)nf * L.sub_cap + align8(L.coord_cap);
}

int sznb_md_compress(int nf, const float *const *h_fields, uint64_t n, double eb_rel, int md_mode, void *d_out,
                     uint64_t out_cap, uint64_t *d_out_len, uint32_t *d_perm_or_null, void *d_ws, uint64_t ws_bytes,
                     hipStream_t stream) {
  return md_compress_impl(nf, h_fields, n, eb_rel, md_mode, d_out, out_cap, d_out_len, d_perm_or_null, d_ws, ws_bytes,
                          stream);
}

int sznb_md_decompress(const void *d_in, uint64_t in_len, int nf, uint64_t n, float *const *h_outs, void *d_ws,
                       uint64_t ws_bytes, hipStream_t stream) {
  return md_decompress_impl(d_in, in_len, nf, n, h_outs, d_ws, ws_bytes, stream);
}

int sznb_profile(int enable) {
  if (enable) {
    g_prof.clear();
    g_evnext = 0;
  }
  g_prof_on = enable != 0;
  return SZNB_OK;
}

int sznb_profile_kernels(const char *names) {
  g_prof_only = names ? names : "";
  return SZNB_OK;
}

int sznb_profile_summary(int max_kernels, char *names, double *total_ms, int *count) {
  std::vector<const char *> keys;
  std::vector<double> tot;
  std::vector<int> cnt;
  for (const ProfRec &r : g_prof) {
    if (hipEventSynchronize(r.b) != hipSuccess) return SZNB_EDEVICE;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return SZNB_EDEVICE;
    size_t i = 0;
    while (i < keys.size() && std::strcmp(keys[i], r.name) != 0) i++;
    if (i == keys.size()) { keys.push_back(r.name); tot.push_back(0.0); cnt.push_back(0); }
    tot[i] += ms;
    cnt[i] += 1;
  }
  const int nk = (int)keys.size();
  for (int i = 0; i < nk && i < max_kernels; i++) {
    std::strncpy(names + 32 * i, keys[i], 31);
    names[32 * i + 31] = 0;
    total_ms[i] = tot[i];
    count[i] = cnt[i];
  }
  return nk;
}

const char *sznb_strerror(int status) {
  switch (status) {
    case SZNB_OK: return "ok";
    case SZNB_EINVAL: return "invalid argument";
    case SZNB_ENONFINITE: return "field holds NaN or Inf";
    case SZNB_EEBTOOSMALL: return "error bound below float32 resolution or lattice too large";
    case SZNB_ENOSPC: return "output buffer or workspace too small";
    case SZNB_ECORRUPT: return "corrupt stream";
    case SZNB_EDEVICE: return "HIP runtime error";
    default: return "unknown status";
  }
}

}  // extern "C"
