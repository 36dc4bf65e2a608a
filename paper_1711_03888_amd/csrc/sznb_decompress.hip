// Decompression kernels of the sznb library (gfx950, wave64).
//
//   d_prep     header validation, one descriptor per block (id, payload
//              word offset, codeword and escape counts, first value) in
//              predictor-grouped order (one workgroup per stream)
//   d_tables   canonical decode tables per (stream, predictor): a 4096-entry
//              first-level table and per-length limits for longer codes
//   d_tasks    group offsets and the pieces (runs of one group's blocks,
//              one per decode workgroup) with their counters
//   d_decode   one wave per block: parallel Huffman decode of the block's
//              ranges from the skip-table entry points (one lane per range),
//              escapes, inverse prediction by a wave scan of affine prefix
//              maps, reconstruction x~ = fl32(fma(p, step, mn))
//   d_const    constant streams
#include "sznb_internal.h"

namespace sznb {

template <class P>
__device__ inline uint32_t rd32(P p, uint64_t off) {
  return (uint32_t)p[off] | ((uint32_t)p[off + 1] << 8) | ((uint32_t)p[off + 2] << 16) | ((uint32_t)p[off + 3] << 24);
}
template <class P>
__device__ inline uint64_t rd64(P p, uint64_t off) {
  return (uint64_t)rd32(p, off) | ((uint64_t)rd32(p, off + 4) << 32);
}
template <class P>
__device__ inline uint16_t rd16(P p, uint64_t off) {
  return (uint16_t)(p[off] | (p[off + 1] << 8));
}

// ---------------------------------------------------------------- prep

// block size and codebook sizes of every header (for the launch layout)
__global__ void d_heads(const DField *__restrict__ D, int nf, uint32_t *heads) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  const DField &df = D[f];
  uint32_t v[4] = {0u, 0u, 0u, 0u};
  if (df.in_len >= (uint64_t)kHdr && rd32(df.in, H_MAGIC) == kMagic) {
    v[0] = rd32(df.in, H_S);
    for (int k = 0; k < 3; k++) v[1 + k] = rd32(df.in, H_NSYM + 4 * k);
  }
  for (int k = 0; k < 4; k++) heads[4 * f + k] = v[k];
}

constexpr int kPrepThreads = 1024;
constexpr uint32_t kPrepBatch = 8;
__global__ __launch_bounds__(kPrepThreads) void d_prep(const DField *__restrict__ D) {
  const DField &df = D[blockIdx.x];
  DState *st = df.st;
  const uint8_t *in = df.in;
  const int t = threadIdx.x;
  __shared__ int s_bad;
  __shared__ uint32_t s_tot[kPrepThreads / kWave][4];
  // the header, read by 32 threads at once and parsed from LDS
  __shared__ uint32_t s_hdr[kHdr / 4];
  if (df.skip) {  // an unused descriptor of an MD container: no stream, no work
    if (t == 0) {
      st->status = 0;
      st->is_const = 0;
      st->nblocks = 0;
      for (int k = 0; k < 3; k++) { st->nsym[k] = 0; st->grp_count[k] = 0; st->grp_start[k] = 0; }
    }
    return;
  }
  if (t < kHdr / 4) s_hdr[t] = df.in_len >= (uint64_t)kHdr ? rd32(G(in), 4ull * t) : 0u;
  __syncthreads();
  if (t == 0) {
    const uint8_t *hb = reinterpret_cast<const uint8_t *>(s_hdr);
    int bad = 0;
    st->status = 0;
    st->is_const = 0;
    st->multi = 0;
    if (df.in_len < (uint64_t)kHdr || rd32(hb, H_MAGIC) != kMagic || rd16(hb, H_VERSION) != 1) bad = 1;
    uint32_t policy = 0, flags = 0, S = 0, nb = 0;
    uint64_t n = 0, total = 0;
    if (!bad) {
      policy = hb[H_POLICY];
      flags = hb[H_FLAGS];
      n = rd64(hb, H_N);
      S = rd32(hb, H_S);
      nb = rd32(hb, H_NB);
      total = rd64(hb, H_TOTAL);
      if (policy > 3 || n != df.n || total > df.in_len || S < kMinBlock || S > kMaxBlock || (S & (S - 1))) bad = 1;
    }
    st->policy = policy; st->S = S; st->n = n;
    st->mn = __uint_as_float(bad ? 0u : rd32(hb, H_MN));
    if (!bad && (flags & 1u)) {
      st->is_const = 1;
      st->nblocks = 0;
    } else if (!bad) {
      const uint64_t nbx = (n + S - 1) / S;
      if (nb != nbx || nb > df.nblocks_max || n == 0) bad = 1;
      Sections sec = sections_of(nb, (int)policy);
      st->step = __longlong_as_double((long long)rd64(hb, H_STEP));
      st->off_pred = rd64(hb, H_OFF_PRED);
      st->off_pfirst = rd64(hb, H_OFF_PFIRST);
      st->off_cwords = rd64(hb, H_OFF_CWORDS);
      st->off_nesc = rd64(hb, H_OFF_NESC);
      const uint64_t off_books = rd64(hb, H_OFF_BOOKS);
      st->off_payload = rd64(hb, H_OFF_PAYLOAD);
      st->payload_words = rd64(hb, H_PWORDS);
      if (st->off_pred != sec.pred || st->off_pfirst != sec.pfirst || st->off_cwords != sec.cwords ||
          st->off_nesc != sec.nesc || off_books != sec.books)
        bad = 1;
      uint64_t o = off_books;
      for (int k = 0; k < 3; k++) {
        const uint32_t ns = rd32(hb, H_NSYM + 4 * k), ml = hb[H_MAXLEN + k];
        st->nsym[k] = ns;
        st->maxlen[k] = ml;
        st->book_off[k] = o;
        if ((ns == 0) != (ml == 0) || ns > (uint32_t)kNSyms || ml > (uint32_t)kLMax) bad = 1;
        o += book_bytes(ns, ml);
      }
      if (policy < 2 && st->nsym[policy] == 0) bad = 1;
      if (o != st->off_payload || st->off_payload + 4 * st->payload_words != total) bad = 1;
      st->nblocks = bad ? 0 : nb;
    }
    s_bad = bad;
  }
  __syncthreads();
  if (s_bad) {
    if (t == 0) { st->status = SZNB_ECORRUPT; st->nblocks = 0; }
    return;
  }
  if (st->is_const) return;
  // block word offsets and predictor groups (the state's fields in registers)
  const uint32_t nb = st->nblocks, policy = st->policy, S = st->S;
  const uint64_t nval = st->n;
  const uint32_t nsym[3] = {st->nsym[0], st->nsym[1], st->nsym[2]};
  const uint32_t mlen[3] = {st->maxlen[0], st->maxlen[1], st->maxlen[2]};
  const uint32_t cwmax = S * kLMax / 32;
  // The block table entries are read kPrepBatch blocks at a time, all loads
  // of a batch issued before any is used.  Streams start at 8-byte aligned
  // addresses (the host checks plain streams; a container's sub-streams sit
  // at multiples of 8 from its aligned start) and the table's sections start
  // at multiples of 8 of the stream and are padded to 8, so a batch starting
  // at a block multiple of 8 is read in 8-byte words, each word loaded only
  // if its first block is in the thread's run (the word then lies inside its
  // section).
  const gptr<const uint8_t> gin = G(in);
  static_assert(kPrepBatch == 8, "a batch is one 8-byte word of predictor bytes");
  const uint32_t per = ((nb + kPrepThreads - 1) / kPrepThreads + 7u) & ~7u;
  const uint32_t lo = min(nb, t * per), hi = min(nb, lo + per);
  const uint64_t ocw = st->off_cwords, one = st->off_nesc, opr = st->off_pred, opf = st->off_pfirst;
  auto w64 = [&](uint64_t off) { return *reinterpret_cast<gptr<const uint64_t>>(gin + off); };
  auto batch = [&](uint32_t b0, uint32_t (&cwv)[kPrepBatch], uint32_t (&nev)[kPrepBatch], uint32_t (&kv)[kPrepBatch]) {
    const bool two = b0 + 4 < hi;
    const uint64_t c0 = w64(ocw + 2ull * b0), c1 = two ? w64(ocw + 2ull * b0 + 8) : 0ull;
    const uint64_t n0 = w64(one + 2ull * b0), n1 = two ? w64(one + 2ull * b0 + 8) : 0ull;
    const uint64_t k8 = policy >= 2 ? w64(opr + b0) : 0ull;
#pragma unroll
    for (uint32_t j = 0; j < kPrepBatch; j++) {
      cwv[j] = (uint32_t)((j < 4 ? c0 : c1) >> (16 * (j & 3))) & 0xffffu;
      nev[j] = (uint32_t)((j < 4 ? n0 : n1) >> (16 * (j & 3))) & 0xffffu;
      kv[j] = policy >= 2 ? (uint32_t)(k8 >> (8 * j)) & 0xffu : policy;
    }
  };
  auto firsts = [&](uint32_t b0, uint32_t (&p0v)[kPrepBatch]) {
#pragma unroll
    for (uint32_t i = 0; i < kPrepBatch / 2; i++) {
      const uint64_t v = b0 + 2 * i < hi ? w64(opf + 4ull * b0 + 8 * i) : 0ull;
      p0v[2 * i] = (uint32_t)v;
      p0v[2 * i + 1] = (uint32_t)(v >> 32);
    }
  };
  uint32_t words = 0, cnt[3] = {0, 0, 0}, bad = 0;
  for (uint32_t b0 = lo; b0 < hi; b0 += kPrepBatch) {
    uint32_t cwv[kPrepBatch], nev[kPrepBatch], kv[kPrepBatch];
    batch(b0, cwv, nev, kv);
#pragma unroll
    for (uint32_t j = 0; j < kPrepBatch; j++) {
      const uint32_t b = b0 + j;
      if (b >= hi) break;
      const uint32_t cw = cwv[j], ne = nev[j], k = kv[j];
      const uint32_t blen = (uint32_t)min((uint64_t)S, nval - (uint64_t)b * S);
      if (k > 2 || (k == 0 ? nsym[0] : k == 1 ? nsym[1] : nsym[2]) == 0 || cw > cwmax || ne > blen) { bad = 1; continue; }
      cnt[k]++;
      words += skip_words(cw, k == 0 ? mlen[0] : k == 1 ? mlen[1] : mlen[2]) + cw + ne;
    }
  }
  // workgroup exclusive scans of (words, cnt0, cnt1, cnt2)
  uint32_t v[4] = {words, cnt[0], cnt[1], cnt[2]}, ex[4], tot[4];
  const int w = t / kWave;
  for (int i = 0; i < 4; i++) {
    uint32_t inc = wave_incl_scan(v[i]);
    ex[i] = inc - v[i];
    if (lane_id() == kWave - 1) s_tot[w][i] = inc;
  }
  bad = wave_max_u32(bad);
  if (lane_id() == 0 && bad) s_bad = 1;
  __syncthreads();
  for (int i = 0; i < 4; i++) {
    tot[i] = 0;
    for (int j = 0; j < kPrepThreads / kWave; j++) {
      if (j < w) ex[i] += s_tot[j][i];
      tot[i] += s_tot[j][i];
    }
  }
  if (s_bad || tot[0] != st->payload_words) {
    if (t == 0) { st->status = SZNB_ECORRUPT; st->nblocks = 0; }
    return;
  }
  uint32_t gstart[3] = {0, tot[1], tot[1] + tot[2]};
  uint32_t run = ex[0], gpos[3] = {gstart[0] + ex[1], gstart[1] + ex[2], gstart[2] + ex[3]};
  // each block's descriptor goes to its predictor group's next slot, so a
  // decoding wave reads everything it needs to start a block in one load
  const gptr<u32x4> desc = G(df.desc);
  for (uint32_t b0 = lo; b0 < hi; b0 += kPrepBatch) {
    uint32_t cwv[kPrepBatch], nev[kPrepBatch], kv[kPrepBatch], p0v[kPrepBatch];
    batch(b0, cwv, nev, kv);
    firsts(b0, p0v);
#pragma unroll
    for (uint32_t j = 0; j < kPrepBatch; j++) {
      const uint32_t b = b0 + j;
      if (b >= hi) break;
      const uint32_t k = kv[j];
      const uint32_t gp = k == 0 ? gpos[0]++ : k == 1 ? gpos[1]++ : gpos[2]++;
      desc[gp] = u32x4{b, run, cwv[j] | (nev[j] << 16), p0v[j]};
      run += skip_words(cwv[j], k == 0 ? mlen[0] : k == 1 ? mlen[1] : mlen[2]) + cwv[j] + nev[j];
    }
  }
  if (t == 0) {
    for (int k = 0; k < 3; k++) { st->grp_count[k] = tot[1 + k]; st->grp_start[k] = gstart[k]; }
  }
}

// --------------------------------------------------------------- tables

__global__ __launch_bounds__(kThreads) void d_tables(const DField *__restrict__ D) {
  const DField &df = D[blockIdx.x / 3];
  const int k = blockIdx.x % 3;
  DState *st = df.st;
  const int t = threadIdx.x;
  __shared__ uint32_t s_cnt[32], s_first[32], s_base[32];
  __shared__ uint64_t s_limit[32];
  __shared__ int s_ok;
  if (st->status != 0 || st->is_const || st->nsym[k] == 0) return;
  const uint8_t *in = df.in;
  const uint32_t ns = st->nsym[k], ml = st->maxlen[k];
  const uint64_t bo = st->book_off[k];
  // the per-length counts, read by ml threads at once
  if (t < 32) s_cnt[t] = (t >= 1 && (uint32_t)t <= ml) ? rd32(G(in), bo + 4ull * (t - 1)) : 0u;
  __syncthreads();
  if (t == 0) {
    uint32_t tot = 0, code = 0, idx = 0;
    int ok = 1;
    for (int l = 0; l < 32; l++) { s_first[l] = 0; s_base[l] = 0; s_limit[l] = 0; }
    for (uint32_t l = 1; l <= ml; l++) tot += s_cnt[l];
    if (tot != ns || s_cnt[ml] == 0) ok = 0;
    for (uint32_t l = 1; l <= ml && ok; l++) {
      s_first[l] = code;
      s_base[l] = idx;
      if ((uint64_t)code + s_cnt[l] > (1ull << l)) ok = 0;  // not a prefix code
      s_limit[l] = ((uint64_t)code + s_cnt[l]) << (32 - l);
      code = (code + s_cnt[l]) << 1;
      idx += s_cnt[l];
    }
    s_ok = ok;
  }
  __syncthreads();
  if (!s_ok) {
    if (t == 0) st->status = SZNB_ECORRUPT;
    return;
  }
  // the canonical symbols (ns 16-bit words at so, a multiple of 4 in an
  // 8-byte aligned stream; the book is padded to 8 bytes) go to the
  // workspace two at a time, four loads per thread in flight.  The first
  // level below reads the few it needs straight from the stream, so it does
  // not wait for this copy.
  const uint64_t so = bo + 4ull * ml;
  const gptr<const uint32_t> sw = reinterpret_cast<gptr<const uint32_t>>(G(in) + so);
  const gptr<uint32_t> symw = reinterpret_cast<gptr<uint32_t>>(G(df.syms) + (uint64_t)k * kNSyms);
  const uint32_t npair = (ns + 1) / 2;
  for (uint32_t i0 = 0; i0 < npair; i0 += 4u * kThreads) {
    uint32_t a[4];
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const uint32_t i = i0 + (uint32_t)u * kThreads + t;
      a[u] = i < npair ? sw[i] : 0u;
    }
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const uint32_t i = i0 + (uint32_t)u * kThreads + t;
      if (i < npair) symw[i] = a[u];
    }
  }
  // first code of every 12-bit window: its symbol and length, then how many
  // whole codes the window holds and their total length (bits 24-27 and
  // 28-31: the counting pass steps over all of them at once)
  __shared__ uint8_t s_len[1u << kLutBits];  // length of a code within the window, 0 if none
  __shared__ uint16_t s_sym[1u << kLutBits];  // its symbol
  uint32_t *lut = df.lut + (uint64_t)k * (2u << kLutBits);
  uint32_t *lut2 = lut + (1u << kLutBits);
  uint32_t ents[(1u << kLutBits) / kThreads];
  for (uint32_t e = t, j = 0; e < (1u << kLutBits); e += kThreads, j++) {
    const uint64_t win = (uint64_t)e << (32 - kLutBits);
    uint32_t len = 1;
    for (uint32_t l = 1; l <= ml; l++) len += s_limit[l] <= win;
    uint32_t ent;
    if (len > ml) ent = kLutInvalid | 0xffffu | (1u << 16);
    else if (len > (uint32_t)kLutBits) {
      // shortest code under this prefix; when the prefix's last window has a
      // code of the same length, every code under it has that length and
      // its canonical index follows from the bits after the prefix
      const uint64_t wl = win | ((1ull << (32 - kLutBits)) - 1u);
      uint32_t ll = 1;
      for (uint32_t l = 1; l <= ml; l++) ll += s_limit[l] <= wl;
      ent = kLutLong | (len << 16);
      if (ll == len) ent |= kLutOne | (s_base[len] - s_first[len] + (e << (len - kLutBits)));
    } else {
      const uint32_t code = (uint32_t)(win >> (32 - len)), si = s_base[len] + (code - s_first[len]);
      ent = ((sw[si >> 1] >> (16u * (si & 1u))) & 0xffffu) | (len << 16);
    }
    ents[j] = ent;
    s_len[e] = (uint8_t)((ent & (kLutInvalid | kLutLong)) ? 0u : len);
    s_sym[e] = (uint16_t)(ent & 0xffffu);
  }
  __syncthreads();
  // second table, in one of two forms: up to three leading codes of the
  // window whose symbols are within 127 of 32768, as signed bytes (bits
  // 0-23), their count (24-25) and total length (26-29); or up to six whose
  // symbols are within 7 of 32768, as signed nibbles (0-23), count (24-26)
  // and length (27-30).  The form that yields more symbols over the 4096
  // windows is kept.
  __shared__ uint32_t s_sum[2], s_nm[2];
  __shared__ uint32_t s_e6[1u << kLutBits];
  if (t < 2) { s_sum[t] = 0; s_nm[t] = 0; }
  __syncthreads();
  uint32_t sum3 = 0, sum6 = 0, nm3 = 0, nm6 = 0;
#pragma unroll
  for (uint32_t e = t, j = 0; e < (1u << kLutBits); e += kThreads, j++) {
    uint32_t pos = 0, cnt = 0, n2 = 0, l2 = 0, d3 = 0, n6 = 0, l6 = 0, d6 = 0;
    bool small = true, tiny = true;
    for (;;) {
      // code at bit pos of the window (bits past the window read as zero;
      // a code is counted only if it ends inside the window)
      const uint32_t w = (e << pos) & ((1u << kLutBits) - 1u);
      const uint32_t l = s_len[w];
      if (!l || pos + l > (uint32_t)kLutBits) break;
      const int32_t dv = (int32_t)s_sym[w] - kRadius;
      if (small && n2 < 3u && dv >= -128 && dv <= 127) {
        d3 |= ((uint32_t)dv & 255u) << (8 * n2);
        n2++;
        l2 = pos + l;
      } else {
        small = false;
      }
      if (tiny && n6 < 6u && dv >= -8 && dv <= 7) {
        d6 |= ((uint32_t)dv & 15u) << (4 * n6);
        n6++;
        l6 = pos + l;
      } else {
        tiny = false;
      }
      pos += l;
      cnt++;
    }
    lut[e] = ents[j] | (cnt << 24) | (pos << 28);
    lut2[e] = d3 | (n2 << 24) | (l2 << 26);
    s_e6[e] = d6 | (n6 << 24) | (l6 << 27);
    sum3 += n2;
    sum6 += n6;
    nm3 += n2 >= 2u;
    nm6 += n6 >= 2u;
  }
  sum3 = wave_sum(sum3);
  sum6 = wave_sum(sum6);
  nm3 = wave_sum(nm3);
  nm6 = wave_sum(nm6);
  if (lane_id() == 0) {
    atomicAdd(&s_sum[0], sum3);
    atomicAdd(&s_sum[1], sum6);
    atomicAdd(&s_nm[0], nm3);
    atomicAdd(&s_nm[1], nm6);
  }
  __syncthreads();
  const uint32_t form = s_sum[1] > s_sum[0] ? 1u : 0u;
  if (form)
    for (uint32_t e = t; e < (1u << kLutBits); e += kThreads) lut2[e] = s_e6[e];
  // the multi-symbol step pays for its extra lookup when at least a quarter
  // of the windows (of the code's own probability mass) offer one
  if (t == 0 && s_nm[form] >= (1u << kLutBits) / 4) atomicOr(&st->multi, (1u << k) | (form << (4 + k)));
  uint32_t *slow = df.slow + (uint64_t)k * kSlowWords;
  if (t < 32) {
    slow[t] = s_first[t];
    slow[32 + t] = s_base[t];
    slow[64 + 2 * t] = (uint32_t)s_limit[t];
    slow[64 + 2 * t + 1] = (uint32_t)(s_limit[t] >> 32);
  }
}

// ---------------------------------------------------------------- tasks

// Decode pieces.  The groups' blocks, taken in (stream, predictor) order,
// form one sequence of C blocks; each group is cut into pieces of at most
// L = ceil(C / G) blocks for a decode grid of G workgroups, so there are at
// most G + np pieces.  Written into tb (np = 3 nf groups):
//   tb[p], p <= np             first block of group p in the sequence (C)
//   tb[np + 1 + p], p <= np    first piece of group p (total Q)
//   tb[2 np + 2]               L
//   tb[2 np + 3 + q]           group of piece q          (q < Q <= np + G)
//   tb[2 np + 3 + QM + q]      blocks of piece q         (QM = np + kMaxDecodeGrid)
//   tb[2 np + 3 + 2 QM + q]    blocks of piece q handed out, zeroed here
__device__ inline uint32_t wg_excl_scan(uint32_t v, uint32_t *s_tot, uint32_t &total) {
  const int w = threadIdx.x / kWave;
  const uint32_t inc = wave_incl_scan(v);
  __syncthreads();  // the previous scan's totals have been read
  if (lane_id() == kWave - 1) s_tot[w] = inc;
  __syncthreads();
  uint32_t run = inc - v;
  total = 0;
  for (int i = 0; i < kThreads / kWave; i++) {
    if (i < w) run += s_tot[i];
    total += s_tot[i];
  }
  return run;
}

__global__ __launch_bounds__(kThreads) void d_tasks(const DField *__restrict__ D, int nf, uint32_t grid,
                                                    uint32_t smax, uint32_t *tb, uint32_t *nconst) {
  __shared__ uint32_t s_tot[kThreads / kWave];
  __shared__ uint32_t s_const;
  const int t = threadIdx.x;
  const int np = 3 * nf;
  const uint32_t QM = (uint32_t)np + kMaxDecodeGrid;
  uint32_t *pgrp = tb + 2 * np + 3, *plen = pgrp + QM, *ctr = plen + QM;
  const int per = (np + kThreads - 1) / kThreads;
  if (t == 0) s_const = 0;
  __syncthreads();
  // a stream whose blocks are longer than the decoder's code regions (laid
  // out for the largest block size the host planned for) is reported
  // corrupt and decodes nothing
  auto fits = [&](const DState *st) { return st->status == 0 && !st->is_const && st->S <= smax; };
  auto blocks = [&](int p) -> uint32_t { return fits(D[p / 3].st) ? D[p / 3].st->grp_count[p % 3] : 0u; };
  uint32_t loc = 0, ncon = 0;
  for (int j = 0; j < per; j++) {
    const int p = t * per + j;
    if (p < np) {
      loc += blocks(p);
      DState *st = D[p / 3].st;
      if (p % 3 == 0 && st->status == 0 && st->is_const) ncon++;
      if (p % 3 == 0 && st->status == 0 && !st->is_const && st->S > smax) st->status = SZNB_ECORRUPT;
    }
  }
  if (ncon) atomicAdd(&s_const, ncon);
  uint32_t C;
  uint32_t pos = wg_excl_scan(loc, s_tot, C);
  const uint32_t L = max(1u, (uint32_t)(((uint64_t)C + grid - 1) / grid));
  uint32_t npc = 0;
  for (int j = 0; j < per; j++) {
    const int p = t * per + j;
    if (p < np) {
      tb[p] = pos;
      const uint32_t c = blocks(p);
      pos += c;
      npc += (c + L - 1) / L;
    }
  }
  uint32_t Q;
  uint32_t q = wg_excl_scan(npc, s_tot, Q);
  for (int j = 0; j < per; j++) {
    const int p = t * per + j;
    if (p < np) {
      tb[np + 1 + p] = q;
      const uint32_t c = blocks(p);
      for (uint32_t i = 0; i * L < c; i++, q++) {
        pgrp[q] = (uint32_t)p;
        plen[q] = min(L, c - i * L);
        ctr[q] = 0;
      }
    }
  }
  if (t == 0) { tb[np] = C; tb[2 * np + 1] = Q; tb[2 * np + 2] = L; }
  __syncthreads();
  if (t == 0) *nconst = s_const;
}

__global__ void d_const(const DField *__restrict__ D, int nf, const uint32_t *nconst) {
  if (*nconst == 0) return;  // no constant stream in the table
  for (int f = 0; f < nf; f++) {
    const DField &df = D[f];
    const DState *st = df.st;
    if (st->status != 0 || !st->is_const) continue;
    const float v = st->mn;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < st->n; i += (uint64_t)gridDim.x * blockDim.x)
      df.out[i] = v;
  }
}

// --------------------------------------------------------------- decode

struct DecTab {
  const uint32_t *lut;     // LDS: 4096 first-level entries
  const uint32_t *lut2;    // LDS: 4096 small-symbol entries
  bool multi;              // use them
  bool multi6;             // in the six-nibble form
  const uint32_t *first;   // LDS: first canonical code of each length
  const uint32_t *base;    // LDS: canonical index of that code
  const uint64_t *limit;   // LDS: end of the left-justified code range of each length
  const uint16_t *lsyms;   // LDS symbols, when they fit
  gptr<const uint16_t> gsyms;  // else the global ones
  bool syms_lds;
  uint32_t maxlen;
};

// Per-lane reader of the block's code region: a 64-bit window holding at
// least 32 unread bits and one word read ahead.  Words past the region read
// as zero: the read-ahead word is fetched at a clamped index and masked when
// it enters the window, so that the load is only waited for one refill
// later.
struct BitReader {
  gptr<const uint32_t> wp;
  uint32_t cw, wi, pend, nb;
  uint64_t buf;
};
__device__ inline void br_init(BitReader &r, gptr<const uint32_t> wp, uint32_t cw, uint32_t pos) {
  r.wp = wp;
  r.cw = cw;
  const uint32_t w = pos >> 5, sh = pos & 31u;
  const uint32_t w0 = w < cw ? wp[w] : 0u, w1 = w + 1 < cw ? wp[w + 1] : 0u;
  r.buf = (((uint64_t)w0 << 32) | w1) << sh;
  r.nb = 64u - sh;
  r.wi = w + 2;
  r.pend = wp[min(r.wi, cw - 1u)];
}
__device__ inline uint32_t br_peek(const BitReader &r) { return (uint32_t)(r.buf >> 32); }
__device__ inline void br_skip(BitReader &r, uint32_t len) {
  r.buf <<= len;
  r.nb -= len;
  if (r.nb < 32u) {
    r.buf |= (uint64_t)(r.wi < r.cw ? r.pend : 0u) << (32u - r.nb);
    r.nb += 32u;
    r.wi++;
    r.pend = r.wp[min(r.wi, r.cw - 1u)];
  }
}

// length of the codeword at the front of a 32-bit window, given its
// first-level entry e (1 for a pattern that is no codeword: speculative
// decoding keeps going)
__device__ inline uint32_t decode_len(const DecTab &T, uint32_t e, uint32_t win) {
  uint32_t len = (e >> 16) & 31u;
  if ((e & (kLutLong | kLutOne)) == kLutLong) {
    while (len <= T.maxlen && (uint64_t)win >= T.limit[len]) len++;
    if (len > T.maxlen) len = 1;
  }
  return len;
}
// symbol | length << 16 (plus the invalid flag for a pattern that is no
// codeword).  kLds: the canonical symbols are known to be in LDS, so that no
// symbol read can come from global memory (such a read would make every
// symbol wait for the bit reader's read-ahead loads as well).
template <bool kLds = false>
__device__ inline uint32_t decode_sym(const DecTab &T, uint32_t win) {
  const uint32_t e = T.lut[win >> (32 - kLutBits)];
  if (!(e & kLutLong)) return e & 0x00ffffffu;
  uint32_t len = (e >> 16) & 31u, idx;
  if (e & kLutOne) {
    // one code length under the prefix: the index is the prefix's first
    // plus the len - kLutBits bits after the prefix
    idx = (e & 0xffffu) + ((win << kLutBits) >> (32 + kLutBits - len));
  } else {
    while (len <= T.maxlen && (uint64_t)win >= T.limit[len]) len++;
    if (len > T.maxlen) return kLutInvalid | 0xffffu | (1u << 16);
    idx = T.base[len] + ((win >> (32 - len)) - T.first[len]);
  }
  return (uint32_t)(kLds || T.syms_lds ? T.lsyms[idx] : T.gsyms[idx]) | (len << 16);
}

// One wave decodes block b of a stream and stores its floats.
// Lane l < R decodes the codewords starting in range l of the block's code
// bits, from the first codeword the skip table points at: one pass counts
// them, a second writes their codes after the counts of the lanes before it
// into the wave's LDS region (u16 per element; the words of row r are
// permuted by XOR with r mod 32, so that lanes writing at the same offset
// of consecutive rows use different banks, with no padding).  The inverse
// prediction then runs row by row: each 64-element row is integrated with
// one (LV), two (LCF) or three (QCF) DPP wave scans carried across rows, and
// the reconstructed floats are stored straight from registers, coalesced.
__device__ __forceinline__ uint32_t qaddr(uint32_t e) { return e ^ (((e >> 6) & 31u) << 1); }

__device__ __forceinline__ void decode_block(const DField &df, gptr<const DState> st, const DecTab &T, u32x4 dsc,
                                             uint32_t k, uint16_t *q16, int *bad_flag) {
  const uint32_t l = lane_id();
  const gptr<const uint8_t> in = G(df.in);
  const uint32_t S = st->S, b = dsc.x;
  const uint32_t len = (uint32_t)min((uint64_t)S, st->n - (uint64_t)b * S);
  const uint32_t cw = dsc.z & 0xffffu, ne = dsc.z >> 16;
  const int32_t p0 = (int32_t)dsc.w;
  const uint32_t R = n_ranges(cw), swd = skip_width(T.maxlen), skw = skip_words(cw, T.maxlen);
  const gptr<const uint32_t> sk = reinterpret_cast<gptr<const uint32_t>>(in + st->off_payload) + dsc.y;
  const gptr<const uint32_t> wp = sk + skw;
  const gptr<const uint32_t> esc = wp + cw;
  uint32_t invalid = 0;

  // bring the block's words into cache with a coalesced sweep, so that the
  // lanes' sequential readers below do not each wait on memory; sixteen
  // loads per lane are issued before the first wait (a typical block is one
  // round trip)
  {
    const uint32_t nw = skw + cw;
    uint32_t sink = 0;
    for (uint32_t i0 = 0; i0 < nw; i0 += 16u * kWave) {
      uint32_t a[16];
#pragma unroll
      for (int u = 0; u < 16; u++) {
        const uint32_t i = i0 + (uint32_t)u * kWave + l;
        a[u] = i < nw ? sk[i] : 0u;
      }
#pragma unroll
      for (int u = 0; u < 16; u++) sink |= a[u];
    }
    asm volatile("" ::"v"(sink));  // the loaded values count as used
  }
  // this lane's range and its first codeword
  uint32_t s = 0, e = 0, start = 0;
  if (l < R) {
    s = range_start(l, cw, R);
    e = range_start(l + 1, cw, R);
    start = s;
    if (l > 0 && swd) {
      const uint32_t bp = (l - 1) * swd, wi = bp >> 5, sh = bp & 31u;
      uint32_t v = sk[wi] << sh;
      if (sh + swd > 32u) v |= sk[wi + 1] >> (32u - sh);
      start = s + (v >> (32u - swd));
    }
  }
  // Single pass for most blocks: each lane decodes its range once and keeps
  // the symbols in registers (two per VGPR; the t-th symbol of every lane
  // goes to the same register, so the indices are static) while it counts
  // them; after the scan of the counts it writes them to the LDS row buffer.
  // A range holding more than kStage codewords, a codebook decoded with the
  // multi-symbol table, or canonical symbols left in global memory take the
  // two passes below instead (count, then decode again into the row buffer).
  constexpr int kStage = 80;
  uint32_t stg[kStage / 2];
  uint32_t pos = start, cnt = 0;
  bool staged = !T.multi && T.syms_lds;
  if (staged) {
    if (pos < e) {
      BitReader br;
      br_init(br, wp, cw, pos);
#pragma unroll
      for (int t = 0; t < kStage; t++) {
        if (pos < e) {
          const uint32_t r = decode_sym<true>(T, br_peek(br));
          const uint32_t ln = (r >> 16) & 31u;
          if (r & kLutInvalid) invalid = 1;
          if (t & 1) stg[t >> 1] |= (r & 0xffffu) << 16;
          else stg[t >> 1] = r & 0xffffu;
          pos += ln;
          br_skip(br, ln);
          cnt++;
        }
      }
    }
    staged = __ballot(pos < e) == 0;  // every range fitted
    if (!staged) {
      pos = start;
      cnt = 0;
      invalid = 0;
    }
  }
  // pass 1: count the codewords of the range
  if (!staged && pos < e) {
    BitReader br;
    br_init(br, wp, cw, pos);
    while (pos < e) {
      const uint32_t win = br_peek(br);
      const uint32_t ent = T.lut[win >> (32 - kLutBits)];
      const uint32_t mc = (ent >> 24) & 15u, ml = ent >> 28;
      uint32_t ln, c = 1;
      if (mc >= 2u && pos + ml <= e) {  // several whole codes, all starting before e
        ln = ml;
        c = mc;
      } else {
        ln = decode_len(T, ent, win);
      }
      pos += ln;
      br_skip(br, ln);
      cnt += c;
    }
  }
  // the codeword that ends a range must be where the next range's entry points
  const uint32_t nstart = __shfl_down(start, 1, kWave);
  if (l + 1 < R && pos != nstart) invalid = 1;
  const uint32_t total = wave_sum(cnt);
  if (total < len) { if (l == 0) *bad_flag = 1; return; }
  const uint32_t o = wave_scan_dpp(cnt) - cnt;
  if (staged) {
#pragma unroll
    for (int t = 0; t < kStage; t++) {
      const uint32_t i = o + (uint32_t)t;
      if ((uint32_t)t < cnt && i < len)
        q16[qaddr(i)] = (uint16_t)((t & 1) ? (stg[t >> 1] >> 16) : (stg[t >> 1] & 0xffffu));
    }
  } else {
    // pass 2: emit the codes
    uint32_t p = start, i = o;
    if (p < e && i < len) {
      BitReader br;
      br_init(br, wp, cw, p);
      if (T.multi && T.multi6) {
        while (p < e && i < len) {
          const uint32_t win = br_peek(br);
          const uint32_t m = T.lut2[win >> (32 - kLutBits)];
          const uint32_t n6 = (m >> 24) & 7u, l6 = (m >> 27) & 15u;
          uint32_t ln, adv;
          if (n6 >= 2u && p + l6 <= e && i + n6 <= len) {  // two to six tiny symbols at once
#pragma unroll
            for (uint32_t u = 0; u < 6u; u++)
              if (u < n6) q16[qaddr(i + u)] = (uint16_t)(kRadius + ((int32_t)(m << (28 - 4 * u)) >> 28));
            ln = l6;
            adv = n6;
          } else {
            const uint32_t r = decode_sym(T, win);
            ln = (r >> 16) & 31u;
            if (r & kLutInvalid) invalid = 1;
            q16[qaddr(i)] = (uint16_t)(r & 0xffffu);
            adv = 1;
          }
          p += ln;
          br_skip(br, ln);
          i += adv;
        }
      } else if (T.multi) {
        while (p < e && i < len) {
          const uint32_t win = br_peek(br);
          const uint32_t m = T.lut2[win >> (32 - kLutBits)];
          const uint32_t n2 = (m >> 24) & 3u, l2 = (m >> 26) & 15u;
          uint32_t ln, adv;
          if (n2 >= 2u && p + l2 <= e && i + n2 <= len) {  // two or three small symbols at once
            q16[qaddr(i)] = (uint16_t)(kRadius + (int32_t)(int8_t)(m & 255u));
            q16[qaddr(i + 1)] = (uint16_t)(kRadius + (int32_t)(int8_t)((m >> 8) & 255u));
            if (n2 == 3u) q16[qaddr(i + 2)] = (uint16_t)(kRadius + (int32_t)(int8_t)((m >> 16) & 255u));
            ln = l2;
            adv = n2;
          } else {
            const uint32_t r = decode_sym(T, win);
            ln = (r >> 16) & 31u;
            if (r & kLutInvalid) invalid = 1;
            q16[qaddr(i)] = (uint16_t)(r & 0xffffu);
            adv = 1;
          }
          p += ln;
          br_skip(br, ln);
          i += adv;
        }
      } else {
        while (p < e && i < len) {
          const uint32_t r = decode_sym(T, br_peek(br));
          const uint32_t ln = (r >> 16) & 31u;
          if (r & kLutInvalid) invalid = 1;
          q16[qaddr(i)] = (uint16_t)(r & 0xffffu);
          p += ln;
          br_skip(br, ln);
          i++;
        }
      }
    }
  }
  __builtin_amdgcn_wave_barrier();
  // inverse prediction and reconstruction, one row of 64 values at a time
  const uint64_t lt = l ? (~0ull >> (64 - l)) : 0ull;
  uint32_t c0 = 0, c1 = 0, c2 = 0, ebase = 0;
  const double step = st->step, mn = (double)st->mn;
  const gptr<float> out = G(df.out) + (uint64_t)b * S;
  if (l == 0 && len && q16[0] != (uint16_t)kRadius) invalid = 1;
  // four rows per step: their scans are independent until the carries,
  // which are added row by row afterwards (integer sums, so the grouping
  // does not change them)
  constexpr int kRows = 4;
  const auto level = [](uint32_t (&v)[kRows], uint32_t &carry) {
    uint32_t sc[kRows];
#pragma unroll
    for (int u = 0; u < kRows; u++) sc[u] = wave_scan_dpp(v[u]);
#pragma unroll
    for (int u = 0; u < kRows; u++) {
      v[u] = sc[u] + carry;
      carry += (uint32_t)__builtin_amdgcn_readlane((int)sc[u], 63);
    }
  };
  for (uint32_t row0 = 0; row0 < len; row0 += kRows * kWave) {
    uint32_t r[kRows];
    uint64_t em[kRows];
#pragma unroll
    for (int u = 0; u < kRows; u++) {
      const uint32_t el = row0 + (uint32_t)u * kWave + l;
      const uint32_t q = el < len ? q16[qaddr(el)] : (uint32_t)kRadius;
      r[u] = q - (uint32_t)kRadius;
      em[u] = __ballot(el < len && q == 0u);
    }
    // escapes take their values in element order
#pragma unroll
    for (int u = 0; u < kRows; u++) {
      if (em[u]) {
        if ((em[u] >> l) & 1ull) {
          const uint32_t ei = ebase + (uint32_t)__popcll(em[u] & lt);
          r[u] = ei < ne ? esc[ei] : 0u;
        }
        ebase += (uint32_t)__popcll(em[u]);
      }
    }
    if (k >= 2) level(r, c2);
    if (k >= 1) level(r, c1);
    level(r, c0);
#pragma unroll
    for (int u = 0; u < kRows; u++) {
      const uint32_t el = row0 + (uint32_t)u * kWave + l;
      if (el < len) out[el] = (float)fma((double)(int32_t)((uint32_t)p0 + r[u]), step, mn);
    }
  }
  if (ebase != ne) invalid = 1;
  if (__ballot(invalid)) { if (l == 0) *bad_flag = 1; }
  __builtin_amdgcn_wave_barrier();
}

// Blocks of piece q (of c blocks) that its own workgroup decodes without the
// counter: three quarters, in whole turns of the nw waves.  Pieces past the
// grid have no workgroup of their own and are all counter-served.
__device__ inline uint32_t static_blocks(uint32_t q, uint32_t c, uint32_t nw) {
  return q < gridDim.x ? c * 3u / 4u / nw * nw : 0u;
}

// Workgroup g of G starts on piece g: its waves take three quarters of the
// piece's blocks in turn and the rest one at a time from the piece's
// counter, so a wave that drew short blocks takes more, and the workgroup
// meets at a barrier only when the piece is used up.  It then helps with the
// piece with the most counter-served blocks left, until none has any.
// Dynamic LDS: lut (4096 words), lut2 (4096 words when some codebook is
// small enough to use it) | first, base (32 words each) | limit (32 u64) |
// symbols (symcap u16, when they fit) | dw code regions of 2 smax bytes.
__global__ void d_decode(const DField *__restrict__ D, int nf, uint32_t *tb, uint32_t smax, uint32_t symcap,
                         uint32_t lut_words) {
  extern __shared__ __align__(16) uint8_t smem[];
  uint32_t *s_lut = reinterpret_cast<uint32_t *>(smem);
  uint32_t *s_first = s_lut + lut_words;
  uint32_t *s_base = s_first + 32;
  uint64_t *s_limit = reinterpret_cast<uint64_t *>(s_base + 32);
  uint16_t *s_syms = reinterpret_cast<uint16_t *>(s_limit + 32);
  uint8_t *regs = reinterpret_cast<uint8_t *>(s_syms) + ((2u * symcap + 15u) & ~15u);
  __shared__ uint64_t s_red[1024 / kWave];
  const int t = threadIdx.x;
  const uint32_t w = t / kWave, nw = blockDim.x / kWave;
  const int np = 3 * nf;
  const uint32_t QM = (uint32_t)np + kMaxDecodeGrid;
  const uint32_t *pgrp = tb + 2 * np + 3, *plen = pgrp + QM;
  uint32_t *ctr = tb + 2 * np + 3 + 2 * QM;
  const uint32_t C = tb[np], Q = tb[2 * np + 1], L = tb[2 * np + 2];
  if (Q == 0) return;
  const uint32_t r0 = blockIdx.x % Q;
  uint32_t piece = blockIdx.x < Q ? blockIdx.x : Q;  // Q: choose below
  int cur = -1;
  bool syms_lds = false;
  uint16_t *q16 = reinterpret_cast<uint16_t *>(regs + (uint64_t)w * 2u * smax);
  // every pass either takes a block or finds a piece used up, so C + Q + 1
  // passes bound the loop
  for (uint32_t pass = 0; pass <= C + Q; pass++) {
    if (piece == Q) {
      // the piece with the most blocks left (counters read coherently; ties
      // go to the first piece at or after this workgroup's own)
      uint64_t key = ~0ull;
      for (uint32_t i = t; i < Q; i += blockDim.x) {
        const uint32_t qq = i + r0 < Q ? i + r0 : i + r0 - Q;
        const uint32_t taken = __hip_atomic_load(&ctr[qq], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t cd = plen[qq] - static_blocks(qq, plen[qq], nw);
        const uint32_t rem = taken < cd ? cd - taken : 0u;
        const uint64_t kq = ((uint64_t)(~rem) << 32) | i;
        key = kq < key ? kq : key;
      }
      key = wave_min_u64(key);
      if (lane_id() == 0) s_red[w] = key;
      __syncthreads();
      key = s_red[0];
      for (uint32_t i = 1; i < nw; i++) key = s_red[i] < key ? s_red[i] : key;
      __syncthreads();  // s_red is read before it is written again
      if (~(uint32_t)(key >> 32) == 0u) break;
      const uint32_t i = (uint32_t)key;
      piece = i + r0 < Q ? i + r0 : i + r0 - Q;
    }
    const int pair = (int)pgrp[piece];
    const int f = pair / 3, k = pair % 3;
    const DField &df = D[f];
    const gptr<const DState> st = G(static_cast<const DState *>(df.st));
    if (pair != cur) {
      const gptr<const uint32_t> gl = G(df.lut) + (uint64_t)k * (2u << kLutBits);
      // eight loads per thread in flight before they are stored
      for (uint32_t i0 = 0; i0 < lut_words; i0 += 8u * blockDim.x) {
        uint32_t a[8];
#pragma unroll
        for (int u = 0; u < 8; u++) {
          const uint32_t i = i0 + (uint32_t)u * blockDim.x + t;
          a[u] = i < lut_words ? gl[i] : 0u;
        }
#pragma unroll
        for (int u = 0; u < 8; u++) {
          const uint32_t i = i0 + (uint32_t)u * blockDim.x + t;
          if (i < lut_words) s_lut[i] = a[u];
        }
      }
      const gptr<const uint32_t> gs = G(df.slow) + (uint64_t)k * kSlowWords;
      for (uint32_t i = t; i < 32u; i += blockDim.x) {
        s_first[i] = gs[i];
        s_base[i] = gs[32 + i];
        s_limit[i] = (uint64_t)gs[64 + 2 * i] | ((uint64_t)gs[64 + 2 * i + 1] << 32);
      }
      const uint32_t ns = st->nsym[k];
      syms_lds = ns <= symcap;
      if (syms_lds) {
        const gptr<const uint16_t> gsy = G(df.syms) + (uint64_t)k * kNSyms;
        for (uint32_t i = t; i < ns; i += blockDim.x) s_syms[i] = gsy[i];
      }
      __syncthreads();
      cur = pair;
    }
    DecTab T2;
    T2.lut = s_lut;
    T2.lut2 = s_lut + (1u << kLutBits);
    T2.multi = lut_words > (1u << kLutBits) && ((st->multi >> k) & 1u);
    T2.multi6 = (st->multi >> (4 + k)) & 1u;
    T2.first = s_first;
    T2.base = s_base;
    T2.limit = s_limit;
    T2.lsyms = s_syms;
    T2.gsyms = G(df.syms) + (uint64_t)k * kNSyms;
    T2.syms_lds = syms_lds;
    T2.maxlen = st->maxlen[k];
    // the piece's blocks: on the workgroup's first pass over its own piece
    // the first cs go to the waves in turn (each wave loads its next
    // descriptor while it decodes a block); the rest, one per wave at a time,
    // from the piece's counter, which other workgroups share
    const uint32_t first = (piece - tb[np + 1 + pair]) * L, c = plen[piece];
    const uint32_t cs = static_blocks(piece, c, nw);
    const gptr<const u32x4> gdesc = G(static_cast<const u32x4 *>(df.desc)) + st->grp_start[k] + first;
    if (pass == 0 && blockIdx.x < Q) {
      uint32_t j = w;
      u32x4 dsc = j < cs ? gdesc[j] : u32x4{0, 0, 0, 0};
      while (j < cs) {
        const uint32_t jn = j + nw;
        const u32x4 dn = jn < cs ? gdesc[jn] : u32x4{0, 0, 0, 0};
        int bad = 0;
        decode_block(df, st, T2, dsc, (uint32_t)k, q16, &bad);
        if (bad && lane_id() == 0) atomicCAS(&df.st->status, 0, SZNB_ECORRUPT);
        j = jn;
        dsc = dn;
      }
    }
    uint32_t *const gctr = ctr + piece;
    uint32_t j = 0;
    if (lane_id() == 0) j = atomicAdd(gctr, 1u);
    j = cs + __builtin_amdgcn_readfirstlane(j);
    while (j < c) {
      uint32_t jn = 0;
      if (lane_id() == 0) jn = atomicAdd(gctr, 1u);
      const u32x4 dsc = gdesc[j];
      int bad = 0;
      decode_block(df, st, T2, dsc, (uint32_t)k, q16, &bad);
      if (bad && lane_id() == 0) atomicCAS(&df.st->status, 0, SZNB_ECORRUPT);
      j = cs + __builtin_amdgcn_readfirstlane(jn);
    }
    __syncthreads();  // every wave is done with the piece (and the tables)
    piece = Q;
  }
}

}  // namespace sznb
