/*
 * sznb oracle -- plain, slow, CPU reference of the error-bounded lossy
 * compressor for 1D float32 particle fields (SZ-style: prediction, linear-
 * scaling quantization, Huffman coding).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header, table or constant
 * generator with the GPU library.
 *
 * Every step is written in the order the method performs it, with plain
 * loops, so that it can be checked against the paper by eye:
 *
 *   value range R = max - min of the field (paper, Problem Statement,
 *     definition of R_vx); absolute bound eb_abs, relative bound
 *     eb_rel = eb_abs / R (same place);
 *   prediction from preceding values: last value x_{i-1} (Sec. 5.1, LV
 *     model), linear curve fit 2x_{i-1} - x_{i-2} (Sec. 5.1, LCF model),
 *     and the quadratic extension 3x_{i-1} - 3x_{i-2} + x_{i-3};
 *   linear-scaling quantization of the prediction error into intervals of
 *     width 2*eb with a large interval count (Sec. 5.1, last paragraph),
 *     realised as rounding onto the lattice mn + step*Z (see lattice());
 *   Huffman coding of the quantization codes (Sec. 2, SZ description;
 *     Sec. 5.2, tailored Huffman encoding).
 *
 * Readings where the paper is silent (block size, warm-up, rounding rule,
 * guard against float32 rounding, tie rules, stream layout) are fixed here
 * and each is marked "reading:".
 *
 * Compile with -O2 -ffp-contract=off (no fused multiply-add contraction, no
 * fast-math): every floating-point step below is one IEEE operation.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OK 0
#define E_INVAL (-1)
#define E_NONFINITE (-2)
#define E_EBSMALL (-3)
#define E_NOSPC (-4)
#define E_CORRUPT (-5)

#define RADIUS 32768         /* 65536 quantization intervals, code 0 = escape */
#define NSYMS 65536
#define LMAX 24              /* reading: Huffman code lengths limited to 24 bits */
#define PMAX (1 << 27)       /* largest lattice index span accepted */
#define HDR 128

/* ---------------------------------------------------------------- helpers */

static uint32_t f2u(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }
static float u2f(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }

static void put_u16(uint8_t *b, uint64_t o, uint16_t v) { memcpy(b + o, &v, 2); }
static void put_u32(uint8_t *b, uint64_t o, uint32_t v) { memcpy(b + o, &v, 4); }
static void put_u64(uint8_t *b, uint64_t o, uint64_t v) { memcpy(b + o, &v, 8); }
static void put_f64(uint8_t *b, uint64_t o, double v) { memcpy(b + o, &v, 8); }
static uint16_t get_u16(const uint8_t *b, uint64_t o) { uint16_t v; memcpy(&v, b + o, 2); return v; }
static uint32_t get_u32(const uint8_t *b, uint64_t o) { uint32_t v; memcpy(&v, b + o, 4); return v; }
static uint64_t get_u64(const uint8_t *b, uint64_t o) { uint64_t v; memcpy(&v, b + o, 8); return v; }
static double get_f64(const uint8_t *b, uint64_t o) { double v; memcpy(&v, b + o, 8); return v; }

static uint64_t align8(uint64_t x) { return (x + 7) & ~(uint64_t)7; }

/* unit in the last place of a float32 magnitude: 2^(E-23) for a normal
 * number with unbiased exponent E, 2^-149 for subnormals and zero */
static double ulp_f32(float m)
{
    uint32_t e = (f2u(m) >> 23) & 0xff;
    if (e == 0) return ldexp(1.0, -149);
    return ldexp(1.0, (int)e - 127 - 23);
}

/* ------------------------------------------------------ range and bound */

typedef struct {
    float mn, mx;       /* field range, zeros canonicalised to +0 */
    double R;           /* value range (paper: R = max - min) */
    double eb_abs;      /* absolute bound after eb_rel conversion */
    double step;        /* lattice spacing 2*(eb_abs - guard) */
    double inv;         /* 1/step */
    int64_t P;          /* lattice index of mx */
    int is_const;       /* R == 0 or n == 0 */
} params_t;

/* Range and bound.  R = max - min (Problem Statement).  If the mode asks for
 * a value-range-relative bound, eb_abs = eb_rel * R (same paragraph).
 * reading: the lattice spacing is 2*(eb_abs - g) with guard g = 2 ulp_f32 of
 * the largest magnitude, so that the float32 rounding of the reconstructed
 * value can never push the error past eb_abs. */
static int range_and_bound(const float *x, uint64_t n, double eb, int eb_rel, params_t *pp)
{
    params_t p;
    memset(&p, 0, sizeof p);
    if (!(eb > 0.0) || !isfinite(eb)) return E_INVAL;
    if (n == 0) { p.is_const = 1; *pp = p; return OK; }
    float mn = x[0], mx = x[0];
    for (uint64_t i = 0; i < n; i++) {
        if (!isfinite(x[i])) return E_NONFINITE;
        if (x[i] < mn) mn = x[i];
        if (x[i] > mx) mx = x[i];
    }
    if (mn == 0.0f) mn = 0.0f; /* -0 -> +0 */
    if (mx == 0.0f) mx = 0.0f;
    p.mn = mn;
    p.mx = mx;
    p.R = (double)mx - (double)mn;
    if (p.R == 0.0) {
        p.is_const = 1;
        p.eb_abs = eb_rel ? eb * p.R : eb;
        *pp = p;
        return OK;
    }
    p.eb_abs = eb_rel ? eb * p.R : eb;
    float am = fabsf(mn) > fabsf(mx) ? fabsf(mn) : fabsf(mx);
    double g = 2.0 * ulp_f32(am);
    double ebp = p.eb_abs - g;
    if (!(ebp > 0.0)) return E_EBSMALL;
    p.step = 2.0 * ebp;
    p.inv = 1.0 / p.step;
    double t = ((double)mx - (double)mn) * p.inv;
    double P = floor(t + 0.5);
    if (P > (double)PMAX) return E_EBSMALL;
    p.P = (int64_t)P;
    *pp = p;
    return OK;
}

/* Linear-scaling quantization as a lattice.  Closed-loop SZ predicts x_i
 * from already reconstructed neighbours and rounds the error to the nearest
 * multiple of 2*eb (Sec. 5.1).  With integer predictor coefficients summing
 * to one and a reconstructed anchor on mn + step*Z, every prediction is a
 * lattice point, so the reconstructed value is the lattice point nearest to
 * x_i: p_i = round((x_i - mn) / step).
 * reading: round half up, two separate fp64 roundings (multiply, then add). */
static int32_t lattice(float xi, const params_t *p)
{
    double t = ((double)xi - (double)p->mn) * p->inv;
    return (int32_t)floor(t + 0.5);
}

/* Reconstruction: x~ = fl32(fma(p, step, mn)). */
static float reconstruct(int32_t pi, const params_t *p)
{
    return (float)fma((double)pi, p->step, (double)p->mn);
}

/* ------------------------------------------------------------ prediction */

/* Residual of predictor k (0 = last value, 1 = linear curve fit, 2 =
 * quadratic curve fit) at position j of a block whose lattice values are
 * q[0..], all relative to the block anchor q[0].
 * reading: values before the block start are taken equal to the anchor, so
 * with d_j = q_j - q_0 (and d_j = 0 for j < 0) the predictions are
 *   LV  : d_{j-1}
 *   LCF : 2 d_{j-1} - d_{j-2}
 *   QCF : 3 d_{j-1} - 3 d_{j-2} + d_{j-3}
 * and the residual is d_j minus the prediction. */
static int32_t residual(const int32_t *q, uint64_t j, int k)
{
    int64_t d0 = (int64_t)q[j] - q[0];
    int64_t d1 = j >= 1 ? (int64_t)q[j - 1] - q[0] : 0;
    int64_t d2 = j >= 2 ? (int64_t)q[j - 2] - q[0] : 0;
    int64_t d3 = j >= 3 ? (int64_t)q[j - 3] - q[0] : 0;
    int64_t pred;
    if (k == 0) pred = d1;
    else if (k == 1) pred = 2 * d1 - d2;
    else pred = 3 * d1 - 3 * d2 + d3;
    return (int32_t)(d0 - pred);
}

/* ------------------------------------------------- per-block selection */

/* LOG[m] = round(2^16 * log2 m), m >= 1 */
static uint32_t LOGT[16385];
static int logt_ready = 0;
static void make_log_table(void)
{
    if (logt_ready) return;
    LOGT[0] = 0;
    for (int m = 1; m <= 16384; m++) LOGT[m] = (uint32_t)floor(65536.0 * log2((double)m) + 0.5);
    logt_ready = 1;
}

/* reading: the best-fit predictor of a block is the one whose residuals have
 * the smallest estimated coded size, estimated as a two-part code: an
 * entropy-coded magnitude class followed by the bits that pick the value
 * inside the class.  Residual r has zigzag index z = 2r (r >= 0) or -2r-1
 * (r < 0); z < 4 is its own class with no extra bits; a larger z with bit
 * length b falls in class 4 + 2(b-3) + (the bit below its leading one), a run
 * of 2^(b-2) values, with b-2 extra bits; an escape (|r| >= 32768) is class
 * 32 with 32 extra bits.  The estimate, in units of 2^-16 bit, is
 *   sum_c n_c (LOG[len] - LOG[n_c]) + 2^16 * sum of extra bits. */
static void res_class(int32_t r, int *cls, int *extra)
{
    if (r >= RADIUS || r <= -RADIUS) { *cls = 32; *extra = 32; return; }
    uint32_t z = r >= 0 ? (uint32_t)r * 2u : (uint32_t)(-(int64_t)r) * 2u - 1u;
    if (z < 4) { *cls = (int)z; *extra = 0; return; }
    int b = 0;
    while ((z >> b) != 0) b++;
    *cls = 4 + 2 * (b - 3) + (int)((z >> (b - 2)) & 1u);
    *extra = b - 2;
}

static uint64_t block_cost(const int32_t *q, uint64_t len, int k)
{
    uint32_t cnt[33];
    uint64_t extra_sum = 0;
    memset(cnt, 0, sizeof cnt);
    for (uint64_t j = 0; j < len; j++) {
        int c, e;
        res_class(residual(q, j, k), &c, &e);
        cnt[c]++;
        extra_sum += (uint64_t)e;
    }
    uint64_t cost = 0;
    for (int c = 0; c < 33; c++)
        if (cnt[c]) cost += (uint64_t)cnt[c] * (uint64_t)(LOGT[len] - LOGT[cnt[c]]);
    return cost + 65536ull * extra_sum;
}

/* argmin over k, ties to the lowest k */
static int select_pred(const int32_t *q, uint64_t len, uint64_t costs[3])
{
    int best = 0;
    for (int k = 0; k < 3; k++) {
        costs[k] = block_cost(q, len, k);
        if (costs[k] < costs[best]) best = k;
    }
    return best;
}

/* -------------------------------------------------------------- Huffman */

typedef struct { uint64_t w; int32_t sym; } leaf_t;

static int leaf_cmp(const void *a, const void *b)
{
    const leaf_t *x = a, *y = b;
    if (x->w != y->w) return x->w < y->w ? -1 : 1;
    return x->sym < y->sym ? -1 : (x->sym > y->sym);
}

/* Huffman code lengths by the two-queue method: leaves sorted by (weight,
 * symbol); each step takes the two lightest of the leaf queue and the queue
 * of merged nodes.  reading: on equal weight the leaf is taken first; the
 * merged queue is first-in first-out.  If a length exceeds LMAX every weight
 * becomes (w+1)/2 (rounded down) and the code is built again. */
static int huffman_lengths(const uint32_t *freq, uint8_t *len)
{
    int nsym = 0;
    memset(len, 0, NSYMS);
    for (int s = 0; s < NSYMS; s++) nsym += freq[s] != 0;
    if (nsym == 0) return 0;
    if (nsym == 1) {
        for (int s = 0; s < NSYMS; s++) if (freq[s]) len[s] = 1;
        return 1;
    }
    leaf_t *L = malloc(sizeof(leaf_t) * nsym);
    uint64_t *w = malloc(sizeof(uint64_t) * NSYMS);
    uint64_t *iw = malloc(sizeof(uint64_t) * nsym);     /* merged weights */
    int32_t *parent = malloc(sizeof(int32_t) * 2 * nsym); /* leaves 0..nsym-1, merged nsym.. */
    int32_t *depth = malloc(sizeof(int32_t) * 2 * nsym);
    for (int s = 0; s < NSYMS; s++) w[s] = freq[s];
    int maxlen;
    for (;;) {
        int k = 0;
        for (int s = 0; s < NSYMS; s++) if (freq[s]) { L[k].w = w[s]; L[k].sym = s; k++; }
        qsort(L, nsym, sizeof(leaf_t), leaf_cmp);
        int lp = 0, ip = 0, ni = 0;
        while ((nsym - lp) + (ni - ip) > 1) {
            int pick[2];
            uint64_t pw[2];
            for (int t = 0; t < 2; t++) {
                int take_leaf;
                if (lp >= nsym) take_leaf = 0;
                else if (ip >= ni) take_leaf = 1;
                else take_leaf = L[lp].w <= iw[ip];
                if (take_leaf) { pick[t] = lp; pw[t] = L[lp].w; lp++; }
                else { pick[t] = nsym + ip; pw[t] = iw[ip]; ip++; }
            }
            iw[ni] = pw[0] + pw[1];
            parent[pick[0]] = nsym + ni;
            parent[pick[1]] = nsym + ni;
            ni++;
        }
        /* depths, root = last merged node */
        int root = nsym + ni - 1;
        depth[root] = 0;
        for (int v = root - 1; v >= nsym; v--) depth[v] = depth[parent[v]] + 1;
        maxlen = 0;
        for (int v = 0; v < nsym; v++) {
            depth[v] = depth[parent[v]] + 1;
            if (depth[v] > maxlen) maxlen = depth[v];
        }
        if (maxlen <= LMAX) {
            for (int v = 0; v < nsym; v++) len[L[v].sym] = (uint8_t)depth[v];
            break;
        }
        for (int s = 0; s < NSYMS; s++) if (freq[s]) w[s] = (w[s] + 1) >> 1;
    }
    free(L); free(w); free(iw); free(parent); free(depth);
    return nsym;
}

/* Canonical code (the rule of RFC 1951, Sec. 3.2.2): symbols ordered by
 * (length, symbol); the first gets code 0, each next one (previous + 1)
 * shifted left by the length difference. */
static void canonical_codes(const uint8_t *len, uint32_t *code, uint16_t *order, int *maxlen_out)
{
    int k = 0, maxlen = 0;
    for (int l = 1; l <= LMAX; l++)
        for (int s = 0; s < NSYMS; s++)
            if (len[s] == l) { order[k++] = (uint16_t)s; maxlen = l; }
    uint32_t c = 0;
    for (int i = 0; i < k; i++) {
        if (i > 0) c = (c + 1) << (len[order[i]] - len[order[i - 1]]);
        code[order[i]] = c;
    }
    *maxlen_out = maxlen;
}

/* ------------------------------------------------------------ bit writer */

typedef struct { uint32_t *w; uint64_t nbits; } bw_t;

static void put_bits(bw_t *b, uint32_t code, int len)
{
    for (int i = len - 1; i >= 0; i--) {
        uint32_t bit = (code >> i) & 1u;
        uint64_t pos = b->nbits++;
        if (bit) b->w[pos >> 5] |= 1u << (31 - (pos & 31));
    }
}

/* ----------------------------------------------------------- skip table */

/* reading: a block's code bits are cut into R word-aligned ranges, range l
 * starting at bit 32 floor(l cw / R) (cw = code words of the block,
 * R = min(64, max(1, floor(cw / 8)))).  For every range after the first the
 * stream stores the distance from the range start to the first codeword that
 * starts at or after it, in w = bitlen(maxlen - 1) bits, MSB first, in words
 * placed ahead of the code words.  A decoder can then begin a codeword in
 * every range without decoding the ones before it. */
static uint32_t n_ranges(uint64_t cw)
{
    uint64_t r = cw / 8;
    if (r < 1) r = 1;
    if (r > 64) r = 64;
    return (uint32_t)r;
}
static uint32_t skip_width(int maxlen)
{
    uint32_t w = 0;
    while ((1 << w) < maxlen) w++;
    return w;
}
static uint64_t skip_words(uint64_t cw, int maxlen)
{
    return ((uint64_t)(n_ranges(cw) - 1) * skip_width(maxlen) + 31) / 32;
}
static uint64_t range_start(uint32_t l, uint64_t cw) { return 32 * ((l * cw) / n_ranges(cw)); }

/* -------------------------------------------------------------- stream */

/* Stream layout (all little-endian), header of 128 bytes:
 *   0 magic 'SZNB'   4 u16 version = 1   6 u8 policy   7 u8 flags (bit0 const,
 *   bit1 eb_rel)   8 u64 n   16 u32 S   20 u32 nblocks   24 f32 mn   28 f32 mx
 *  32 f64 eb_abs   40 f64 step   48 u32 n_sym[3]   60 u8 max_len[3] (+1 pad)
 *  64 u64 payload_words   72 u64 total_bytes   80.. u64 section offsets:
 *  pred, pfirst, cwords, nesc, books, payload.
 * Sections, each 8-byte aligned: pred u8[nb] (best-fit and learned policies
 * only), pfirst i32[nb], cwords u16[nb], nesc u16[nb]; books: for each
 * predictor k with n_sym[k] > 0, blcount u32[max_len[k]] then syms
 * u16[n_sym[k]] in canonical order, padded to 8 bytes; payload u32[].  Each
 * block's payload is its skip table (see above), its code bits (MSB first,
 * coded with the codebook of the block's predictor) zero-padded to a 32-bit
 * word, then its escaped residuals as i32 words in element order.
 * reading: one Huffman codebook per predictor -- a block is entropy coded with
 * the code built from the residuals of all blocks that chose the same
 * predictor, so blocks with different residual laws do not share a code. */

static int block_log2_of(uint32_t mode)
{
    uint32_t b = (mode >> 8) & 15u;
    if (b == 0) return 12;
    return (int)b;
}

int sznbref_compress_blocks(const float *x, uint64_t n, double eb, uint32_t mode,
                            const uint8_t *forced_pred, uint8_t **out, size_t *out_len);

int sznbref_compress(const float *x, uint64_t n, double eb, uint32_t mode, uint8_t **out, size_t *out_len)
{
    return sznbref_compress_blocks(x, n, eb, mode, NULL, out, out_len);
}

static void write_header_common(uint8_t *b, int policy, int flags, uint64_t n, uint64_t S,
                                const params_t *p)
{
    memcpy(b, "SZNB", 4);
    put_u16(b, 4, 1);
    b[6] = (uint8_t)policy;
    b[7] = (uint8_t)flags;
    put_u64(b, 8, n);
    put_u32(b, 16, (uint32_t)S);
    put_u32(b, 24, f2u(p->mn));
    put_u32(b, 28, f2u(p->mx));
    put_f64(b, 32, p->eb_abs);
}

/* forced_pred: optional per-block predictor ids (used for the learned
 * policy, whose choice is made outside this function); NULL otherwise. */
int sznbref_compress_blocks(const float *x, uint64_t n, double eb, uint32_t mode,
                            const uint8_t *forced_pred, uint8_t **out, size_t *out_len)
{
    *out = NULL;
    *out_len = 0;
    int policy = (int)(mode & 3u);
    int eb_rel = (mode >> 4) & 1u;
    int bl = block_log2_of(mode);
    if (bl < 10 || bl > 14) return E_INVAL;
    if (mode & ~(uint32_t)(3u | 16u | (15u << 8))) return E_INVAL;
    if (n >= (1ull << 31)) return E_INVAL;
    if (policy == 3 && forced_pred == NULL) return E_INVAL;
    uint64_t S = 1ull << bl;
    params_t p;
    int st = range_and_bound(x, n, eb, eb_rel, &p);
    if (st) return st;

    if (p.is_const) {
        uint8_t *b = calloc(1, HDR);
        write_header_common(b, policy, 1 | (eb_rel << 1), n, S, &p);
        put_u64(b, 72, HDR);
        *out = b;
        *out_len = HDR;
        return OK;
    }

    uint64_t nb = (n + S - 1) / S;
    int32_t *q = malloc(sizeof(int32_t) * n);
    for (uint64_t i = 0; i < n; i++) q[i] = lattice(x[i], &p);

    /* predictor of each block */
    uint8_t *pred = malloc(nb);
    make_log_table();
    for (uint64_t b = 0; b < nb; b++) {
        uint64_t len = (b + 1) * S <= n ? S : n - b * S;
        if (policy == 0) pred[b] = 0;
        else if (policy == 1) pred[b] = 1;
        else if (policy == 2) { uint64_t c[3]; pred[b] = (uint8_t)select_pred(q + b * S, len, c); }
        else pred[b] = forced_pred[b];
        if (pred[b] > 2) { free(q); free(pred); return E_INVAL; }
    }

    /* codes and one histogram per predictor */
    uint16_t *code = malloc(sizeof(uint16_t) * n);
    int32_t *res = malloc(sizeof(int32_t) * n);
    uint32_t *freq = calloc(3 * (uint64_t)NSYMS, sizeof(uint32_t));
    for (uint64_t b = 0; b < nb; b++) {
        uint64_t len = (b + 1) * S <= n ? S : n - b * S;
        for (uint64_t j = 0; j < len; j++) {
            int32_t r = residual(q + b * S, j, pred[b]);
            res[b * S + j] = r;
            uint16_t c = (r > -RADIUS && r < RADIUS) ? (uint16_t)(r + RADIUS) : 0;
            code[b * S + j] = c;
            freq[(uint64_t)pred[b] * NSYMS + c]++;
        }
    }

    /* one canonical Huffman code per predictor in use */
    uint8_t *len = calloc(3 * (uint64_t)NSYMS, 1);
    uint32_t *cw = calloc(3 * (uint64_t)NSYMS, sizeof(uint32_t));
    uint16_t *order = malloc(sizeof(uint16_t) * 3 * NSYMS);
    int nsym[3], maxlen[3];
    for (int k = 0; k < 3; k++) {
        nsym[k] = huffman_lengths(freq + (uint64_t)k * NSYMS, len + (uint64_t)k * NSYMS);
        maxlen[k] = 0;
        if (nsym[k]) canonical_codes(len + (uint64_t)k * NSYMS, cw + (uint64_t)k * NSYMS,
                                     order + (uint64_t)k * NSYMS, &maxlen[k]);
    }

    /* per-block sizes */
    uint16_t *cwords = malloc(sizeof(uint16_t) * nb);
    uint16_t *nesc = malloc(sizeof(uint16_t) * nb);
    uint64_t payload_words = 0;
    for (uint64_t b = 0; b < nb; b++) {
        uint64_t blen = (b + 1) * S <= n ? S : n - b * S;
        const uint8_t *lk = len + (uint64_t)pred[b] * NSYMS;
        uint64_t bits = 0, ne = 0;
        for (uint64_t j = 0; j < blen; j++) {
            bits += lk[code[b * S + j]];
            ne += code[b * S + j] == 0;
        }
        cwords[b] = (uint16_t)((bits + 31) / 32);
        nesc[b] = (uint16_t)ne;
        payload_words += skip_words(cwords[b], maxlen[pred[b]]) + cwords[b] + ne;
    }

    uint64_t off_pred = 0, o = HDR;
    if (policy >= 2) { off_pred = o; o = align8(o + nb); }
    uint64_t off_pfirst = o; o = align8(o + 4 * nb);
    uint64_t off_cwords = o; o = align8(o + 2 * nb);
    uint64_t off_nesc = o; o = align8(o + 2 * nb);
    uint64_t off_books = o;
    for (int k = 0; k < 3; k++)
        if (nsym[k]) o = align8(o + 4 * (uint64_t)maxlen[k] + 2 * (uint64_t)nsym[k]);
    uint64_t off_payload = o;
    uint64_t total = off_payload + 4 * payload_words;

    uint8_t *s = calloc(1, total);
    write_header_common(s, policy, eb_rel << 1, n, S, &p);
    put_u32(s, 20, (uint32_t)nb);
    put_f64(s, 40, p.step);
    for (int k = 0; k < 3; k++) {
        put_u32(s, 48 + 4 * (uint64_t)k, (uint32_t)nsym[k]);
        s[60 + k] = (uint8_t)maxlen[k];
    }
    put_u64(s, 64, payload_words);
    put_u64(s, 72, total);
    put_u64(s, 80, off_pred);
    put_u64(s, 88, off_pfirst);
    put_u64(s, 96, off_cwords);
    put_u64(s, 104, off_nesc);
    put_u64(s, 112, off_books);
    put_u64(s, 120, off_payload);
    for (uint64_t b = 0; b < nb; b++) {
        if (policy >= 2) s[off_pred + b] = pred[b];
        put_u32(s, off_pfirst + 4 * b, (uint32_t)q[b * S]);
        put_u16(s, off_cwords + 2 * b, cwords[b]);
        put_u16(s, off_nesc + 2 * b, nesc[b]);
    }
    o = off_books;
    for (int k = 0; k < 3; k++) {
        if (!nsym[k]) continue;
        const uint8_t *lk = len + (uint64_t)k * NSYMS;
        for (int l = 1; l <= maxlen[k]; l++) {
            uint32_t c = 0;
            for (int t = 0; t < NSYMS; t++) c += lk[t] == l;
            put_u32(s, o + 4 * (uint64_t)(l - 1), c);
        }
        uint64_t so = o + 4 * (uint64_t)maxlen[k];
        for (int i = 0; i < nsym[k]; i++) put_u16(s, so + 2 * (uint64_t)i, order[(uint64_t)k * NSYMS + i]);
        o = align8(so + 2 * (uint64_t)nsym[k]);
    }

    uint64_t wpos = 0;
    for (uint64_t b = 0; b < nb; b++) {
        uint64_t blen = (b + 1) * S <= n ? S : n - b * S;
        const uint8_t *lk = len + (uint64_t)pred[b] * NSYMS;
        const uint32_t *ck = cw + (uint64_t)pred[b] * NSYMS;
        bw_t bw;
        bw.w = calloc((uint64_t)cwords[b] + 1, sizeof(uint32_t));
        bw.nbits = 0;
        uint64_t *cstart = malloc(sizeof(uint64_t) * (blen + 1));
        for (uint64_t j = 0; j < blen; j++) {
            cstart[j] = bw.nbits;
            put_bits(&bw, ck[code[b * S + j]], lk[code[b * S + j]]);
        }
        /* skip table: first codeword start at or after each range start */
        const uint64_t cwn = cwords[b];
        const uint32_t R = n_ranges(cwn), wdt = skip_width(maxlen[pred[b]]);
        const uint64_t skw = skip_words(cwn, maxlen[pred[b]]);
        bw_t sk;
        sk.w = calloc(skw + 1, sizeof(uint32_t));
        sk.nbits = 0;
        uint64_t j = 0;
        for (uint32_t l = 1; l < R; l++) {
            uint64_t st = range_start(l, cwn);
            while (j < blen && cstart[j] < st) j++;
            put_bits(&sk, (uint32_t)(cstart[j] - st), (int)wdt);
        }
        for (uint64_t k = 0; k < skw; k++) put_u32(s, off_payload + 4 * (wpos + k), sk.w[k]);
        wpos += skw;
        for (uint64_t k = 0; k < cwords[b]; k++) put_u32(s, off_payload + 4 * (wpos + k), bw.w[k]);
        wpos += cwords[b];
        free(bw.w);
        free(sk.w);
        free(cstart);
        for (uint64_t j = 0; j < blen; j++)
            if (code[b * S + j] == 0) { put_u32(s, off_payload + 4 * wpos, (uint32_t)res[b * S + j]); wpos++; }
    }

    free(q); free(pred); free(code); free(res); free(freq); free(len); free(cw); free(order);
    free(cwords); free(nesc);
    *out = s;
    *out_len = total;
    return OK;
}

/* ------------------------------------------------------------ decompress */

typedef struct {
    int maxlen;
    uint32_t cnt[LMAX + 1], first[LMAX + 2], index[LMAX + 2];
    uint64_t off_syms;
} book_t;

int sznbref_decompress(const uint8_t *s, size_t slen, float **out, uint64_t *n_out)
{
    *out = NULL;
    *n_out = 0;
    if (slen < HDR || memcmp(s, "SZNB", 4) != 0 || get_u16(s, 4) != 1) return E_CORRUPT;
    int policy = s[6];
    int flags = s[7];
    uint64_t n = get_u64(s, 8);
    uint64_t S = get_u32(s, 16);
    uint64_t nb = get_u32(s, 20);
    float mn = u2f(get_u32(s, 24));
    double step = get_f64(s, 40);
    uint64_t total = get_u64(s, 72);
    if (total > slen || policy > 3 || n >= (1ull << 31)) return E_CORRUPT;
    if (S < 1024 || S > 16384 || (S & (S - 1))) return E_CORRUPT;
    float *y = malloc(sizeof(float) * (n ? n : 1));
    if (flags & 1) {
        for (uint64_t i = 0; i < n; i++) y[i] = mn;
        *out = y;
        *n_out = n;
        return OK;
    }
    if (nb != (n + S - 1) / S) { free(y); return E_CORRUPT; }
    uint64_t pw = get_u64(s, 64);
    uint64_t off_pred = get_u64(s, 80), off_pfirst = get_u64(s, 88), off_cwords = get_u64(s, 96);
    uint64_t off_nesc = get_u64(s, 104), off_books = get_u64(s, 112), off_payload = get_u64(s, 120);
    if (off_payload + 4 * pw > total || off_books > off_payload) { free(y); return E_CORRUPT; }
    /* the block tables must sit where the writer puts them: a corrupt offset
     * would send the table reads below outside the stream */
    {
        uint64_t e = HDR, e_pred = 0;
        if (policy >= 2) { e_pred = e; e = align8(e + nb); }
        uint64_t e_pfirst = e; e = align8(e + 4 * nb);
        uint64_t e_cwords = e; e = align8(e + 2 * nb);
        uint64_t e_nesc = e; e = align8(e + 2 * nb);
        if (off_pred != e_pred || off_pfirst != e_pfirst || off_cwords != e_cwords || off_nesc != e_nesc ||
            off_books != e) {
            free(y);
            return E_CORRUPT;
        }
    }

    /* canonical decoding tables: first code and first index per length */
    book_t bk[3];
    uint64_t o = off_books;
    for (int k = 0; k < 3; k++) {
        uint32_t nsym = get_u32(s, 48 + 4 * (uint64_t)k);
        int maxlen = s[60 + k];
        bk[k].maxlen = 0;
        if (nsym == 0) continue;
        if (maxlen < 1 || maxlen > LMAX || nsym > NSYMS || o + 4 * (uint64_t)maxlen + 2 * (uint64_t)nsym > off_payload) {
            free(y);
            return E_CORRUPT;
        }
        bk[k].maxlen = maxlen;
        memset(bk[k].cnt, 0, sizeof bk[k].cnt);
        uint32_t tot = 0;
        for (int l = 1; l <= maxlen; l++) { bk[k].cnt[l] = get_u32(s, o + 4 * (uint64_t)(l - 1)); tot += bk[k].cnt[l]; }
        if (tot != nsym) { free(y); return E_CORRUPT; }
        uint32_t c = 0, idx = 0;
        for (int l = 1; l <= maxlen; l++) {
            bk[k].first[l] = c;
            bk[k].index[l] = idx;
            c = (c + bk[k].cnt[l]) << 1;
            idx += bk[k].cnt[l];
        }
        bk[k].off_syms = o + 4 * (uint64_t)maxlen;
        o = align8(bk[k].off_syms + 2 * (uint64_t)nsym);
    }

    int32_t *r = malloc(sizeof(int32_t) * S);
    uint64_t wpos = 0;
    for (uint64_t b = 0; b < nb; b++) {
        uint64_t blen = (b + 1) * S <= n ? S : n - b * S;
        int k = policy == 0 ? 0 : policy == 1 ? 1 : s[off_pred + b];
        int32_t p0 = (int32_t)get_u32(s, off_pfirst + 4 * b);
        uint64_t cwn = get_u16(s, off_cwords + 2 * b);
        uint64_t ne = get_u16(s, off_nesc + 2 * b);
        if (k > 2 || bk[k].maxlen == 0) { free(y); free(r); return E_CORRUPT; }
        const book_t *B = &bk[k];
        const uint64_t skw = skip_words(cwn, B->maxlen);
        if (wpos + skw + cwn + ne > pw) { free(y); free(r); return E_CORRUPT; }
        const uint64_t sbase = off_payload + 4 * wpos;
        uint64_t base = sbase + 4 * skw;
        uint64_t bit = 0, esc = 0;
        const uint32_t R = n_ranges(cwn), wdt = skip_width(B->maxlen);
        uint32_t rnext = 1;  /* next range whose skip is checked */
        uint64_t sbit = 0;
        for (uint64_t j = 0; j < blen; j++) {
            /* every range start passed on the way to this codeword must point at it */
            while (rnext < R && range_start(rnext, cwn) <= bit) {
                uint32_t v = 0;
                for (uint32_t t = 0; t < wdt; t++, sbit++)
                    v = (v << 1) | ((get_u32(s, sbase + 4 * (sbit >> 5)) >> (31 - (sbit & 31))) & 1u);
                if (range_start(rnext, cwn) + v != bit) { free(y); free(r); return E_CORRUPT; }
                rnext++;
            }
            /* canonical decode, one bit at a time */
            uint32_t v = 0;
            int l = 0, found = 0;
            uint32_t sym = 0;
            while (l < B->maxlen) {
                if (bit >= 32 * cwn) { free(y); free(r); return E_CORRUPT; }
                uint32_t wd = get_u32(s, base + 4 * (bit >> 5));
                v = (v << 1) | ((wd >> (31 - (bit & 31))) & 1u);
                bit++;
                l++;
                if (v >= B->first[l] && v - B->first[l] < B->cnt[l]) {
                    sym = get_u16(s, B->off_syms + 2 * (uint64_t)(B->index[l] + v - B->first[l]));
                    found = 1;
                    break;
                }
            }
            if (!found) { free(y); free(r); return E_CORRUPT; }
            if (sym == 0) {
                if (esc >= ne) { free(y); free(r); return E_CORRUPT; }
                r[j] = (int32_t)get_u32(s, base + 4 * (cwn + esc));
                esc++;
            } else {
                r[j] = (int32_t)sym - RADIUS;
            }
        }
        if (esc != ne || r[0] != 0 || rnext != R) { free(y); free(r); return E_CORRUPT; }
        /* invert the prediction: d_j = q_j - q_0 from residuals, values before
         * the block equal to the anchor */
        int64_t d1 = 0, d2 = 0, d3 = 0;
        for (uint64_t j = 0; j < blen; j++) {
            int64_t pred;
            if (k == 0) pred = d1;
            else if (k == 1) pred = 2 * d1 - d2;
            else pred = 3 * d1 - 3 * d2 + d3;
            int64_t d0 = pred + r[j];
            int32_t pi = (int32_t)((int64_t)p0 + d0);
            y[b * S + j] = (float)fma((double)pi, step, (double)mn);
            d3 = d2; d2 = d1; d1 = d0;
        }
        wpos += skw + cwn + ne;
    }
    free(r);
    *out = y;
    *n_out = n;
    return OK;
}

/* ---------------------------------------------------- learned selector */

/* The learned policy replaces the exhaustive trial of select_pred by a small
 * network that reads cheap statistics of the block.  Not in the paper (its
 * methods fix one predictor each, Sec. 5.1); the definitions here are this
 * compressor's own.
 *
 * Features of a block of lattice values p_0..p_{len-1}, read on the sample
 * J = {j < len : j = 0 mod 4} of m = |J| positions (exact integer sums and
 * counts, so they do not depend on any summation order), with Dp_j and D2p_j
 * the LV and LCF residuals of residual() and P' = max(P, 1):
 *   0  sum_J p / (m P')              1  (max_J p - min_J p) / P'
 *   2  F(sum_J |Dp|) - F(m)          3  F(sum_J |D2p|) - F(m)
 *   4  F(max_J |Dp|)                 5  F(max_J |D2p|)
 *   6  #_J(Dp = 0) / m               7  #_J(D2p = 0) / m
 *   8  #_J(|Dp| <= 1) / m            9  #_J(|D2p| <= 1) / m
 *   10 #_J(Dp_j Dp_{j-1} < 0) / m   (Dp_{-1} = 0)
 *   11 F(sum_J bitlen |Dp|) - F(m)   12 F(sum_J bitlen |D2p|) - F(m)
 *   13 #_J(|Dp| >= 32768) / m        14 F(P')        15 1
 * F(v) = bit length of v plus the 8 bits after its leading one, over 256 (a
 * fixed-point log2 that is exact in float32); every ratio is one fp64
 * division rounded to float32. */
static float flog(uint64_t v)
{
    int b = 0;
    while (b < 64 && (v >> b) != 0) b++;
    if (b == 0) return 0.0f;
    uint64_t frac = b - 1 >= 8 ? (v >> (b - 9)) & 255u : (v << (9 - b)) & 255u;
    return (float)b + (float)frac / 256.0f;
}

static float ratio_f(uint64_t a, uint64_t b) { return (float)((double)a / (double)b); }

static uint32_t bitlen32(uint32_t v)
{
    uint32_t b = 0;
    while (b < 32 && (v >> b) != 0) b++;
    return b;
}

#define FEAT_STRIDE 4

static void block_features(const int32_t *q, uint64_t len, int64_t P, float f[16])
{
    uint64_t Pp = P > 0 ? (uint64_t)P : 1u;
    int64_t sum_p = 0, mx = q[0], mn = q[0];
    uint64_t s1 = 0, s2 = 0, m1 = 0, m2 = 0, z1 = 0, z2 = 0, o1 = 0, o2 = 0, sc = 0, b1 = 0, b2 = 0, esc = 0;
    uint64_t m = 0;
    for (uint64_t j = 0; j < len; j += FEAT_STRIDE) {
        m++;
        sum_p += q[j];
        if (q[j] > mx) mx = q[j];
        if (q[j] < mn) mn = q[j];
        int32_t d1 = residual(q, j, 0), d2 = residual(q, j, 1);
        int32_t prev = j >= 1 ? residual(q, j - 1, 0) : 0;
        uint32_t a1 = d1 < 0 ? (uint32_t)(-(int64_t)d1) : (uint32_t)d1;
        uint32_t a2 = d2 < 0 ? (uint32_t)(-(int64_t)d2) : (uint32_t)d2;
        s1 += a1; s2 += a2;
        if (a1 > m1) m1 = a1;
        if (a2 > m2) m2 = a2;
        if (a1 == 0) z1++;
        if (a2 == 0) z2++;
        if (a1 <= 1) o1++;
        if (a2 <= 1) o2++;
        if ((d1 > 0 && prev < 0) || (d1 < 0 && prev > 0)) sc++;
        b1 += bitlen32(a1);
        b2 += bitlen32(a2);
        if (a1 >= RADIUS) esc++;
    }
    float fm = flog(m);
    f[0] = ratio_f((uint64_t)sum_p, m * Pp);
    f[1] = ratio_f((uint64_t)(mx - mn), Pp);
    f[2] = flog(s1) - fm;
    f[3] = flog(s2) - fm;
    f[4] = flog(m1);
    f[5] = flog(m2);
    f[6] = ratio_f(z1, m);
    f[7] = ratio_f(z2, m);
    f[8] = ratio_f(o1, m);
    f[9] = ratio_f(o2, m);
    f[10] = ratio_f(sc, m);
    f[11] = flog(b1) - fm;
    f[12] = flog(b2) - fm;
    f[13] = ratio_f(esc, m);
    f[14] = flog(Pp);
    f[15] = 1.0f;
}

/* bfloat16 rounding, round to nearest, ties to even (finite inputs) */
static float bf16_round(float x)
{
    uint32_t u = f2u(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return u2f(u & 0xffff0000u);
}

/* Network 16 -> 32 -> 32 -> 3, ReLU.  Parameters in this order: W1[32][16],
 * b1[32], W2[32][32], b2[32], W3[3][32], b3[3] (1699 floats).  Inference:
 * inputs and weights rounded to bfloat16, biases kept in float32; each
 * neuron starts from its bias and adds w_k x_k for k ascending with one
 * fused multiply-add each; hidden outputs are ReLU then bfloat16-rounded. */
#define MLP_NPARAM 1699
static void mlp_logits(const float *w, const float feat[16], float z[3])
{
    const float *W1 = w, *B1 = w + 512, *W2 = w + 544, *B2 = w + 1568, *W3 = w + 1600, *B3 = w + 1696;
    float x[16], h1[32], h2[32];
    for (int k = 0; k < 16; k++) x[k] = bf16_round(feat[k]);
    for (int j = 0; j < 32; j++) {
        float acc = B1[j];
        for (int k = 0; k < 16; k++) acc = fmaf(bf16_round(W1[16 * j + k]), x[k], acc);
        h1[j] = bf16_round(acc > 0.0f ? acc : 0.0f);
    }
    for (int j = 0; j < 32; j++) {
        float acc = B2[j];
        for (int k = 0; k < 32; k++) acc = fmaf(bf16_round(W2[32 * j + k]), h1[k], acc);
        h2[j] = bf16_round(acc > 0.0f ? acc : 0.0f);
    }
    for (int j = 0; j < 3; j++) {
        float acc = B3[j];
        for (int k = 0; k < 32; k++) acc = fmaf(bf16_round(W3[32 * j + k]), h2[k], acc);
        z[j] = acc;
    }
}

/* argmax of the logits (ties to the lowest index) unless the margin to the
 * runner-up is below tau (or not a number): then the exhaustive trial. */
static int select_learned(const int32_t *q, uint64_t len, int64_t P, const float *w, float tau, int *fallback)
{
    float f[16], z[3];
    block_features(q, len, P, f);
    mlp_logits(w, f, z);
    int top = 0;
    for (int k = 1; k < 3; k++)
        if (z[k] > z[top]) top = k;
    float second = -INFINITY;
    for (int k = 0; k < 3; k++)
        if (k != top && z[k] > second) second = z[k];
    float margin = z[top] - second;
    if (!(margin >= tau)) {
        uint64_t c[3];
        *fallback = 1;
        return select_pred(q, len, c);
    }
    *fallback = 0;
    return top;
}

int sznbref_features(const int32_t *q, uint64_t n, uint32_t S, int64_t P, float *feat)
{
    for (uint64_t b = 0; b * S < n; b++) {
        uint64_t len = (b + 1) * S <= n ? S : n - b * S;
        block_features(q + b * S, len, P, feat + 16 * b);
    }
    return OK;
}

int sznbref_mlp_logits(const float *w, const float *feat, uint64_t nb, float *z)
{
    for (uint64_t b = 0; b < nb; b++) mlp_logits(w, feat + 16 * b, z + 3 * b);
    return OK;
}

float sznbref_bf16(float x) { return bf16_round(x); }

int sznbref_select_learned(const int32_t *q, uint64_t n, uint32_t S, int64_t P, const float *w, float tau,
                           uint8_t *pred, uint8_t *fallback)
{
    make_log_table();
    for (uint64_t b = 0; b * S < n; b++) {
        uint64_t len = (b + 1) * S <= n ? S : n - b * S;
        int fb;
        pred[b] = (uint8_t)select_learned(q + b * S, len, P, w, tau, &fb);
        fallback[b] = (uint8_t)fb;
    }
    return OK;
}

/* learned policy end to end: range, lattice, per-block learned choice, then
 * the same stream as every other policy */
int sznbref_compress_learned(const float *x, uint64_t n, double eb, uint32_t mode, const float *w, float tau,
                             uint8_t **out, size_t *out_len)
{
    if ((mode & 3u) != 3u) return E_INVAL;
    int bl = block_log2_of(mode);
    if (bl < 10 || bl > 14) return E_INVAL;
    if (n >= (1ull << 31)) return E_INVAL;
    params_t p;
    int st = range_and_bound(x, n, eb, (mode >> 4) & 1u, &p);
    if (st) return st;
    uint64_t S = 1ull << bl, nb = (n + S - 1) / S;
    uint8_t *pred = calloc(nb ? nb : 1, 1), *fb = calloc(nb ? nb : 1, 1);
    if (!p.is_const) {
        int32_t *q = malloc(sizeof(int32_t) * n);
        for (uint64_t i = 0; i < n; i++) q[i] = lattice(x[i], &p);
        sznbref_select_learned(q, n, (uint32_t)S, p.P, w, tau, pred, fb);
        free(q);
    }
    st = sznbref_compress_blocks(x, n, eb, mode, pred, out, out_len);
    free(pred);
    free(fb);
    return st;
}

void sznbref_free(void *p) { free(p); }

/* ------------------------------------------- introspection for the tests */

/* out: mn, mx, R, eb_abs, step, inv, P, is_const */
int sznbref_params(const float *x, uint64_t n, double eb, int eb_rel, double *out)
{
    params_t p;
    int st = range_and_bound(x, n, eb, eb_rel, &p);
    if (st) return st;
    out[0] = p.mn; out[1] = p.mx; out[2] = p.R; out[3] = p.eb_abs;
    out[4] = p.step; out[5] = p.inv; out[6] = (double)p.P; out[7] = p.is_const;
    return OK;
}

int sznbref_lattice(const float *x, uint64_t n, double eb, int eb_rel, int32_t *q)
{
    params_t p;
    int st = range_and_bound(x, n, eb, eb_rel, &p);
    if (st) return st;
    if (p.is_const) { for (uint64_t i = 0; i < n; i++) q[i] = 0; return OK; }
    for (uint64_t i = 0; i < n; i++) q[i] = lattice(x[i], &p);
    return OK;
}

int sznbref_residuals(const int32_t *q, uint64_t n, uint32_t S, int k, int32_t *r)
{
    for (uint64_t b = 0; b * S < n; b++) {
        uint64_t len = (b + 1) * S <= n ? S : n - b * S;
        for (uint64_t j = 0; j < len; j++) r[b * S + j] = residual(q + b * S, j, k);
    }
    return OK;
}

/* costs: 3 per block */
int sznbref_select(const int32_t *q, uint64_t n, uint32_t S, uint8_t *pred, uint64_t *costs)
{
    make_log_table();
    for (uint64_t b = 0; b * S < n; b++) {
        uint64_t len = (b + 1) * S <= n ? S : n - b * S;
        pred[b] = (uint8_t)select_pred(q + b * S, len, costs + 3 * b);
    }
    return OK;
}

int sznbref_block_cost(const int32_t *q, uint64_t len, int k, uint64_t *cost)
{
    make_log_table();
    if (len == 0 || len > 16384) return E_INVAL;
    *cost = block_cost(q, len, k);
    return OK;
}

void sznbref_log_table(uint32_t *tab)
{
    make_log_table();
    memcpy(tab, LOGT, sizeof LOGT);
}

int sznbref_res_class(int32_t r, int *cls, int *extra)
{
    res_class(r, cls, extra);
    return OK;
}

/* lengths for a 65536-entry frequency table; returns n_sym */
int sznbref_huffman_lengths(const uint32_t *freq, uint8_t *len)
{
    return huffman_lengths(freq, len);
}

int sznbref_canonical(const uint8_t *len, uint32_t *code, uint16_t *order)
{
    int m;
    canonical_codes(len, code, order, &m);
    return m;
}

void sznbref_reconstruct_array(const int64_t *p, uint64_t n, double step, float mn, float *out)
{
    params_t q;
    memset(&q, 0, sizeof q);
    q.step = step;
    q.mn = mn;
    for (uint64_t i = 0; i < n; i++) out[i] = reconstruct((int32_t)p[i], &q);
}

float sznbref_reconstruct(int32_t pi, double step, float mn)
{
    params_t p;
    memset(&p, 0, sizeof p);
    p.step = step;
    p.mn = mn;
    return reconstruct(pi, &p);
}
