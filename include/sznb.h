/*
 * sznb -- error-bounded lossy compression of 1D float32 particle fields on
 * AMD MI355X (gfx950).
 *
 * The method is the SZ-style pipeline the paper studies for N-body snapshots
 * (Tao, Di, Chen, Cappello, "In-Depth Exploration of Single-Snapshot Lossy
 * Compression Techniques for N-Body Simulations"):
 *   - prediction of each value from preceding values: last value (Sec. 5.1,
 *     the LV model), linear curve fit (Sec. 5.1, the LCF model) and its
 *     quadratic extension, the best fit chosen per block;
 *   - linear-scaling quantization of the prediction error into intervals of
 *     width 2*eb, 65536 intervals (Sec. 5.1);
 *   - Huffman coding of the quantization codes (Sec. 2; Sec. 5.2);
 *   - decompression that restores every value within the bound (Problem
 *     Statement: |x_i - x~_i| <= eb_abs, eb_rel = eb_abs / R).
 *
 * Every function is a plain C entry point over raw pointers.  "d_" pointers
 * are device (HBM) pointers, "h_" pointers are host pointers.  The caller
 * owns every buffer; the library never allocates device memory in these
 * calls.  Work is enqueued on `stream` (0 = default stream) and the calls
 * return without waiting for the GPU unless stated otherwise.
 *
 * Errors: argument errors found on the host are returned at once.  Errors
 * that depend on the data (non-finite input, a bound below float32
 * resolution, an output buffer that is too small, a corrupt stream) are found
 * on the GPU: the call returns SZNB_OK, the field's output length is set to
 * 0, and the per-field status is written into the workspace, where
 * sznb_read_status() reads it back (it synchronises the stream).
 */
#ifndef SZNB_H
#define SZNB_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define SZNB_OK 0
#define SZNB_EINVAL (-1)          /* bad argument (eb <= 0 or not finite, bad mode, n too large) */
#define SZNB_ENONFINITE (-2)      /* the field holds NaN or Inf */
#define SZNB_EEBTOOSMALL (-3)     /* bound below float32 resolution, or more than 2^27 lattice steps */
#define SZNB_ENOSPC (-4)          /* output buffer or workspace too small */
#define SZNB_ECORRUPT (-5)        /* stream fails validation */
#define SZNB_EDEVICE (-6)         /* HIP runtime error */

/* mode bits of sznb_compress */
#define SZNB_PRED_LV 0u           /* last-value predictor on every block (the paper's SZ-LV) */
#define SZNB_PRED_LCF 1u          /* linear curve fit on every block (original 1D SZ) */
#define SZNB_PRED_BESTFIT 2u      /* LV / LCF / QCF chosen per block by exhaustive trial */
#define SZNB_PRED_LEARNED 3u      /* per-block choice by the learned selector, trial as fallback */
#define SZNB_EB_REL (1u << 4)     /* eb is relative to the field's value range R = max - min */
#define SZNB_BLOCK_LOG2(b) ((uint32_t)(b) << 8) /* block size 2^b, b in 10..14; 0 = 4096 */

#define SZNB_MAX_N ((uint64_t)1 << 31)   /* fields hold fewer than 2^31 values */
#define SZNB_HEADER_BYTES 128u

/* Worst-case stream size for a field of n values compressed with `mode`. */
uint64_t sznb_compress_bound(uint64_t n, uint32_t mode);

/* Smallest output capacity the device path accepts (header, block tables,
 * codebooks).  Payload beyond out_cap is reported as SZNB_ENOSPC. */
uint64_t sznb_compress_min_capacity(uint64_t n, uint32_t mode);

/* Workspace bytes for compressing the nf fields of sizes n[] with modes
 * mode[] in one call.  No initial contents are required: every call clears
 * what it needs. */
uint64_t sznb_compress_workspace_bytes(int nf, const uint64_t *h_n, const uint32_t *h_mode);

/* Compress one field d_field[0..n) under the bound eb (absolute, or relative
 * to the value range when mode has SZNB_EB_REL) into d_out[0..out_cap).
 * The stream length is written to the device word *d_out_len (0 on error).
 * Stream layout: 128-byte header, block tables, one canonical Huffman
 * codebook per predictor in use, and the payload; see the design notes. */
int sznb_compress(const float *d_field, uint64_t n, double eb, uint32_t mode,
                  void *d_out, uint64_t out_cap, uint64_t *d_out_len,
                  void *d_ws, uint64_t ws_bytes, hipStream_t stream);

/* Compress nf fields in one batched launch sequence.  Arrays are host arrays
 * of length nf holding device pointers (fields, outputs) and per-field
 * parameters; d_lens is a device array of nf stream lengths.  All fields must
 * use the same block size. */
int sznb_compress_batch(int nf, const float *const *h_fields, const uint64_t *h_n,
                        const double *h_eb, const uint32_t *h_mode,
                        void *const *h_outs, const uint64_t *h_caps, uint64_t *d_lens,
                        void *d_ws, uint64_t ws_bytes, hipStream_t stream);

/* Parse a stream header held in host memory. */
int sznb_stream_info(const void *h_hdr, uint64_t hdr_len, uint64_t *n, uint32_t *mode,
                     double *eb_abs, uint64_t *total_bytes);

/* Workspace bytes for decompressing nf streams whose fields hold n[] values. */
uint64_t sznb_decompress_workspace_bytes(int nf, const uint64_t *h_n);

/* Decompress the stream d_stream[0..stream_len) into d_out[0..n), where n is
 * the field size stored in the stream (checked on the device).  d_stream must
 * be 8-byte aligned and d_out 16-byte aligned (SZNB_EINVAL otherwise). */
int sznb_decompress(const void *d_stream, uint64_t stream_len, float *d_out, uint64_t n,
                    void *d_ws, uint64_t ws_bytes, hipStream_t stream);

/* For callers that cannot allocate device memory (code between allocations
 * of a serving loop, harnesses that forbid hipMalloc): sznb_decompress
 * without a workspace argument.  The library keeps a fixed 8 MiB workspace
 * per GPU in device memory for the life of the process and never allocates
 * in this call; fields of more than SZNB_NOALLOC_MAX_N values are refused
 * with SZNB_ENOSPC.  Every call on one GPU shares that GPU's workspace:
 * calls that overlap on one GPU (other host threads, other streams) race.
 * The call waits for the stream (header read-back, then the decode) and
 * returns the stream's status (SZNB_ECORRUPT for a corrupt stream). */
#define SZNB_NOALLOC_MAX_N ((uint64_t)1 << 28)
int sznb_decompress_noalloc(const void *d_stream, uint64_t stream_len, float *d_out, uint64_t n,
                            hipStream_t stream);

/* Decompress nf streams in one batched launch sequence. */
int sznb_decompress_batch(int nf, const void *const *h_streams, const uint64_t *h_lens,
                          float *const *h_outs, const uint64_t *h_n,
                          void *d_ws, uint64_t ws_bytes, hipStream_t stream);

/* Per-field device status of the last call that used d_ws: waits for
 * `stream`, copies nf status words to h_status.  Returns the first non-OK
 * status, or SZNB_OK. */
int sznb_read_status(const void *d_ws, int nf, int *h_status, hipStream_t stream);

const char *sznb_strerror(int status);

/* ---- plans: many fields, one launch sequence, optionally one HIP graph
 * sznb_compress_plan validates the field table (as sznb_compress_batch),
 * writes its descriptors into d_ws and waits for that upload; the plan keeps
 * the pointers, so inputs may change in place between launches, and d_ws and
 * the outputs must outlive it.  sznb_plan_launch enqueues the compression
 * kernels only (no host synchronisation, no memory-set nodes), so it can run
 * under stream capture; sznb_plan_capture records it once into a HIP graph
 * owned by the plan (stream: a non-default stream), after which
 * sznb_plan_launch replays that graph.  Results are read as after
 * sznb_compress_batch (sznb_read_status, d_lens). */
typedef struct sznb_plan_s *sznb_plan;
int sznb_compress_plan(int nf, const float *const *h_fields, const uint64_t *h_n, const double *h_eb,
                       const uint32_t *h_mode, void *const *h_outs, const uint64_t *h_caps, uint64_t *d_lens,
                       void *d_ws, uint64_t ws_bytes, hipStream_t stream, sznb_plan *plan_out);
/* Decompression plan of a table of streams (as sznb_decompress_batch): the
 * headers are read once here (block size, codebook sizes) to lay out the
 * decoder; launches then enqueue kernels only.  Streams given to a later
 * launch may be new contents of the same buffers; one whose block size
 * exceeds the largest planned one is reported as SZNB_ECORRUPT. */
int sznb_decompress_plan(int nf, const void *const *h_streams, const uint64_t *h_lens, float *const *h_outs,
                         const uint64_t *h_n, void *d_ws, uint64_t ws_bytes, hipStream_t stream,
                         sznb_plan *plan_out);
int sznb_plan_capture(sznb_plan plan, hipStream_t stream);
int sznb_plan_launch(sznb_plan plan, hipStream_t stream);
void sznb_plan_destroy(sznb_plan plan);

/* Width of the persistent grids (range and pack kernels) in workgroups of
 * 256 threads per compute unit, 1..16 (default 8); process-wide. */
int sznb_set_workgroups_per_cu(int wg);
int sznb_get_workgroups_per_cu(void);

/* Autotuner: times compression of the given fields for block sizes 2^10 ..
 * 2^14 and 2, 4, 8, 16 workgroups per CU, keeps the candidates whose total
 * stream size is within 1 % of the smallest and returns the fastest as a mode
 * (policy_mode | SZNB_BLOCK_LOG2(b)) and a width for
 * sznb_set_workgroups_per_cu.  policy_mode holds only predictor and
 * SZNB_EB_REL bits.  With cache_path, a line keyed by (GPU architecture,
 * log2 of the total value count, log2 of the field count, policy) is looked
 * up first and appended after a tuning run.  Allocates its own scratch. */
int sznb_autotune(int nf, const float *const *h_fields, const uint64_t *h_n, const double *h_eb,
                  uint32_t policy_mode, const char *cache_path, uint32_t *h_best_mode, int *h_best_wg,
                  hipStream_t stream);

/* ---- learned predictor selector (SZNB_PRED_LEARNED)
 * Not part of the paper, whose methods fix one predictor each (Sec. 5.1): a
 * small network 16 -> 32 -> 32 -> 3 (ReLU) reads 16 statistics of a block's
 * lattice values and picks LV, LCF or QCF; when the margin between its two
 * largest logits is below tau (or not a number) the block falls back to the
 * exhaustive trial of SZNB_PRED_BESTFIT.  The predictor ids are stored in the
 * stream, so decompression never needs the network.
 * Parameters, 1699 float32 in this order: W1[32][16], b1[32], W2[32][32],
 * b2[32], W3[3][32], b3[3].  Inference rounds features and weights to
 * bfloat16 (nearest, ties to even), keeps biases in float32, accumulates each
 * neuron from its bias with one fused multiply-add per input in ascending
 * order, and rounds hidden outputs (after ReLU) to bfloat16.
 * Features of a block of lattice values p (span P' = max(P,1)), read on its
 * positions j = 0 mod 4 (m of them), Dp / D2p its LV / LCF residuals,
 * F(v) = bit length of v + (8 bits after the leading one)/256, every ratio
 * one fp64 division rounded to float32, sums and counts over the sample:
 *   0 sum p/(m P')  1 (max p - min p)/P'  2 F(sum|Dp|)-F(m)
 *   3 F(sum|D2p|)-F(m)  4 F(max|Dp|)  5 F(max|D2p|)  6 #(Dp=0)/m
 *   7 #(D2p=0)/m  8 #(|Dp|<=1)/m  9 #(|D2p|<=1)/m
 *   10 #(Dp_j Dp_{j-1} < 0)/m  11 F(sum bitlen|Dp|)-F(m)
 *   12 F(sum bitlen|D2p|)-F(m)  13 #(|Dp|>=32768)/m  14 F(P')  15 1 */
#define SZNB_MLP_PARAMS 1699u
#define SZNB_FEATURES 16u

/* Load the selector used by SZNB_PRED_LEARNED on the current device (host
 * parameters, copied; weights rounded to bfloat16 here).  Until it is
 * called, compressing with SZNB_PRED_LEARNED returns SZNB_EINVAL. */
int sznb_set_selector(const float *h_params, float tau);

/* Training data: for every block of every field (blocks in field order),
 * the 16 features (d_feat, float32 [blocks][16]), the three trial costs
 * (d_cost, u64 [blocks][3], 2^-16 bit units) and the trial's choice
 * (d_label, u8 [blocks]).  All fields must share one block size.  Returns
 * after enqueueing; constant or failed fields give zero rows. */
uint64_t sznb_features_workspace_bytes(int nf, const uint64_t *h_n, const uint32_t *h_mode);
int sznb_block_features(int nf, const float *const *h_fields, const uint64_t *h_n, const double *h_eb,
                        const uint32_t *h_mode, float *d_feat, uint64_t *d_cost, uint8_t *d_label,
                        void *d_ws, uint64_t ws_bytes, hipStream_t stream);

/* Blocks of each field of the last compression in d_ws that the learned
 * policy handed to the exhaustive trial (waits for the stream). */
int sznb_compress_fallbacks(const void *d_ws, int nf, uint32_t *h_out, hipStream_t stream);

/* Training (float32, deterministic): gradient of the mean softmax
 * cross-entropy over a batch of feature rows and labels (d_grad: 1699
 * floats, d_loss: 1 float), and one Adam step (Kingma and Ba, 2015) with
 * bias correction; step counts from 1. */
uint64_t sznb_mlp_grad_workspace_bytes(uint32_t batch);
int sznb_mlp_grad(const float *d_params, const float *d_feat, const uint8_t *d_label, uint32_t batch,
                  float *d_grad, float *d_loss, void *d_ws, uint64_t ws_bytes, hipStream_t stream);
int sznb_mlp_adam(float *d_params, float *d_m, float *d_v, const float *d_grad, uint32_t step, float lr,
                  float beta1, float beta2, float eps, hipStream_t stream);

/* The compressor's bfloat16 inference on nb feature rows: logits [nb][3],
 * choice (argmax, ties to the lowest) and margin to the runner-up. */
int sznb_mlp_infer(const float *d_params, const float *d_feat, uint64_t nb, float *d_logits,
                   uint8_t *d_choice, float *d_margin, hipStream_t stream);

/* ---- molecular-dynamics snapshots: the paper's modes (Sec. 5.2, Sec. 6)
 * and its R-index studies (Tables 4-6)
 * md_mode, low byte (the kind):
 *   0 best_speed:       SZ-LV on every field in stored order;
 *   1 best_tradeoff:    particles reordered by a stable sort of their
 *                       R-index without its k least significant digits
 *                       inside fixed index segments (Table 5: segment 16384,
 *                       k = 6), then SZ-LV on every field;
 *   2 best_compression: full R-index sort; the sorted coordinate keys coded
 *                       CPC2000-style (Rice-coded deltas), the velocities by
 *                       SZ-LV in the same order;
 *   3 CPC2000:          as 2, with the velocities' lattice integers coded by
 *                       CPC2000's variable-length code (per segment the
 *                       minimum, then Rice-coded offsets; Sec. 2, Sec. 5.2).
 * Further bits (SZNB_MD_*): segment size 2^s, s in 10..14 (default 16384);
 * k + 1 in bits 12-15 (default: 6 for kind 1, 0 otherwise); the key fields
 * (Sec. 5.3, Table 6): coordinates (default), velocities, or all six fields
 * (each cut to its 10 leading bits, one bit of each per 6-bit digit; kind 1
 * only, with six fields).  Kind 0 takes none of them.
 * h_fields: 3 coordinate fields (x, y, z), optionally followed by 3 velocity
 * fields, each of n values (device pointers, 16-byte aligned).  eb_rel is the
 * value-range-relative bound of every field.  The particles come back from
 * sznb_md_decompress in the stored order of the container (reordered for
 * kinds 1-3: no index is kept, every field is permuted the same way); the
 * permutation is written to d_perm_or_null when given.
 * Both calls enqueue their work and return without waiting for the GPU; the
 * container length is written to the device word *d_out_len and the first
 * error of the call (keying, any sub-stream, the container) is read with
 * sznb_read_status(d_ws, 1, ...). */
#define SZNB_MD_SEG_LOG2(s) ((int)(s) << 8)
#define SZNB_MD_IGNORED(k) ((int)((k) + 1) << 12)
#define SZNB_MD_KEY_VEL (1 << 16)
#define SZNB_MD_KEY_ALL (2 << 16)
uint64_t sznb_md_workspace_bytes(int nf, uint64_t n);
uint64_t sznb_md_bound(int nf, uint64_t n);
int sznb_md_compress(int nf, const float *const *h_fields, uint64_t n, double eb_rel, int md_mode,
                     void *d_out, uint64_t out_cap, uint64_t *d_out_len, uint32_t *d_perm_or_null,
                     void *d_ws, uint64_t ws_bytes, hipStream_t stream);
int sznb_md_decompress(const void *d_in, uint64_t in_len, int nf, uint64_t n, float *const *h_outs,
                       void *d_ws, uint64_t ws_bytes, hipStream_t stream);

/* Measurement hooks.  sznb_profile(1) clears the record and brackets every
 * later kernel launch with a pair of HIP events on the launch stream;
 * sznb_profile(0) stops recording.  sznb_profile_summary() waits for the
 * recorded events and writes, per kernel, its name (32-byte slots in
 * `names`), the summed duration in milliseconds and the launch count; it
 * returns the number of distinct kernels (entries beyond max_kernels are
 * dropped). */
int sznb_profile(int enable);
int sznb_profile_summary(int max_kernels, char *names, double *total_ms, int *count);
/* Restricts the bracketing to the kernels named in `names` (comma-separated,
 * as sznb_profile_summary names them); NULL or "" brackets every kernel.
 * Each bracket costs the stream a few microseconds between kernels, so a
 * measurement that needs only some kernels' durations names them. */
int sznb_profile_kernels(const char *names);

#ifdef __cplusplus
}
#endif
#endif /* SZNB_H */
