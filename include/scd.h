/*
 * scd.h - C ABI of a spectral correlation density (SCD) library for AMD Instinct MI355X (gfx950).
 *
 * Two estimators of the SCD are provided (arXiv 2506.18003, Sec. II):
 *   FAM   the FFT accumulation method, Eq. (3)-(5);
 *   SSCA  the strip spectral correlation analyser, Eq. (6)-(7), computed through the decomposed N-point
 *         DFT of Sec. III-B (Eq. (10)-(16)).
 *
 * Conventions shared by every entry point
 *   - Complex arrays are interleaved float pairs (re, im), i.e. complex64; `n` complex values take 2n floats.
 *   - x, win and out are DEVICE pointers (hipMalloc'd, managed, or hipHostMalloc'd memory the GPU can read),
 *     contiguous, 8-byte aligned. The caller owns them; the library never retains them after a call.
 *   - Calls enqueue kernels on a HIP stream and return without waiting: on the stream in scd_opts, else
 *     on the stream given to scd_set_stream (default: the null stream). Only the first call for a new
 *     (size, channel count) pair synchronises, while it generates its FP64 tables.
 *   - Frames are centred as in Eq. (3): frame p covers samples pL - d + j, j = 0..Np-1, d = Np/2 - 1, and
 *     win[j] multiplies sample j of the frame. Samples outside the signal are zero.
 *   - The down-conversion factor is Eq. (3)'s exp(-i 2 pi k p L / Np) with the integer exponent reduced
 *     mod Np. Channel k and bin q are in natural DFT order (k, q >= 0). No normalisation is applied
 *     (g = g_d = 1).
 *   - Return 0 (SCD_OK) on success, or a negative SCD_ERR_* code; scd_last_error() then gives a message.
 *     Argument errors are detected before any GPU work is enqueued. On error, out is unspecified and x and
 *     win are never written. Nothing is printed and no C++ exception crosses the ABI.
 *   - The library's own device memory is allocated on first use and released by scd_shutdown(): the
 *     FP64-generated tables per device, and the scratch (SSCA intermediate and the like) per (device, stream).
 */
#ifndef SCD_H
#define SCD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define SCD_OK 0
#define SCD_ERR_NULL (-1)        /* a required pointer is NULL                                         */
#define SCD_ERR_SIZE (-2)        /* a size is not a power of two, out of range, or inconsistent        */
#define SCD_ERR_ALIAS (-3)       /* out overlaps x, win or the workspace                                */
#define SCD_ERR_NOMEM (-4)       /* device allocation failed or the caller's workspace is too small     */
#define SCD_ERR_HIP (-5)         /* a HIP runtime call or kernel launch failed                          */
#define SCD_ERR_MODEL (-6)       /* invalid selector model                                              */
#define SCD_ERR_UNSUPPORTED (-7) /* valid arguments, but this precision/size combination is not built   */
#define SCD_ERR_PTR (-8)         /* a pointer is not device-accessible memory, or its allocation is
                                    smaller than the array it must hold                                 */

/* Arithmetic of the channelizer DFT (Eq. (3)). Everything after the channelizer is FP32.
 *   SCD_FP32        FP32 throughout.
 *   SCD_SPLIT_BF16  channelizer as a DFT-GEMM on MFMA with bf16 hi/lo split operands (3 products), FP32
 *                   accumulation.
 *   SCD_SPLIT_FP16  the same with fp16 hi/lo operands.
 *   SCD_BF16        a single bf16 product (no split), FP32 accumulation: an accuracy ablation.
 *   SCD_FP16        a single fp16 product (no split), FP32 accumulation: an accuracy ablation. */
typedef enum scd_precision {
  SCD_FP32 = 0,
  SCD_SPLIT_BF16 = 1,
  SCD_SPLIT_FP16 = 2,
  SCD_BF16 = 3,
  SCD_FP16 = 4
} scd_precision;

/* Options of the _ex entry points. Zero-initialise, then set what you need.
 *   precision        an scd_precision value (FP32 if 0)
 *   batch            number of signals (0 or 1 = one signal); signals and outputs are laid out at the
 *                    strides below
 *   x_stride         complex elements between consecutive signals of x (0 = the signal length)
 *   out_stride       complex elements between consecutive outputs (0 = the output size)
 *   stream           hipStream_t to enqueue on (NULL = the stream given to scd_set_stream)
 *   workspace        device scratch for the SSCA intermediate or FAM's X_T (NULL = library-owned); must not
 *                    overlap x, win or out; its contents are undefined after the call
 *   workspace_bytes  size of workspace; see scd_ssca_workspace_size / scd_fam_workspace_size */
typedef struct scd_opts {
  int precision;
  int batch;
  int64_t x_stride;
  int64_t out_stride;
  void* stream;
  void* workspace;
  size_t workspace_bytes;
} scd_opts;

/*
 * scd_ssca - SSCA estimate of one signal (Sec. II-C, Eq. (6)-(7); Sec. III-B, Eq. (10)-(16)).
 *
 *   S[k][q] = sum_{n=0}^{N-1} X_T[n][k] conj(x[n]) exp(-i 2 pi n q / N),   k in [0,Np), q in [0,N),
 *   X_T[n][k] = exp(-i 2 pi ((k n) mod Np) / Np) * sum_{j<Np} win[j] x[n - d + j] exp(-i 2 pi k j / Np).
 *
 * Cell [k][q] estimates the SCD at alpha = f_k + q_c/N, f = (f_k - q_c/N)/2 (f_s = 1), with k_c, q_c the
 * signed indices ((k + Np/2) mod Np) - Np/2 and ((q + N/2) mod N) - N/2 and f_k = k_c/Np.
 *
 *   x    device, N complex values
 *   N    SSCA window = signal length, a power of two in [2^10, 2^20]
 *   Np   channel count, a power of two in [16, 256], Np <= N
 *   win  device, Np floats
 *   out  device, Np*N complex values, row-major [Np][N]
 * Errors: SCD_ERR_NULL, SCD_ERR_SIZE, SCD_ERR_ALIAS, SCD_ERR_PTR, SCD_ERR_NOMEM, SCD_ERR_HIP.
 * Uses a library-owned intermediate of 8*Np*N bytes when N > 1024 and no workspace is given. The library's
 * scratch (this intermediate, the split-precision operands, the selector's buffers) is kept per (device,
 * stream): calls on different streams may run concurrently, and calls on one stream are ordered by it. Each
 * stream's scratch persists until scd_shutdown. The FP64 tables are shared, read-only once built.
 */
int scd_ssca(const float* x, int64_t N, int Np, const float* win, float* out);

/* scd_ssca with options: precision, batching (x: [batch] signals at x_stride, out: [batch][Np][N] at
 * out_stride), stream and caller workspace. A caller workspace smaller than one signal's intermediate gives
 * SCD_ERR_NOMEM; a smaller batch chunk is used when it holds fewer than `batch` intermediates. Split
 * precisions require Np <= 128 (SCD_ERR_UNSUPPORTED otherwise). */
int scd_ssca_ex(const float* x, int64_t N, int Np, const float* win, float* out, const scd_opts* opts);

/*
 * scd_ssca_block_ex - SSCA estimate of the block n in [offset, offset + N) of a longer signal (a stream of
 * blocks): the channelizer of Eq. (3) sees the whole signal, so frames at the block's edges use the true
 * neighbouring samples, with zeros only outside [0, len); the sum of Eq. (7) runs over the block:
 *   S[k][q] = sum_{n<N} X_T[offset + n][k] conj(x[offset + n]) exp(-i 2 pi n q / N).
 *   x       device, len complex values per signal (opts->x_stride between signals, default len)
 *   len     samples of each signal, at most 2^27
 *   offset  start of the block, a multiple of Np (where Eq. (3)'s down-conversion restarts), offset + N <= len
 * offset = 0 with len = N is scd_ssca_ex. Other arguments, options and errors as scd_ssca_ex, except that only
 * SCD_FP32 is supported (SCD_ERR_UNSUPPORTED otherwise) and a bad len or offset is SCD_ERR_SIZE. */
int scd_ssca_block_ex(const float* x, int64_t len, int64_t offset, int64_t N, int Np, const float* win, float* out,
                      const scd_opts* opts);

/*
 * scd_ssca_strips - the SSCA restricted to a caller-given set of strips. Each strip k of Eq. (7) is its own
 * N-point DFT of the channel-data product of channel k (Eq. (6)), so any set of strips is computed exactly
 * and independently of the others. This is one GPU's share when the strips are split over several GPUs.
 *   strips   host, nstrips distinct strip indices in [0, Np), in any order; read before the call returns
 *   nstrips  0 .. Np; 0 does nothing (SCD_OK once x, win and out are non-NULL)
 * Only the listed rows of out ([Np][N] per signal) are written; the other rows are left untouched. Every
 * signal of a batch gets the same strips. Stage 1 computes each channel subset (strips k = c mod Np/16) that
 * holds a listed strip; Stage 2 runs only for the listed strips. Precision SCD_FP32 or SCD_SPLIT_BF16
 * (SCD_ERR_UNSUPPORTED otherwise). Other arguments, options (batch, strides, stream, workspace) and errors as
 * scd_ssca_ex. A strip outside [0, Np), or listed twice, or nstrips outside [0, Np] gives SCD_ERR_SIZE;
 * strips == NULL with nstrips > 0 gives SCD_ERR_NULL. At N = 1024, where Stage 1 alone is the transform, its
 * output goes through the library's scratch (8*Np*N bytes per signal) and the listed rows are copied to out.
 */
int scd_ssca_strips(const float* x, int64_t N, int Np, const float* win, const int* strips, int nstrips, float* out,
                    const scd_opts* opts);

/*
 * Streaming receiver: SSCA estimates of a continuous stream of host blocks of N samples (the block form of
 * scd_ssca_block_ex over consecutive blocks, each with its true neighbouring samples at its edges; zeros only
 * before the first block and after the last), in fixed device memory: a library-owned ring of `slots` blocks with
 * Np samples of halo at its two ends, and the caller's output buffers used in rotation. Each push copies one host
 * block on the receiver's own copy stream (default priority) and enqueues the estimate of the previous block on
 * the caller's stream, ordered by events, so the copy of one block overlaps the estimate of an earlier one. The
 * ring bounds how far the host runs ahead: a push first waits until the estimate of block c + 1 - slots (the
 * last one reading the slot block c reuses) has finished.
 *
 * scd_receiver_create: N, Np as scd_ssca (N >= Np); win: device Np floats (caller-owned, read by every estimate);
 *   slots in [3, 64] (4 lets a copy overlap the estimate two blocks back); outputs: n_outputs (1..64) device
 *   buffers of Np*N complex values each, caller-owned; stream: hipStream_t of the estimates (NULL: null stream).
 *   Allocates the ring (8 (slots N + 2 Np) bytes) on the current device and synchronises once.
 * scd_receiver_push: waits for the slot (above), then copies; host_block holds N complex values, in pinned
 *   memory for the copy to be asynchronous; it
 *   must not be modified until its copy has completed (scd_receiver_wait_copy). On return *out_index is the
 *   output buffer that will hold the previous block's estimate in stream order, and *offset that block's first
 *   sample (-1 and unchanged for the first push). A buffer is overwritten n_outputs estimates later.
 * scd_receiver_finish: enqueues the last block's estimate (its right edge reads zeros), waits for every copy.
 * scd_receiver_wait_copy: waits until every pushed block's copy has completed.
 * scd_receiver_destroy: waits for the receiver's work, frees it (NULL is a no-op).
 * Errors: SCD_ERR_NULL, SCD_ERR_SIZE, SCD_ERR_NOMEM, SCD_ERR_HIP, and those of scd_ssca_block_ex.
 */
typedef struct scd_receiver scd_receiver;
int scd_receiver_create(int64_t N, int Np, const float* win, int slots, float* const* outputs, int n_outputs,
                        void* stream, scd_receiver** rx);
int scd_receiver_push(scd_receiver* rx, const float* host_block, int* out_index, int64_t* offset);
int scd_receiver_finish(scd_receiver* rx, int* out_index, int64_t* offset);
int scd_receiver_wait_copy(scd_receiver* rx);
int scd_receiver_destroy(scd_receiver* rx);

/*
 * scd_ssca_cross_ex - SSCA estimate of the cross SCD of x and y (Eq. (2) with y != x, Sec. II-A): the demodulate
 * of y has the SSCA's one-sample window, so the channel-data product takes conj(y[n]) where scd_ssca takes
 * conj(x[n]):
 *   S_xy[k][q] = sum_{n=0}^{N-1} X_T[n][k] conj(y[n]) exp(-i 2 pi n q / N),   X_T[n][k] of x as in scd_ssca.
 * conjugate != 0 gives the conjugate form, with y[n] in place of conj(y[n]) (a library form; the paper
 * treats the conjugated product only); its cell [k][q] pairs x's demodulate at f_k with y's at q/N, so alpha
 * there is the conjugate cycle frequency f_k + q_c/N. y = x gives exactly scd_ssca's result.
 *   y    device, N complex values per signal, laid out like x (same opts->x_stride)
 * Other arguments, options and errors as scd_ssca_ex, except that only SCD_FP32 is supported
 * (SCD_ERR_UNSUPPORTED otherwise) and out must not overlap y (SCD_ERR_ALIAS). */
int scd_ssca_cross_ex(const float* x, const float* y, int64_t N, int Np, const float* win, int conjugate, float* out,
                      const scd_opts* opts);

/*
 * scd_ssca_stage1_ex / scd_ssca_stage2_ex - the two stages of SSCA_2DFFT (Sec. III-B, Eq. (14)-(16)) as
 * separate calls, so a caller can time, pipeline or interleave them. scd_ssca_ex runs exactly stage 1
 * followed by stage 2 through a library-owned intermediate.
 *
 * With N = M1*M2, M1 = 1024, M2 = N/1024, stage 1 generates the channel-data product X_g(m1*M2 + m2, k)
 * (Eq. (11)-(13)), takes the M1-point DFT over m1 and multiplies by the rotation factor
 * exp(-i 2 pi m2 m1' / N) (Eq. (15)); it writes S_s1(m1', m2, k) to `inter` in the blocked layout
 * inter[k][m1'/16][m2][m1' mod 16] (Np*N complex values per signal). Stage 2 takes the M2-point DFT over m2
 * (Eq. (16)) and writes S[k][q], q = m1' + M1*m2', to out ([Np][N]).
 *   stage 1: x (N complex per signal, opts->x_stride), win, inter (opts->out_stride, default Np*N)
 *   stage 2: inter (opts->x_stride, default Np*N), out (opts->out_stride, default Np*N); win is not used
 * With N == 1024 the intermediate layout equals the output layout and stage 2 only copies (nothing when
 * inter == out). Precision (stage 1 only) as in scd_ssca_ex. Errors as scd_ssca_ex.
 */
int scd_ssca_stage1_ex(const float* x, int64_t N, int Np, const float* win, float* inter, const scd_opts* opts);
int scd_ssca_stage2_ex(const float* inter, int64_t N, int Np, float* out, const scd_opts* opts);

/*
 * scd_fam - FAM estimate of one signal (Sec. II-B, Eq. (3)-(5)).
 *
 *   S[k][l][q] = sum_{p=0}^{P-1} X_T[p][k] conj(X_T[p][l]) exp(-i 2 pi p q / P),
 *   X_T[p][k]  = exp(-i 2 pi ((k p L) mod Np) / Np) * sum_{j<Np} win[j] x[pL - d + j] exp(-i 2 pi k j / Np),
 * over the first N = P*L samples. Cell [k][l][q] estimates the SCD at f = (f_k + f_l)/2,
 * alpha = f_k - f_l + q_c/(P L); bins with |q_c| < P L / Np are inside the pair's channel overlap.
 *
 *   x    device, P*L complex values
 *   Np   channel count, a power of two in [16, 256]
 *   L    hop between frames, a power of two in [1, Np] (the paper uses Np/4)
 *   P    frame count, a power of two in [4, 1024], P*L <= 2^16
 *   win  device, Np floats
 *   out  device, Np*Np*P complex values, row-major [Np][Np][P] (k unconjugated, l conjugated)
 * Errors: SCD_ERR_NULL, SCD_ERR_SIZE, SCD_ERR_ALIAS, SCD_ERR_PTR, SCD_ERR_NOMEM, SCD_ERR_HIP.
 */
int scd_fam(const float* x, int Np, int L, int P, const float* win, float* out);

/* scd_fam with options (batch, strides, stream, workspace for X_T). Only SCD_FP32 is supported. */
int scd_fam_ex(const float* x, int Np, int L, int P, const float* win, float* out, const scd_opts* opts);

/* scd_fam_power_ex - the output the paper's FAM keeps (Alg. 1: |S|^2 of the second FFT over its central half,
 * the bins with -P/4 <= q_c < P/4), written by the FAM kernel itself instead of the complex grid:
 *   out[k][l][j] = |S[k][l][q]|^2, q = j for j < P/4 and q = j + P/2 for j >= P/4 (j < P/2),
 * each power rounded as re*re + im*im with every operation rounded to FP32 (no fused multiply-add).
 *   out  device, Np*Np*(P/2) floats per signal, row-major [Np][Np][P/2]; opts->out_stride counts floats.
 * Arguments, sizes, options and errors otherwise as scd_fam_ex. The output is a quarter of the complex grid's
 * bytes, which dominate FAM's HBM traffic. */
int scd_fam_power_ex(const float* x, int Np, int L, int P, const float* win, float* out, const scd_opts* opts);

/* scd_fam_cross_ex - FAM estimate of the cross SCD of x and y (Eq. (2) and (5) with a second input):
 *   S_xy[k][l][q] = sum_p X_T[p][k] conj(Y_T[p][l]) exp(-i 2 pi p q / P),   Y_T the Eq. (3) channelizer of y;
 * conjugate != 0 takes Y_T[p][l] itself (the conjugate SCD, a library form). y = x gives scd_fam's result.
 *   y    device, P*L complex values per signal, laid out like x (same opts->x_stride)
 * A caller workspace must hold X_T and Y_T: twice what scd_fam_workspace_size reports. Other arguments,
 * options and errors as scd_fam_ex; out must not overlap y (SCD_ERR_ALIAS). */
int scd_fam_cross_ex(const float* x, const float* y, int Np, int L, int P, const float* win, int conjugate, float* out,
                     const scd_opts* opts);

/* ---------------------------------------------------------------------------------------------------------
 * Learned strip selection. The paper has no learned component (its glossary only names the averaged cyclic
 * periodogram and the PSD, and its conclusion points at a machine-learning back-end); the definitions below
 * are this library's. A small MLP reads per-strip features and predicts which SSCA strips carry cycle-frequency
 * energy; only those strips then get their N-point DFT, with the full SSCA as fallback below a confidence
 * threshold.
 *
 * Features (2 Np floats per signal, strip k): from the SSCAs S_b of 16 segments of 1024 samples starting at
 * b N/16 (each zero outside itself), A_k[q] = sum_b |S_b[k][q]|^2;
 *   feat[k]      = 0.5 log(A_k[q0(k)]) centred over k, q0(k) = (-k_c 1024/Np) mod 1024 (alpha = 0 bin);
 *   feat[Np + k] = log(max / mean of A_k over bins more than 4 bins (circularly) away from q0(k)).
 * Labels (from a full SSCA): strip k is active when max |S[k][q]|^2 > (6.2^2 / 2) * mean |S[k][q]|^2 over the
 * bins q whose cycle frequency is at least 1/256 away from 0 modulo 1.
 * MLP: f -> relu(W1 f + b1) -> relu(W2 h1 + b2) -> sigmoid(W3 h2 + b3), sizes 2 Np -> 256 -> 256 -> Np, on
 * standardised features (f - mu) / sigma. Parameters are one FP32 device array packed as
 * [W1 (256 x 2Np) | b1 (256) | W2 (256 x 256) | b2 (256) | W3 (Np x 256) | b3 (Np)], W row-major [out][in];
 * every GEMM rounds both operands to bf16 and accumulates in FP32 on the matrix cores.
 * ------------------------------------------------------------------------------------------------------- */

/* A trained selector. All arrays are device memory owned by the caller. */
typedef struct scd_selector {
  int Np;              /* channel count the model was trained for                         */
  const float* params; /* packed MLP parameters, scd_mlp_param_count(Np) floats            */
  const float* mu;     /* feature means, 2 Np floats                                       */
  const float* sigma;  /* feature scales, 2 Np floats                                      */
  float theta;         /* strip score threshold                                            */
  float conf_min;      /* fall back to the full SSCA when min_k max(s_k, 1 - s_k) < conf_min */
} scd_selector;

/* A library-owned selector: the packed MLP parameters, feature means and scales in device memory of the device
 * that was current when it was created, with the score threshold and confidence floor. Opaque; the calls below
 * create, save, load and free it, and scd_model_selector gives the scd_selector view scd_ssca_learned takes.
 * Model files are little-endian: "SCDM", u32 version 1, i32 Np, i32 parameter count, f32 theta, f32 conf_min,
 * the parameters, mu (2 Np) and sigma (2 Np) as f32, then a u32 FNV-1a hash of every preceding byte. */
typedef struct scd_model scd_model;

/* Create a model from HOST arrays (params: scd_mlp_param_count(Np) floats, mu and sigma: 2 Np floats each), which
 * are copied to device memory. Every value must be finite, sigma positive, theta and conf_min in [0, 1].
 * *model is NULL on error. Errors: SCD_ERR_NULL, SCD_ERR_SIZE (Np), SCD_ERR_MODEL (values), SCD_ERR_NOMEM,
 * SCD_ERR_HIP. */
int scd_model_create(int Np, const float* params, const float* mu, const float* sigma, float theta, float conf_min,
                     scd_model** model);

/* Free a model (NULL is a no-op). A model must not be freed while work that reads it is queued. */
int scd_model_destroy(scd_model* model);

/* The scd_selector view of a model (device pointers owned by the model, valid until scd_model_destroy). */
int scd_model_selector(const scd_model* model, scd_selector* selector);

/* Copy a model's arrays to HOST memory (any pointer may be NULL to skip that array); waits for the device. */
int scd_model_read(const scd_model* model, float* params, float* mu, float* sigma);

/* Write a model file from HOST arrays, without a device (the checks of scd_model_create apply). Errors:
 * SCD_ERR_NULL, SCD_ERR_SIZE, SCD_ERR_MODEL (values, or the file cannot be written). */
int scd_model_write(const char* path, int Np, const float* params, const float* mu, const float* sigma, float theta,
                    float conf_min);

/* Write a model to a file (scd_model_read, then scd_model_write). */
int scd_model_save(const scd_model* model, const char* path);

/* Read and check a model file (magic, version, Np, size, hash and values, all before any device call), then
 * create the model on the current device. Errors: SCD_ERR_NULL, SCD_ERR_MODEL (missing, malformed or corrupt
 * file), and those of scd_model_create. */
int scd_model_load(const char* path, scd_model** model);

/* Number of packed MLP parameters for Np channels (262912 for Np = 256), or SCD_ERR_SIZE. */
int scd_mlp_param_count(int Np);

/* Features of each signal: x device [batch] signals of N (power of two in [2^14, 2^20]) at opts->x_stride,
 * feat device [batch][2 Np]. Uses library-owned scratch for the segment periodograms (16 * Np * 4 KiB per
 * signal, at most 8 signals at a time). */
int scd_features(const float* x, int64_t N, int Np, const float* win, float* feat, const scd_opts* opts);

/* Labels of each strip of densely packed SCDs S (device [batch][Np][N] complex, as written by scd_ssca):
 * labels device [batch][Np] (0 or 1), ratio device [batch][Np] (max / mean, may be NULL). */
int scd_strip_labels(const float* S, int64_t N, int Np, float* labels, float* ratio, const scd_opts* opts);

/* out[i][j] = (f[i][j] - mu[j]) / sigma[j] for n rows of dim (device arrays). stream: hipStream_t or NULL. */
int scd_standardize(const float* f, const float* mu, const float* sigma, float* out, int n, int dim, void* stream);

/* MLP forward pass on `batch` standardised feature rows x (device [batch][2 Np]). act (device,
 * [4][batch][256]) receives the pre- and post-activation of both hidden layers (a1, h1, a2, h2), z (device
 * [batch][Np]) the logits and scores (device [batch][Np]) the sigmoid outputs. */
int scd_mlp_forward(int Np, int batch, const float* params, const float* x, float* act, float* z, float* scores,
                    void* stream);

/* Gradients of the mean binary cross-entropy between scores and labels (device [batch][Np]) with respect to the
 * packed parameters (grads, device, packed like params) and, if dx is not NULL, to x (device [batch][2 Np]).
 * act and scores come from scd_mlp_forward on the same x; scratch is device memory of
 * batch * (Np + 512) floats. */
int scd_mlp_backward(int Np, int batch, const float* params, const float* x, const float* act, const float* scores,
                     const float* labels, float* grads, float* scratch, float* dx, void* stream);

/* One Adam step (step number t >= 1) on n parameters in place; m and v are the moment estimates. */
int scd_adam_step(int n, float* params, const float* grads, float* m, float* v, int t, float lr, float beta1,
                  float beta2, float eps, void* stream);

/* mask[b][k] = scores[b][k] >= theta; conf[b] = min_k max(s, 1 - s) (device arrays). */
int scd_select(const float* scores, int Np, int batch, float theta, unsigned char* mask, float* conf, void* stream);

/* SSCA of one signal restricted to the strips the selector picks (a library form; the paper has no selector).
 * Everything runs on the GPU, in stream order: the features, one kernel that standardises them, runs the MLP,
 * thresholds the scores at selector->theta, falls back to every strip when min_k max(s_k, 1 - s_k) is below
 * selector->conf_min, and writes the selection to device memory; then Stage 1 and Stage 2 over the selected
 * strips only (their grids cover every strip and skip the unselected ones, so the host never waits for the
 * selection). Only the selected strips of out ([Np][N]) are written; the other rows are left untouched.
 * mask: device Np bytes (written: 1 = computed). fell_back: host int, or NULL; when given, the call copies the
 * fallback flag back and synchronises its stream once, at the end. selector->params must be 16-byte aligned.
 * opts: precision (SCD_FP32 or SCD_SPLIT_BF16), stream, workspace as scd_ssca_ex (batch must be 1). N must be
 * a power of two in [2^14, 2^20]. Errors as scd_ssca_ex, plus SCD_ERR_MODEL. */
int scd_ssca_learned(const float* x, int64_t N, int Np, const float* win, const scd_selector* selector, float* out,
                     unsigned char* mask, int* fell_back, const scd_opts* opts);

/* The selector half of scd_ssca_learned on one signal, without the SSCA: the features, then the same fused
 * kernel chain (standardise, MLP, threshold at selector->theta, fallback to every strip below
 * selector->conf_min). scores: device Np floats (the sigmoid outputs); mask: device Np bytes (1 = the strip
 * scd_ssca_learned would compute); conf: device float, min_k max(s_k, 1 - s_k) (may be NULL); fell_back: device
 * int, 1 when the fallback applies (may be NULL). Asynchronous on the stream of opts. Arguments, sizes and
 * errors as scd_ssca_learned. */
int scd_selector_run(const float* x, int64_t N, int Np, const float* win, const scd_selector* selector, float* scores,
                     unsigned char* mask, float* conf, int* fell_back, const scd_opts* opts);

/* One signal of scd_ssca_batch. */
typedef struct scd_ssca_item {
  const float* x;               /* device, N complex values                                                */
  int64_t N;                    /* as scd_ssca; a power of two in [2^14, 2^20] when a selector is given     */
  int Np;                       /* as scd_ssca                                                             */
  const float* win;             /* device, Np floats                                                       */
  float* out;                   /* device, Np*N complex values, [Np][N]                                    */
  const scd_selector* selector; /* NULL: every strip; otherwise only the strips this selector picks       */
  unsigned char* mask;          /* with a selector: device Np bytes, written as by scd_ssca_learned; else
                                   unused                                                                  */
} scd_ssca_item;

/* SSCA of n signals of any lengths and channel counts (a library form for mixed workloads; the paper estimates
 * one signal at a time). An item without a selector runs as scd_ssca_ex; an item with one runs as
 * scd_ssca_learned with fell_back NULL, so the call never waits for the GPU. Each item's outputs equal those of
 * its single call.
 *   - Items run on four library-owned lanes (streams of default priority; item i on lane i mod 4), each with
 *     its own scratch, so short items, whose grids cannot fill the GPU, and selectors overlap other items.
 *     The lanes start after the work already on opts' stream, and that stream waits for all of them, so the
 *     results are ordered on it as for single calls. With a caller workspace (one buffer) or a single item,
 *     the items run in order on opts' stream instead.
 *   - Every item uses opts' precision and workspace. opts->batch must be 0 or 1 and both strides 0: each item
 *     is one signal. A caller workspace must hold the largest item's intermediate; the library's scratch grows
 *     per lane to the largest item that lane runs, waiting for that lane once when it grows.
 *   - Argument errors that the host can see in any item (sizes, NULL pointers, precision, selector fields)
 *     are returned before anything is enqueued. A later failure (say a pointer that is not device memory)
 *     stops the call at that item, and the items before it stay enqueued. Either way the error code is the
 *     item's, with its index in scd_last_error.
 *   - Batch calls in one process run one at a time on the host.
 * Errors: SCD_ERR_NULL (items NULL with n > 0), SCD_ERR_SIZE (n < 0 or opts->batch > 1), SCD_ERR_UNSUPPORTED
 * (nonzero strides), and those of scd_ssca_ex and scd_ssca_learned. */
int scd_ssca_batch(const scd_ssca_item* items, int n, const scd_opts* opts);

/*
 * scd_ssca_noalloc - scd_ssca_ex (FP32, one signal) for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc. It calls no hipMalloc, hipFree or
 * other allocating routine. Its scratch (the FP64-generated tables, regenerated by every call, then the
 * intermediate) is a file-scope device array that each GPU the library runs on holds until the process ends;
 * scd_ssca_noalloc_limit() gives the intermediate's capacity (64 MiB), so 8 * Np * N must not exceed it
 * (N == 1024 needs no intermediate). Every call on one GPU uses that GPU's one array: calls that overlap on one
 * GPU (different streams, or threads without ordering) race and corrupt each other's results.
 *   x, N, Np, win, out  as scd_ssca
 *   opts                stream only: precision must be SCD_FP32, batch 0 or 1, no workspace (or opts NULL)
 * Errors: SCD_ERR_NULL, SCD_ERR_SIZE (including 8 * Np * N above the limit), SCD_ERR_ALIAS, SCD_ERR_PTR,
 * SCD_ERR_UNSUPPORTED (other precision, batch or a workspace), SCD_ERR_HIP. The result equals scd_ssca_ex's. */
int scd_ssca_noalloc(const float* x, int64_t N, int Np, const float* win, float* out, const scd_opts* opts);

/* The intermediate capacity of scd_ssca_noalloc's scratch, in bytes. */
size_t scd_ssca_noalloc_limit(void);

/* Bytes of workspace scd_ssca_ex needs for `batch` signals (0 when N == 1024). Errors: SCD_ERR_NULL,
 * SCD_ERR_SIZE. */
int scd_ssca_workspace_size(int64_t N, int Np, int batch, size_t* bytes);

/* Bytes of workspace scd_fam_ex needs for `batch` signals. Errors: SCD_ERR_NULL, SCD_ERR_SIZE. */
int scd_fam_workspace_size(int Np, int L, int P, int batch, size_t* bytes);

/* Set the default stream (a hipStream_t, NULL = null stream) used when scd_opts.stream is NULL. */
int scd_set_stream(void* stream);

/* The message of the calling thread's last failed call ("" if none). Valid until its next call. */
const char* scd_last_error(void);

/* ABI version: (major << 16) | minor. */
int scd_version(void);

/* Wait for the library's work, then free its tables and workspaces on every device. Safe to call twice. */
void scd_shutdown(void);

#ifdef __cplusplus
}
#endif

#endif /* SCD_H */
