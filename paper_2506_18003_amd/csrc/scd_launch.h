// Internal (not exported) launchers shared between the kernel files and the C ABI layer.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace scd {

// Offsets (in float2) of the per-plan FP64-generated tables inside one device allocation.
constexpr int kTabTw1024 = 0;     // omega_1024^j, j < 1024
constexpr int kTabRotLo = 1024;   // omega_N^j,    j < 1024 (SSCA rotation factors, low part)
constexpr int kTabRoots = 2048;   // omega_Np^e,   e < Np   (down-conversion factors)
constexpr int kTabSize = 2048 + 256;

// Channelizer precisions (values of scd_precision in scd.h).
constexpr int SCD_PREC_FP32 = 0;
constexpr int SCD_PREC_SPLIT_BF16 = 1;
constexpr int SCD_PREC_SPLIT_FP16 = 2;
constexpr int SCD_PREC_BF16 = 3;
constexpr int SCD_PREC_FP16 = 4;
constexpr int kMfmaPad = 256;  // zero samples on each side of the 16-bit copies of x

// Which strips an SSCA launch computes, built on the GPU and read by the kernels from device memory. Stage 1
// runs the channel subsets sub[0..nsub) (subset c holds the strips k = c (mod Np/16)), or, in its paired
// form, the subset pairs pair[0..npair) (pair p holds subsets p and p + Np/32), and stores strip k only if
// bit k of keep is set; stage 2 runs strips ch[0..nch). Grids are sized for every subset and strip, and the
// workgroups past the counts exit.
struct ChanSel {
  unsigned keep[8];
  unsigned char sub[16];
  unsigned char pair[8];
  unsigned char ch[256];
  int nsub, npair, nch;
};
// A selection as the launchers take it: the grid sizes (host; the most units the selection can hold) and the
// ChanSel in device memory; dev == nullptr means every strip (sub[i] = i, pair[i] = i, ch[k] = k, all kept).
struct SelArg {
  const ChanSel* dev;
  int nsub, npair, nch;
};
inline SelArg selarg_all(int Np) { return SelArg{nullptr, Np / 16, Np / 32, Np}; }

hipError_t launch_gen_roots(float2* dst, int count, int M, hipStream_t stream);

// Set the calling thread's scd_last_error message and return `code` (SCD_ERR_HIP for set_hip_error).
int set_error(int code, const char* msg);
int set_hip_error(hipError_t e, const char* what);

// SSCA Stage 1 (channelizer + CDP + M1-point DFT + rotation) of `batch` signals. x: [batch][N] at stride xbs;
// win: device float[Np]; T: [batch] blocked intermediates [Np][M1/16][M2][16] at stride tbs (float2 elements).
// With N == 1024 the intermediate layout equals the output layout [Np][N]. ymode 1 (cross) or 2 (conjugate)
// takes the channel-data product with conj(y[n]) or y[n] instead of conj(x[n]); y is laid out like x, and a
// cross form runs without a selection (sel.dev == nullptr). xlen/xoff estimate the block [xoff, xoff + N) of a
// signal of xlen samples at x (xoff a multiple of Np; 0 and 0 = the whole signal, xlen = N).
hipError_t launch_ssca_pass1_fp32(const float2* x, int N, int Np, const float* win, const float2* tabs, float2* T,
                                  int batch, int64_t xbs, int64_t tbs, const SelArg& sel, hipStream_t stream,
                                  const float2* y = nullptr, int ymode = 0, int xlen = 0, int xoff = 0);

// SSCA Stage 1 with the channelizer on MFMA in 16-bit (split or plain) precision, Np <= 128. scratch: device
// memory of ssca_mfma_scratch_bytes(N, Np, batch) bytes for the 16-bit copies of x and the DFT weights,
// filled by this call. Other arguments as launch_ssca_pass1_fp32.
size_t ssca_mfma_scratch_bytes(int N, int Np, int batch);
hipError_t launch_ssca_pass1_mfma(int prec, const float2* x, int N, int Np, const float* win, const float2* tabs,
                                  void* scratch, float2* T, int batch, int64_t xbs, int64_t tbs, const SelArg& sel,
                                  hipStream_t stream);

// SSCA Stage 2 (M2-point DFT over m2) of `batch` intermediates into out: [batch][Np][N] at stride obs. A no-op
// when N == 1024.
hipError_t launch_ssca_pass2(const float2* T, int N, int Np, const float2* tabs, float2* out, int batch,
                             int64_t tbs, int64_t obs, const SelArg& sel, hipStream_t stream);

// FAM of `batch` signals. x: [batch][P*L] at stride xbs; xt: [batch][Np][P] scratch; out: complex
// [batch][Np][Np][P], or with `power` float [batch][Np][Np][P/2] (|S|^2 of the bins -P/4 <= q_c < P/4); obs in elements.
// With y (laid out like x) the cross form: xt must then hold 2 * batch * Np * P values (X_T, then Y_T), and conj
// takes Y_T itself instead of its conjugate.
hipError_t launch_fam_fp32(const float2* x, int Np, int L, int P, const float* win, const float2* tabs,
                           float2* xt, void* out, bool power, int batch, int64_t xbs, int64_t obs,
                           hipStream_t stream, const float2* y = nullptr, bool conj = false);

// ---- learned strip selector (learn.hip) ----
constexpr int kHidden = 256;
struct MlpLayout {  // offsets (floats) of the packed parameters [W1 b1 W2 b2 W3 b3]
  int in, out, W1, b1, W2, b2, W3, b3, total;
};
__host__ __device__ inline MlpLayout mlp_layout(int Np) {
  MlpLayout L;
  L.in = 2 * Np;
  L.out = Np;
  L.W1 = 0;
  L.b1 = L.W1 + kHidden * L.in;
  L.W2 = L.b1 + kHidden;
  L.b2 = L.W2 + kHidden * kHidden;
  L.W3 = L.b2 + kHidden;
  L.b3 = L.W3 + Np * kHidden;
  L.total = L.b3 + Np;
  return L;
}
// Selector features of nsig signals of N samples, xs complex apart: the segment periodograms go to P
// ([nsig][16][Np][1024] floats of device scratch), then feat [nsig][2 Np] (PSD, centred over k if `centre`;
// ACP). tabs: the tables of N = 1024 and this Np.
hipError_t launch_features(const float2* x, int64_t xs, int64_t N, int Np, int nsig, const float* win,
                           const float2* tabs, float* P, float* feat, hipStream_t stream, bool centre = true);
// S: [nsig][Np][N] -> labels [nsig][Np] (0/1), ratio [nsig][Np] (may be null).
hipError_t launch_labels(const float2* S, int64_t N, int Np, int nsig, float* labels, float* ratio,
                         hipStream_t stream);
hipError_t launch_standardize(const float* f, const float* mu, const float* sigma, float* out, int n, int dim,
                              hipStream_t stream);
hipError_t launch_mlp_forward(int Np, int B, const float* params, const float* x, float* act, float* z, float* sc,
                              hipStream_t stream);
hipError_t launch_mlp_backward(int Np, int B, const float* params, const float* x, const float* act, const float* sc,
                               const float* y, float* grads, float* scratch, float* dx, hipStream_t stream);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int n, int t, float lr, float b1, float b2,
                       float eps, hipStream_t stream);
hipError_t launch_select(const float* sc, int Np, int nsig, float theta, unsigned char* mask, float* conf,
                         hipStream_t stream);
// Selector inference of one signal: centre the PSD part of the raw feat [2 Np] and standardise, MLP (activations in h: 2 * 256 + Np floats of
// device scratch), strip mask (device Np bytes), confidence, fallback to every strip when the confidence is
// below conf_min (fell = 1), and the ChanSel the SSCA kernels read.
hipError_t launch_select_infer(const float* feat, const float* mu, const float* sigma, const float* params, int Np,
                               float theta, float conf_min, float* h, unsigned char* mask, float* conf, int* fell,
                               ChanSel* sel, hipStream_t stream);

}  // namespace scd
