// Kernels of the learned strip selector: features, labels, the MLP (bf16 MFMA GEMMs with FP32 accumulation)
// with its backward pass and Adam, and the strip selection.
//
// Features of a signal (2 Np floats): from the SSCA S_b of B_F = 16 segments of N_C = 1024 samples (each zero
// outside itself; Eq. (6)-(7) with N = N_C, so M1 = 1024 and M2 = 1),
//   A_k[q]  = sum_b |S_b[k][q]|^2 (averaged cyclic periodogram of strip k),
//   PSD_k   = 0.5 log(A_k[q0(k)] + 1e-30) centred over k, q0(k) = (-k_c N_C / Np) mod N_C (alpha = 0 bin),
//   ACP_k   = log(max / mean of A_k over the bins farther than 4 (circularly) from q0(k)).
// Labels from a full SSCA S [Np][N]: strip k is active if max |S|^2 exceeds T = 6.2^2/2 times the mean |S|^2
// over the bins whose cycle frequency is at least 1/256 away from 0 modulo 1.
// MLP: 2 Np -> 256 -> 256 -> Np, ReLU, ReLU, sigmoid; parameters packed as [W1 b1 W2 b2 W3 b3] (FP32 master,
// row-major W[out][in]); every GEMM rounds both operands to bf16 and accumulates in FP32 on
// v_mfma_f32_32x32x16_bf16.
#include <hip/hip_runtime.h>

#include "scd_device.h"
#include "scd_launch.h"

namespace scd {

namespace {

constexpr int kNC = 1024;
constexpr int kBF = 16;
constexpr float kLabelT = 6.2f * 6.2f / 2.0f;

__device__ __forceinline__ int signed_idx(int i, int n) { return ((i + n / 2) & (n - 1)) - n / 2; }

// Block-wide reductions of one float per thread (256 threads).
__device__ float block_sum(float v, float* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  const float r = red[0];
  __syncthreads();
  return r;
}
__device__ float block_max(float v, float* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) red[tid] = fmaxf(red[tid], red[tid + s]);
    __syncthreads();
  }
  const float r = red[0];
  __syncthreads();
  return r;
}

constexpr int kSegThreads = 512;
constexpr int kSegStride = kNC + kNC / 16;  // one float2 of padding per 16 elements

// Periodograms P_b[k][q] = |S_b[k][q]|^2 of the B_F feature segments. One workgroup per (channel parity h,
// subset c, segment b, signal): the 8 channels k = c + S (2 kk + h), kk < 8, S = Np / 16. Thread t owns the
// adjacent frames m1 = 2t and 2t + 1 (frame n = m1 centred, samples outside the segment zero). Per frame:
//   - the complex-windowed fold of the frame to 16 residues, A[j0] = sum_j1 hc[j0 + 16 j1] x[n - d + j0 + 16 j1],
//     hc[j] = w[j] omega_Np^{(c j) mod Np}. The two frames' windows overlap, so each pair of samples read
//     from LDS (and each pair of hc values) serves both frames' folds;
//   - the parity-h half of its 16-point DFT: one decimation-in-frequency step,
//     e[j0] = (A[j0] + (-1)^h A[j0 + 8]) omega_16^{h j0}, then an 8-point DFT (output kk is channel index 2 kk + h);
//   - the down-conversion factor omega_Np^{(k n) mod Np} and conj(x[n]) (Eq. (6); M2 = 1, so n = m1).
// Then the 1024-point DFT over m1 of the 8 channels in LDS, whose last stage writes |S_b[k][q]|^2.
// P is [sig][B_F][Np][N_C]; the signals are xs complex apart and segment b starts at b N / B_F.
template <int NP>
__global__ __launch_bounds__(kSegThreads) void seg_periodogram_kernel(const float2* __restrict__ x, int64_t xs,
                                                                     int64_t N, const float* __restrict__ win,
                                                                     const float2* __restrict__ tabs,
                                                                     float* __restrict__ P) {
  constexpr int S = NP / 16;
  constexpr int D = NP / 2 - 1;
  constexpr int XL = kNC + NP - 1;  // samples the frames touch: n - D + j for n < N_C, j < NP
  __shared__ float2 buf[8 * kSegStride];
  __shared__ float2 tw[kNC];  // omega_1024^e
  __shared__ __align__(16) float2 xl[XL + 1];  // xl[i] = segment sample i - D (zero outside the segment)
  __shared__ __align__(16) float2 hc[NP];
  __shared__ float2 rt[NP];   // omega_Np^e
  const int h = blockIdx.x & 1, c = blockIdx.x >> 1, b = blockIdx.y, sig = blockIdx.z;
  const int tid = threadIdx.x;
  const float2* seg = x + sig * xs + static_cast<int64_t>(b) * (N / kBF);
  {
    // Samples outside the segment read as zero through a range-checked buffer load; every load of a thread is
    // issued before its first LDS write.
    constexpr int PER = (XL + 1 + kSegThreads - 1) / kSegThreads;
    const auto sr = make_rsrc(seg, kNC * 8);
    float2 v[PER];
#pragma unroll
    for (int r = 0; r < PER; ++r) v[r] = load_c64(sr, tid + r * kSegThreads - D);
#pragma unroll
    for (int r = 0; r < PER; ++r)
      if (tid + r * kSegThreads < XL + 1) xl[tid + r * kSegThreads] = v[r];
  }
  lds_copy<kNC, kSegThreads>(tw, tabs + kTabTw1024, tid);
  for (int j = tid; j < NP; j += kSegThreads) {
    rt[j] = tabs[kTabRoots + j];
    hc[j] = cscale(tabs[kTabRoots + ((c * j) & (NP - 1))], win[j]);
  }
  __syncthreads();
  // Fold of frames 2t (a0) and 2t + 1 (a1). xw[j] is tap j of frame 2t and tap j - 1 of frame 2t + 1; each
  // residue sums its taps in increasing order.
  float2 a0[16], a1[16];
#pragma unroll
  for (int j0 = 0; j0 < 16; ++j0) {
    a0[j0] = make_float2(0.f, 0.f);
    a1[j0] = make_float2(0.f, 0.f);
  }
  const float2* xw = xl + 2 * tid;
  float2 hprev = make_float2(0.f, 0.f);  // hc[j - 1]
#pragma unroll 1
  for (int j1 = 0; j1 < NP / 16; ++j1) {
#pragma unroll
    for (int j0 = 0; j0 < 16; j0 += 2) {
      const int j = 16 * j1 + j0;
      const float4 xv = *reinterpret_cast<const float4*>(xw + j);  // 16-byte aligned: 2 tid + j is even
      const float4 hv = *reinterpret_cast<const float4*>(hc + j);
      const float2 x0 = make_float2(xv.x, xv.y), x1 = make_float2(xv.z, xv.w);
      const float2 h0 = make_float2(hv.x, hv.y), h1 = make_float2(hv.z, hv.w);
      a0[j0] = cfma(a0[j0], h0, x0);
      a0[j0 + 1] = cfma(a0[j0 + 1], h1, x1);
      if (j > 0) a1[(j0 + 15) & 15] = cfma(a1[(j0 + 15) & 15], hprev, x0);
      a1[j0] = cfma(a1[j0], h0, x1);
      hprev = h1;
    }
  }
  a1[15] = cfma(a1[15], hprev, xw[NP]);  // tap Np - 1 of frame 2t + 1
#pragma unroll
  for (int f = 0; f < 2; ++f) {
    const int m1 = 2 * tid + f;
    float2* a = f ? a1 : a0;
    float2 e[8];
    if (h == 0) {
#pragma unroll
      for (int j0 = 0; j0 < 8; ++j0) e[j0] = cadd(a[j0], a[j0 + 8]);
    } else {
#pragma unroll
      for (int j0 = 0; j0 < 8; ++j0) e[j0] = cmul(csub(a[j0], a[j0 + 8]), tw[64 * j0]);
    }
    dft8(e);
    const float2 xn = xl[m1 + D];
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      const int k = c + S * (2 * kk + h);
      buf[kk * kSegStride + m1 + (m1 >> 4)] = cmul(e[kk], cmulc(rt[(k * m1) & (NP - 1)], xn));
    }
  }
  __syncthreads();
  float* Pb = P + (static_cast<int64_t>(sig) * kBF + b) * NP * kNC;
  auto st = [&](int bq, int q, float2 v) {
    const int k = c + S * (2 * bq + h);
    Pb[k * kNC + q] = fmaf(v.x, v.x, v.y * v.y);
  };
  NoLoad ld;
  lds_fft<kNC, 8, kSegThreads, false, LdsLayout<kSegStride, 1, 4>, kNC>(buf, tw, tid, ld, st);
}

// One workgroup per (strip k, signal): A_k[q] = sum_b P_b[k][q] in segment order; feat [sig][2 Np] gets the
// raw (uncentred) PSD_k and ACP_k. Every load of a thread is issued before the sums; the four reductions
// share one pass across the wave and one through LDS.
__global__ __launch_bounds__(256) void acp_features_kernel(const float* __restrict__ P, int Np,
                                                           float* __restrict__ feat) {
  constexpr int QT = kNC / 256;  // bins per thread: q = QT tid + r
  static_assert(QT == 4, "one float4 of bins per thread and segment");
  __shared__ float red[4][4];
  const int k = blockIdx.x, sig = blockIdx.y, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const float* base = P + (static_cast<int64_t>(sig) * kBF * Np + k) * kNC + QT * tid;
  const int q0 = (-signed_idx(k, Np) * (kNC / Np)) & (kNC - 1);
  float4 pv[kBF];
#pragma unroll
  for (int b = 0; b < kBF; ++b) pv[b] = *reinterpret_cast<const float4*>(base + static_cast<int64_t>(b) * Np * kNC);
  float a[QT] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int b = 0; b < kBF; ++b) {
    a[0] += pv[b].x;
    a[1] += pv[b].y;
    a[2] += pv[b].z;
    a[3] += pv[b].w;
  }
  float sum = 0.f, mx = 0.f, a0 = 0.f, cnt = 0.f;
#pragma unroll
  for (int r = 0; r < QT; ++r) {
    const int q = QT * tid + r;
    if (q == q0) a0 = a[r];
    if (abs(signed_idx((q - q0) & (kNC - 1), kNC)) > 4) {
      sum += a[r];
      mx = fmaxf(mx, a[r]);
      cnt += 1.f;
    }
  }
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) {
    sum += __shfl_xor(sum, m, 64);
    cnt += __shfl_xor(cnt, m, 64);
    a0 += __shfl_xor(a0, m, 64);
    mx = fmaxf(mx, __shfl_xor(mx, m, 64));
  }
  if (lane == 0) {
    red[w][0] = sum;
    red[w][1] = cnt;
    red[w][2] = a0;
    red[w][3] = mx;
  }
  __syncthreads();
  if (tid == 0) {
    const float tot = (red[0][0] + red[1][0]) + (red[2][0] + red[3][0]);
    const float n = (red[0][1] + red[1][1]) + (red[2][1] + red[3][1]);
    const float a0s = (red[0][2] + red[1][2]) + (red[2][2] + red[3][2]);
    const float m = fmaxf(fmaxf(red[0][3], red[1][3]), fmaxf(red[2][3], red[3][3]));
    feat[sig * 2 * Np + k] = 0.5f * logf(a0s + 1e-30f);
    feat[sig * 2 * Np + Np + k] = logf(m / (tot / n));
  }
}

// Centre the PSD half of each signal's features (one workgroup per signal).
__global__ __launch_bounds__(256) void centre_psd_kernel(float* __restrict__ feat, int Np) {
  __shared__ float red[256];
  const int sig = blockIdx.x, tid = threadIdx.x;
  float s = 0.f;
  for (int k = tid; k < Np; k += 256) s += feat[sig * 2 * Np + k];
  const float mean = block_sum(s, red) / static_cast<float>(Np);
  for (int k = tid; k < Np; k += 256) feat[sig * 2 * Np + k] -= mean;
}

// One workgroup per (strip k, signal): S [sig][Np][N].
__global__ __launch_bounds__(256) void labels_kernel(const float2* __restrict__ S, int64_t N, int Np,
                                                     float* __restrict__ labels, float* __restrict__ ratio) {
  __shared__ float red[256];
  const int k = blockIdx.x, sig = blockIdx.y, tid = threadIdx.x;
  const float2* row = S + (static_cast<int64_t>(sig) * Np + k) * N;
  const int n = static_cast<int>(N);
  const int shift = signed_idx(k, Np) * (n / Np);
  const int guard = n / 256;
  float sum = 0.f, mx = 0.f;
  for (int q = tid; q < n; q += 256) {
    const int d = abs(signed_idx((q + shift) & (n - 1), n));
    if (d >= guard) {
      const float2 v = row[q];
      const float p = fmaf(v.x, v.x, v.y * v.y);
      sum += p;
      mx = fmaxf(mx, p);
    }
  }
  const float tot = block_sum(sum, red);
  const float m = block_max(mx, red);
  if (tid == 0) {
    const float r = m / (tot / static_cast<float>(n - (2 * guard - 1)));
    if (ratio) ratio[sig * Np + k] = r;
    labels[sig * Np + k] = (r > kLabelT) ? 1.f : 0.f;
  }
}

// out[b][i] = (f[b][i] - mu[i]) / sigma[i]
__global__ void standardize_kernel(const float* __restrict__ f, const float* __restrict__ mu,
                                   const float* __restrict__ sigma, float* __restrict__ out, int n, int dim) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n * dim) out[e] = (f[e] - mu[e % dim]) / sigma[e % dim];
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

enum { kEpiStore = 0, kEpiBiasRelu = 1, kEpiBiasSigmoid = 2 };

// C[M][N] = sum_k A(m,k) B(k,n) with A(m,k) = TA ? A[k*lda + m] : A[m*lda + k] and
// B(k,n) = TB ? B[n*ldb + k] : B[k*ldb + n]; both operands rounded to bf16, FP32 accumulation. One wave per
// 32 x 32 tile of C. Epilogues: store; C = acc + bias[n] and C2 = relu(C); C = acc + bias[n] and
// C2 = sigmoid(C). Out-of-range operand elements read as zero and out-of-range outputs are not written.
template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(64) void gemm_bf16_kernel(const float* __restrict__ A, int lda, const float* __restrict__ B,
                                                       int ldb, float* __restrict__ C, float* __restrict__ C2,
                                                       const float* __restrict__ bias, int M, int N, int K) {
  const int l = threadIdx.x, g = l >> 5, lc = l & 31;
  const int m0 = blockIdx.y * 32, n0 = blockIdx.x * 32;
  f32x16 acc = {};
  for (int k0 = 0; k0 < K; k0 += 16) {
    bf16x8 a, b;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const int k = k0 + 8 * g + v;
      const int m = m0 + lc, n = n0 + lc;
      float av = 0.f, bv = 0.f;
      if (m < M && k < K) av = TA ? A[static_cast<int64_t>(k) * lda + m] : A[static_cast<int64_t>(m) * lda + k];
      if (n < N && k < K) bv = TB ? B[static_cast<int64_t>(n) * ldb + k] : B[static_cast<int64_t>(k) * ldb + n];
      a[v] = static_cast<__bf16>(av);
      b[v] = static_cast<__bf16>(bv);
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int m = m0 + 8 * (r / 4) + 4 * g + (r % 4), n = n0 + lc;
    if (m < M && n < N) {
      float v = acc[r];
      const int64_t o = static_cast<int64_t>(m) * N + n;
      if constexpr (EPI == kEpiStore) {
        C[o] = v;
      } else {
        v += bias[n];
        C[o] = v;
        C2[o] = (EPI == kEpiBiasRelu) ? fmaxf(v, 0.f) : 1.f / (1.f + expf(-v));
      }
    }
  }
}

// dz = (s - y) / count
__global__ void bce_grad_kernel(const float* __restrict__ s, const float* __restrict__ y, float* __restrict__ dz,
                                int n, float inv_count) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) dz[e] = (s[e] - y[e]) * inv_count;
}

// d *= (a > 0)
__global__ void relu_mask_kernel(float* __restrict__ d, const float* __restrict__ a, int n) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n && !(a[e] > 0.f)) d[e] = 0.f;
}

// db[j] = sum_i d[i][j]
__global__ void colsum_kernel(const float* __restrict__ d, float* __restrict__ db, int rows, int cols) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < cols) {
    float s = 0.f;
    for (int i = 0; i < rows; ++i) s += d[static_cast<int64_t>(i) * cols + j];
    db[j] = s;
  }
}

__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int n, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) {
    const float ge = g[e];
    const float me = b1 * m[e] + (1.f - b1) * ge;
    const float ve = b2 * v[e] + (1.f - b2) * ge * ge;
    m[e] = me;
    v[e] = ve;
    p[e] -= lr * (me / c1) / (sqrtf(ve / c2) + eps);
  }
}

// mask[k] = s[k] >= theta; conf[sig] = min_k max(s[k], 1 - s[k]); one workgroup per signal.
__global__ __launch_bounds__(256) void select_kernel(const float* __restrict__ s, int Np, float theta,
                                                     unsigned char* __restrict__ mask, float* __restrict__ conf) {
  __shared__ float red[256];
  const int sig = blockIdx.x, tid = threadIdx.x;
  float c = 1.f;
  for (int k = tid; k < Np; k += 256) {
    const float v = s[sig * Np + k];
    mask[sig * Np + k] = (v >= theta) ? 1 : 0;
    c = fminf(c, fmaxf(v, 1.f - v));
  }
  red[tid] = c;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) red[tid] = fminf(red[tid], red[tid + st]);
    __syncthreads();
  }
  if (tid == 0) conf[sig] = red[0];
}

__device__ __forceinline__ float bf16r(float v) { return static_cast<float>(static_cast<__bf16>(v)); }

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// v from another lane by a DPP pattern; lanes of rows outside ROW_MASK get 0.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp_f(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROW_MASK, 0xf, false));
}
// Sum over the wave, held by lane 63: pairs and quads (quad permutations), 8 and 16 lanes (half-row and row
// mirrors), then rows 0 + 1 and 2 + 3 (row broadcast of lane 15), then all four (row broadcast of lane 31).
// DPP moves are plain VALU operations, with none of the LDS latency of a cross-lane shuffle.
__device__ __forceinline__ float wave_sum_lane63(float v) {
  v += dpp_f<0xb1>(v);        // quad_perm [1, 0, 3, 2]
  v += dpp_f<0x4e>(v);        // quad_perm [2, 3, 0, 1]
  v += dpp_f<0x141>(v);       // row_half_mirror
  v += dpp_f<0x140>(v);       // row_mirror
  v += dpp_f<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_f<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  return v;
}

// Selector inference of one signal in two launches of 1024-thread workgroups (16 waves):
//   - infer_l12_kernel, kInferBlocks workgroups. Each standardises the raw features (the PSD part centred over k
//     first, then each input rounded to bf16). Workgroup g then computes rows [64 g, 64 g + 64) of the first
//     layer, and the second layer's partial sums over those same 64 hidden inputs for all 256 of its rows. So
//     each workgroup's CU fetches a quarter of W1 and of W2, all of its loads issued at once. The cold weights
//     (the SSCA's traffic evicts them between calls) arrive over four CUs instead of one;
//   - infer_l3_select_kernel, one workgroup: the second layer's rows from the partials (summed in workgroup
//     order, then the bias), the third layer, and the selection: mask, confidence min_k max(s_k, 1 - s_k),
//     fallback to every strip below conf_min, and the channel selection the SSCA kernels read (strip list in
//     increasing k from wave ballots and per-wave counts, subset and pair lists from the kept strips).
// A dense row is out[o] = act(sum_i bf16(W[o][i]) in[i] + b[o]) with FP32 accumulation: each lane sums its
// inputs i = 64 c + lane in order of c, and a DPP reduction sums the lanes. The activations (h1, h2, the Np
// scores) are also written to act.
constexpr int kInferThreads = 1024;
constexpr int kInferWaves = kInferThreads / 64;
constexpr int kInferBlocks = 4;                     // workgroups of the first launch
constexpr int kInferRows1 = kHidden / kInferBlocks; // first-layer rows (and second-layer inputs) per workgroup
static_assert(kInferRows1 == 64 && kInferRows1 % kInferWaves == 0, "one wave-wide chunk of h1 per workgroup");

// One dense layer: wave w owns the NOUT / 16 consecutive rows from w NOUT / 16. Its weights are loaded in
// batches of RB rows (every load of a batch in flight at once, at most 64 registers), one batch when they fit.
// ACT: 0 = ReLU then bf16 rounding (the next layer's operand), 1 = sigmoid. `bias`, `in` and `out` are in LDS.
template <int NIN, int NOUT>
struct Dense {
  static constexpr int C = NIN >= 64 ? NIN / 64 : 1;  // weight loads per row and lane
  static constexpr int R = NOUT / kInferWaves;        // rows per wave
  static constexpr int RB = R * C <= 64 ? R : 64 / C; // rows per batch of loads
  static_assert(NOUT % kInferWaves == 0 && R % RB == 0, "rows must split evenly over the waves");
  __device__ __forceinline__ static void load(const float* __restrict__ W, int r0, int w, int lane, float (&wv)[RB][C]) {
    const bool live = NIN >= 64 || lane < NIN;
#pragma unroll
    for (int u = 0; u < RB; ++u)
#pragma unroll
      for (int cc = 0; cc < C; ++cc)
        wv[u][cc] = live ? W[static_cast<int64_t>(w * R + r0 + u) * NIN + 64 * cc + lane] : 0.f;
  }
  template <int ACT>
  __device__ __forceinline__ static void rows(const float (&wv)[RB][C], const float* bias, const float* in,
                                              float* out, int r0, int w, int lane) {
    const bool live = NIN >= 64 || lane < NIN;
    float xv[C];
#pragma unroll
    for (int cc = 0; cc < C; ++cc) xv[cc] = live ? in[64 * cc + lane] : 0.f;
#pragma unroll
    for (int u = 0; u < RB; ++u) {
      float acc = 0.f;
#pragma unroll
      for (int cc = 0; cc < C; ++cc) acc = fmaf(bf16r(wv[u][cc]), xv[cc], acc);
      acc = wave_sum_lane63(acc);
      const int o = w * R + r0 + u;
      if (lane == 63) {
        acc += bias[o];
        out[o] = (ACT == 0) ? bf16r(fmaxf(acc, 0.f)) : 1.f / (1.f + expf(-acc));
      }
    }
  }
  // The whole layer; `first` holds the weights of the first batch if they were loaded ahead.
  template <int ACT>
  __device__ __forceinline__ static void run(const float* __restrict__ W, const float* bias, const float* in,
                                             float* out, int w, int lane, float (&first)[RB][C]) {
    rows<ACT>(first, bias, in, out, 0, w, lane);
    for (int r0 = RB; r0 < R; r0 += RB) {
      float wv[RB][C];
      load(W, r0, w, lane, wv);
      rows<ACT>(wv, bias, in, out, r0, w, lane);
    }
  }
};

template <int NP>
__global__ __launch_bounds__(kInferThreads) void infer_l12_kernel(const float* __restrict__ feat,
                                                                  const float* __restrict__ mu,
                                                                  const float* __restrict__ sigma,
                                                                  const float* __restrict__ params,
                                                                  float* __restrict__ act, float* __restrict__ part) {
  constexpr int NIN = 2 * NP;
  constexpr int C1 = NIN >= 64 ? NIN / 64 : 1;      // first-layer loads per row and lane
  constexpr int R1 = kInferRows1 / kInferWaves;    // first-layer rows per wave
  constexpr int R2 = kHidden / kInferWaves;        // second-layer rows per wave
  __shared__ float x0[NIN];
  __shared__ float h1[kInferRows1];
  __shared__ float red[1];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = blockIdx.x;
  const MlpLayout L = mlp_layout(NP);
  const bool live = NIN >= 64 || lane < NIN;
  // Every weight this workgroup needs, in flight while the features are standardised.
  float w1[R1][C1], w2[R2];
#pragma unroll
  for (int u = 0; u < R1; ++u)
#pragma unroll
    for (int cc = 0; cc < C1; ++cc)
      w1[u][cc] = live ? params[L.W1 + static_cast<int64_t>(kInferRows1 * g + R1 * w + u) * NIN + 64 * cc + lane] : 0.f;
#pragma unroll
  for (int u = 0; u < R2; ++u) w2[u] = params[L.W2 + static_cast<int64_t>(R2 * w + u) * kHidden + kInferRows1 * g + lane];
  if (w == 0) {
    float ps = 0.f;
    // Loads first, then the sums in the same order as a strided loop (which would wait for each load in turn).
    constexpr int PS = (NP + 63) / 64;
    float fv[PS];
#pragma unroll
    for (int r = 0; r < PS; ++r) fv[r] = (NP % 64 == 0 || lane + 64 * r < NP) ? feat[min(lane + 64 * r, NP - 1)] : 0.f;
#pragma unroll
    for (int r = 0; r < PS; ++r) ps += fv[r];
    ps = wave_sum(ps);
    if (lane == 0) red[0] = ps / static_cast<float>(NP);
  }
  __syncthreads();
  const float mean = red[0];
  for (int i = tid; i < NIN; i += kInferThreads) x0[i] = bf16r((feat[i] - (i < NP ? mean : 0.f) - mu[i]) / sigma[i]);
  __syncthreads();
  float xv[C1];
#pragma unroll
  for (int cc = 0; cc < C1; ++cc) xv[cc] = live ? x0[64 * cc + lane] : 0.f;
#pragma unroll
  for (int u = 0; u < R1; ++u) {
    float acc = 0.f;
#pragma unroll
    for (int cc = 0; cc < C1; ++cc) acc = fmaf(bf16r(w1[u][cc]), xv[cc], acc);
    acc = wave_sum_lane63(acc);
    const int r = R1 * w + u;
    if (lane == 63) {
      const float h = bf16r(fmaxf(acc + params[L.b1 + kInferRows1 * g + r], 0.f));
      h1[r] = h;
      act[kInferRows1 * g + r] = h;
    }
  }
  __syncthreads();
  const float hv = h1[lane];
#pragma unroll
  for (int u = 0; u < R2; ++u) {
    const float p = wave_sum_lane63(bf16r(w2[u]) * hv);
    if (lane == 63) part[g * kHidden + R2 * w + u] = p;
  }
}

template <int NP>
__global__ __launch_bounds__(kInferThreads) void infer_l3_select_kernel(
    const float* __restrict__ params, const float* __restrict__ part, float theta, float conf_min,
    float* __restrict__ act, unsigned char* __restrict__ mask, float* __restrict__ conf_out,
    int* __restrict__ fell, ChanSel* __restrict__ sel) {
  constexpr int S = NP / 16;
  __shared__ float b3[NP];
  __shared__ float h2[kHidden];
  __shared__ float sc[NP];
  __shared__ float red[kInferWaves];
  __shared__ int wcnt[kInferWaves];
  __shared__ unsigned long long wbits[kInferWaves];
  __shared__ unsigned char keep[NP];
  __shared__ unsigned char used[16];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const MlpLayout L = mlp_layout(NP);
  using D3 = Dense<kHidden, NP>;
  float w3[D3::RB][D3::C];  // the third layer's first batch, in flight while the second layer is finished
  D3::load(params + L.W3, 0, w, lane, w3);
  if (tid < kHidden) {
    float acc = part[tid];
#pragma unroll
    for (int gg = 1; gg < kInferBlocks; ++gg) acc += part[gg * kHidden + tid];
    const float h = bf16r(fmaxf(acc + params[L.b2 + tid], 0.f));
    h2[tid] = h;
    act[kHidden + tid] = h;
  }
  if (tid < NP) b3[tid] = params[L.b3 + tid];
  __syncthreads();
  D3::template run<1>(params + L.W3, b3, h2, sc, w, lane, w3);
  __syncthreads();
  const float s = tid < NP ? sc[tid] : 0.5f;
  if (tid < NP) act[2 * kHidden + tid] = s;
  float c = tid < NP ? fmaxf(s, 1.f - s) : 1.f;
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) c = fminf(c, __shfl_xor(c, m, 64));
  if (lane == 0) red[w] = c;
  __syncthreads();
  float conf = red[0];
#pragma unroll
  for (int i = 1; i < kInferWaves; ++i) conf = fminf(conf, red[i]);
  const bool fb = conf < conf_min;
  const bool kp = tid < NP && (fb || s >= theta);
  if (tid < NP) {
    keep[tid] = kp ? 1 : 0;
    mask[tid] = kp ? 1 : 0;
  }
  const unsigned long long bal = __ballot(kp);
  if (lane == 0) {
    wcnt[w] = __popcll(bal);
    wbits[w] = bal;
  }
  __syncthreads();
  int base = 0;
  for (int i = 0; i < w; ++i) base += wcnt[i];
  if (kp) sel->ch[base + __popcll(bal & ((1ull << lane) - 1ull))] = static_cast<unsigned char>(tid);
  if (tid < 8) sel->keep[tid] = static_cast<unsigned>(wbits[tid >> 1] >> (32 * (tid & 1)));
  if (tid < S) {  // subset tid holds the strips k = tid (mod S)
    unsigned char u = 0;
    for (int k = tid; k < NP; k += S) u |= keep[k];
    used[tid] = u;
  }
  __syncthreads();
  if (tid == 0) {
    int nsub = 0, npair = 0, nch = 0;
    for (int i = 0; i < S; ++i)
      if (used[i]) sel->sub[nsub++] = static_cast<unsigned char>(i);
    for (int i = 0; i < S / 2; ++i)
      if (used[i] || used[i + S / 2]) sel->pair[npair++] = static_cast<unsigned char>(i);
    for (int i = 0; i < kInferWaves; ++i) nch += wcnt[i];
    sel->nch = nch;
    sel->nsub = nsub;
    sel->npair = npair;
    *conf_out = conf;
    *fell = fb ? 1 : 0;
  }
}

template <int NP>
hipError_t select_infer(const float* feat, const float* mu, const float* sigma, const float* params, float theta,
                        float conf_min, float* act, unsigned char* mask, float* conf, int* fell, ChanSel* sel,
                        hipStream_t s) {
  float* part = act + 3 * kHidden;  // kInferBlocks x 256 partial sums of the second layer
  hipLaunchKernelGGL(infer_l12_kernel<NP>, dim3(kInferBlocks), dim3(kInferThreads), 0, s, feat, mu, sigma, params,
                     act, part);
  hipLaunchKernelGGL(infer_l3_select_kernel<NP>, dim3(1), dim3(kInferThreads), 0, s, params, part, theta, conf_min,
                     act, mask, conf, fell, sel);
  return hipGetLastError();
}

template <int NP>
hipError_t seg_features(const float2* x, int64_t xs, int64_t N, int nsig, const float* win, const float2* tabs,
                        float* P, float* feat, hipStream_t s, bool centre) {
  hipLaunchKernelGGL(seg_periodogram_kernel<NP>, dim3(2 * (NP / 16), kBF, nsig), dim3(kSegThreads), 0, s, x, xs, N,
                     win, tabs, P);
  hipLaunchKernelGGL(acp_features_kernel, dim3(NP, nsig), dim3(256), 0, s, P, NP, feat);
  if (centre) hipLaunchKernelGGL(centre_psd_kernel, dim3(nsig), dim3(256), 0, s, feat, NP);
  return hipGetLastError();
}

inline dim3 blocks1(int64_t n) { return dim3(static_cast<unsigned>((n + 255) / 256)); }

template <bool TA, bool TB, int EPI>
hipError_t gemm(const float* A, int lda, const float* B, int ldb, float* C, float* C2, const float* bias, int M, int N,
                int K, hipStream_t s) {
  hipLaunchKernelGGL((gemm_bf16_kernel<TA, TB, EPI>), dim3((N + 31) / 32, (M + 31) / 32), dim3(64), 0, s, A, lda, B, ldb,
                     C, C2, bias, M, N, K);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_features(const float2* x, int64_t xs, int64_t N, int Np, int nsig, const float* win,
                           const float2* tabs, float* P, float* feat, hipStream_t s, bool centre) {
  switch (Np) {
    case 16: return seg_features<16>(x, xs, N, nsig, win, tabs, P, feat, s, centre);
    case 32: return seg_features<32>(x, xs, N, nsig, win, tabs, P, feat, s, centre);
    case 64: return seg_features<64>(x, xs, N, nsig, win, tabs, P, feat, s, centre);
    case 128: return seg_features<128>(x, xs, N, nsig, win, tabs, P, feat, s, centre);
    case 256: return seg_features<256>(x, xs, N, nsig, win, tabs, P, feat, s, centre);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_labels(const float2* S, int64_t N, int Np, int nsig, float* labels, float* ratio, hipStream_t s) {
  hipLaunchKernelGGL(labels_kernel, dim3(Np, nsig), dim3(256), 0, s, S, N, Np, labels, ratio);
  return hipGetLastError();
}

hipError_t launch_standardize(const float* f, const float* mu, const float* sigma, float* out, int n, int dim,
                              hipStream_t s) {
  hipLaunchKernelGGL(standardize_kernel, blocks1(static_cast<int64_t>(n) * dim), dim3(256), 0, s, f, mu, sigma, out, n,
                     dim);
  return hipGetLastError();
}

// act: [a1 h1 a2 h2] each [B][256]; z, s: [B][Np].
hipError_t launch_mlp_forward(int Np, int B, const float* params, const float* x, float* act, float* z, float* sc,
                              hipStream_t s) {
  const MlpLayout L = mlp_layout(Np);
  float* a1 = act;
  float* h1 = a1 + static_cast<int64_t>(B) * kHidden;
  float* a2 = h1 + static_cast<int64_t>(B) * kHidden;
  float* h2 = a2 + static_cast<int64_t>(B) * kHidden;
  hipError_t e = gemm<false, true, kEpiBiasRelu>(x, L.in, params + L.W1, L.in, a1, h1, params + L.b1, B, kHidden,
                                                  L.in, s);
  if (e == hipSuccess)
    e = gemm<false, true, kEpiBiasRelu>(h1, kHidden, params + L.W2, kHidden, a2, h2, params + L.b2, B, kHidden,
                                        kHidden, s);
  if (e == hipSuccess)
    e = gemm<false, true, kEpiBiasSigmoid>(h2, kHidden, params + L.W3, kHidden, z, sc, params + L.b3, B, Np, kHidden,
                                           s);
  return e;
}

// scratch: dz [B][Np], d2 [B][256], d1 [B][256]; grads packed like params; dx [B][2 Np] (may be null).
hipError_t launch_mlp_backward(int Np, int B, const float* params, const float* x, const float* act, const float* sc,
                               const float* y, float* grads, float* scratch, float* dx, hipStream_t s) {
  const MlpLayout L = mlp_layout(Np);
  const float* a1 = act;
  const float* h1 = a1 + static_cast<int64_t>(B) * kHidden;
  const float* a2 = h1 + static_cast<int64_t>(B) * kHidden;
  const float* h2 = a2 + static_cast<int64_t>(B) * kHidden;
  float* dz = scratch;
  float* d2 = dz + static_cast<int64_t>(B) * Np;
  float* d1 = d2 + static_cast<int64_t>(B) * kHidden;
  const int nz = B * Np;
  hipLaunchKernelGGL(bce_grad_kernel, blocks1(nz), dim3(256), 0, s, sc, y, dz, nz, 1.f / static_cast<float>(nz));
  hipError_t e = hipGetLastError();
  // layer 3: dW3 = dz^T h2, db3 = colsum dz, d2 = (dz W3) * (a2 > 0)
  if (e == hipSuccess) e = gemm<true, false, kEpiStore>(dz, Np, h2, kHidden, grads + L.W3, nullptr, nullptr, Np, kHidden, B, s);
  hipLaunchKernelGGL(colsum_kernel, blocks1(Np), dim3(256), 0, s, dz, grads + L.b3, B, Np);
  if (e == hipSuccess) e = gemm<false, false, kEpiStore>(dz, Np, params + L.W3, kHidden, d2, nullptr, nullptr, B, kHidden, Np, s);
  hipLaunchKernelGGL(relu_mask_kernel, blocks1(B * kHidden), dim3(256), 0, s, d2, a2, B * kHidden);
  // layer 2
  if (e == hipSuccess) e = gemm<true, false, kEpiStore>(d2, kHidden, h1, kHidden, grads + L.W2, nullptr, nullptr, kHidden, kHidden, B, s);
  hipLaunchKernelGGL(colsum_kernel, blocks1(kHidden), dim3(256), 0, s, d2, grads + L.b2, B, kHidden);
  if (e == hipSuccess) e = gemm<false, false, kEpiStore>(d2, kHidden, params + L.W2, kHidden, d1, nullptr, nullptr, B, kHidden, kHidden, s);
  hipLaunchKernelGGL(relu_mask_kernel, blocks1(B * kHidden), dim3(256), 0, s, d1, a1, B * kHidden);
  // layer 1
  if (e == hipSuccess) e = gemm<true, false, kEpiStore>(d1, kHidden, x, L.in, grads + L.W1, nullptr, nullptr, kHidden, L.in, B, s);
  hipLaunchKernelGGL(colsum_kernel, blocks1(kHidden), dim3(256), 0, s, d1, grads + L.b1, B, kHidden);
  if (e == hipSuccess && dx)
    e = gemm<false, false, kEpiStore>(d1, kHidden, params + L.W1, L.in, dx, nullptr, nullptr, B, L.in, kHidden, s);
  if (e == hipSuccess) e = hipGetLastError();
  return e;
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int n, int t, float lr, float b1, float b2,
                       float eps, hipStream_t s) {
  const float c1 = 1.f - powf(b1, static_cast<float>(t)), c2 = 1.f - powf(b2, static_cast<float>(t));
  hipLaunchKernelGGL(adam_kernel, blocks1(n), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_select_infer(const float* feat, const float* mu, const float* sigma, const float* params, int Np,
                               float theta, float conf_min, float* h, unsigned char* mask, float* conf, int* fell,
                               ChanSel* sel, hipStream_t s) {
  switch (Np) {
    case 16: return select_infer<16>(feat, mu, sigma, params, theta, conf_min, h, mask, conf, fell, sel, s);
    case 32: return select_infer<32>(feat, mu, sigma, params, theta, conf_min, h, mask, conf, fell, sel, s);
    case 64: return select_infer<64>(feat, mu, sigma, params, theta, conf_min, h, mask, conf, fell, sel, s);
    case 128: return select_infer<128>(feat, mu, sigma, params, theta, conf_min, h, mask, conf, fell, sel, s);
    case 256: return select_infer<256>(feat, mu, sigma, params, theta, conf_min, h, mask, conf, fell, sel, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_select(const float* sc, int Np, int nsig, float theta, unsigned char* mask, float* conf,
                         hipStream_t s) {
  hipLaunchKernelGGL(select_kernel, dim3(nsig), dim3(256), 0, s, sc, Np, theta, mask, conf);
  return hipGetLastError();
}

}  // namespace scd
