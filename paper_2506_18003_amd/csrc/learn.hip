// Kernels of the learned strip selector: features, labels, the MLP (bf16 MFMA GEMMs with FP32 accumulation)
// with its backward pass and Adam, and the strip selection.
//
// Features of a signal (2 Np floats): from the SSCA S_b of B_F = 16 segments of N_C = 1024 samples,
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

// One workgroup per (strip k, signal): seg is [sig][B_F][Np][N_C] complex; feat [sig][2 Np] gets the raw
// (uncentred) PSD_k and ACP_k.
__global__ __launch_bounds__(256) void acp_features_kernel(const float2* __restrict__ seg, int Np,
                                                           float* __restrict__ feat) {
  __shared__ float red[256];
  const int k = blockIdx.x, sig = blockIdx.y, tid = threadIdx.x;
  const float2* base = seg + (static_cast<int64_t>(sig) * kBF * Np + k) * kNC;
  const int q0 = (-signed_idx(k, Np) * (kNC / Np)) & (kNC - 1);
  float sum = 0.f, mx = 0.f, a0 = 0.f;
  int cnt = 0;
  for (int q = tid; q < kNC; q += 256) {
    float a = 0.f;
    for (int b = 0; b < kBF; ++b) {
      const float2 v = base[static_cast<int64_t>(b) * Np * kNC + q];
      a = fmaf(v.x, v.x, fmaf(v.y, v.y, a));
    }
    if (q == q0) a0 = a;
    const int d = abs(signed_idx((q - q0) & (kNC - 1), kNC));
    if (d > 4) {
      sum += a;
      mx = fmaxf(mx, a);
      ++cnt;
    }
  }
  const float tot = block_sum(sum, red);
  const float n = block_sum(static_cast<float>(cnt), red);
  const float m = block_max(mx, red);
  const float a0s = block_sum(a0, red);
  if (tid == 0) {
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

// out[o] = sum_i bf16(W[o][i]) in[i] + b[o] for o < nout, in FP32 (in[] already bf16-valued, in LDS).
__device__ __forceinline__ float dense_row(const float* __restrict__ W, const float* in, int nin, int o) {
  const float4* w = reinterpret_cast<const float4*>(W + static_cast<int64_t>(o) * nin);
  float acc = 0.f;
  for (int i = 0; i < nin / 4; ++i) {
    const float4 v = w[i];
    acc = fmaf(bf16r(v.x), in[4 * i], acc);
    acc = fmaf(bf16r(v.y), in[4 * i + 1], acc);
    acc = fmaf(bf16r(v.z), in[4 * i + 2], acc);
    acc = fmaf(bf16r(v.w), in[4 * i + 3], acc);
  }
  return acc;
}

// Selector inference of one signal in one workgroup: standardised features -> MLP (every product of bf16-rounded
// operands, FP32 accumulation, as in the GEMM kernels) -> strip scores -> mask, confidence, fallback and the
// channel selection of the SSCA kernels. Thread o computes output o of each layer from its weight row.
__global__ __launch_bounds__(256) void select_infer_kernel(const float* __restrict__ feat, const float* __restrict__ mu,
                                                           const float* __restrict__ sigma,
                                                           const float* __restrict__ params, int Np, float theta,
                                                           float conf_min, unsigned char* __restrict__ mask,
                                                           float* __restrict__ conf_out, int* __restrict__ fell,
                                                           ChanSel* __restrict__ sel) {
  __shared__ float xin[512];
  __shared__ float h1[kHidden], h2[kHidden];
  __shared__ float red[256];
  __shared__ unsigned char keep[256];
  const int tid = threadIdx.x;
  const MlpLayout L = mlp_layout(Np);
  for (int i = tid; i < L.in; i += 256) xin[i] = bf16r((feat[i] - mu[i]) / sigma[i]);
  __syncthreads();
  h1[tid] = bf16r(fmaxf(dense_row(params + L.W1, xin, L.in, tid) + params[L.b1 + tid], 0.f));
  __syncthreads();
  h2[tid] = bf16r(fmaxf(dense_row(params + L.W2, h1, kHidden, tid) + params[L.b2 + tid], 0.f));
  __syncthreads();
  float s = 0.f, c = 1.f;
  if (tid < Np) {
    const float z = dense_row(params + L.W3, h2, kHidden, tid) + params[L.b3 + tid];
    s = 1.f / (1.f + expf(-z));
    c = fmaxf(s, 1.f - s);
  }
  red[tid] = c;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) red[tid] = fminf(red[tid], red[tid + st]);
    __syncthreads();
  }
  const float conf = red[0];
  const bool fb = conf < conf_min;
  if (tid < Np) {
    const unsigned char m = (fb || s >= theta) ? 1 : 0;
    keep[tid] = m;
    mask[tid] = m;
  }
  __syncthreads();
  if (tid == 0) {
    const int S = Np / 16;
    unsigned kb[8] = {};
    bool used[16] = {};
    int nch = 0, nsub = 0, npair = 0;
    for (int k = 0; k < Np; ++k) {
      if (!keep[k]) continue;
      kb[k >> 5] |= 1u << (k & 31);
      sel->ch[nch++] = static_cast<unsigned char>(k);
      used[k % S] = true;  // strip k belongs to subset k mod S
    }
    for (int i = 0; i < S; ++i)
      if (used[i]) sel->sub[nsub++] = static_cast<unsigned char>(i);
    for (int i = 0; i < S / 2; ++i)
      if (used[i] || used[i + S / 2]) sel->pair[npair++] = static_cast<unsigned char>(i);
    for (int w = 0; w < 8; ++w) sel->keep[w] = kb[w];
    sel->nch = nch;
    sel->nsub = nsub;
    sel->npair = npair;
    *conf_out = conf;
    *fell = fb ? 1 : 0;
  }
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

hipError_t launch_acp_features(const float2* seg, int Np, int nsig, float* feat, hipStream_t s) {
  hipLaunchKernelGGL(acp_features_kernel, dim3(Np, nsig), dim3(256), 0, s, seg, Np, feat);
  hipLaunchKernelGGL(centre_psd_kernel, dim3(nsig), dim3(256), 0, s, feat, Np);
  return hipGetLastError();
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
                               float theta, float conf_min, unsigned char* mask, float* conf, int* fell, ChanSel* sel,
                               hipStream_t s) {
  if (Np > 256 || 2 * Np > 512) return hipErrorInvalidValue;
  hipLaunchKernelGGL(select_infer_kernel, dim3(1), dim3(256), 0, s, feat, mu, sigma, params, Np, theta, conf_min, mask,
                     conf, fell, sel);
  return hipGetLastError();
}

hipError_t launch_select(const float* sc, int Np, int nsig, float theta, unsigned char* mask, float* conf,
                         hipStream_t s) {
  hipLaunchKernelGGL(select_kernel, dim3(nsig), dim3(256), 0, s, sc, Np, theta, mask, conf);
  return hipGetLastError();
}

}  // namespace scd
