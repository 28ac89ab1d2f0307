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

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// One dense layer of selector inference, spread over the GPU: wave w of block b computes row o = 4 b + w,
// out[o] = act(sum_i bf16(W[o][i]) in[i] + b[o]) with FP32 accumulation. Its lanes read 64 consecutive weights
// per load (whole 256-byte runs, all NIN/64 loads in flight) and the row sum is reduced across the wave.
// FIRST: in = bf16(standardised features) computed here from the raw features (PSD not yet centred: each wave
// subtracts the mean PSD itself), mu and sigma; otherwise in is the previous layer's output (already
// bf16-valued). ACT: 0 = ReLU then bf16 rounding (the next layer's operand), 1 = sigmoid.
template <int NIN, bool FIRST, int ACT>
__global__ __launch_bounds__(256) void mlp_infer_layer_kernel(const float* __restrict__ W, const float* __restrict__ bias,
                                                              const float* __restrict__ in,
                                                              const float* __restrict__ mu,
                                                              const float* __restrict__ sigma, int nout,
                                                              float* __restrict__ out) {
  constexpr int C = NIN >= 64 ? NIN / 64 : 1;
  const int lane = threadIdx.x & 63;
  const int o = 4 * blockIdx.x + (threadIdx.x >> 6);
  if (o >= nout) return;
  const bool live = NIN >= 64 || lane < NIN;
  float wv[C], xv[C];
#pragma unroll
  for (int cc = 0; cc < C; ++cc) wv[cc] = live ? W[static_cast<int64_t>(o) * NIN + 64 * cc + lane] : 0.f;
  float mean = 0.f;
  if constexpr (FIRST) {
    constexpr int NPF = NIN / 2;  // PSD entries
    float ps = 0.f;
    for (int i = lane; i < NPF; i += 64) ps += in[i];
    mean = wave_sum(ps) / static_cast<float>(NPF);
  }
#pragma unroll
  for (int cc = 0; cc < C; ++cc) {
    const int i = 64 * cc + lane;
    float v = 0.f;
    if (live) v = FIRST ? bf16r((in[i] - (i < NIN / 2 ? mean : 0.f) - mu[i]) / sigma[i]) : in[i];
    xv[cc] = v;
  }
  float acc = 0.f;
#pragma unroll
  for (int cc = 0; cc < C; ++cc) acc = fmaf(bf16r(wv[cc]), xv[cc], acc);
  acc = wave_sum(acc);
  if (lane == 0) {
    acc += bias[o];
    out[o] = (ACT == 0) ? bf16r(fmaxf(acc, 0.f)) : 1.f / (1.f + expf(-acc));
  }
}

// Strip selection of one signal from its scores: mask, confidence min_k max(s_k, 1 - s_k), fallback to every
// strip below conf_min, and the channel selection the SSCA kernels read (strip list in increasing k from wave
// ballots and per-wave counts, subset and pair lists from the kept strips).
template <int NP>
__global__ __launch_bounds__(256) void select_finish_kernel(const float* __restrict__ sc, float theta, float conf_min,
                                                            unsigned char* __restrict__ mask,
                                                            float* __restrict__ conf_out, int* __restrict__ fell,
                                                            ChanSel* __restrict__ sel) {
  __shared__ float red[4];
  __shared__ int wcnt[4];
  __shared__ unsigned long long wbits[4];
  __shared__ unsigned char keep[NP];
  __shared__ unsigned char used[16];
  constexpr int S = NP / 16;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const float s = tid < NP ? sc[tid] : 0.5f;
  float c = tid < NP ? fmaxf(s, 1.f - s) : 1.f;
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) c = fminf(c, __shfl_xor(c, m, 64));
  if (lane == 0) red[w] = c;
  __syncthreads();
  const float conf = fminf(fminf(red[0], red[1]), fminf(red[2], red[3]));
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
    int nsub = 0, npair = 0;
    for (int i = 0; i < S; ++i)
      if (used[i]) sel->sub[nsub++] = static_cast<unsigned char>(i);
    for (int i = 0; i < S / 2; ++i)
      if (used[i] || used[i + S / 2]) sel->pair[npair++] = static_cast<unsigned char>(i);
    sel->nch = wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
    sel->nsub = nsub;
    sel->npair = npair;
    *conf_out = conf;
    *fell = fb ? 1 : 0;
  }
}

template <int NP>
hipError_t select_infer(const float* feat, const float* mu, const float* sigma, const float* params, float theta,
                        float conf_min, float* h, unsigned char* mask, float* conf, int* fell, ChanSel* sel,
                        hipStream_t s) {
  const MlpLayout L = mlp_layout(NP);
  float* h1 = h;
  float* h2 = h + kHidden;
  float* sc = h + 2 * kHidden;
  hipLaunchKernelGGL((mlp_infer_layer_kernel<2 * NP, true, 0>), dim3(kHidden / 4), dim3(256), 0, s, params + L.W1,
                     params + L.b1, feat, mu, sigma, kHidden, h1);
  hipLaunchKernelGGL((mlp_infer_layer_kernel<kHidden, false, 0>), dim3(kHidden / 4), dim3(256), 0, s, params + L.W2,
                     params + L.b2, h1, mu, sigma, kHidden, h2);
  hipLaunchKernelGGL((mlp_infer_layer_kernel<kHidden, false, 1>), dim3(NP / 4), dim3(256), 0, s, params + L.W3,
                     params + L.b3, h2, mu, sigma, NP, sc);
  hipLaunchKernelGGL(select_finish_kernel<NP>, dim3(1), dim3(256), 0, s, sc, theta, conf_min, mask, conf, fell, sel);
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

hipError_t launch_acp_features(const float2* seg, int Np, int nsig, float* feat, hipStream_t s, bool centre) {
  hipLaunchKernelGGL(acp_features_kernel, dim3(Np, nsig), dim3(256), 0, s, seg, Np, feat);
  if (centre) hipLaunchKernelGGL(centre_psd_kernel, dim3(nsig), dim3(256), 0, s, feat, Np);
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
