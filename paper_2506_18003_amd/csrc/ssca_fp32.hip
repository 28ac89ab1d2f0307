// Plain FP32 SSCA (Sec. II-C, Eq. (6)-(7)) computed as the paper's SSCA_2DFFT (Sec. III-B, Eq. (10)-(16)),
// with N = M1 * M2, M1 = 1024 and M2 = N / 1024.
//
// Pass 1 (one workgroup per (m2, channel subset)): generates the channel-data product X_g only where Stage 1
// needs it. For every m1 it forms the centred, windowed frame n = m1*M2 + m2 (Eq. (3), L = 1), evaluates the
// 16 channels k = c + S*k' (S = Np/16) of the subset with a pruned DFT, applies the down-conversion factor
// omega_Np^{(k n) mod Np} and the conjugate sample conj(x[n]) (Eq. (6)), and writes X_g(m1, m2, k) into an
// LDS column. It then takes the M1-point DFT of each column (Stage 1), multiplies by the rotation factor
// omega_N^{m2 m1'} and stores the result to HBM in a blocked layout T[k][m1'/16][m2][m1' % 16], so both this
// store and pass 2's load move whole 128-byte runs.
//
// Pass 2 (one workgroup per (16 consecutive m1', k)): Stage 2, the M2-point DFT over m2 of 16 rows at once,
// stored at S[k][q] with q = m1' + M1*m2' (16 consecutive q per run).
//
// Pruned channel-subset DFT: with j = j0 + 16*j1 (j0 < 16, j1 < S) and k = c + S*k',
//   sum_j v[j] omega_Np^{k j} = sum_{j0} omega_16^{k' j0} [ sum_{j1} (w[j] omega_Np^{c j}) x[n-d+j] ],
// so each subset costs one complex-windowed fold of the frame to 16 points plus a 16-point DFT.
#include <type_traits>

#include "scd_device.h"
#include "scd_launch.h"

namespace scd {

namespace {

constexpr int kM1 = 1024;
constexpr int kP1Threads = 256;
constexpr int kCols = 16;
constexpr int kColStride = kM1 + kM1 / 16;  // one float2 of padding per 16 elements
constexpr int kP2Threads = 256;

template <int NP>
__global__ __launch_bounds__(kP1Threads) void ssca_pass1_fp32(const float2* __restrict__ x, int N, int M2,
                                                             int m2shift, const float* __restrict__ win,
                                                             const float2* __restrict__ tabs,
                                                             float2* __restrict__ T, int64_t xbs, int64_t tbs) {
  constexpr int S = NP / 16;
  constexpr int D = NP / 2 - 1;
  __shared__ float2 col[kCols * kColStride];
  __shared__ float2 tw[1024];
  __shared__ float2 rlo[1024];
  __shared__ float2 hc[NP];
  __shared__ float2 rt[NP];

  const int tid = threadIdx.x;
  const int m2 = blockIdx.x;
  const int c = blockIdx.y;
  x += blockIdx.z * xbs;
  T += blockIdx.z * tbs;

  for (int i = tid; i < 1024; i += kP1Threads) {
    tw[i] = tabs[kTabTw1024 + i];
    rlo[i] = tabs[kTabRotLo + i];
  }
  for (int i = tid; i < NP; i += kP1Threads) {
    const float2 r = tabs[kTabRoots + i];
    rt[i] = r;
    hc[i] = cscale(tabs[kTabRoots + ((c * i) & (NP - 1))], win[i]);
  }
  __syncthreads();

  // Channelizer, down-conversion and channel-data product for frames m1 = tid + f*256.
#pragma unroll 1
  for (int f = 0; f < kM1 / kP1Threads; ++f) {
    const int m1 = tid + f * kP1Threads;
    const int n = m1 * M2 + m2;
    const int base = n - D;
    float2 u[16];
#pragma unroll
    for (int j0 = 0; j0 < 16; ++j0) u[j0] = make_float2(0.f, 0.f);
#pragma unroll
    for (int j1 = 0; j1 < S; ++j1) {
#pragma unroll
      for (int j0 = 0; j0 < 16; ++j0) {
        const int idx = base + j0 + 16 * j1;
        const float2 xv = (static_cast<unsigned>(idx) < static_cast<unsigned>(N)) ? x[idx] : make_float2(0.f, 0.f);
        u[j0] = cfma(u[j0], hc[j0 + 16 * j1], xv);
      }
    }
    dft16(u);
    const float2 xn = x[n];
#pragma unroll
    for (int kp = 0; kp < 16; ++kp) {
      const int k = c + S * kp;
      const float2 pc = cmulc(rt[(k * n) & (NP - 1)], xn);
      col[kp * kColStride + m1 + (m1 >> 4)] = cmul(u[kp], pc);
    }
  }
  __syncthreads();

  // Stage 1: M1-point DFT over m1, rotation omega_N^{m2 m1'}, blocked store.
  const int hishift = 10 - m2shift;  // omega_N^{1024 a_hi} = omega_1024^{a_hi * 1024 / M2}
  auto st = [&](int b, int m, float2 v) {
    const int k = c + S * b;
    const int a = m2 * m;
    const float2 rot = cmul(rlo[a & 1023], tw[((a >> 10) << hishift) & 1023]);
    T[((k * (kM1 / 16) + (m >> 4)) * M2 + m2) * 16 + (m & 15)] = cmul(v, rot);
  };
  NoLoad ld;
  lds_fft<kM1, kCols, kP1Threads, false, LdsLayout<kColStride, 1, 4>>(col, tw, tid, ld, st);
}

template <int M2>
__global__ __launch_bounds__(kP2Threads) void ssca_pass2_fp32(const float2* __restrict__ T,
                                                             const float2* __restrict__ tabs,
                                                             float2* __restrict__ out, int N, int64_t tbs,
                                                             int64_t obs) {
  __shared__ float2 buf[M2 * 16];
  __shared__ float2 tw[1024];
  const int tid = threadIdx.x;
  const int mb = blockIdx.x;  // block of 16 consecutive m1'
  const int k = blockIdx.y;
  for (int i = tid; i < 1024; i += kP2Threads) tw[i] = tabs[kTabTw1024 + i];
  __syncthreads();
  const float2* src = T + blockIdx.z * tbs + (static_cast<int64_t>(k) * (kM1 / 16) + mb) * (M2 * 16);
  float2* dst = out + blockIdx.z * obs + static_cast<int64_t>(k) * N + mb * 16;
  auto ld = [&](int b, int m) { return src[m * 16 + b]; };
  auto st = [&](int b, int m, float2 v) { dst[b + kM1 * m] = v; };
  lds_fft<M2, 16, kP2Threads, true, LdsLayout<1, 16>>(buf, tw, tid, ld, st);
}

template <int NP>
hipError_t pass1(const float2* x, int N, int M2, int m2shift, const float* win, const float2* tabs, float2* T,
                 int batch, int64_t xbs, int64_t tbs, hipStream_t s) {
  dim3 grid(M2, NP / 16, batch);
  hipLaunchKernelGGL(ssca_pass1_fp32<NP>, grid, dim3(kP1Threads), 0, s, x, N, M2, m2shift, win, tabs, T, xbs, tbs);
  return hipGetLastError();
}

template <int M2>
hipError_t pass2(const float2* T, const float2* tabs, float2* out, int N, int Np, int batch, int64_t tbs,
                 int64_t obs, hipStream_t s) {
  dim3 grid(kM1 / 16, Np, batch);
  hipLaunchKernelGGL(ssca_pass2_fp32<M2>, grid, dim3(kP2Threads), 0, s, T, tabs, out, N, tbs, obs);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_ssca_pass1_fp32(const float2* x, int N, int Np, const float* win, const float2* tabs, float2* T,
                                  int batch, int64_t xbs, int64_t tbs, hipStream_t s) {
  const int M2 = N / kM1;
  int m2shift = 0;
  while ((1 << m2shift) < M2) ++m2shift;
  switch (Np) {
    case 16: return pass1<16>(x, N, M2, m2shift, win, tabs, T, batch, xbs, tbs, s);
    case 32: return pass1<32>(x, N, M2, m2shift, win, tabs, T, batch, xbs, tbs, s);
    case 64: return pass1<64>(x, N, M2, m2shift, win, tabs, T, batch, xbs, tbs, s);
    case 128: return pass1<128>(x, N, M2, m2shift, win, tabs, T, batch, xbs, tbs, s);
    case 256: return pass1<256>(x, N, M2, m2shift, win, tabs, T, batch, xbs, tbs, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_ssca_pass2(const float2* T, int N, int Np, const float2* tabs, float2* out, int batch, int64_t tbs,
                             int64_t obs, hipStream_t s) {
  switch (N / kM1) {
    case 1: return hipSuccess;
    case 2: return pass2<2>(T, tabs, out, N, Np, batch, tbs, obs, s);
    case 4: return pass2<4>(T, tabs, out, N, Np, batch, tbs, obs, s);
    case 8: return pass2<8>(T, tabs, out, N, Np, batch, tbs, obs, s);
    case 16: return pass2<16>(T, tabs, out, N, Np, batch, tbs, obs, s);
    case 32: return pass2<32>(T, tabs, out, N, Np, batch, tbs, obs, s);
    case 64: return pass2<64>(T, tabs, out, N, Np, batch, tbs, obs, s);
    case 128: return pass2<128>(T, tabs, out, N, Np, batch, tbs, obs, s);
    case 256: return pass2<256>(T, tabs, out, N, Np, batch, tbs, obs, s);
    case 512: return pass2<512>(T, tabs, out, N, Np, batch, tbs, obs, s);
    case 1024: return pass2<1024>(T, tabs, out, N, Np, batch, tbs, obs, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace scd
