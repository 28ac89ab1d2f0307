// FFT accumulation method (Sec. II-B, Eq. (3)-(5)) in FP32.
//
// fam_chan: the channelizer of Eq. (3) with hop L over P frames. A workgroup loads F = 4096/Np centred,
//   windowed frames into LDS (zero outside [0, P*L)), takes their Np-point DFTs, applies the down-conversion
//   omega_Np^{(k p L) mod Np} and stores X_T channel-major, xt[k][p], so the pair kernel reads rows.
//   X_T is at most 256 x 1024 complex (2 MiB) and stays in L2.
// fam_pair: for channel k and a tile of KLT channels l, forms z[p] = X_T[p][k] conj(X_T[p][l]) (the conjugate
//   multiplication of Eq. (5)) while loading, takes the P-point DFT of the KLT products in LDS and stores
//   S[k][l][q] as one contiguous KLT*P run (the output stream dominates FAM's HBM traffic). Row k, which all
//   KLT products share, is staged in LDS once, so each thread's global loads are only its rows l. The LDS
//   rows carry one float2 of padding per 16 elements (radix-16 stages write 16-element strides), and when
//   every stage has the same radix each sequence's butterflies stay in one wave, so the stages need no
//   workgroup barrier. KLT is 16, or 64 for P <= 64 (short transforms: more of them per workgroup). In the power
//   form it stores only |S|^2 of the bins the paper keeps after its second FFT (Alg. 1), -P/4 <= q_c < P/4, in the
//   order q = 0..P/4-1, P-P/4..P-1: a quarter of the complex output's bytes.
#include <type_traits>

#include "scd_device.h"
#include "scd_launch.h"

namespace scd {

namespace {

constexpr int kChanThreads = 256;
constexpr int kPairThreads = 256;

template <int NP>
__global__ __launch_bounds__(kChanThreads) void fam_chan_fp32(const float2* __restrict__ x, int L, int P,
                                                             const float* __restrict__ win,
                                                             const float2* __restrict__ tabs,
                                                             float2* __restrict__ xt, int64_t xbs,
                                                             int64_t xtbs) {
  constexpr int F = 4096 / NP;
  constexpr int D = NP / 2 - 1;
  __shared__ float2 buf[F * NP];
  __shared__ float2 tw[1024];
  __shared__ float2 rt[NP];
  const int tid = threadIdx.x;
  const int p0 = blockIdx.x * F;
  const int len = P * L;
  x += blockIdx.y * xbs;
  xt += blockIdx.y * xtbs;
  lds_copy<1024, kChanThreads>(tw, tabs + kTabTw1024, tid);
  lds_copy<NP, kChanThreads>(rt, tabs + kTabRoots, tid);
  // Samples outside [0, P L), and every sample of the frames p >= P, read as zero through a range-checked
  // buffer load, so all of a thread's loads are in flight before its first LDS write.
  constexpr int PER = F * NP / kChanThreads;
  const auto xr = make_rsrc(x, len * 8);
  float2 xv[PER];
  float wv[PER];
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    const int e = tid + r * kChanThreads;
    const int f = e / NP, j = e % NP;
    const int p = p0 + f;
    xv[r] = load_c64(xr, p < P ? p * L - D + j : -1);
    wv[r] = win[j];
  }
#pragma unroll
  for (int r = 0; r < PER; ++r) buf[tid + r * kChanThreads] = cscale(xv[r], wv[r]);
  __syncthreads();
  auto st = [&](int f, int k, float2 v) {
    const int p = p0 + f;
    if (p < P) xt[static_cast<int64_t>(k) * P + p] = cmul(v, rt[(k * p * L) & (NP - 1)]);
  };
  NoLoad ld;
  lds_fft<NP, F, kChanThreads, true, LdsLayout<NP, 1>>(buf, tw, tid, ld, st);
}

// |v|^2 as re*re + im*im with each operation rounded to FP32 (no fused multiply-add), as the documented
// power form is defined.
__device__ __forceinline__ float power_rn(float2 v) {
#pragma clang fp contract(off)
  return v.x * v.x + v.y * v.y;
}

// Rows l come from yt: X_T itself for the auto SCD, y's channelizer output for the cross SCD. CONJ multiplies
// by Y_T[p][l] itself (the conjugate form) instead of its conjugate.
template <int P, int KLT, bool POWER, bool CONJ>
__global__ __launch_bounds__(kPairThreads) void fam_pair_fp32(const float2* __restrict__ xt,
                                                             const float2* __restrict__ yt, int Np,
                                                             const float2* __restrict__ tabs,
                                                             void* __restrict__ out, int64_t xtbs,
                                                             int64_t obs) {
  constexpr int TWN = P < 16 ? 16 : P;  // omega_P^e (at least the 16 roots a radix-16 stage may index)
  constexpr int BS = P + P / 16;        // padded LDS row
  using Lay = LdsLayout<BS, 1, 4>;
  constexpr bool WAVE = uniform_radix<P, 1>() && 64 % (P / StageRadix<P, 1>::value) == 0;
  __shared__ float2 buf[KLT * BS];
  __shared__ float2 tw[TWN];
  __shared__ float2 rk[P];  // row k of X_T
  const int tid = threadIdx.x;
  const int l0 = blockIdx.x * KLT;
  const int k = blockIdx.y;
  xt += blockIdx.z * xtbs;
  yt += blockIdx.z * xtbs;
  lds_copy<TWN, kPairThreads, 1024 / TWN>(tw, tabs + kTabTw1024, tid);
  lds_copy<P, kPairThreads>(rk, xt + static_cast<int64_t>(k) * P, tid);
  __syncthreads();
  const float2* rl = yt + static_cast<int64_t>(l0) * P;
  auto ld = [&](int b, int m) { return CONJ ? cmul(rk[m], rl[b * P + m]) : cmulc(rk[m], rl[b * P + m]); };
  // The output is written once and never read back here: stream it past the caches.
  if constexpr (POWER) {
    constexpr int H = P / 4;
    float* dst = static_cast<float*>(out) + blockIdx.z * obs + (static_cast<int64_t>(k) * Np + l0) * (P / 2);
    auto st = [&](int b, int m, float2 v) {
      if (m < H || m >= P - H)
        __builtin_nontemporal_store(power_rn(v), dst + b * (P / 2) + (m < H ? m : m - P / 2));
    };
    lds_fft<P, KLT, kPairThreads, false, Lay, TWN, WAVE>(buf, tw, tid, ld, st);
  } else {
    float2* dst = static_cast<float2*>(out) + blockIdx.z * obs + (static_cast<int64_t>(k) * Np + l0) * P;
    auto st = [&](int b, int m, float2 v) { st1_nt(dst + b * P + m, v); };
    lds_fft<P, KLT, kPairThreads, false, Lay, TWN, WAVE>(buf, tw, tid, ld, st);
  }
}

template <int NP>
hipError_t chan(const float2* x, int L, int P, const float* win, const float2* tabs, float2* xt, int batch,
                int64_t xbs, hipStream_t s) {
  constexpr int F = 4096 / NP;
  dim3 grid((P + F - 1) / F, batch);
  hipLaunchKernelGGL(fam_chan_fp32<NP>, grid, dim3(kChanThreads), 0, s, x, L, P, win, tabs, xt, xbs,
                     static_cast<int64_t>(NP) * P);
  return hipGetLastError();
}

template <int P, int KLT>
hipError_t pair_tile(const float2* xt, const float2* yt, bool conj, int Np, const float2* tabs, void* out, bool power,
                     int batch, int64_t obs, hipStream_t s) {
  dim3 grid(Np / KLT, Np, batch);
  const int64_t xtbs = static_cast<int64_t>(Np) * P;
  if (power)
    hipLaunchKernelGGL((fam_pair_fp32<P, KLT, true, false>), grid, dim3(kPairThreads), 0, s, xt, yt, Np, tabs, out,
                       xtbs, obs);
  else if (conj)
    hipLaunchKernelGGL((fam_pair_fp32<P, KLT, false, true>), grid, dim3(kPairThreads), 0, s, xt, yt, Np, tabs, out,
                       xtbs, obs);
  else
    hipLaunchKernelGGL((fam_pair_fp32<P, KLT, false, false>), grid, dim3(kPairThreads), 0, s, xt, yt, Np, tabs, out,
                       xtbs, obs);
  return hipGetLastError();
}

// Channels l per workgroup: 64 for P <= 64 (at most Np), else 16. Np is a power of two >= 16.
template <int P>
hipError_t pair(const float2* xt, const float2* yt, bool conj, int Np, const float2* tabs, void* out, bool power,
                int batch, int64_t obs, hipStream_t s) {
  if constexpr (P <= 64) {
    if (Np >= 64) return pair_tile<P, 64>(xt, yt, conj, Np, tabs, out, power, batch, obs, s);
    if (Np == 32) return pair_tile<P, 32>(xt, yt, conj, Np, tabs, out, power, batch, obs, s);
  }
  return pair_tile<P, 16>(xt, yt, conj, Np, tabs, out, power, batch, obs, s);
}

}  // namespace

hipError_t launch_fam_fp32(const float2* x, int Np, int L, int P, const float* win, const float2* tabs, float2* xt,
                           void* out, bool power, int batch, int64_t xbs, int64_t obs, hipStream_t s,
                           const float2* y, bool conj) {
  auto channelize = [&](const float2* in, float2* dst) -> hipError_t {
    switch (Np) {
      case 16: return chan<16>(in, L, P, win, tabs, dst, batch, xbs, s);
      case 32: return chan<32>(in, L, P, win, tabs, dst, batch, xbs, s);
      case 64: return chan<64>(in, L, P, win, tabs, dst, batch, xbs, s);
      case 128: return chan<128>(in, L, P, win, tabs, dst, batch, xbs, s);
      case 256: return chan<256>(in, L, P, win, tabs, dst, batch, xbs, s);
      default: return hipErrorInvalidValue;
    }
  };
  hipError_t e = channelize(x, xt);
  if (e != hipSuccess) return e;
  // The cross forms channelize y into the second half of the scratch.
  float2* yt = xt;
  if (y) {
    yt = xt + static_cast<int64_t>(batch) * Np * P;
    if ((e = channelize(y, yt)) != hipSuccess) return e;
  }
  switch (P) {
    case 4: return pair<4>(xt, yt, conj, Np, tabs, out, power, batch, obs, s);
    case 8: return pair<8>(xt, yt, conj, Np, tabs, out, power, batch, obs, s);
    case 16: return pair<16>(xt, yt, conj, Np, tabs, out, power, batch, obs, s);
    case 32: return pair<32>(xt, yt, conj, Np, tabs, out, power, batch, obs, s);
    case 64: return pair<64>(xt, yt, conj, Np, tabs, out, power, batch, obs, s);
    case 128: return pair<128>(xt, yt, conj, Np, tabs, out, power, batch, obs, s);
    case 256: return pair<256>(xt, yt, conj, Np, tabs, out, power, batch, obs, s);
    case 512: return pair<512>(xt, yt, conj, Np, tabs, out, power, batch, obs, s);
    case 1024: return pair<1024>(xt, yt, conj, Np, tabs, out, power, batch, obs, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace scd
