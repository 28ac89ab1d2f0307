// SSCA Stage 1 with the channelizer DFT on the matrix cores (MFMA), in split or plain 16-bit precision.
//
// The channel-subset DFT of Eq. (3) is a complex GEMM Y[frame][k'] = sum_j x[frame][j] W[j][k'] with
// W[j][k'] = w[j] omega_Np^{(c + S k') j}. It is computed realified and transposed on
// v_mfma_f32_32x32x16_{bf16,f16}: the 32 rows are the 16 channels' (re, im) outputs, the 32 columns are
// frames and K = 2 Np runs over the frame's interleaved (re, im) samples:
//   rows 2k'   : [ Re W, -Im W ] . [x_re, x_im]     rows 2k'+1 : [ Im W,  Re W ] . [x_re, x_im].
// In the split forms both operands carry a hi and a lo 16-bit part (v = hi + lo, lo = v - hi rounded) and the
// GEMM sums W_hi X_hi + W_hi X_lo + W_lo X_hi in FP32, which leaves an error of order 2^-16 (bf16) or 2^-22
// (fp16) relative to the operands instead of the 2^-8 / 2^-11 of a single 16-bit product. The plain forms
// (one product) exist as the accuracy ablation. The weights are generated in FP64 on the GPU before the split.
//
// Everything after the channelizer (down-conversion, channel-data product, the M1-point DFT, rotation, the
// blocked store) is FP32 and organised as in the FP32 Stage 1 (see ssca_fp32.hip); only the frame <-> lane
// mapping follows the MFMA output layout: lane l of wave w holds, for frames t' = 64 w + 32 u + (l mod 32)
// (u < 2) of each 256-frame chunk, the 8 channels k' in {0,1,4,5,8,9,12,13} + 2 (l / 32).
#include <type_traits>

#include "scd_device.h"
#include "scd_launch.h"

namespace scd {

namespace {

constexpr int kM1 = 1024;
constexpr int kThreads = 256;
constexpr int kSeq = 256;
constexpr int kSeqStride = kSeq + kSeq / 16;
constexpr int kHalfSeqs = 32;
constexpr int kXchgFloats = kHalfSeqs * kSeqStride;
constexpr int kJS = 8;                   // complex samples per sub-chunk = one K-step of 16 reals
constexpr int kRow = kJS + 4;            // LDS words per frame row (4 words of padding break bank conflicts)
constexpr int kPlaneWords = kThreads * kRow;
constexpr int kStageWords = 2 * kPlaneWords;  // hi and lo planes

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
// The same 16 bytes when only 4-byte alignment is known (rows of the 16-bit copies of x start anywhere).
typedef unsigned u32x4_a4 __attribute__((ext_vector_type(4), aligned(4)));

template <int PREC>
struct Prec {
  static constexpr bool kSplit = (PREC == SCD_PREC_SPLIT_BF16 || PREC == SCD_PREC_SPLIT_FP16);
  static constexpr bool kBf16 = (PREC == SCD_PREC_SPLIT_BF16 || PREC == SCD_PREC_BF16);
  using T16 = typename std::conditional<kBf16, __bf16, _Float16>::type;
  using V8 = typename std::conditional<kBf16, bf16x8, f16x8>::type;
  __device__ __forceinline__ static f32x16 mfma(V8 a, V8 b, f32x16 c) {
    if constexpr (kBf16) return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    else return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};

template <class T16>
__device__ __forceinline__ unsigned short bits16(T16 v) {
  return __builtin_bit_cast(unsigned short, v);
}

// x -> 16-bit hi and lo planes, one 32-bit word (re, im) per sample, with kMfmaPad zero samples on each side.
// INTERLEAVE: one plane of word pairs (hi, lo) per sample instead (hi points to it; lo unused).
template <int PREC, bool INTERLEAVE = false>
__global__ void split_x_kernel(const float2* __restrict__ x, int N, unsigned* __restrict__ hi,
                               unsigned* __restrict__ lo) {
  using P = Prec<PREC>;
  using T16 = typename P::T16;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = e - kMfmaPad;
  if (e >= N + 2 * kMfmaPad) return;
  float2 v = make_float2(0.f, 0.f);
  if (n >= 0 && n < N) v = x[n];
  const T16 hr = static_cast<T16>(v.x), hm = static_cast<T16>(v.y);
  const T16 lr = static_cast<T16>(v.x - static_cast<float>(hr)), lm = static_cast<T16>(v.y - static_cast<float>(hm));
  const unsigned wh = bits16(hr) | (static_cast<unsigned>(bits16(hm)) << 16);
  const unsigned wl = bits16(lr) | (static_cast<unsigned>(bits16(lm)) << 16);
  if constexpr (INTERLEAVE) {
    reinterpret_cast<uint2*>(hi)[e] = make_uint2(wh, wl);
  } else {
    hi[e] = wh;
    lo[e] = wl;
  }
}

// Realified, transposed channel-subset DFT weights in FP64, split into 16-bit hi and lo:
// W[c][row][k] for row = 2 k' + comp, k = 2 j + xcomp, stored row-major with K = 2 Np.
template <int PREC>
__global__ void mfma_weights_kernel(const float* __restrict__ win, int Np, int S, unsigned short* __restrict__ whi,
                                    unsigned short* __restrict__ wlo) {
  using T16 = typename Prec<PREC>::T16;
  const int K = 2 * Np;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= S * 32 * K) return;
  const int c = e / (32 * K), row = (e / K) % 32, k = e % K;
  const int kp = row >> 1, comp = row & 1, j = k >> 1, xcomp = k & 1;
  const int ch = c + S * kp;
  double s, co;
  sincospi(-2.0 * static_cast<double>((ch * j) & (Np - 1)) / static_cast<double>(Np), &s, &co);
  const double hr = static_cast<double>(win[j]) * co, hm = static_cast<double>(win[j]) * s;
  const double v = (comp == 0) ? (xcomp == 0 ? hr : -hm) : (xcomp == 0 ? hm : hr);
  const T16 h = static_cast<T16>(v);
  whi[e] = bits16(h);
  wlo[e] = bits16(static_cast<T16>(v - static_cast<double>(h)));
}

template <int NP, int PREC, bool PHASE_BY_M2, bool SEL>
__global__ __launch_bounds__(kThreads, 2) void ssca_pass1_mfma(const float2* __restrict__ x, int N, int M2,
                                                              int m2shift, const unsigned* __restrict__ xhi,
                                                              const unsigned* __restrict__ xlo,
                                                              const unsigned short* __restrict__ whi_g,
                                                              const unsigned short* __restrict__ wlo_g,
                                                              const float2* __restrict__ tabs,
                                                              float2* __restrict__ T, int64_t xbs, int64_t pbs,
                                                              int64_t tbs, const ChanSel* __restrict__ sel) {
  using P = Prec<PREC>;
  using V8 = typename P::V8;
  constexpr int S = NP / 16;
  constexpr int D = NP / 2 - 1;
  constexpr int K = 2 * NP;
  constexpr int NSUB = NP / kJS;
  constexpr int kStageFloats = kStageWords;  // one float2 slot per two words
  constexpr int kBufFloats = kStageFloats > kXchgFloats ? kStageFloats : kXchgFloats;
  __shared__ float2 buf[kBufFloats];
  __shared__ float2 tw[1024];
  __shared__ float2 stp[16];
  __shared__ float2 rt[NP];
  unsigned* words = reinterpret_cast<unsigned*>(buf);

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6, g = lane >> 5, lc = lane & 31;
  int m2, u;
  block_to_m2_unit_xcd(M2, m2shift, m2, u);
  if (SEL && u >= sel->nsub) return;
  const int c = SEL ? sel->sub[u] : u;
  x += blockIdx.y * xbs;
  xhi += blockIdx.y * pbs;
  xlo += blockIdx.y * pbs;
  T += blockIdx.y * tbs;
  const float2* rlo = tabs + kTabRotLo;
  const unsigned short* whi = whi_g + c * 32 * K;
  const unsigned short* wlo = wlo_g + c * 32 * K;
  const auto xr = make_rsrc(x, N * 8);
  const int hishift = 10 - m2shift;

  lds_copy<1024, kThreads>(tw, tabs + kTabTw1024, tid);
  lds_copy<NP, kThreads>(rt, tabs + kTabRoots, tid);
  if (tid < 16) stp[tid] = rot_factor(rlo, tabs + kTabTw1024, 64 * m2 * tid, hishift);

  // Sub-chunk s: frames m1 = 256 (s / NSUB) + i (i < 256), samples kJS (s % NSUB) + [0, kJS). Each thread moves
  // 4 x 16 bytes: (frame i, sample group q2 of 4, plane).
  u32x4 pf[4];
  auto issue = [&](int s) {
    const int sbase = (256 * (s / NSUB)) * M2 + m2 - D + (s % NSUB) * kJS + kMfmaPad;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + kThreads * q;  // 0 .. 1023
      const int i = e >> 2, q2 = (e >> 1) & 1, plane = e & 1;
      const unsigned* src = (plane ? xlo : xhi) + sbase + i * M2 + 4 * q2;
      pf[q] = *reinterpret_cast<const u32x4_a4*>(src);
    }
  };
  auto stash = [&](int s) {
    unsigned* b = words + (s & 1) * kStageWords;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + kThreads * q;
      const int i = e >> 2, q2 = (e >> 1) & 1, plane = e & 1;
      *reinterpret_cast<u32x4*>(b + plane * kPlaneWords + i * kRow + 4 * q2) = pf[q];
    }
  };
  issue(0);
  stash(0);
  issue(1);

  float2 col[4][2][8];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    f32x16 acc[2] = {};
#pragma unroll 1
    for (int sub = 0; sub < NSUB; ++sub) {
      const int s = f * NSUB + sub;
      __syncthreads();
      // Weight operand: row lc, K range 16 sub + 8 g .. +8.
      const V8 wh = __builtin_bit_cast(V8, *reinterpret_cast<const u32x4*>(whi + lc * K + 16 * sub + 8 * g));
      V8 wl;
      if constexpr (P::kSplit) wl = __builtin_bit_cast(V8, *reinterpret_cast<const u32x4*>(wlo + lc * K + 16 * sub + 8 * g));
      const unsigned* b = words + (s & 1) * kStageWords;
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int fr = 64 * wave + 32 * u + lc;
        const V8 xh = __builtin_bit_cast(V8, *reinterpret_cast<const u32x4*>(b + fr * kRow + 4 * g));
        acc[u] = P::mfma(wh, xh, acc[u]);
        if constexpr (P::kSplit) {
          const V8 xl = __builtin_bit_cast(V8, *reinterpret_cast<const u32x4*>(b + kPlaneWords + fr * kRow + 4 * g));
          acc[u] = P::mfma(wh, xl, acc[u]);
          acc[u] = P::mfma(wl, xh, acc[u]);
        }
      }
      if (s + 1 < 4 * NSUB) stash(s + 1);
      if (s + 2 < 4 * NSUB) issue(s + 2);
    }
    // acc[u][r]: row 8 (r/4) + 4 g + r%4 of frame 64 w + 32 u + lc; rows 2k' (re), 2k'+1 (im).
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int n = (64 * wave + 32 * u + lc + 256 * f) * M2 + m2;
      const float2 xn = load_c64(xr, n);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const float2 y = make_float2(acc[u][2 * q], acc[u][2 * q + 1]);
        if constexpr (PHASE_BY_M2) {
          col[f][u][q] = cmulc(y, xn);
        } else {
          const int kp = 4 * (q >> 1) + 2 * g + (q & 1);
          col[f][u][q] = cmul(y, cmulc(rt[((c + S * kp) * n) & (NP - 1)], xn));
        }
      }
    }
  }

  // 4-point DFT over f and twiddle omega_1024^{t' r}.
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int tp = 64 * wave + 32 * u + lc;
    const float2 t1 = tw[tp], t2 = tw[2 * tp], t3 = tw[3 * tp];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      float2 a[4] = {col[0][u][q], col[1][u][q], col[2][u][q], col[3][u][q]};
      dft4(a);
      col[0][u][q] = a[0];
      col[1][u][q] = cmul(a[1], t1);
      col[2][u][q] = cmul(a[2], t2);
      col[3][u][q] = cmul(a[3], t3);
    }
  }

  // Two exchanges: half h holds the 8 channels of lane group g == h as sequences b = 4 q + r.
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    __syncthreads();
    if (g == h) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int tp = 64 * wave + 32 * u + lc;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
#pragma unroll
          for (int r = 0; r < 4; ++r) buf[(q * 4 + r) * kSeqStride + tp + (tp >> 4)] = col[r][u][q];
        }
      }
    }
    __syncthreads();
    auto st = [&](int b, int m, float2 v) {
      const int q = b >> 2;
      const int kp = 4 * (q >> 1) + 2 * h + (q & 1);
      const int k = c + S * kp;
      const int rj = (b & 3) + 4 * (m & 15);
      float2 base = rot_factor(rlo, tw, m2 * rj, hishift);
      if constexpr (PHASE_BY_M2) base = cmul(base, rt[(k * m2) & (NP - 1)]);
      const int i = m >> 4;
      st1_nt(T + ((k * (kM1 / 16) + (rj >> 4)) * M2 + m2) * 16 + (rj & 15) + i * (64 * M2), cmul(v, cmul(base, stp[i])));
    };
    NoLoad ld;
    lds_fft<kSeq, kHalfSeqs, kThreads, false, LdsLayout<kSeqStride, 1, 4>>(buf, tw, tid, ld, st);
  }
}

// Paired form (32 <= Np <= 128). One workgroup of 512 threads computes the subsets c and c + Np/32 of one
// m2, so every x sample it loads serves 32 channels. Wave w owns frames t' = 32 w + (lane mod 32) of each
// 256-frame group and reads their 16-bit samples straight from the plane (no LDS staging); in the split forms
// the plane interleaves each sample's hi and lo words, so at each K-step the two lanes of a frame load one
// 64-byte run holding both operands, and consecutive K-steps continue along the same line. Each K-step's weights (both subsets, hi and lo) are loaded once and serve the wave's four frame
// tiles. After the channelizer, threads 256 s .. 256 s + 255 run subset s's 256-point DFTs in LDS
// exactly as the single-subset form; the rotation comes from a per-workgroup LDS table.
constexpr int kPairThreads = 512;
#ifndef KUNROLL
#define KUNROLL 2
#endif

// Weights of the paired form: W[c][kappa][row][16] (one K-step's 32 rows contiguous); lane group g of K-step
// kappa holds, for v < 8, component v % 2 of sample 8 kappa + 4 g + v / 2.
template <int PREC>
__global__ void mfma_weights_pair_kernel(const float* __restrict__ win, int Np, int S, unsigned short* __restrict__ whi,
                                         unsigned short* __restrict__ wlo) {
  using T16 = typename Prec<PREC>::T16;
  const int nks = Np / 8;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= S * nks * 512) return;
  const int kk = e & 15, row = (e >> 4) & 31, kap = (e >> 9) % nks, c = (e >> 9) / nks;
  const int g = kk >> 3, v = kk & 7;
  const int j = 8 * kap + 4 * g + (v >> 1), xcomp = v & 1;
  const int kp = row >> 1, comp = row & 1;
  const int ch = c + S * kp;
  double sn, co;
  sincospi(-2.0 * static_cast<double>((ch * j) & (Np - 1)) / static_cast<double>(Np), &sn, &co);
  const double hr = static_cast<double>(win[j]) * co, hm = static_cast<double>(win[j]) * sn;
  const double val = (comp == 0) ? (xcomp == 0 ? hr : -hm) : (xcomp == 0 ? hm : hr);
  const T16 h = static_cast<T16>(val);
  whi[e] = bits16(h);
  wlo[e] = bits16(static_cast<T16>(val - static_cast<double>(h)));
}

template <int NP, int PREC, bool PHASE_BY_M2, bool SEL>
__global__ __launch_bounds__(kPairThreads, 1) void ssca_pass1_mfma_pair(
    const float2* __restrict__ x, int N, int M2, int m2shift, const unsigned* __restrict__ xhi,
    const unsigned* __restrict__ xlo, const unsigned short* __restrict__ whi_g, const unsigned short* __restrict__ wlo_g,
    const float2* __restrict__ tabs, float2* __restrict__ T, int64_t xbs, int64_t pbs, int64_t tbs,
    const ChanSel* __restrict__ sel) {
  using P = Prec<PREC>;
  using V8 = typename P::V8;
  constexpr int S = NP / 16;
  constexpr int D = NP / 2 - 1;
  constexpr int NKS = NP / 8;  // K-steps of 16 reals
  static_assert(NP >= 32 && NP <= 128, "the paired MFMA form covers 32 <= Np <= 128");
  __shared__ float2 buf[2 * kXchgFloats];
  __shared__ float2 tw[kSeq];
  __shared__ float2 rot[kM1];
  __shared__ float2 rt[NP];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6, g = lane >> 5, lc = lane & 31;
  const int half = tid >> 8, t = tid & 255;
  int m2, u;
  block_to_m2_unit_xcd(M2, m2shift, m2, u);
  if (SEL && u >= sel->npair) return;
  const int cg = SEL ? sel->pair[u] : u;
  x += blockIdx.y * xbs;
  xhi += blockIdx.y * pbs;
  (void)xlo;  // the paired form reads the interleaved plane (hi and lo words) through xhi
  T += blockIdx.y * tbs;
  const auto trs = make_rsrc_u(T, static_cast<unsigned>(NP) * 8u * static_cast<unsigned>(N));  // one signal's T
  const float2* rlo = tabs + kTabRotLo;
  const float2* tw_g = tabs + kTabTw1024;
  const auto xr = make_rsrc(x, N * 8);
  const int hishift = 10 - m2shift;
  lds_copy<kSeq, kPairThreads, 4>(tw, tw_g, tid);
  rot_fill<kPairThreads>(rot, rlo, tw_g, m2, hishift, tid);
  lds_copy<NP, kPairThreads>(rt, tabs + kTabRoots, tid);
  __syncthreads();

  // Weight offsets (elements) of subset cg + sb S/2 at this lane's row and K group; K-step kappa adds 512 kappa.
  const int woff0 = cg * NKS * 512 + lc * 16 + 8 * g;
  const int woff1 = woff0 + (S / 2) * NKS * 512;
  const int tp = 32 * wave + lc;  // frame within each 256-frame group

  // Channelizer: K-step by K-step, each weight load serves the four frame tiles (f) of this wave, whose
  // accumulators acc[f][sb] all stay in registers.
  f32x16 acc[4][2] = {};
#pragma unroll KUNROLL
  for (int kap = 0; kap < NKS; ++kap) {
    const int so = 8 * kap;
    V8 wh[2], wl[2];
#pragma unroll
    for (int sb = 0; sb < 2; ++sb) {
      const int wo = (sb ? woff1 : woff0) + kap * 512;
      wh[sb] = __builtin_bit_cast(V8, *reinterpret_cast<const u32x4*>(whi_g + wo));
      if constexpr (P::kSplit) wl[sb] = __builtin_bit_cast(V8, *reinterpret_cast<const u32x4*>(wlo_g + wo));
    }
    V8 xh[4], xl[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      const int e = ((tp + 256 * f) * M2 + m2) - D + kMfmaPad + 4 * g + so;
      if constexpr (P::kSplit) {
        // interleaved plane: words (hi, lo) of samples e .. e+3
        const u32x4 a = *reinterpret_cast<const u32x4_a4*>(xhi + 2 * e);
        const u32x4 b = *reinterpret_cast<const u32x4_a4*>(xhi + 2 * e + 4);
        xh[f] = __builtin_bit_cast(V8, u32x4{a.x, a.z, b.x, b.z});
        xl[f] = __builtin_bit_cast(V8, u32x4{a.y, a.w, b.y, b.w});
      } else {
        xh[f] = __builtin_bit_cast(V8, u32x4(*reinterpret_cast<const u32x4_a4*>(xhi + e)));
      }
    }
    // Product by product over the 8 accumulators, so consecutive MFMAs are independent.
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
      for (int sb = 0; sb < 2; ++sb) acc[f][sb] = P::mfma(wh[sb], xh[f], acc[f][sb]);
    if constexpr (P::kSplit) {
#pragma unroll
      for (int f = 0; f < 4; ++f)
#pragma unroll
        for (int sb = 0; sb < 2; ++sb) acc[f][sb] = P::mfma(wh[sb], xl[f], acc[f][sb]);
#pragma unroll
      for (int f = 0; f < 4; ++f)
#pragma unroll
        for (int sb = 0; sb < 2; ++sb) acc[f][sb] = P::mfma(wl[sb], xh[f], acc[f][sb]);
    }
  }

  // acc[f][sb][r]: row 8 (r/4) + 4 g + r%4 of frame tp + 256 f; rows 2k' (re), 2k'+1 (im): q = r/2 is channel
  // k' = 4 (q/2) + 2 g + q%2 of subset cg + sb S/2.
  float2 col[4][2][8];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    const int n = (tp + 256 * f) * M2 + m2;
    const float2 xn = load_c64(xr, n);
#pragma unroll
    for (int sb = 0; sb < 2; ++sb) {
      const int cs = cg + sb * (S / 2);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const float2 y = make_float2(acc[f][sb][2 * q], acc[f][sb][2 * q + 1]);
        const int k = cs + S * (4 * (q >> 1) + 2 * g + (q & 1));
        if constexpr (PHASE_BY_M2) col[f][sb][q] = cmul(cmulc(y, xn), rt[(k * m2) & (NP - 1)]);
        else col[f][sb][q] = cmul(y, cmulc(rt[(k * n) & (NP - 1)], xn));
      }
    }
  }

  // 4-point DFT over f and twiddle omega_1024^{t' r}.
  const float2 t1 = tw_g[tp], t2 = tw_g[2 * tp], t3 = tw_g[3 * tp];
#pragma unroll
  for (int sb = 0; sb < 2; ++sb) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      float2 a[4] = {col[0][sb][q], col[1][sb][q], col[2][sb][q], col[3][sb][q]};
      dft4(a);
      col[0][sb][q] = a[0];
      col[1][sb][q] = cmul(a[1], t1);
      col[2][sb][q] = cmul(a[2], t2);
      col[3][sb][q] = cmul(a[3], t3);
    }
  }

  // Exchange h covers channels k' = 8 h .. 8 h + 7 of both subsets: every lane writes its q = 4 h .. 4 h + 3
  // (channel k' = 4 (q/2) + 2 g + q%2) as sequences b = 4 (k' - 8 h) + r of subset sb's buffer, whose 256-point
  // DFTs threads 256 sb .. 256 sb + 255 then take.
  const int chalf = cg + half * (S / 2);
  float2* xb = buf + half * kXchgFloats;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    __syncthreads();
#pragma unroll
    for (int sb = 0; sb < 2; ++sb) {
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        const int kk = 4 * (qq >> 1) + 2 * g + (qq & 1);
#pragma unroll
        for (int r = 0; r < 4; ++r)
          buf[sb * kXchgFloats + (kk * 4 + r) * kSeqStride + tp + (tp >> 4)] = col[r][sb][4 * h + qq];
      }
    }
    __syncthreads();
    // Output m = j + 16 i of sequence b goes to T[k][j / 4 + 4 i][m2][4 (j % 4) + b % 4] (as in the FP32 Stage 1):
    // a per-butterfly lane offset plus a scalar offset of i * 4 M2 * 16 elements.
    auto st = [&](int b, int m, float2 v) {
      const int k = chalf + S * (8 * h + (b >> 2));
      const int jj = m & 15, ii = m >> 4;
      const int m1p = (b & 3) + 4 * jj + 64 * ii;
      const unsigned voff = static_cast<unsigned>((((k * (kM1 / 16) + (jj >> 2)) * M2 + m2) * 16 + 4 * (jj & 3) +
                                                   (b & 3)) * 8);
      const unsigned soff = static_cast<unsigned>(ii) * (4u * 16u * 8u * static_cast<unsigned>(M2));
      store_c64<false>(trs, cmul(v, rot[m1p]), voff, soff);
    };
    NoLoad ld;
    // Wave-local radix-16 stages, as in the paired FP32 Stage 1.
    lds_fft<kSeq, kHalfSeqs, kThreads, false, LdsLayout<kSeqStride, 1, 4>, kSeq, true>(xb, tw, t, ld, st);
  }
}

template <int NP, int PREC>
hipError_t pass1(const float2* x, int N, int M2, int m2shift, const float* win, const float2* tabs, void* scratch,
                 float2* T, int batch, int64_t xbs, int64_t tbs, const SelArg& sel, hipStream_t s) {
  constexpr int S = NP / 16;
  if (sel.nsub <= 0) return hipSuccess;
  const int64_t plane = N + 2 * kMfmaPad;
  unsigned* xhi = static_cast<unsigned*>(scratch);
  unsigned* xlo = xhi + plane * batch;
  unsigned short* whi = reinterpret_cast<unsigned short*>(xlo + plane * batch);
  unsigned short* wlo = whi + S * 32 * 2 * NP;
  const int nw = S * 32 * 2 * NP;
  constexpr bool PAIR = NP >= 32;
  if constexpr (PAIR)
    hipLaunchKernelGGL(mfma_weights_pair_kernel<PREC>, dim3((nw + 255) / 256), dim3(256), 0, s, win, NP, S, whi, wlo);
  else
    hipLaunchKernelGGL(mfma_weights_kernel<PREC>, dim3((nw + 255) / 256), dim3(256), 0, s, win, NP, S, whi, wlo);
  if constexpr (PAIR && Prec<PREC>::kSplit) {
    // one interleaved plane of 2 words per sample, [batch][2 plane] (the hi and lo regions, back to back)
    for (int b = 0; b < batch; ++b)
      hipLaunchKernelGGL((split_x_kernel<PREC, true>), dim3((plane + 255) / 256), dim3(256), 0, s, x + b * xbs, N,
                         xhi + 2 * b * plane, xhi);
  } else {
    for (int b = 0; b < batch; ++b)
      hipLaunchKernelGGL(split_x_kernel<PREC>, dim3((plane + 255) / 256), dim3(256), 0, s, x + b * xbs, N,
                         xhi + b * plane, xlo + b * plane);
  }
  if constexpr (PAIR) {
    if (sel.npair <= 0) return hipSuccess;
    // Strip selection (learned form) is built for the split-bf16 channelizer only.
    if (sel.dev && PREC != SCD_PREC_SPLIT_BF16) return hipErrorInvalidValue;
    dim3 pgrid(M2 * sel.npair, batch);
    // plane stride per signal: 2 plane words (interleaved split forms) or plane words (one 16-bit plane)
    const int64_t pstride = Prec<PREC>::kSplit ? 2 * plane : plane;
    auto pgo = [&](auto kern) {
      hipLaunchKernelGGL(kern, pgrid, dim3(kPairThreads), 0, s, x, N, M2, m2shift, xhi, xlo, whi, wlo, tabs, T, xbs,
                         pstride, tbs, sel.dev);
    };
    if constexpr (PREC == SCD_PREC_SPLIT_BF16) {
      if (sel.dev) {
        if (M2 % NP == 0) pgo(ssca_pass1_mfma_pair<NP, PREC, true, true>);
        else pgo(ssca_pass1_mfma_pair<NP, PREC, false, true>);
        return hipGetLastError();
      }
    }
    if (M2 % NP == 0) pgo(ssca_pass1_mfma_pair<NP, PREC, true, false>);
    else pgo(ssca_pass1_mfma_pair<NP, PREC, false, false>);
    return hipGetLastError();
  } else {
    dim3 grid(M2 * sel.nsub, batch);
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, grid, dim3(kThreads), 0, s, x, N, M2, m2shift, xhi, xlo, whi, wlo, tabs, T, xbs, plane,
                         tbs, sel.dev);
    };
    // Strip selection (learned form) is built for the split-bf16 channelizer only.
    if (sel.dev && PREC != SCD_PREC_SPLIT_BF16) return hipErrorInvalidValue;
    if constexpr (PREC == SCD_PREC_SPLIT_BF16) {
      if (sel.dev) {
        if (M2 % NP == 0) go(ssca_pass1_mfma<NP, PREC, true, true>);
        else go(ssca_pass1_mfma<NP, PREC, false, true>);
        return hipGetLastError();
      }
    }
    if (M2 % NP == 0) go(ssca_pass1_mfma<NP, PREC, true, false>);
    else go(ssca_pass1_mfma<NP, PREC, false, false>);
    return hipGetLastError();
  }
}

template <int PREC>
hipError_t pass1_np(const float2* x, int N, int Np, const float* win, const float2* tabs, void* scratch, float2* T,
                    int batch, int64_t xbs, int64_t tbs, const SelArg& sel, hipStream_t s) {
  const int M2 = N / kM1;
  int m2shift = 0;
  while ((1 << m2shift) < M2) ++m2shift;
  switch (Np) {
    case 16: return pass1<16, PREC>(x, N, M2, m2shift, win, tabs, scratch, T, batch, xbs, tbs, sel, s);
    case 32: return pass1<32, PREC>(x, N, M2, m2shift, win, tabs, scratch, T, batch, xbs, tbs, sel, s);
    case 64: return pass1<64, PREC>(x, N, M2, m2shift, win, tabs, scratch, T, batch, xbs, tbs, sel, s);
    case 128: return pass1<128, PREC>(x, N, M2, m2shift, win, tabs, scratch, T, batch, xbs, tbs, sel, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

size_t ssca_mfma_scratch_bytes(int N, int Np, int batch) {
  const size_t plane = static_cast<size_t>(N) + 2 * kMfmaPad;
  const size_t S = static_cast<size_t>(Np) / 16;
  return 2 * 4 * plane * static_cast<size_t>(batch) + 2 * 2 * S * 32 * 2 * static_cast<size_t>(Np);
}

hipError_t launch_ssca_pass1_mfma(int prec, const float2* x, int N, int Np, const float* win, const float2* tabs,
                                  void* scratch, float2* T, int batch, int64_t xbs, int64_t tbs, const SelArg& sel,
                                  hipStream_t s) {
  switch (prec) {
    case SCD_PREC_SPLIT_BF16: return pass1_np<SCD_PREC_SPLIT_BF16>(x, N, Np, win, tabs, scratch, T, batch, xbs, tbs, sel, s);
    case SCD_PREC_SPLIT_FP16: return pass1_np<SCD_PREC_SPLIT_FP16>(x, N, Np, win, tabs, scratch, T, batch, xbs, tbs, sel, s);
    case SCD_PREC_BF16: return pass1_np<SCD_PREC_BF16>(x, N, Np, win, tabs, scratch, T, batch, xbs, tbs, sel, s);
    case SCD_PREC_FP16: return pass1_np<SCD_PREC_FP16>(x, N, Np, win, tabs, scratch, T, batch, xbs, tbs, sel, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace scd
