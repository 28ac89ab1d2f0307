// Plain FP32 SSCA (Sec. II-C, Eq. (6)-(7)) computed as the paper's SSCA_2DFFT (Sec. III-B, Eq. (10)-(16)),
// with N = M1 * M2, M1 = 1024 and M2 = N / 1024.
//
// Stage 1 (one workgroup per (m2, channel subset or subset pair)): generates the channel-data product X_g
// only where Stage 1 needs it. For every m1 it forms the centred, windowed frame n = m1*M2 + m2 (Eq. (3),
// L = 1), evaluates the 16 channels k = c + S*k' (S = Np/16) of each subset with a pruned DFT, applies the
// down-conversion factor omega_Np^{(k n) mod Np} and the conjugate sample conj(x[n]) (Eq. (6)), and keeps
// X_g(m1, m2, k) in registers. It then takes the M1-point DFT over m1, multiplies by the rotation factor
// omega_N^{m2 m1'} and stores the result to HBM in a blocked layout T[k][m1'/16][m2][m1' % 16], so both this
// store and Stage 2's load move whole 128-byte runs.
//
// Stage 2 (one workgroup per (16 consecutive m1', k)): the M2-point DFT over m2 of the 16 rows, stored at
// S[k][q] with q = m1' + M1*m2' (16 consecutive q per run).
//
// Pruned channel-subset DFT: with the subset's complex window hc[j] = w[j] omega_Np^{(c j) mod Np},
// j = j0 + 16*j1 (j0 < 16, j1 < S) and k = c + S*k',
//   sum_j w[j] x[n-d+j] omega_Np^{k j} = sum_{j0} omega_16^{k' j0} [ sum_{j1} hc[j] x[n-d+j] ],
// so each subset costs one complex-windowed fold of the frame to 16 points plus a 16-point DFT.
#include <type_traits>

#include "scd_device.h"
#include "scd_launch.h"

namespace scd {

namespace {

constexpr int kM1 = 1024;
constexpr int kP1Threads = 256;       // one frame per thread in each chunk of 256 frames
constexpr int kSeq = 256;             // the M1-point DFT is 4 (registers) x 256 (LDS)
constexpr int kSeqStride = kSeq + kSeq / 16;  // one float2 of padding per 16 elements
constexpr int kHalfSeqs = 32;         // 8 channels x 4 residues per LDS exchange
constexpr int kXchgFloats = kHalfSeqs * kSeqStride;
constexpr int kP2Threads = 256;
constexpr int kPairMinBlocks = 256;   // paired Stage-1 grids at least this large (one block per CU)
constexpr int kSingleMinBlocks = 4096;  // single-subset grids this large fill two blocks per CU for eight rounds

// Stage 1. Blocks run m2 fastest (see block_to_m2_unit for how that spreads x over the XCDs' L2 caches). With
// a selection in device memory the grid covers every subset and the workgroups past the selected count exit
// at once, so the host never needs to know the selection. A selected subset writes all its strips to the
// intermediate (Stage 2 reads and writes only the selected ones): a per-strip test on every store cost more
// than the stores it saved. A workgroup computes one channel subset (PAIR
// false: strips k = c mod Np/16) or a subset pair (PAIR true, Np >= 32: subsets c and c + Np/32) for one m2,
// with 256 threads per subset; thread t of a subset owns frames m1 = t + 256 f (f < 4).
//
// Fold: for each group f of 256 frames, lane (frame i, residue j0 = tid % 16) forms
//   A = sum_{j1 < Np/16} hc[j0 + 16 j1] x[n - d + j0 + 16 j1]
// over the rounds that cover the group. A wave's loads cover 4 frames x 16 consecutive samples (whole
// 128-byte lines, straight from L2, with loads for the next rounds kept in flight in a register ring), and
// only 16 folded values per frame (and the frame's own sample x[n]) pass through LDS, where thread t picks up
// frame t's row. In a pair the same loads serve both subsets: with j = j0 + 32 m + 16 e, the 32-channel
// subset c (strips c mod Np/32) is the 32-point DFT of u[j0 + 16 e] = sum_m hc[j0 + 32 m + 16 e] x[...]; its
// even outputs are the 16-point DFT of u[j0] + u[j0 + 16] (subset c) and its odd outputs that of
// (u[j0] - u[j0 + 16]) omega_32^{j0} (subset c + Np/32). Each thread then takes the 16-point DFT and
// multiplies by conj(x[n]) and the down-conversion's constant part (the k'-dependent part is the column shift
// of the fold's LDS row), keeping the 16 channel values in registers.
//
// The M1 = 1024-point DFT over m1 = t + 256 f is a 4-point DFT over f in registers, a twiddle
// omega_1024^{t r}, and a 256-point DFT over t in LDS (two halves of 8 channels), giving m1' = r + 4 s. Its
// last radix stage stores to HBM, multiplying by the rotation factor omega_N^{m2 m1'} from a per-workgroup
// LDS table. These are plain (cached) stores: measured faster than nontemporal ones here, while Stage 2,
// which streams T in and S out once, keeps nontemporal loads and stores.
//
// YM selects the second input of the channel-data product: 0 the auto SCD (conj(x[n]) from the fold), 1 the
// cross SCD (conj(y[n]), Eq. (2) with y != x), 2 the conjugate form (y[n]); the cross forms load y[n].
template <int NP, bool PHASE_BY_M2, bool SEL, bool PAIR, int YM>
__global__ __launch_bounds__(PAIR ? 2 * kP1Threads : kP1Threads, PAIR ? 1 : 2) void ssca_pass1_fp32(
    const float2* __restrict__ x, const float2* __restrict__ y, int N, int xlen, int xoff, int M2, int m2shift,
    const float* __restrict__ win, const float2* __restrict__ tabs, float2* __restrict__ T, int64_t xbs,
    int64_t tbs, const ChanSel* __restrict__ sel) {
  constexpr int S = NP / 16;
  constexpr int D = NP / 2 - 1;
  constexpr int NH = PAIR ? 2 : 1;      // channel subsets per workgroup
  constexpr int NTH = NH * kP1Threads;
  constexpr int NT = NP / 16;           // taps per lane and round
  constexpr int FPR = NTH / 16;         // frames per round
  constexpr int RPG = 256 / FPR;        // rounds per group of 256 frames
  constexpr int NR = 4 * RPG;
  constexpr int PF = 16 / NT < NR ? 16 / NT : NR;  // rounds of loads in flight
  constexpr int kURow = 17;             // LDS row of one frame's folded values (16 + 1 padding)
  constexpr int kUBuf = kP1Threads * kURow;
  static_assert(2 * kUBuf <= kXchgFloats, "fold buffers must fit in the exchange buffer");
  static_assert(!PAIR || NT % 2 == 0, "a subset pair needs Np >= 32");
  __shared__ float2 buf[NH * kXchgFloats];
  __shared__ float2 tw[kSeq];   // omega_256^e
  __shared__ float2 rot[kM1];   // rotation factors omega_N^{m2 m1'} of this m2
  __shared__ float2 rt[NP];

  const int tid = threadIdx.x;
  const int half = PAIR ? (tid >> 8) : 0;
  const int t = tid & (kP1Threads - 1);
  int m2, u;
  // Paired workgroups at M2 = 1024 take a contiguous m2 range per XCD: 3% (Np = 128) and 5% (Np = 256) faster
  // there; at M2 = 512 the same order measured 8% slower, and elsewhere it made no difference.
  if (PAIR && M2 == kM1) block_to_m2_unit_xcd(M2, m2shift, m2, u);
  else block_to_m2_unit(M2, m2shift, m2, u);
  if (SEL && u >= (PAIR ? sel->npair : sel->nsub)) return;
  const int cg = SEL ? (PAIR ? sel->pair[u] : sel->sub[u]) : u;
  const int c = cg + half * (S / 2);  // this thread's subset
  x += blockIdx.y * xbs;
  T += blockIdx.y * tbs;
  const auto trs = make_rsrc_u(T, static_cast<unsigned>(NP) * 8u * static_cast<unsigned>(N));  // one signal's T
  const float2* rlo = tabs + kTabRotLo;
  // x holds xlen samples and the block starts at xoff (0 and N for a whole signal): frames at the block's
  // edges read the neighbouring samples, and only samples outside x read as zero.
  const auto xr = make_rsrc(x, xlen * 8);
  const int hishift = 10 - m2shift;

  const float2* tw_g = tabs + kTabTw1024;
  lds_copy<kSeq, NTH, 4>(tw, tw_g, tid);
  rot_fill<NTH>(rot, rlo, tw_g, m2, hishift, tid);
  if constexpr (!PHASE_BY_M2) lds_copy<NP, NTH>(rt, tabs + kTabRoots, tid);

  const int j0 = tid & 15, fi = tid >> 4;
  float2 hl[NT];  // the subset's complex window w[j] omega_Np^{(cg j) mod Np} at j = j0 + 16 j1
#pragma unroll
  for (int j1 = 0; j1 < NT; ++j1) {
    const int j = j0 + 16 * j1;
    hl[j1] = cscale(tabs[kTabRoots + ((cg * j) & (NP - 1))], win[j]);
  }
  const float2 w32 = tw_g[32 * j0];  // omega_32^{j0}
  // The down-conversion factor of frame n splits as omega_Np^{(c + S k') n} = omega_Np^{c n} omega_16^{k' n}. Its
  // k'-dependent part is a cyclic shift of the 16-point DFT's input by n, applied by storing residue j0 at column
  // (j0 + n) mod 16; the constant part omega_Np^{c n} goes into conj(x[n]). When Np divides M2, n = m2 (mod Np)
  // for every frame, so both are fixed for the workgroup; otherwise the column follows each round's frame and
  // the constant each thread's frame.
  const int jcol = PHASE_BY_M2 ? ((j0 + m2) & 15) : (j0 + fi * M2 + m2);
  const float2 cphase = PHASE_BY_M2 ? tabs[kTabRoots + ((c * m2) & (NP - 1))] : make_float2(1.f, 0.f);
  // Round g folds frames m1 = FPR g + fi; its NT samples sit at x[base + 16 j1].
  const int base0 = xoff + fi * M2 + m2 - D + j0;
  float2 ring[PF][NT];
  auto issue = [&](int g) {
#pragma unroll
    for (int j1 = 0; j1 < NT; ++j1) ring[g % PF][j1] = load_c64(xr, base0 + FPR * g * M2 + 16 * j1);
  };
#pragma unroll
  for (int g = 0; g < PF; ++g) issue(g);

  float2 col[4][16];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    float2* ub = buf + (f & 1) * NH * kUBuf;
#pragma unroll
    for (int r = 0; r < RPG; ++r) {
      const int g = RPG * f + r;
      // the column of frame m1 = 256 f + FPR r + fi, n = m1 M2 + m2
      const int row = (FPR * r + fi) * kURow + (PHASE_BY_M2 ? jcol : ((jcol + (256 * f + FPR * r) * M2) & 15));
      // Tap j = D of frame m1 is the frame's own sample x[n] (n - D + j = n): the lane of residue D mod 16
      // holds it as tap D / 16 and parks it in the row's padding slot for the channel-data product.
      if (YM == 0 && j0 == (D & 15)) ub[(FPR * r + fi) * kURow + 16] = ring[g % PF][D >> 4];
      if constexpr (PAIR) {
        float2 ea = cmul(hl[0], ring[g % PF][0]);
        float2 eb = cmul(hl[1], ring[g % PF][1]);
#pragma unroll
        for (int j1 = 2; j1 < NT; j1 += 2) {
          ea = cfma(ea, hl[j1], ring[g % PF][j1]);
          eb = cfma(eb, hl[j1 + 1], ring[g % PF][j1 + 1]);
        }
        if (g + PF < NR) issue(g + PF);
        ub[row] = cadd(ea, eb);
        ub[kUBuf + row] = cmul(csub(ea, eb), w32);
      } else {
        float2 acc = cmul(hl[0], ring[g % PF][0]);
#pragma unroll
        for (int j1 = 1; j1 < NT; ++j1) acc = cfma(acc, hl[j1], ring[g % PF][j1]);
        if (g + PF < NR) issue(g + PF);
        ub[row] = acc;
      }
    }
    __syncthreads();
    float2 u[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) u[j] = ub[half * kUBuf + t * kURow + j];
    dft16(u);
    const int n = (t + 256 * f) * M2 + m2;
    float2 xn;  // the sample whose conjugate the channel-data product takes
    if constexpr (YM == 0) {
      xn = ub[t * kURow + 16];
    } else {
      xn = load_c64(make_rsrc(y + blockIdx.y * xbs, N * 8), n);
      if constexpr (YM == 2) xn = cconj(xn);
    }
    // x[n] conj(omega_Np^{c n})
    const float2 xp = cmulc(xn, PHASE_BY_M2 ? cphase : rt[(c * n) & (NP - 1)]);
#pragma unroll
    for (int kp = 0; kp < 16; ++kp) col[f][kp] = cmulc(u[kp], xp);
  }

  // 4-point DFT over f and twiddle omega_1024^{t r}: col[r][k'] now holds residue r of channel k'.
  const float2 t1 = tw_g[t], t2 = tw_g[2 * t], t3 = tw_g[3 * t];
#pragma unroll
  for (int kp = 0; kp < 16; ++kp) {
    float2 a[4] = {col[0][kp], col[1][kp], col[2][kp], col[3][kp]};
    dft4(a);
    col[0][kp] = a[0];
    col[1][kp] = cmul(a[1], t1);
    col[2][kp] = cmul(a[2], t2);
    col[3][kp] = cmul(a[3], t3);
  }

  float2* xb = buf + half * kXchgFloats;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
#pragma unroll
      for (int r = 0; r < 4; ++r) xb[(kk * 4 + r) * kSeqStride + t + (t >> 4)] = col[r][8 * h + kk];
    }
    __syncthreads();
    if constexpr (SEL && !PAIR) {
      // Stage 2 reads only selected strips: a half whose eight strips k = c + S (8 h + kk) are all unselected
      // skips its DFTs and stores (the whole workgroup: c is uniform). The test comes after the exchange writes,
      // so the half's channel values leave the registers on both paths; skipping the writes as well made this
      // kernel spill.
      unsigned any = 0;
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) {
        const int k = c + S * (8 * h + kk);
        any |= sel->keep[k >> 5] >> (k & 31);
      }
      if (!(any & 1u)) continue;
    }
    // Last radix-16 stage output m = j + 16 i of sequence b = 4 kk + r is m1' = (r + 4 j) + 64 i, stored at
    // T[k][m1' / 16][m2][m1' % 16] = T[k][j / 4 + 4 i][m2][4 (j % 4) + r]: a per-butterfly lane offset plus
    // i * 4 M2 * 16 elements, the latter a scalar offset of the buffer store.
    auto st = [&](int b, int m, float2 v) {
      const int k = c + S * (8 * h + (b >> 2));
      const int jj = m & 15, ii = m >> 4;
      const int m1p = (b & 3) + 4 * jj + 64 * ii;
      const unsigned voff = static_cast<unsigned>((((k * (kM1 / 16) + (jj >> 2)) * M2 + m2) * 16 + 4 * (jj & 3) +
                                                   (b & 3)) * 8);
      const unsigned soff = static_cast<unsigned>(ii) * (4u * 16u * 8u * static_cast<unsigned>(M2));
      store_c64<false>(trs, cmul(v, rot[m1p]), voff, soff);
    };
    // Each 256-point sequence's butterflies stay in one wave in both radix-16 stages, so past the barrier above
    // the stages need no workgroup barrier. That pays in a paired workgroup (one per CU: a barrier stalls the
    // whole CU), not measurably in the single-subset one.
    NoLoad ld;
    lds_fft<kSeq, kHalfSeqs, kP1Threads, false, LdsLayout<kSeqStride, 1, 4>, kSeq, PAIR>(xb, tw, t, ld, st);
  }
}

// Stage 2. A workgroup owns 16 consecutive m1' of channel k: one 128-byte run of the blocked intermediate per
// m2, and one 128-byte run of the output per m2'. Each thread works on pairs of adjacent rows, so every global
// and LDS access moves 16 bytes; element (row b, m) sits at LDS m*16 + b. The stage structure is the
// Stockham one of lds_fft, applied to row pairs: the first stage streams straight from HBM and the last
// stage streams straight to HBM (nontemporal: each byte is touched once). NT threads share the 16 rows; tw
// holds omega_TWN^e for e < TWN.
template <int L, int NS, int NT, int TWN>
__device__ __forceinline__ void p2_stage(const float2* __restrict__ src, float2* __restrict__ dst, float2* buf,
                                         const float2* tw, int tid) {
  constexpr int R = StageRadix<L, NS>::value;
  constexpr int NBF = 8 * (L / R);  // (row pair, butterfly) work items
  constexpr int PER = (NBF + NT - 1) / NT;
  constexpr bool FIRST = NS == 1, LAST = NS * R == L;
  float2 a[PER][R], b[PER][R];
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int bf = tid + p * NT;
    if (NBF % NT == 0 || bf < NBF) {
      const int rp = bf & 7, j = bf >> 3, k = j % NS;
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int m = j + i * (L / R);
        if constexpr (FIRST) {
          ld2_nt(src + m * 16 + 2 * rp, a[p][i], b[p][i]);
        } else {
          const float4 t = *reinterpret_cast<const float4*>(buf + m * 16 + 2 * rp);
          a[p][i] = make_float2(t.x, t.y);
          b[p][i] = make_float2(t.z, t.w);
        }
      }
      if constexpr (NS > 1) {
#pragma unroll
        for (int i = 1; i < R; ++i) {
          const float2 w = tw[(i * k * (TWN / (NS * R))) & (TWN - 1)];
          a[p][i] = cmul(a[p][i], w);
          b[p][i] = cmul(b[p][i], w);
        }
      }
      dft<R>(a[p]);
      dft<R>(b[p]);
    }
  }
  if constexpr (!FIRST) __syncthreads();
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int bf = tid + p * NT;
    if (NBF % NT == 0 || bf < NBF) {
      const int rp = bf & 7, j = bf >> 3, k = j % NS;
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int m = (j / NS) * NS * R + k + i * NS;
        if constexpr (LAST) st2_nt(dst + 2 * rp + kM1 * m, a[p][i], b[p][i]);
        else *reinterpret_cast<float4*>(buf + m * 16 + 2 * rp) = make_float4(a[p][i].x, a[p][i].y, b[p][i].x, b[p][i].y);
      }
    }
  }
  if constexpr (!LAST) __syncthreads();
  if constexpr (!LAST) p2_stage<L, NS * R, NT, TWN>(src, dst, buf, tw, tid);
}

// Stage 2's workgroups of one channel, in launch order w < GX (GX a multiple of 8), to their blocks. The XCDs
// receive workgroups round robin, w = x, x + 8, ... on XCD x; giving XCD x the blocks [x GX/8, (x + 1) GX/8)
// makes each XCD write runs of GX/8 adjacent blocks of a strip instead of single blocks 8 apart.
template <int GX>
__device__ __forceinline__ int xcd_run(unsigned w) {
  static_assert(GX % 8 == 0, "a multiple of the 8 XCDs");
  return static_cast<int>((w & 7u) * (GX / 8) + (w >> 3));
}

// For short strips (M2 <= 64) a block of 16 m1' holds only 16 M2 points, too few for a whole workgroup: one wave
// takes each block, a workgroup takes four blocks of one channel, and LDS holds only the M2 twiddles they use.
// Longer strips give each block the whole workgroup and the 1024-entry table.
template <int M2>
struct P2Shape {
  static constexpr int NT = M2 >= 128 ? kP2Threads : 64;  // threads per block of 16 m1'
  static constexpr int G = kP2Threads / NT;                // blocks per workgroup
  static constexpr int TWN = M2 >= 128 ? 1024 : M2;        // twiddle entries: omega_TWN^e
};

template <int M2>
__global__ __launch_bounds__(kP2Threads) void ssca_pass2_fp32(const float2* __restrict__ T,
                                                             const float2* __restrict__ tabs,
                                                             float2* __restrict__ out, int N, int64_t tbs,
                                                             int64_t obs, const ChanSel* __restrict__ sel) {
  using Sh = P2Shape<M2>;
  __shared__ float2 buf[Sh::G * M2 * 16];
  __shared__ float2 tw[Sh::TWN];
  const int tid = threadIdx.x;
  const int g = tid / Sh::NT;
  const int mb = xcd_run<kM1 / 16 / Sh::G>(blockIdx.x) * Sh::G + g;  // block of 16 consecutive m1'
  if (sel && static_cast<int>(blockIdx.y) >= sel->nch) return;
  const int k = sel ? sel->ch[blockIdx.y] : static_cast<int>(blockIdx.y);
  // Stage 2 keeps plain strided table loops (one load in flight per thread): on the 32 x 32 kernel they
  // measured about 3% faster than lds_copy's all-loads-first fill; the cause was not isolated.
  for (int i = tid; i < Sh::TWN; i += kP2Threads) tw[i] = tabs[kTabTw1024 + i * (1024 / Sh::TWN)];
  __syncthreads();
  const float2* src = T + blockIdx.z * tbs + (static_cast<int64_t>(k) * (kM1 / 16) + mb) * (M2 * 16);
  float2* dst = out + blockIdx.z * obs + static_cast<int64_t>(k) * N + mb * 16;
  p2_stage<M2, 1, Sh::NT, Sh::TWN>(src, dst, buf + g * (M2 * 16), tw, tid % Sh::NT);
}

// Stage 2 for M2 = 1024 as 32 x 32, with m2 = j + 32 i and m2' = i' + 32 j':
//   X[i' + 32 j'] = sum_j omega_32^{j j'} omega_1024^{j i'} sum_i omega_32^{i i'} x[j + 32 i].
// Thread (row pair rp, j) loads x[j + 32 i] (i < 32) of its two rows straight from HBM, takes both 32-point
// DFTs over i in registers and applies omega_1024^{j i'}. The exchange runs in two halves of i' (16 each,
// 66 KB of LDS); thread (row, i') then takes the 32-point DFT over j and stores X[i' + 32 j'] of its row.
// Two workgroups share a CU, so one workgroup's HBM traffic overlaps another's arithmetic.
constexpr int kP2XStride = 32 * 16 + 16;  // LDS stride of one i': 32 j x 16 rows, plus 16 float2 of padding

__global__ __launch_bounds__(kP2Threads, 2) void ssca_pass2_fp32_32x32(const float2* __restrict__ T,
                                                                      const float2* __restrict__ tabs,
                                                                      float2* __restrict__ out, int N, int64_t tbs,
                                                                      int64_t obs, const ChanSel* __restrict__ sel) {
  __shared__ float2 buf[16 * kP2XStride];
  __shared__ float2 tw[1024];
  const int tid = threadIdx.x;
  const int mb = xcd_run<kM1 / 16>(blockIdx.x);  // block of 16 consecutive m1'
  if (sel && static_cast<int>(blockIdx.y) >= sel->nch) return;
  const int k = sel ? sel->ch[blockIdx.y] : static_cast<int>(blockIdx.y);
  for (int i = tid; i < 1024; i += kP2Threads) tw[i] = tabs[kTabTw1024 + i];  // plain loop (see ssca_pass2_fp32)
  const float2* src = T + blockIdx.z * tbs + (static_cast<int64_t>(k) * (kM1 / 16) + mb) * (1024 * 16);
  // S[k][q] of this workgroup's rows: q = 16 mb + row + 1024 (i' + 32 j'), through a buffer over strip k.
  const auto ors = make_rsrc_u(out + blockIdx.z * obs + static_cast<int64_t>(k) * N, 8u * static_cast<unsigned>(N));
  const int rp = tid & 7, j = tid >> 3;
  float2 a[32], b[32];
#pragma unroll
  for (int i = 0; i < 32; ++i) ld2_nt(src + (j + 32 * i) * 16 + 2 * rp, a[i], b[i]);
  dft32(a);
  dft32(b);
  __syncthreads();
#pragma unroll
  for (int ip = 1; ip < 32; ++ip) {
    const float2 w = tw[(j * ip) & 1023];
    a[ip] = cmul(a[ip], w);
    b[ip] = cmul(b[ip], w);
  }
  const int row = tid & 15, ipl = tid >> 4;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (h) __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q)
      *reinterpret_cast<float4*>(buf + q * kP2XStride + j * 16 + 2 * rp) =
          make_float4(a[16 * h + q].x, a[16 * h + q].y, b[16 * h + q].x, b[16 * h + q].y);
    __syncthreads();
    float2 v[32];
#pragma unroll
    for (int jj = 0; jj < 32; ++jj) v[jj] = buf[ipl * kP2XStride + jj * 16 + row];
    dft32(v);
    const int ip = 16 * h + ipl;
    const unsigned voff = static_cast<unsigned>(mb * 16 + row + kM1 * ip) * 8u;
#pragma unroll
    for (int jp = 0; jp < 32; ++jp) store_c64<true>(ors, v[jp], voff, static_cast<unsigned>(jp) * (32u * kM1 * 8u));
  }
}

template <int NP>
hipError_t pass1(const float2* x, int N, int M2, int m2shift, const float* win, const float2* tabs,
                 float2* T, int batch, int64_t xbs, int64_t tbs, const SelArg& sel, hipStream_t s,
                 const float2* y, int ymode, int xlen, int xoff) {
  if (sel.nsub <= 0) return hipSuccess;
  if (ymode != 0 && sel.dev) return hipErrorInvalidValue;  // the cross forms run on every strip
  // Subset pairs halve the x traffic and the fold work per strip, but a paired workgroup holds 256 KB of
  // channel values and fills a CU alone, so every CU computes and then stores its intermediate in step with the
  // others and the stores hardly overlap any arithmetic (at N = 2^20, Np = 64: 0.243 ms, of which 0.100 ms
  // comes back when the stores are left out). Two single-subset workgroups share a CU and overlap one's stores
  // with the other's arithmetic (0.216 ms, 0.033 ms of it stores), which outweighs the extra fold work once the
  // single-subset grid fills the GPU for several rounds. Pairs serve the grids in between, and grids too small to
  // give every CU a paired workgroup (e.g. short segments) run single subsets.
  auto go = [&](auto kern, bool pair) {
    dim3 grid(M2 * (pair ? sel.npair : sel.nsub), batch);
    hipLaunchKernelGGL(kern, grid, dim3((pair ? 2 : 1) * kP1Threads), 0, s, x, y, N, xlen, xoff, M2, m2shift, win,
                       tabs, T, xbs, tbs, sel.dev);
  };
  auto launch_phase = [&](auto pair_tag, auto phase_tag) {
    constexpr bool PAIR = decltype(pair_tag)::value;
    constexpr bool PH = decltype(phase_tag)::value;
    if (sel.dev) go(ssca_pass1_fp32<NP, PH, true, PAIR, 0>, PAIR);
    else if (ymode == 1) go(ssca_pass1_fp32<NP, PH, false, PAIR, 1>, PAIR);
    else if (ymode == 2) go(ssca_pass1_fp32<NP, PH, false, PAIR, 2>, PAIR);
    else go(ssca_pass1_fp32<NP, PH, false, PAIR, 0>, PAIR);
  };
  auto launch = [&](auto pair_tag) {
    if (M2 % NP == 0) launch_phase(pair_tag, std::true_type{});
    else launch_phase(pair_tag, std::false_type{});
  };
  if constexpr (NP >= 32) {
    const int64_t single_blocks = static_cast<int64_t>(M2) * sel.nsub * batch;
    const int64_t pair_blocks = static_cast<int64_t>(M2) * sel.npair * batch;
    // A pair computes both its subsets, so a selection that leaves pairs half used runs single subsets. At
    // Np >= 128 a lane folds Np/16 >= 8 taps, and the pair's shared fold wins at every grid measured (N = 2^18 to
    // 2^20: 10-20% faster at Np = 128, 27-30% at Np = 256). At Np = 32 and 64 pairs won by 7-14% on grids of up
    // to 2048 single-subset blocks (Np = 32 at N = 2^18..2^20, Np = 64 at 2^17..2^19); at 4096 (Np = 64,
    // N = 2^20) the two measured equal or single subsets faster.
    const bool pairs_full = sel.nsub >= 2 * sel.npair;
    const bool pairs_pay = NP >= 128 || single_blocks < kSingleMinBlocks;
    if (pairs_full && pairs_pay && pair_blocks >= kPairMinBlocks) launch(std::true_type{});
    else launch(std::false_type{});
  } else {
    launch(std::false_type{});
  }
  return hipGetLastError();
}

template <int M2>
hipError_t pass2(const float2* T, const float2* tabs, float2* out, int N, int batch, int64_t tbs, int64_t obs,
                 const SelArg& sel, hipStream_t s) {
  if (sel.nch <= 0) return hipSuccess;
  if constexpr (M2 == 1024) {
    dim3 grid(kM1 / 16, sel.nch, batch);
    hipLaunchKernelGGL(ssca_pass2_fp32_32x32, grid, dim3(kP2Threads), 0, s, T, tabs, out, N, tbs, obs, sel.dev);
  } else {
    dim3 grid(kM1 / 16 / P2Shape<M2>::G, sel.nch, batch);
    hipLaunchKernelGGL(ssca_pass2_fp32<M2>, grid, dim3(kP2Threads), 0, s, T, tabs, out, N, tbs, obs, sel.dev);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_ssca_pass1_fp32(const float2* x, int N, int Np, const float* win, const float2* tabs,
                                  float2* T, int batch, int64_t xbs, int64_t tbs, const SelArg& sel, hipStream_t s,
                                  const float2* y, int ymode, int xlen, int xoff) {
  if (xlen == 0) xlen = N;
  const int M2 = N / kM1;
  int m2shift = 0;
  while ((1 << m2shift) < M2) ++m2shift;
  switch (Np) {
    case 16: return pass1<16>(x, N, M2, m2shift, win, tabs, T, batch, xbs, tbs, sel, s, y, ymode, xlen, xoff);
    case 32: return pass1<32>(x, N, M2, m2shift, win, tabs, T, batch, xbs, tbs, sel, s, y, ymode, xlen, xoff);
    case 64: return pass1<64>(x, N, M2, m2shift, win, tabs, T, batch, xbs, tbs, sel, s, y, ymode, xlen, xoff);
    case 128: return pass1<128>(x, N, M2, m2shift, win, tabs, T, batch, xbs, tbs, sel, s, y, ymode, xlen, xoff);
    case 256: return pass1<256>(x, N, M2, m2shift, win, tabs, T, batch, xbs, tbs, sel, s, y, ymode, xlen, xoff);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_ssca_pass2(const float2* T, int N, int Np, const float2* tabs, float2* out, int batch, int64_t tbs,
                             int64_t obs, const SelArg& sel, hipStream_t s) {
  (void)Np;
  switch (N / kM1) {
    case 1: return hipSuccess;
    case 2: return pass2<2>(T, tabs, out, N, batch, tbs, obs, sel, s);
    case 4: return pass2<4>(T, tabs, out, N, batch, tbs, obs, sel, s);
    case 8: return pass2<8>(T, tabs, out, N, batch, tbs, obs, sel, s);
    case 16: return pass2<16>(T, tabs, out, N, batch, tbs, obs, sel, s);
    case 32: return pass2<32>(T, tabs, out, N, batch, tbs, obs, sel, s);
    case 64: return pass2<64>(T, tabs, out, N, batch, tbs, obs, sel, s);
    case 128: return pass2<128>(T, tabs, out, N, batch, tbs, obs, sel, s);
    case 256: return pass2<256>(T, tabs, out, N, batch, tbs, obs, sel, s);
    case 512: return pass2<512>(T, tabs, out, N, batch, tbs, obs, sel, s);
    case 1024: return pass2<1024>(T, tabs, out, N, batch, tbs, obs, sel, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace scd
