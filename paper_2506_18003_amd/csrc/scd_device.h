// Device-side building blocks shared by the SCD kernels (gfx950, wave64).
//
// * complex float2 arithmetic;
// * forward DFTs of 2, 4, 8 and 16 points held in registers (natural order in and out), with the trivial
//   twiddles of the 8- and 16-point forms written as rotations rather than multiplications;
// * a Stockham-ordered, mixed-radix (16, then 8/4/2) in-LDS FFT over a batch of sequences, whose first stage
//   may read from a caller functor (e.g. straight from HBM) and whose last stage may hand its outputs to a
//   caller functor (e.g. to apply a rotation factor and store to HBM).
//
// Twiddles come from an LDS copy of omega_1024^e = exp(-2 pi i e / 1024), e < 1024, which the host generates
// in FP64 on the GPU (tables.hip); every stage of every transform here is at most 1024 points long.
#pragma once
#include <hip/hip_runtime.h>

namespace scd {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.y, b.x, -a.x * b.y));
}
__device__ __forceinline__ float2 cfma(float2 acc, float2 a, float2 b) {  // acc + a*b
  return make_float2(fmaf(a.x, b.x, fmaf(-a.y, b.y, acc.x)), fmaf(a.x, b.y, fmaf(a.y, b.x, acc.y)));
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
// multiply by -i
__device__ __forceinline__ float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }

// Raw buffer resource over `bytes` bytes at p (gfx9 word 3). Loads through it at byte offsets >= bytes (which
// includes negative element indices converted to unsigned) return zero, so out-of-range samples read as the
// zero padding of the signal without a compare or a fault.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, bytes, 0x00020000);
}

// The complex sample at element index idx (may be negative or past the end: zero then).
__device__ __forceinline__ float2 load_c64(__amdgpu_buffer_rsrc_t r, int idx) {
  // Bit-cast the whole 64-bit result: extracting its two lanes separately let the compiler drop the second
  // dword of the load.
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, static_cast<unsigned>(idx) * 8u, 0, 0));
}

// Raw buffer resource over `bytes` bytes (up to 4 GiB - 1) for stores: 8-byte stores at a per-lane byte offset
// voff plus a wave-uniform byte offset soff. Splitting the address this way keeps the per-store address
// arithmetic out of the vector ALU: a loop-invariant voff per lane, and soff (a compile-time multiple of a
// kernel argument) in a scalar register.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc_u(const void* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, static_cast<int>(bytes), 0x00020000);
}
typedef unsigned int v2u_t __attribute__((ext_vector_type(2)));
template <bool NT>
__device__ __forceinline__ void store_c64(__amdgpu_buffer_rsrc_t r, float2 v, unsigned voff, unsigned soff) {
  // Cache policy bit 1 is the nontemporal hint on gfx950.
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u_t, v), r, static_cast<int>(voff),
                                        static_cast<int>(soff), NT ? 2 : 0);
}

// Streaming (nontemporal) 16-byte global accesses of two adjacent complex values.
typedef float v4f_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void ld2_nt(const float2* p, float2& a, float2& b) {
  const v4f_t t = __builtin_nontemporal_load(reinterpret_cast<const v4f_t*>(p));
  a = make_float2(t.x, t.y);
  b = make_float2(t.z, t.w);
}
__device__ __forceinline__ void st2_nt(float2* p, float2 a, float2 b) {
  const v4f_t t = {a.x, a.y, b.x, b.y};
  __builtin_nontemporal_store(t, reinterpret_cast<v4f_t*>(p));
}
__device__ __forceinline__ void st1_nt(float2* p, float2 a) {
  typedef float v2f_t __attribute__((ext_vector_type(2)));
  const v2f_t t = {a.x, a.y};
  __builtin_nontemporal_store(t, reinterpret_cast<v2f_t*>(p));
}

// LDS table fills. A strided copy loop whose trip count the compiler cannot see waits for each load before
// the next, so a thread that copies R entries pays R memory latencies before its workgroup can start. These
// fills issue every load of a thread first, at indices clamped into range so that no load sits behind a
// branch, and only then write LDS.
//
// dst[i] = src[i * STRIDE] for 0 <= i < N, by NT threads.
template <int N, int NT, int STRIDE = 1>
__device__ __forceinline__ void lds_copy(float2* dst, const float2* __restrict__ src, int tid) {
  constexpr int PER = (N + NT - 1) / NT;
  float2 v[PER];
#pragma unroll
  for (int r = 0; r < PER; ++r) v[r] = src[min(tid + r * NT, N - 1) * STRIDE];
#pragma unroll
  for (int r = 0; r < PER; ++r)
    if (N % NT == 0 || tid + r * NT < N) dst[tid + r * NT] = v[r];
}

// omega_N^a for 0 <= a < N from the two-level table: rlo[e] = omega_N^e and tw[e] = omega_1024^e (e < 1024),
// omega_N^a = omega_N^{a mod 1024} omega_1024^{(a / 1024) 1024 / M2}, with hishift = log2(1024 / M2).
__device__ __forceinline__ int rot_lo(int a) { return a & 1023; }
__device__ __forceinline__ int rot_hi(int a, int hishift) { return ((a >> 10) << hishift) & 1023; }
__device__ __forceinline__ float2 rot_factor(const float2* rlo, const float2* tw, int a, int hishift) {
  return cmul(rlo[rot_lo(a)], tw[rot_hi(a, hishift)]);
}

// rot[i] = omega_N^{m2 i} for i < 1024, by NT threads (NT divides 1024), loads first as in lds_copy.
template <int NT>
__device__ __forceinline__ void rot_fill(float2* rot, const float2* rlo, const float2* tw, int m2, int hishift,
                                         int tid) {
  constexpr int PER = 1024 / NT;
  float2 lo[PER], hi[PER];
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    const int a = m2 * (tid + r * NT);
    lo[r] = rlo[rot_lo(a)];
    hi[r] = tw[rot_hi(a, hishift)];
  }
#pragma unroll
  for (int r = 0; r < PER; ++r) rot[tid + r * NT] = cmul(lo[r], hi[r]);
}

constexpr float kC8 = 0.70710678118654752440f;   // cos(pi/4)
constexpr float kC16 = 0.92387953251128675613f;  // cos(pi/8)
constexpr float kS16 = 0.38268343236508977173f;  // sin(pi/8)

// a * omega_16^E for a compile-time exponent E (omega_16 = exp(-2 pi i / 16)).
template <int E>
__device__ __forceinline__ float2 rot16(float2 a) {
  constexpr int e = ((E % 16) + 16) % 16;
  if constexpr (e == 0) return a;
  else if constexpr (e == 4) return mul_mi(a);
  else if constexpr (e == 8) return make_float2(-a.x, -a.y);
  else if constexpr (e == 12) return make_float2(-a.y, a.x);
  else if constexpr (e == 2) return make_float2((a.x + a.y) * kC8, (a.y - a.x) * kC8);
  else if constexpr (e == 6) return make_float2((a.y - a.x) * kC8, -(a.x + a.y) * kC8);
  else if constexpr (e == 10) return make_float2(-(a.x + a.y) * kC8, (a.x - a.y) * kC8);
  else if constexpr (e == 14) return make_float2((a.x - a.y) * kC8, (a.x + a.y) * kC8);
  else {
    // general: cos(2 pi e/16) - i sin(2 pi e/16), built from cos/sin(pi/8) by quadrant
    constexpr int q = e / 4, r = e % 4;  // r is 1 or 3
    constexpr float c0 = (r == 1) ? kC16 : kS16;
    constexpr float s0 = (r == 1) ? kS16 : kC16;
    // omega_16^r = (c0, -s0); then rotate by (-i)^q
    float2 b = make_float2(fmaf(a.x, c0, a.y * s0), fmaf(a.y, c0, -a.x * s0));
    if constexpr (q == 0) return b;
    else if constexpr (q == 1) return mul_mi(b);
    else if constexpr (q == 2) return make_float2(-b.x, -b.y);
    else return make_float2(-b.y, b.x);
  }
}

__device__ __forceinline__ void dft2(float2* a) {
  float2 t = a[0];
  a[0] = cadd(t, a[1]);
  a[1] = csub(t, a[1]);
}

__device__ __forceinline__ void dft4(float2* a) {
  float2 s02 = cadd(a[0], a[2]), d02 = csub(a[0], a[2]);
  float2 s13 = cadd(a[1], a[3]), d13 = mul_mi(csub(a[1], a[3]));
  a[0] = cadd(s02, s13);
  a[2] = csub(s02, s13);
  a[1] = cadd(d02, d13);
  a[3] = csub(d02, d13);
}

// 4-point DFT of a[o], a[o+s], a[o+2s], a[o+3s], in place.
template <int O, int S>
__device__ __forceinline__ void dft4s(float2* a) {
  float2 t[4] = {a[O], a[O + S], a[O + 2 * S], a[O + 3 * S]};
  dft4(t);
  a[O] = t[0]; a[O + S] = t[1]; a[O + 2 * S] = t[2]; a[O + 3 * S] = t[3];
}

// 8-point DFT = 2 x 4: A[n1][k2] = DFT4_{n2} a[n1 + 2 n2]; A *= w8^{n1 k2}; X[k2 + 4 k1] = DFT2_{n1}.
__device__ __forceinline__ void dft8(float2* a) {
  float2 e[4] = {a[0], a[2], a[4], a[6]};
  float2 o[4] = {a[1], a[3], a[5], a[7]};
  dft4(e);
  dft4(o);
  o[1] = rot16<2>(o[1]);
  o[2] = rot16<4>(o[2]);
  o[3] = rot16<6>(o[3]);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    a[k] = cadd(e[k], o[k]);
    a[k + 4] = csub(e[k], o[k]);
  }
}

// 16-point DFT = 4 x 4: A[n1][k2] = DFT4_{n2} a[n1 + 4 n2]; A *= w16^{n1 k2}; X[k2 + 4 k1] = DFT4_{n1} A.
__device__ __forceinline__ void dft16(float2* a) {
  float2 t[16];
#pragma unroll
  for (int n1 = 0; n1 < 4; ++n1) {
    float2 v[4] = {a[n1], a[n1 + 4], a[n1 + 8], a[n1 + 12]};
    dft4(v);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) t[n1 * 4 + k2] = v[k2];
  }
  t[5] = rot16<1>(t[5]);  t[6] = rot16<2>(t[6]);  t[7] = rot16<3>(t[7]);
  t[9] = rot16<2>(t[9]);  t[10] = rot16<4>(t[10]); t[11] = rot16<6>(t[11]);
  t[13] = rot16<3>(t[13]); t[14] = rot16<6>(t[14]); t[15] = rot16<9>(t[15]);
#pragma unroll
  for (int k2 = 0; k2 < 4; ++k2) {
    float2 v[4] = {t[k2], t[4 + k2], t[8 + k2], t[12 + k2]};
    dft4(v);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) a[k2 + 4 * k1] = v[k1];
  }
}

constexpr float kC32a = 0.98078528040323044913f;  // cos(pi/16)
constexpr float kS32a = 0.19509032201612826785f;  // sin(pi/16)
constexpr float kC32b = 0.83146961230254523708f;  // cos(3 pi/16)
constexpr float kS32b = 0.55557023301960222474f;  // sin(3 pi/16)

// a * omega_32^E for a compile-time exponent E.
template <int E>
__device__ __forceinline__ float2 rot32(float2 a) {
  constexpr int e = ((E % 32) + 32) % 32;
  if constexpr (e % 2 == 0) {
    return rot16<e / 2>(a);
  } else {
    // omega_32^e = cos(pi e/16) - i sin(pi e/16); first-quadrant angle pi r/16 (r odd), then (-i)^q
    constexpr int q = e / 8, r = e % 8;
    constexpr float c0 = r == 1 ? kC32a : r == 3 ? kC32b : r == 5 ? kS32b : kS32a;
    constexpr float s0 = r == 1 ? kS32a : r == 3 ? kS32b : r == 5 ? kC32b : kC32a;
    float2 b = make_float2(fmaf(a.x, c0, a.y * s0), fmaf(a.y, c0, -a.x * s0));
    if constexpr (q == 0) return b;
    else if constexpr (q == 1) return mul_mi(b);
    else if constexpr (q == 2) return make_float2(-b.x, -b.y);
    else return make_float2(-b.y, b.x);
  }
}

template <int K>
__device__ __forceinline__ void rot32_odd_half(float2* o) {
  if constexpr (K < 16) {
    o[K] = rot32<K>(o[K]);
    rot32_odd_half<K + 1>(o);
  }
}

// 32-point DFT = 2 x 16: X[k] = E[k] + omega_32^k O[k], X[k + 16] = E[k] - omega_32^k O[k], with E and O the
// 16-point DFTs of the even and odd samples.
__device__ __forceinline__ void dft32(float2* a) {
  float2 e[16], o[16];
#pragma unroll
  for (int n = 0; n < 16; ++n) {
    e[n] = a[2 * n];
    o[n] = a[2 * n + 1];
  }
  dft16(e);
  dft16(o);
  rot32_odd_half<1>(o);
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    a[k] = cadd(e[k], o[k]);
    a[k + 16] = csub(e[k], o[k]);
  }
}

template <int R>
__device__ __forceinline__ void dft(float2* a) {
  if constexpr (R == 2) dft2(a);
  else if constexpr (R == 4) dft4(a);
  else if constexpr (R == 8) dft8(a);
  else if constexpr (R == 16) dft16(a);
  else if constexpr (R == 32) dft32(a);
  else static_assert(R == 1, "unsupported radix");
}

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }

// Radix of the stage that starts with sub-transform length NS in a length-L transform: 16 while at least
// 4 bits remain, then the remaining 2^b.
template <int L, int NS>
struct StageRadix {
  static constexpr int rem = ilog2(L) - ilog2(NS);
  static constexpr int value = rem >= 4 ? 16 : (1 << rem);
};

// Default LDS addressing: element m of sequence b sits at b*BS + m*MS (+ PAD extra float2 per 16 elements
// along m, which breaks the 16-element stride of radix-16 writes across LDS banks).
template <int BS, int MS, int PADSH = 0>
struct LdsLayout {
  __device__ __forceinline__ static int at(int b, int m) {
    if constexpr (PADSH > 0) return b * BS + (m + (m >> PADSH)) * MS;
    else return b * BS + m * MS;
  }
};

// Block index -> (m2, unit) of a Stage-1 grid of M2 x units blocks: m2 fastest. Blocks go to the 8 XCDs round
// robin, so XCD x works on m2 = x (mod 8): the frames of m2 and m2 + 8 share all but 8 of their samples and the
// concurrently running blocks of one XCD read neighbouring stretches of x from its L2. (A remap giving each XCD a
// contiguous m2 range measured about 3% slower.)
__device__ __forceinline__ void block_to_m2_unit(int M2, int m2shift, int& m2, int& u) {
  m2 = blockIdx.x & (M2 - 1);
  u = blockIdx.x >> m2shift;
}

// Alternative mapping (units a power of two): XCD x (blocks b = x mod 8) takes the contiguous range
// m2 in [x M2/8, (x+1) M2/8) with the units of one m2 adjacent; plain order if M2 < 8. The split-precision
// Stage 1, which reads twice the operand bytes per sample, measured faster with it.
__device__ __forceinline__ void block_to_m2_unit_xcd(int M2, int m2shift, int& m2, int& u) {
  const int b = blockIdx.x;
  const int ushift = __builtin_ctz(gridDim.x >> m2shift);
  if ((M2 & 7) == 0) {
    const int idx = b >> 3;
    m2 = (b & 7) * (M2 >> 3) + (idx >> ushift);
    u = idx & ((1 << ushift) - 1);
  } else {
    m2 = b & (M2 - 1);
    u = b >> m2shift;
  }
}

struct NoLoad {};
struct NoStore {};

// One Stockham stage (radix R, sub-transform length NS) over NB sequences of length L, run by NT threads.
// Butterfly j of sequence b reads elements j + i*L/R (i < R), multiplies element i by
// omega_{NS R}^{i (j mod NS)}, takes an R-point DFT and writes output i to (j/NS)*NS*R + (j mod NS) + i*NS.
// BFAST selects the enumeration of butterflies over threads: sequence index fastest (true) or j fastest.
// All threads read their inputs before the barrier and write after it, so the stage runs in place.
// Ordering between the phases of a stage. WAVE false: a workgroup barrier. WAVE true: only the issuing wave's
// own LDS accesses need ordering (LDS executes one wave's instructions in order), so a compiler fence and a
// wave barrier suffice.
template <bool WAVE>
__device__ __forceinline__ void stage_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

template <int L, int NB, int NT, int NS, bool BFAST, class Lay, int TWN, bool WAVE = false, class LoadF, class StoreF>
__device__ __forceinline__ void stockham_stage(float2* buf, const float2* tw, int tid, LoadF& ld, StoreF& st) {
  static_assert(TWN >= L, "the twiddle table must hold at least L roots");
  constexpr int R = StageRadix<L, NS>::value;
  constexpr int NBF = NB * (L / R);
  constexpr int PER = (NBF + NT - 1) / NT;
  constexpr bool FIRST = (NS == 1);
  constexpr bool LAST = (NS * R == L);
  constexpr bool LOAD_EXT = FIRST && !std::is_same<LoadF, NoLoad>::value;
  constexpr bool STORE_EXT = LAST && !std::is_same<StoreF, NoStore>::value;
  float2 v[PER][R];
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int bf = tid + p * NT;
    if (NBF % NT == 0 || bf < NBF) {
      const int b = BFAST ? (bf % NB) : (bf / (L / R));
      const int j = BFAST ? (bf / NB) : (bf % (L / R));
      const int k = j % NS;
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int m = j + i * (L / R);
        if constexpr (LOAD_EXT) v[p][i] = ld(b, m);
        else v[p][i] = buf[Lay::at(b, m)];
      }
      if constexpr (NS > 1) {
#pragma unroll
        for (int i = 1; i < R; ++i) v[p][i] = cmul(v[p][i], tw[(i * k * (TWN / (NS * R))) & (TWN - 1)]);
      }
      dft<R>(v[p]);
    }
  }
  // In place: every read of the stage before any write. With WAVE and an external store nothing is written.
  if constexpr (!LOAD_EXT && !(WAVE && STORE_EXT)) stage_sync<WAVE>();
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int bf = tid + p * NT;
    if (NBF % NT == 0 || bf < NBF) {
      const int b = BFAST ? (bf % NB) : (bf / (L / R));
      const int j = BFAST ? (bf / NB) : (bf % (L / R));
      const int k = j % NS;
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int m = (j / NS) * NS * R + k + i * NS;
        if constexpr (STORE_EXT) st(b, m, v[p][i]);
        else buf[Lay::at(b, m)] = v[p][i];
      }
    }
  }
  if constexpr (!STORE_EXT) stage_sync<WAVE>();
}

template <int L, int NB, int NT, int NS, bool BFAST, class Lay, int TWN, bool WAVE = false, class LoadF, class StoreF>
__device__ __forceinline__ void stockham_from(float2* buf, const float2* tw, int tid, LoadF& ld, StoreF& st) {
  if constexpr (NS < L) {
    stockham_stage<L, NB, NT, NS, BFAST, Lay, TWN, WAVE>(buf, tw, tid, ld, st);
    constexpr int R = StageRadix<L, NS>::value;
    stockham_from<L, NB, NT, NS * R, BFAST, Lay, TWN, WAVE>(buf, tw, tid, ld, st);
  }
}

// First stage of a length-L transform split in two, so a caller can start the first stage's loads early:
// FirstStage<...>::gather reads its inputs through `ld` into registers; FirstStage<...>::scatter takes the
// R-point DFTs and writes the results to LDS, followed by a barrier. Then stockham_rest runs the remaining
// stages.
template <int L, int NB, int NT, bool BFAST>
struct FirstStage {
  static constexpr int R = StageRadix<L, 1>::value;
  static constexpr int NBF = NB * (L / R);
  static constexpr int PER = (NBF + NT - 1) / NT;
  template <class LoadF>
  __device__ __forceinline__ static void gather(float2 (&v)[PER][R], int tid, LoadF& ld) {
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int bf = tid + p * NT;
      if (NBF % NT == 0 || bf < NBF) {
        const int b = BFAST ? (bf % NB) : (bf / (L / R));
        const int j = BFAST ? (bf / NB) : (bf % (L / R));
#pragma unroll
        for (int i = 0; i < R; ++i) v[p][i] = ld(b, j + i * (L / R));
      }
    }
  }
  // When this stage is the only one (R == L) its outputs go to `st`; otherwise to LDS, then a barrier.
  template <class Lay, class StoreF>
  __device__ __forceinline__ static void scatter(float2 (&v)[PER][R], float2* buf, int tid, StoreF& st) {
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int bf = tid + p * NT;
      if (NBF % NT == 0 || bf < NBF) {
        const int b = BFAST ? (bf % NB) : (bf / (L / R));
        const int j = BFAST ? (bf / NB) : (bf % (L / R));
        dft<R>(v[p]);
#pragma unroll
        for (int i = 0; i < R; ++i) {
          if constexpr (R == L) st(b, i, v[p][i]);
          else buf[Lay::at(b, j * R + i)] = v[p][i];
        }
      }
    }
    if constexpr (R != L) __syncthreads();
  }
};

template <int L, int NB, int NT, bool BFAST, class Lay, int TWN = 1024, class StoreF>
__device__ __forceinline__ void stockham_rest(float2* buf, const float2* tw, int tid, StoreF& st) {
  NoLoad ld;
  stockham_from<L, NB, NT, StageRadix<L, 1>::value, BFAST, Lay, TWN>(buf, tw, tid, ld, st);
}

// Forward DFT of NB length-L sequences (L a power of two, 2 <= L <= 1024), natural order in and out.
// Requires a barrier before the call if the data were just written to LDS by other threads. On return the
// outputs are either in LDS (followed by a barrier) or were handed to `st(b, m, value)`.
// `tw` holds omega_TWN^e for e < TWN (TWN >= L, a power of two).
//
// WAVE true drops the workgroup barriers between and inside the stages. That is valid when every stage has the
// same butterfly count per sequence, L / R <= 64 dividing 64, with sequences enumerated j fastest (BFAST
// false) over a multiple of 64 threads: then the threads of a sequence lie in one wave in every stage, and
// only that wave touches the sequence's LDS. The caller still needs a workgroup barrier before the call if
// other waves wrote the inputs, and after it before the buffer is reused.
template <int L, int NS>
constexpr bool uniform_radix() {
  constexpr int R = StageRadix<L, NS>::value;
  if constexpr (R != StageRadix<L, 1>::value) return false;
  else if constexpr (NS * R >= L) return true;
  else return uniform_radix<L, NS * R>();
}
static_assert(uniform_radix<256, 1>() && uniform_radix<16, 1>() && uniform_radix<4, 1>() && !uniform_radix<32, 1>() &&
                  !uniform_radix<64, 1>() && !uniform_radix<512, 1>() && !uniform_radix<1024, 1>(),
              "uniform_radix: every stage's radix equals the first's");
template <int L, int NB, int NT, bool BFAST, class Lay, int TWN = 1024, bool WAVE = false, class LoadF, class StoreF>
__device__ __forceinline__ void lds_fft(float2* buf, const float2* tw, int tid, LoadF& ld, StoreF& st) {
  static_assert(L >= 2 && L <= 1024 && (L & (L - 1)) == 0, "length must be a power of two in [2, 1024]");
  static_assert(!WAVE || (!BFAST && NT % 64 == 0 && uniform_radix<L, 1>() && 64 % (L / StageRadix<L, 1>::value) == 0),
                "wave-local stages need one wave per sequence in every stage");
  stockham_from<L, NB, NT, 1, BFAST, Lay, TWN, WAVE>(buf, tw, tid, ld, st);
}

}  // namespace scd
