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
constexpr int kHcFloats = 16 * 256;  // complex windows of every channel subset (S * Np <= 4096)

// Channelizer precisions (values of scd_precision in scd.h).
constexpr int SCD_PREC_FP32 = 0;
constexpr int SCD_PREC_SPLIT_BF16 = 1;
constexpr int SCD_PREC_SPLIT_FP16 = 2;
constexpr int SCD_PREC_BF16 = 3;
constexpr int SCD_PREC_FP16 = 4;
constexpr int kMfmaPad = 256;  // zero samples on each side of the 16-bit copies of x

hipError_t launch_gen_roots(float2* dst, int count, int M, hipStream_t stream);

// SSCA Stage 1 (channelizer + CDP + M1-point DFT + rotation) of `batch` signals. x: [batch][N] at stride xbs;
// T: [batch] blocked intermediates [Np][M1/16][M2][16] at stride tbs (float2 elements). With N == 1024 the
// intermediate layout equals the output layout [Np][N]. hc: kHcFloats float2 of device scratch that this call
// fills with the subsets' complex windows before stage 1 reads them.
hipError_t launch_ssca_pass1_fp32(const float2* x, int N, int Np, const float* win, const float2* tabs, float2* hc,
                                  float2* T, int batch, int64_t xbs, int64_t tbs, hipStream_t stream);

// SSCA Stage 1 with the channelizer on MFMA in 16-bit (split or plain) precision, Np <= 128. scratch: device
// memory of ssca_mfma_scratch_bytes(N, Np, batch) bytes for the 16-bit copies of x and the DFT weights,
// filled by this call. Other arguments as launch_ssca_pass1_fp32.
size_t ssca_mfma_scratch_bytes(int N, int Np, int batch);
hipError_t launch_ssca_pass1_mfma(int prec, const float2* x, int N, int Np, const float* win, const float2* tabs,
                                  void* scratch, float2* T, int batch, int64_t xbs, int64_t tbs, hipStream_t stream);

// SSCA Stage 2 (M2-point DFT over m2) of `batch` intermediates into out: [batch][Np][N] at stride obs. A no-op
// when N == 1024.
hipError_t launch_ssca_pass2(const float2* T, int N, int Np, const float2* tabs, float2* out, int batch,
                             int64_t tbs, int64_t obs, hipStream_t stream);

// FAM of `batch` signals. x: [batch][P*L] at stride xbs; xt: [batch][Np][P] scratch; out: [batch][Np][Np][P].
hipError_t launch_fam_fp32(const float2* x, int Np, int L, int P, const float* win, const float2* tabs,
                           float2* xt, float2* out, int batch, int64_t xbs, int64_t obs, hipStream_t stream);

}  // namespace scd
