// FP64 generation, on the GPU, of the roots of unity the estimators use.
//
// dst[j] = omega_M^j = exp(-2 pi i j / M) for j < count, evaluated as sincospi(-2 j / M) in double precision
// (j / M is exact in binary for M a power of two, so the only rounding is the FP64 sincospi and the final
// conversion to FP32). This covers the channelizer's down-conversion factors exp(-i 2 pi k n L / Np) (the
// integer exponent is reduced mod Np before lookup), the in-LDS FFT twiddles omega_1024, and the rotation
// factors exp(-i 2 pi m2 m1' / N) of the decomposed N-point DFT (Eq. 10), which a two-level lookup builds as
// omega_N^{a mod 1024} * omega_1024^{(a / 1024) * 1024 / M2}.
#include "scd_launch.h"

namespace scd {

__global__ void gen_roots_kernel(float2* __restrict__ dst, int count, int M) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < count) {
    double s, c;
    sincospi(-2.0 * static_cast<double>(j) / static_cast<double>(M), &s, &c);
    dst[j] = make_float2(static_cast<float>(c), static_cast<float>(s));
  }
}

hipError_t launch_gen_roots(float2* dst, int count, int M, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  const int nt = 256;
  hipLaunchKernelGGL(gen_roots_kernel, dim3((count + nt - 1) / nt), dim3(nt), 0, stream, dst, count, M);
  return hipGetLastError();
}

}  // namespace scd
