// Streaming SSCA receiver (the C-ABI scd_receiver_* calls): estimates a continuous stream of host blocks of N
// samples in fixed device memory, each block with its true neighbouring samples at its edges.
//
// Device ring: [H | slot 0 | slot 1 | ... | slot R-1 | H], H = Np samples, each slot N samples. Block c goes to
// slot c mod R with one host-to-device copy. A block's left and right neighbours sit in the adjacent slots, so
// its edge frames (reaching Np/2 - 1 samples left and Np/2 right) read the true samples without any copy, except
// across the ring's wrap: when block c lands in slot 0, the last H samples of block c - 1 (slot R-1) are copied
// into the zone before slot 0, and the first H samples of block c into the zone after slot R-1. The estimate of
// block c - 1 (scd_ssca_block_ex over its slot and halos, into one of the caller's output buffers in rotation) is
// enqueued on the compute stream once block c's copies have landed. Before the copy of block c, push waits on
// the host for the estimate of block c + 1 - R, the last one that reads the memory the copy overwrites; with
// R >= 4 the copy then runs while the estimate of the block before is still computing. The wait is on the host,
// not a stream-side wait in front of the copy: with a pending cross-stream wait the runtime held the host inside
// the copy call (0.45 ms per 8 MiB block on some systems) and left a gap between estimates.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "scd.h"
#include "scd_launch.h"

struct scd_receiver {
  int device;
  int64_t N;
  int Np, H, slots;
  const float* win;
  std::vector<float*> outs;  // caller-owned output buffers, [Np][N] complex each
  float2* ring;              // library-owned: 2 H + slots * N complex
  hipStream_t compute;       // the caller's stream
  hipStream_t copy;          // the receiver's copy stream (default priority)
  std::vector<hipEvent_t> copied, estimated;  // per block, indexed by block mod slots
  int64_t count;
};

namespace {

float2* slot_ptr(const scd_receiver* r, int64_t c) { return r->ring + r->H + (c % r->slots) * r->N; }

// Estimate block b into output buffer b mod n_outputs, after block `after`'s copies (b + 1, or b itself for the
// last block).
int estimate(scd_receiver* r, int64_t b, int64_t after, int* out_index, int64_t* offset) {
  hipError_t e = hipStreamWaitEvent(r->compute, r->copied[after % r->slots], 0);
  if (e != hipSuccess) return scd::set_hip_error(e, "receiver: wait for copy");
  const int oi = static_cast<int>(b % static_cast<int64_t>(r->outs.size()));
  scd_opts o{};
  o.stream = r->compute;
  const float* x = reinterpret_cast<const float*>(slot_ptr(r, b) - r->H);
  const int rc = scd_ssca_block_ex(x, r->N + 2 * r->H, r->H, r->N, r->Np, r->win, r->outs[oi], &o);
  if (rc) return rc;
  e = hipEventRecord(r->estimated[b % r->slots], r->compute);
  if (e != hipSuccess) return scd::set_hip_error(e, "receiver: record estimate");
  if (out_index) *out_index = oi;
  if (offset) *offset = b * r->N;
  return SCD_OK;
}

void release(scd_receiver* r) {
  for (auto ev : r->copied) (void)hipEventDestroy(ev);
  for (auto ev : r->estimated) (void)hipEventDestroy(ev);
  if (r->copy) (void)hipStreamDestroy(r->copy);
  if (r->ring) (void)hipFree(r->ring);
  delete r;
}

}  // namespace

extern "C" {

int scd_receiver_create(int64_t N, int Np, const float* win, int slots, float* const* outputs, int n_outputs,
                        void* stream, scd_receiver** rx) {
  if (!rx) return scd::set_error(SCD_ERR_NULL, "NULL receiver handle");
  *rx = nullptr;
  if (!win || !outputs) return scd::set_error(SCD_ERR_NULL, "NULL argument");
  if (N < 1024 || N > (1 << 20) || (N & (N - 1)))
    return scd::set_error(SCD_ERR_SIZE, "N must be a power of two in [2^10, 2^20]");
  if (Np < 16 || Np > 256 || (Np & (Np - 1)))
    return scd::set_error(SCD_ERR_SIZE, "Np must be a power of two in [16, 256]");
  if (slots < 3 || slots > 64) return scd::set_error(SCD_ERR_SIZE, "slots must lie in [3, 64]");
  if (n_outputs < 1 || n_outputs > 64) return scd::set_error(SCD_ERR_SIZE, "n_outputs must lie in [1, 64]");
  for (int i = 0; i < n_outputs; ++i)
    if (!outputs[i]) return scd::set_error(SCD_ERR_NULL, "NULL output buffer");
  auto* r = new scd_receiver{};
  r->N = N;
  r->Np = Np;
  r->H = Np;
  r->slots = slots;
  r->win = win;
  r->outs.assign(outputs, outputs + n_outputs);
  r->compute = static_cast<hipStream_t>(stream);
  hipError_t e = hipGetDevice(&r->device);
  const size_t ring_bytes = sizeof(float2) * (2 * static_cast<size_t>(r->H) + static_cast<size_t>(slots) * N);
  if (e == hipSuccess) e = hipMalloc(&r->ring, ring_bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    release(r);
    return scd::set_error(SCD_ERR_NOMEM, "receiver: ring allocation failed");
  }
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&r->copy, hipStreamNonBlocking);
  r->copied.assign(slots, nullptr);
  r->estimated.assign(slots, nullptr);
  for (int i = 0; i < slots && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&r->copied[i], hipEventDisableTiming);
  for (int i = 0; i < slots && e == hipSuccess; ++i)
    e = hipEventCreateWithFlags(&r->estimated[i], hipEventDisableTiming);
  // Only the zone before slot 0 needs zeros up front (the first block's left neighbour); finish() clears the
  // last block's right halo itself.
  if (e == hipSuccess) e = hipMemsetAsync(r->ring, 0, ring_bytes, r->copy);
  if (e == hipSuccess) e = hipStreamSynchronize(r->copy);
  if (e != hipSuccess) {
    const int rc = scd::set_hip_error(e, "receiver set-up");
    release(r);
    return rc;
  }
  *rx = r;
  return SCD_OK;
}

int scd_receiver_push(scd_receiver* r, const float* host_block, int* out_index, int64_t* offset) {
  if (!r || !host_block) return scd::set_error(SCD_ERR_NULL, "NULL argument");
  if (out_index) *out_index = -1;
  const int64_t c = r->count;
  const int64_t N = r->N, H = r->H;
  const int s = static_cast<int>(c % r->slots);
  hipError_t e = hipSuccess;
  if (c + 1 - r->slots >= 0) e = hipEventSynchronize(r->estimated[(c + 1) % r->slots]);
  float2* dst = slot_ptr(r, c);
  if (e == hipSuccess) e = hipMemcpyAsync(dst, host_block, sizeof(float2) * N, hipMemcpyHostToDevice, r->copy);
  if (e == hipSuccess && s == 0 && c >= 1) {
    float2* last = r->ring + H + static_cast<int64_t>(r->slots) * N;  // the zone after slot R-1
    e = hipMemcpyAsync(r->ring, last - H, sizeof(float2) * H, hipMemcpyDeviceToDevice, r->copy);
    if (e == hipSuccess) e = hipMemcpyAsync(last, dst, sizeof(float2) * H, hipMemcpyDeviceToDevice, r->copy);
  }
  if (e == hipSuccess) e = hipEventRecord(r->copied[s], r->copy);
  if (e != hipSuccess) return scd::set_hip_error(e, "receiver: block copy");
  r->count = c + 1;
  return c >= 1 ? estimate(r, c - 1, c, out_index, offset) : SCD_OK;
}

int scd_receiver_finish(scd_receiver* r, int* out_index, int64_t* offset) {
  if (!r) return scd::set_error(SCD_ERR_NULL, "NULL receiver");
  if (out_index) *out_index = -1;
  if (r->count == 0) return SCD_OK;
  const int64_t L = r->count - 1;
  // Nothing follows the last block: its right halo (the next slot's head, or the zone after slot R-1) reads
  // zeros. The copy stream has finished writing there once the last block's copies have landed.
  hipError_t e = hipStreamWaitEvent(r->compute, r->copied[L % r->slots], 0);
  if (e == hipSuccess) e = hipMemsetAsync(slot_ptr(r, L) + r->N, 0, sizeof(float2) * r->H, r->compute);
  if (e != hipSuccess) return scd::set_hip_error(e, "receiver: final halo");
  const int rc = estimate(r, L, L, out_index, offset);
  if (rc) return rc;
  e = hipStreamSynchronize(r->copy);
  if (e != hipSuccess) return scd::set_hip_error(e, "receiver: copies");
  return SCD_OK;
}

int scd_receiver_wait_copy(scd_receiver* r) {
  if (!r) return scd::set_error(SCD_ERR_NULL, "NULL receiver");
  if (r->count == 0) return SCD_OK;
  const hipError_t e = hipEventSynchronize(r->copied[(r->count - 1) % r->slots]);
  if (e != hipSuccess) return scd::set_hip_error(e, "receiver: wait for copies");
  return SCD_OK;
}

int scd_receiver_destroy(scd_receiver* r) {
  if (!r) return SCD_OK;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(r->device);
  (void)hipStreamSynchronize(r->copy);
  (void)hipStreamSynchronize(r->compute);
  release(r);
  (void)hipSetDevice(cur);
  return SCD_OK;
}

}  // extern "C"
