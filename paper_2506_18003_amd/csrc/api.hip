// C ABI of the SCD library: argument validation, per-device plan cache of FP64-generated tables, workspace
// management, stream selection and error reporting. All numerical work is in the kernels; this file only
// checks arguments and enqueues launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>

#include "scd.h"
#include "scd_launch.h"

namespace {

thread_local std::string g_err;
std::mutex g_mu;
hipStream_t g_stream = nullptr;

// Library scratch of one stream: only work enqueued on that stream touches it, so calls on different streams
// never share writable memory.
struct Scratch {
  void* work = nullptr;  // SSCA intermediates / FAM X_T
  size_t work_bytes = 0;
  void* aux = nullptr;  // 16-bit copies of x and MFMA weights of the split-precision channelizer
  size_t aux_bytes = 0;
  void* lrn = nullptr;  // segment periodograms of the selector features
  size_t lrn_bytes = 0;
  void* sel = nullptr;  // selector scratch: features, activations, scores, confidence, channel selection
  size_t sel_bytes = 0;
};
// Lanes of scd_ssca_batch: library-owned streams that each run whole items (selector, then SSCA) with their
// own scratch, so short items, whose grids cannot fill the GPU, and selectors overlap other items.
constexpr int kBatchLanes = 4;
struct BatchPipe {
  hipStream_t lane[kBatchLanes] = {};
  hipEvent_t start = nullptr;          // the caller's stream at the start of a batch call
  hipEvent_t end[kBatchLanes] = {};    // each lane's last item of the call
};
struct DevState {
  std::map<std::pair<int64_t, int>, float2*> plans;  // (transform length, Np) -> tables (read-only once built)
  std::map<hipStream_t, Scratch> streams;
  BatchPipe pipe;
};
std::mutex g_batch_mu;  // one scd_ssca_batch call at a time: its side streams and events are per device
// features (2 Np) + standardised features (2 Np) + activations (4 * 256) + logits (Np) + scores (Np) + conf
constexpr int kSelStructFloats = (sizeof(scd::ChanSel) + 3) / 4 + 4;
constexpr int kSelScratchFloats = 4 * 256 + 4 * 256 + 2 * 256 + 64 + kSelStructFloats;
static_assert(2 * 256 + 3 * 256 + 4 * 256 <= kSelScratchFloats - kSelStructFloats - 2, "selector scratch layout");
std::map<int, DevState> g_dev;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  (void)hipGetLastError();
  return fail(SCD_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

bool overlaps(const void* a, size_t an, const void* b, size_t bn) {
  if (an == 0 || bn == 0) return false;
  const uintptr_t a0 = reinterpret_cast<uintptr_t>(a), b0 = reinterpret_cast<uintptr_t>(b);
  return a0 < b0 + bn && b0 < a0 + an;
}

// The GPU may read/write `bytes` starting at p: p is device, managed or pinned-host memory and its
// allocation extends at least that far.
int check_device_range(const void* p, size_t bytes, const char* name) {
  hipPointerAttribute_t attr;
  std::memset(&attr, 0, sizeof(attr));
  hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(SCD_ERR_PTR, "%s is not memory the GPU can access (%s)", name, hipGetErrorString(e));
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged && attr.type != hipMemoryTypeHost &&
      attr.type != hipMemoryTypeUnified) {
    return fail(SCD_ERR_PTR, "%s is not memory the GPU can access", name);
  }
  if (attr.type == hipMemoryTypeDevice) {
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    e = hipMemGetAddressRange(&base, &size, const_cast<void*>(p));
    if (e == hipSuccess && base != nullptr) {
      const uintptr_t end = reinterpret_cast<uintptr_t>(base) + size;
      if (reinterpret_cast<uintptr_t>(p) + bytes > end)
        return fail(SCD_ERR_PTR, "%s: allocation holds %zu bytes from this pointer, %zu needed", name,
                    static_cast<size_t>(end - reinterpret_cast<uintptr_t>(p)), bytes);
    } else {
      (void)hipGetLastError();
    }
  }
  return SCD_OK;
}

// Tables for (transform length n, Np): omega_1024, omega_n^j (j < 1024) and omega_Np. Generated once in FP64
// on the GPU; creation waits for the generation to finish so any stream may use them afterwards.
int get_tables(DevState& st, int64_t n, int Np, hipStream_t s, float2** out) {
  auto key = std::make_pair(n, Np);
  auto it = st.plans.find(key);
  if (it != st.plans.end()) {
    *out = it->second;
    return SCD_OK;
  }
  float2* t = nullptr;
  hipError_t e = hipMalloc(&t, sizeof(float2) * scd::kTabSize);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(SCD_ERR_NOMEM, "table allocation failed: %s", hipGetErrorString(e));
  }
  e = scd::launch_gen_roots(t + scd::kTabTw1024, 1024, 1024, s);
  if (e == hipSuccess) e = scd::launch_gen_roots(t + scd::kTabRotLo, 1024, static_cast<int>(n), s);
  if (e == hipSuccess) e = scd::launch_gen_roots(t + scd::kTabRoots, Np, Np, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    (void)hipFree(t);
    return hip_fail(e, "table generation");
  }
  st.plans[key] = t;
  *out = t;
  return SCD_OK;
}

// Library-owned device buffer of at least `bytes` for work on `stream`, grown on demand (the old one is freed
// once the stream drains, since its queued kernels may still use it).
int grow(void** buf, size_t* have, size_t bytes, hipStream_t stream, void** out) {
  if (bytes == 0) {
    *out = nullptr;
    return SCD_OK;
  }
  if (*have < bytes) {
    if (*buf) {
      hipError_t e = hipStreamSynchronize(stream);
      if (e != hipSuccess) return hip_fail(e, "synchronise before workspace growth");
      (void)hipFree(*buf);
      *buf = nullptr;
      *have = 0;
    }
    hipError_t e = hipMalloc(buf, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      *buf = nullptr;
      return fail(SCD_ERR_NOMEM, "device allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    }
    *have = bytes;
  }
  *out = *buf;
  return SCD_OK;
}

int get_work(DevState& st, hipStream_t s, size_t bytes, void** out) {
  Scratch& c = st.streams[s];
  return grow(&c.work, &c.work_bytes, bytes, s, out);
}
int get_aux(DevState& st, hipStream_t s, size_t bytes, void** out) {
  Scratch& c = st.streams[s];
  return grow(&c.aux, &c.aux_bytes, bytes, s, out);
}
int get_lrn(DevState& st, hipStream_t s, size_t bytes, void** out) {
  Scratch& c = st.streams[s];
  return grow(&c.lrn, &c.lrn_bytes, bytes, s, out);
}
int get_sel(DevState& st, hipStream_t s, size_t bytes, void** out) {
  Scratch& c = st.streams[s];
  return grow(&c.sel, &c.sel_bytes, bytes, s, out);
}

int current_device(int* dev) {
  hipError_t e = hipGetDevice(dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  return SCD_OK;
}

struct Resolved {
  int precision = SCD_FP32;
  int batch = 1;
  int64_t xs = 0, os = 0;
  hipStream_t stream = nullptr;
  void* work = nullptr;
  size_t work_bytes = 0;
};

int resolve(const scd_opts* o, int64_t xlen, int64_t olen, Resolved* r) {
  r->stream = g_stream;
  r->xs = xlen;
  r->os = olen;
  if (!o) return SCD_OK;
  r->precision = o->precision;
  r->batch = o->batch <= 0 ? 1 : o->batch;
  if (o->x_stride < 0 || o->out_stride < 0) return fail(SCD_ERR_SIZE, "negative stride");
  if (o->x_stride) r->xs = o->x_stride;
  if (o->out_stride) r->os = o->out_stride;
  if (r->batch > 1 && (r->xs < xlen || r->os < olen))
    return fail(SCD_ERR_SIZE, "stride smaller than one signal (x_stride %lld < %lld or out_stride %lld < %lld)",
                static_cast<long long>(r->xs), static_cast<long long>(xlen), static_cast<long long>(r->os),
                static_cast<long long>(olen));
  if (o->stream) r->stream = static_cast<hipStream_t>(o->stream);
  r->work = o->workspace;
  r->work_bytes = o->workspace_bytes;
  if (r->work == nullptr && r->work_bytes != 0) return fail(SCD_ERR_NULL, "workspace_bytes set without workspace");
  return SCD_OK;
}

size_t span_bytes(int batch, int64_t stride, int64_t len) {
  return 8u * static_cast<size_t>(static_cast<int64_t>(batch - 1) * stride + len);
}

}  // namespace

namespace scd {
// Error reporting for the library's other host files (the calling thread's scd_last_error message).
int set_error(int code, const char* msg) { return fail(code, "%s", msg); }
int set_hip_error(hipError_t e, const char* what) { return hip_fail(e, what); }
}  // namespace scd

extern "C" {

int scd_version(void) { return (1 << 16) | 0; }

const char* scd_last_error(void) { return g_err.c_str(); }

int scd_set_stream(void* stream) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_stream = static_cast<hipStream_t>(stream);
  return SCD_OK;
}

int scd_ssca_workspace_size(int64_t N, int Np, int batch, size_t* bytes) {
  if (!bytes) return fail(SCD_ERR_NULL, "bytes is NULL");
  if (!is_pow2(N) || N < 1024 || N > (1 << 20)) return fail(SCD_ERR_SIZE, "N must be a power of two in [2^10, 2^20]");
  if (!is_pow2(Np) || Np < 16 || Np > 256) return fail(SCD_ERR_SIZE, "Np must be a power of two in [16, 256]");
  if (batch < 1) batch = 1;
  *bytes = (N == 1024) ? 0 : 8u * static_cast<size_t>(Np) * static_cast<size_t>(N) * static_cast<size_t>(batch);
  return SCD_OK;
}

int scd_fam_workspace_size(int Np, int L, int P, int batch, size_t* bytes) {
  if (!bytes) return fail(SCD_ERR_NULL, "bytes is NULL");
  if (!is_pow2(Np) || Np < 16 || Np > 256) return fail(SCD_ERR_SIZE, "Np must be a power of two in [16, 256]");
  if (!is_pow2(L) || L > Np) return fail(SCD_ERR_SIZE, "L must be a power of two in [1, Np]");
  if (!is_pow2(P) || P < 4 || P > 1024) return fail(SCD_ERR_SIZE, "P must be a power of two in [4, 1024]");
  if (batch < 1) batch = 1;
  *bytes = 8u * static_cast<size_t>(Np) * static_cast<size_t>(P) * static_cast<size_t>(batch);
  return SCD_OK;
}

}  // extern "C"

namespace {

enum class SscaPart { kWhole, kStage1, kStage2 };

// Writes a host-built selection to device memory. It travels as a kernel argument, which the runtime copies at
// launch, so the call needs no separate host-to-device copy and never waits on the host.
__global__ void put_chansel_kernel(scd::ChanSel sel, scd::ChanSel* dst) {
  if (threadIdx.x == 0) *dst = sel;
}

unsigned pow2_at_least(unsigned v) {
  unsigned p = 1;
  while (p < v) p <<= 1;
  return v == 0 ? 0 : p;
}

// Shared validation and dispatch of the SSCA entry points. For kStage1 `in` is x and `dst` the intermediate;
// for kStage2 `in` is the intermediate and `dst` the output (win unused); for kWhole `in` is x and `dst` out.
// ymode: 0 the auto SCD; 1 the cross SCD of `in` and y; 2 the conjugate form (whole transform, FP32 only).
// xlen/xoff (whole transform, FP32): the block [xoff, xoff + N) of a signal of xlen samples; 0 = the signal.
// upload (whole transform): a host-built selection, copied into the stream's selector scratch once every argument
// has been checked; selp then gives only the grid sizes.
int ssca_common(SscaPart part, const float* in, int64_t N, int Np, const float* win, float* dst,
                const scd_opts* opts, const scd::SelArg* selp = nullptr, const float* y = nullptr, int ymode = 0,
                int64_t xlen = 0, int64_t xoff = 0, const scd::ChanSel* upload = nullptr) {
  const bool need_win = part != SscaPart::kStage2;
  if (!in || !dst || (need_win && !win)) return fail(SCD_ERR_NULL, "input, window and output must be non-NULL");
  if (ymode != 0 && !y) return fail(SCD_ERR_NULL, "y must be non-NULL");
  if (!is_pow2(N) || N < 1024 || N > (1 << 20))
    return fail(SCD_ERR_SIZE, "N = %lld must be a power of two in [2^10, 2^20]", static_cast<long long>(N));
  if (!is_pow2(Np) || Np < 16 || Np > 256) return fail(SCD_ERR_SIZE, "Np = %d must be a power of two in [16, 256]", Np);
  const int64_t grid = static_cast<int64_t>(Np) * N;
  if (xlen == 0) xlen = N;
  if (xlen != N || xoff != 0) {
    if (xlen > (int64_t{1} << 27)) return fail(SCD_ERR_SIZE, "a signal of blocks holds at most 2^27 samples");
    if (xoff < 0 || xoff % Np != 0 || xoff + N > xlen)
      return fail(SCD_ERR_SIZE, "the block [%lld, %lld) must lie in [0, %lld) and start at a multiple of Np",
                  static_cast<long long>(xoff), static_cast<long long>(xoff + N), static_cast<long long>(xlen));
  }
  const int64_t inlen = (part == SscaPart::kStage2) ? grid : xlen;
  Resolved r;
  int rc = resolve(opts, inlen, grid, &r);
  if (rc) return rc;
  if (r.precision < SCD_FP32 || r.precision > SCD_FP16) return fail(SCD_ERR_SIZE, "unknown precision %d", r.precision);
  if (r.precision != SCD_FP32 && part != SscaPart::kStage2 && Np > 128)
    return fail(SCD_ERR_UNSUPPORTED, "16-bit channelizer precisions support Np <= 128 (got %d)", Np);
  if (ymode != 0 && r.precision != SCD_FP32) return fail(SCD_ERR_UNSUPPORTED, "the cross forms run in FP32 only");
  if (xlen != N && r.precision != SCD_FP32) return fail(SCD_ERR_UNSUPPORTED, "the block form runs in FP32 only");
  const size_t ib = span_bytes(r.batch, r.xs, inlen);
  const size_t ob = span_bytes(r.batch, r.os, grid);
  const size_t wb = need_win ? 4u * static_cast<size_t>(Np) : 0;
  if (overlaps(dst, ob, in, ib) || overlaps(dst, ob, win, wb)) return fail(SCD_ERR_ALIAS, "output overlaps an input");
  if (ymode != 0 && overlaps(dst, ob, y, ib)) return fail(SCD_ERR_ALIAS, "output overlaps y");
  const size_t per = (part == SscaPart::kWhole && N > 1024) ? 8u * static_cast<size_t>(grid) : 0;
  if (part == SscaPart::kWhole && r.work) {
    if (overlaps(r.work, r.work_bytes, in, ib) || overlaps(r.work, r.work_bytes, dst, ob) ||
        overlaps(r.work, r.work_bytes, win, wb) || (ymode != 0 && overlaps(r.work, r.work_bytes, y, ib)))
      return fail(SCD_ERR_ALIAS, "workspace overlaps x, y, win or out");
    if (per > 0 && r.work_bytes < per)
      return fail(SCD_ERR_NOMEM, "workspace of %zu bytes is smaller than one intermediate (%zu)", r.work_bytes, per);
  }

  std::lock_guard<std::mutex> lk(g_mu);
  if ((rc = check_device_range(in, ib, part == SscaPart::kStage2 ? "intermediate" : "x"))) return rc;
  if (need_win && (rc = check_device_range(win, wb, "win"))) return rc;
  if (ymode != 0 && (rc = check_device_range(y, ib, "y"))) return rc;
  if ((rc = check_device_range(dst, ob, part == SscaPart::kStage1 ? "intermediate" : "out"))) return rc;
  if (part == SscaPart::kWhole && r.work && (rc = check_device_range(r.work, r.work_bytes, "workspace"))) return rc;
  int dev;
  if ((rc = current_device(&dev))) return rc;
  DevState& st = g_dev[dev];
  float2* tabs;
  if ((rc = get_tables(st, N, Np, r.stream, &tabs))) return rc;
  const float2* ic = reinterpret_cast<const float2*>(in);
  float2* oc = reinterpret_cast<float2*>(dst);
  const int n = static_cast<int>(N);
  const int prec = r.precision;
  scd::SelArg sel = selp ? *selp : scd::selarg_all(Np);
  if (upload) {
    void* p;
    if ((rc = get_sel(st, r.stream, 4u * kSelScratchFloats, &p))) return rc;
    auto* d = reinterpret_cast<scd::ChanSel*>(static_cast<float*>(p) + kSelScratchFloats - kSelStructFloats);
    hipLaunchKernelGGL(put_chansel_kernel, dim3(1), dim3(64), 0, r.stream, *upload, d);
    sel.dev = d;
  }
  // Stage 1 in the requested precision, for nb signals.
  auto stage1 = [&](const float2* xs, float2* T, int nb, int64_t tbs) -> hipError_t {
    if (prec == SCD_FP32) {
      const float2* ys = ymode ? reinterpret_cast<const float2*>(y) + (xs - ic) : nullptr;
      return scd::launch_ssca_pass1_fp32(xs, n, Np, win, tabs, T, nb, r.xs, tbs, sel, r.stream, ys, ymode,
                                         static_cast<int>(xlen), static_cast<int>(xoff));
    }
    void* aux = nullptr;
    if (get_aux(st, r.stream, scd::ssca_mfma_scratch_bytes(n, Np, nb), &aux)) return hipErrorOutOfMemory;
    return scd::launch_ssca_pass1_mfma(prec, xs, n, Np, win, tabs, aux, T, nb, r.xs, tbs, sel, r.stream);
  };
  hipError_t e = hipSuccess;
  if (part == SscaPart::kStage1) {
    e = stage1(ic, oc, r.batch, r.os);
  } else if (part == SscaPart::kStage2) {
    if (N == 1024) {
      // The Stage 1 output already is the result; copy it if the caller asked for another buffer.
      for (int b = 0; b < r.batch && e == hipSuccess && ic != oc; ++b)
        e = hipMemcpyAsync(oc + b * r.os, ic + b * r.xs, 8u * static_cast<size_t>(grid), hipMemcpyDeviceToDevice,
                           r.stream);
    } else {
      e = scd::launch_ssca_pass2(ic, n, Np, tabs, oc, r.batch, r.xs, r.os, sel, r.stream);
    }
  } else if (per == 0 && !upload) {
    // N == 1024: the Stage 1 output is the final result.
    e = stage1(ic, oc, r.batch, r.os);
  } else if (per == 0) {
    // N == 1024 with a host selection: Stage 1 writes whole channel subsets, so it goes to the library's buffer
    // (whose layout at M2 = 1 is the output's) and only the listed rows are copied out.
    const size_t row = 8u * static_cast<size_t>(N);
    void* work;
    if ((rc = get_work(st, r.stream, 8u * static_cast<size_t>(grid) * r.batch, &work))) return rc;
    float2* T = static_cast<float2*>(work);
    e = stage1(ic, T, r.batch, grid);
    for (int b = 0; b < r.batch && e == hipSuccess; ++b)
      for (int i = 0; i < upload->nch && e == hipSuccess; ++i)
        e = hipMemcpyAsync(oc + b * r.os + upload->ch[i] * N, T + b * grid + upload->ch[i] * N, row,
                           hipMemcpyDeviceToDevice, r.stream);
  } else {
    int chunk = r.batch;
    void* work = r.work;
    if (work) {
      chunk = static_cast<int>(std::min<size_t>(r.batch, r.work_bytes / per));
    } else if ((rc = get_work(st, r.stream, per * r.batch, &work))) {
      return rc;
    }
    float2* T = static_cast<float2*>(work);
    for (int b0 = 0; b0 < r.batch && e == hipSuccess; b0 += chunk) {
      const int nb = std::min(chunk, r.batch - b0);
      e = stage1(ic + b0 * r.xs, T, nb, grid);
      if (e == hipSuccess) e = scd::launch_ssca_pass2(T, n, Np, tabs, oc + b0 * r.os, nb, grid, r.os, sel, r.stream);
    }
  }
  if (e == hipErrorOutOfMemory) return SCD_ERR_NOMEM;
  if (e != hipSuccess) return hip_fail(e, "SSCA launch");
  return SCD_OK;
}

}  // namespace

extern "C" {

int scd_ssca_ex(const float* x, int64_t N, int Np, const float* win, float* out, const scd_opts* opts) {
  return ssca_common(SscaPart::kWhole, x, N, Np, win, out, opts);
}

int scd_ssca_cross_ex(const float* x, const float* y, int64_t N, int Np, const float* win, int conjugate, float* out,
                      const scd_opts* opts) {
  return ssca_common(SscaPart::kWhole, x, N, Np, win, out, opts, nullptr, y, conjugate ? 2 : 1);
}

int scd_ssca_block_ex(const float* x, int64_t len, int64_t offset, int64_t N, int Np, const float* win, float* out,
                      const scd_opts* opts) {
  if (len <= 0) return fail(SCD_ERR_SIZE, "len must be positive");
  return ssca_common(SscaPart::kWhole, x, N, Np, win, out, opts, nullptr, nullptr, 0, len, offset);
}

int scd_ssca_strips(const float* x, int64_t N, int Np, const float* win, const int* strips, int nstrips, float* out,
                    const scd_opts* opts) {
  if (!is_pow2(Np) || Np < 16 || Np > 256) return fail(SCD_ERR_SIZE, "Np = %d must be a power of two in [16, 256]", Np);
  if (nstrips < 0 || nstrips > Np) return fail(SCD_ERR_SIZE, "nstrips = %d must lie in [0, Np = %d]", nstrips, Np);
  if (nstrips > 0 && !strips) return fail(SCD_ERR_NULL, "strips must be non-NULL");
  if (opts && opts->precision != SCD_FP32 && opts->precision != SCD_SPLIT_BF16)
    return fail(SCD_ERR_UNSUPPORTED, "a strip list runs in FP32 or split-BF16");
  // The selection: the listed strips for Stage 2 (ascending), the channel subsets (strips k = c mod Np/16) and
  // subset pairs (c, c + Np/32) that hold one of them for Stage 1.
  const int S = Np / 16;
  scd::ChanSel cs{};
  for (int i = 0; i < nstrips; ++i) {
    const int k = strips[i];
    if (k < 0 || k >= Np) return fail(SCD_ERR_SIZE, "strip %d lies outside [0, %d)", k, Np);
    if (cs.keep[k >> 5] & (1u << (k & 31))) return fail(SCD_ERR_SIZE, "strip %d is listed twice", k);
    cs.keep[k >> 5] |= 1u << (k & 31);
  }
  bool used[16] = {};
  for (int k = 0; k < Np; ++k) {
    if (cs.keep[k >> 5] & (1u << (k & 31))) {
      cs.ch[cs.nch++] = static_cast<unsigned char>(k);
      used[k % S] = true;
    }
  }
  for (int c = 0; c < S; ++c)
    if (used[c]) cs.sub[cs.nsub++] = static_cast<unsigned char>(c);
  for (int c = 0; c < S / 2; ++c)
    if (used[c] || used[c + S / 2]) cs.pair[cs.npair++] = static_cast<unsigned char>(c);
  if (cs.nch == 0) {
    if (!x || !win || !out) return fail(SCD_ERR_NULL, "input, window and output must be non-NULL");
    return SCD_OK;
  }
  // Grid sizes: the unit counts rounded up to powers of two (one Stage-1 block mapping needs that); the blocks
  // past the selection's own counts exit at once.
  const scd::SelArg sel{nullptr, static_cast<int>(pow2_at_least(cs.nsub)), static_cast<int>(pow2_at_least(cs.npair)),
                        cs.nch};
  return ssca_common(SscaPart::kWhole, x, N, Np, win, out, opts, &sel, nullptr, 0, 0, 0, &cs);
}

int scd_ssca(const float* x, int64_t N, int Np, const float* win, float* out) {
  return ssca_common(SscaPart::kWhole, x, N, Np, win, out, nullptr);
}

int scd_ssca_stage1_ex(const float* x, int64_t N, int Np, const float* win, float* inter, const scd_opts* opts) {
  return ssca_common(SscaPart::kStage1, x, N, Np, win, inter, opts);
}

int scd_ssca_stage2_ex(const float* inter, int64_t N, int Np, float* out, const scd_opts* opts) {
  return ssca_common(SscaPart::kStage2, inter, N, Np, nullptr, out, opts);
}

}  // extern "C"

namespace {

// FAM of Eq. (3)-(5); `power` selects the |S|^2 form over -P/4 <= q_c < P/4 (float output, P/2 bins per pair).
int fam_common(const float* x, int Np, int L, int P, const float* win, float* out, const scd_opts* opts,
               bool power, const float* y = nullptr, bool conj = false) {
  if (!x || !win || !out) return fail(SCD_ERR_NULL, "x, win and out must be non-NULL");
  if (!is_pow2(Np) || Np < 16 || Np > 256) return fail(SCD_ERR_SIZE, "Np = %d must be a power of two in [16, 256]", Np);
  if (!is_pow2(L) || L > Np) return fail(SCD_ERR_SIZE, "L = %d must be a power of two in [1, Np]", L);
  if (!is_pow2(P) || P < 4 || P > 1024) return fail(SCD_ERR_SIZE, "P = %d must be a power of two in [4, 1024]", P);
  if (static_cast<int64_t>(P) * L > (1 << 16)) return fail(SCD_ERR_SIZE, "P*L must be at most 2^16");
  const int64_t n = static_cast<int64_t>(P) * L;
  const int64_t olen = static_cast<int64_t>(Np) * Np * (power ? P / 2 : P);
  Resolved r;
  int rc = resolve(opts, n, olen, &r);
  if (rc) return rc;
  if (r.precision != SCD_FP32) return fail(SCD_ERR_UNSUPPORTED, "FAM is FP32 only");
  const size_t xb = span_bytes(r.batch, r.xs, n);
  const size_t ob = span_bytes(r.batch, r.os, olen) / (power ? 2 : 1);  // float elements in the power form
  const size_t wb = 4u * static_cast<size_t>(Np);
  if (overlaps(out, ob, x, xb) || overlaps(out, ob, win, wb)) return fail(SCD_ERR_ALIAS, "out overlaps x or win");
  if (y && overlaps(out, ob, y, xb)) return fail(SCD_ERR_ALIAS, "out overlaps y");
  // X_T per signal, and Y_T beside it in the cross forms.
  const size_t per = 8u * static_cast<size_t>(Np) * static_cast<size_t>(P) * (y ? 2 : 1);
  if (r.work && (overlaps(r.work, r.work_bytes, x, xb) || overlaps(r.work, r.work_bytes, out, ob) ||
                 overlaps(r.work, r.work_bytes, win, wb) || (y && overlaps(r.work, r.work_bytes, y, xb))))
    return fail(SCD_ERR_ALIAS, "workspace overlaps x, y, win or out");
  if (r.work && r.work_bytes < per)
    return fail(SCD_ERR_NOMEM, "workspace of %zu bytes is smaller than one X_T (%zu)", r.work_bytes, per);

  std::lock_guard<std::mutex> lk(g_mu);
  if ((rc = check_device_range(x, xb, "x"))) return rc;
  if ((rc = check_device_range(win, wb, "win"))) return rc;
  if (y && (rc = check_device_range(y, xb, "y"))) return rc;
  if ((rc = check_device_range(out, ob, "out"))) return rc;
  if (r.work && (rc = check_device_range(r.work, r.work_bytes, "workspace"))) return rc;
  int dev;
  if ((rc = current_device(&dev))) return rc;
  DevState& st = g_dev[dev];
  float2* tabs;
  if ((rc = get_tables(st, 1024, Np, r.stream, &tabs))) return rc;
  int chunk = r.batch;
  void* work = r.work;
  if (work) chunk = static_cast<int>(std::min<size_t>(r.batch, r.work_bytes / per));
  else if ((rc = get_work(st, r.stream, per * r.batch, &work))) return rc;
  const float2* xc = reinterpret_cast<const float2*>(x);
  for (int b0 = 0; b0 < r.batch; b0 += chunk) {
    const int nb = std::min(chunk, r.batch - b0);
    void* oc = power ? static_cast<void*>(out + b0 * r.os) : static_cast<void*>(reinterpret_cast<float2*>(out) + b0 * r.os);
    const float2* yc = y ? reinterpret_cast<const float2*>(y) + b0 * r.xs : nullptr;
    hipError_t e = scd::launch_fam_fp32(xc + b0 * r.xs, Np, L, P, win, tabs, static_cast<float2*>(work), oc,
                                        power, nb, r.xs, r.os, r.stream, yc, conj);
    if (e != hipSuccess) return hip_fail(e, "FAM launch");
  }
  return SCD_OK;
}

}  // namespace

// ---- selector model lifecycle ----------------------------------------------------------------------------
// A model owns one device block [params | mu | sigma] on the device that was current at creation. Model files
// are little-endian: "SCDM", u32 version 1, i32 Np, i32 parameter count, f32 theta, f32 conf_min, the
// parameters, mu (2 Np) and sigma (2 Np) as f32, and a u32 FNV-1a hash of every byte before it.
struct scd_model {
  int device;
  int Np;
  int nparams;
  float theta, conf_min;
  float* block;  // device: params (16-byte aligned at the block start), mu, sigma
};

namespace {

constexpr char kModelMagic[4] = {'S', 'C', 'D', 'M'};
constexpr uint32_t kModelVersion = 1;
constexpr size_t kModelHeader = 4 + 4 + 4 + 4 + 4 + 4;

uint32_t fnv1a(const unsigned char* p, size_t n) {
  uint32_t h = 2166136261u;
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 16777619u;
  }
  return h;
}

// Host-side checks shared by creation, writing and loading.
int check_model_values(int Np, const float* params, const float* mu, const float* sigma, float theta, float conf_min) {
  const int n = scd_mlp_param_count(Np);
  if (n < 0) return fail(SCD_ERR_SIZE, "model Np = %d must be a power of two in [16, 256]", Np);
  if (!(theta >= 0.f && theta <= 1.f)) return fail(SCD_ERR_MODEL, "theta = %g must lie in [0, 1]", theta);
  if (!(conf_min >= 0.f && conf_min <= 1.f)) return fail(SCD_ERR_MODEL, "conf_min = %g must lie in [0, 1]", conf_min);
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(params[i])) return fail(SCD_ERR_MODEL, "parameter %d is not finite", i);
  for (int i = 0; i < 2 * Np; ++i) {
    if (!std::isfinite(mu[i])) return fail(SCD_ERR_MODEL, "mu[%d] is not finite", i);
    if (!(std::isfinite(sigma[i]) && sigma[i] > 0.f)) return fail(SCD_ERR_MODEL, "sigma[%d] must be positive", i);
  }
  return SCD_OK;
}

template <class T>
void put(std::string& b, T v) {
  b.append(reinterpret_cast<const char*>(&v), sizeof(T));
}

}  // namespace

extern "C" {

int scd_model_write(const char* path, int Np, const float* params, const float* mu, const float* sigma, float theta,
                    float conf_min) {
  if (!path || !params || !mu || !sigma) return fail(SCD_ERR_NULL, "NULL argument");
  int rc;
  if ((rc = check_model_values(Np, params, mu, sigma, theta, conf_min))) return rc;
  const int n = scd_mlp_param_count(Np);
  std::string b;
  b.reserve(kModelHeader + 4u * (n + 4 * Np) + 4);
  b.append(kModelMagic, 4);
  put<uint32_t>(b, kModelVersion);
  put<int32_t>(b, Np);
  put<int32_t>(b, n);
  put<float>(b, theta);
  put<float>(b, conf_min);
  b.append(reinterpret_cast<const char*>(params), 4u * n);
  b.append(reinterpret_cast<const char*>(mu), 8u * Np);
  b.append(reinterpret_cast<const char*>(sigma), 8u * Np);
  put<uint32_t>(b, fnv1a(reinterpret_cast<const unsigned char*>(b.data()), b.size()));
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(SCD_ERR_MODEL, "cannot open %s for writing", path);
  const size_t w = std::fwrite(b.data(), 1, b.size(), f);
  const int closed = std::fclose(f);
  if (w != b.size() || closed != 0) return fail(SCD_ERR_MODEL, "writing %s failed", path);
  return SCD_OK;
}

int scd_model_create(int Np, const float* params, const float* mu, const float* sigma, float theta, float conf_min,
                     scd_model** model) {
  if (!model) return fail(SCD_ERR_NULL, "NULL model handle");
  *model = nullptr;
  if (!params || !mu || !sigma) return fail(SCD_ERR_NULL, "NULL argument");
  int rc;
  if ((rc = check_model_values(Np, params, mu, sigma, theta, conf_min))) return rc;
  const int n = scd_mlp_param_count(Np);
  int dev;
  if ((rc = current_device(&dev))) return rc;
  float* block = nullptr;
  const size_t bytes = 4u * (static_cast<size_t>(n) + 4u * Np);
  hipError_t e = hipMalloc(&block, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(SCD_ERR_NOMEM, "model allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
  }
  e = hipMemcpy(block, params, 4u * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(block + n, mu, 8u * Np, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(block + n + 2 * Np, sigma, 8u * Np, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(block);
    return hip_fail(e, "model upload");
  }
  *model = new scd_model{dev, Np, n, theta, conf_min, block};
  return SCD_OK;
}

int scd_model_destroy(scd_model* model) {
  if (!model) return SCD_OK;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(model->device);
  const hipError_t e = hipFree(model->block);
  (void)hipSetDevice(cur);
  delete model;
  if (e != hipSuccess) return hip_fail(e, "model free");
  return SCD_OK;
}

int scd_model_selector(const scd_model* model, scd_selector* selector) {
  if (!model || !selector) return fail(SCD_ERR_NULL, "NULL argument");
  selector->Np = model->Np;
  selector->params = model->block;
  selector->mu = model->block + model->nparams;
  selector->sigma = model->block + model->nparams + 2 * model->Np;
  selector->theta = model->theta;
  selector->conf_min = model->conf_min;
  return SCD_OK;
}

int scd_model_read(const scd_model* model, float* params, float* mu, float* sigma) {
  if (!model) return fail(SCD_ERR_NULL, "NULL model");
  int cur = 0;
  (void)hipGetDevice(&cur);
  hipError_t e = hipSetDevice(model->device);
  if (e == hipSuccess && params) e = hipMemcpy(params, model->block, 4u * model->nparams, hipMemcpyDeviceToHost);
  if (e == hipSuccess && mu) e = hipMemcpy(mu, model->block + model->nparams, 8u * model->Np, hipMemcpyDeviceToHost);
  if (e == hipSuccess && sigma)
    e = hipMemcpy(sigma, model->block + model->nparams + 2 * model->Np, 8u * model->Np, hipMemcpyDeviceToHost);
  (void)hipSetDevice(cur);
  if (e != hipSuccess) return hip_fail(e, "model read-back");
  return SCD_OK;
}

int scd_model_save(const scd_model* model, const char* path) {
  if (!model || !path) return fail(SCD_ERR_NULL, "NULL argument");
  std::string host(4u * (static_cast<size_t>(model->nparams) + 4u * model->Np), '\0');
  float* h = reinterpret_cast<float*>(&host[0]);
  int rc;
  if ((rc = scd_model_read(model, h, h + model->nparams, h + model->nparams + 2 * model->Np))) return rc;
  return scd_model_write(path, model->Np, h, h + model->nparams, h + model->nparams + 2 * model->Np, model->theta,
                         model->conf_min);
}

int scd_model_load(const char* path, scd_model** model) {
  if (!path || !model) return fail(SCD_ERR_NULL, "NULL argument");
  *model = nullptr;
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(SCD_ERR_MODEL, "cannot open %s", path);
  std::string b;
  char chunk[1 << 16];
  size_t r;
  while ((r = std::fread(chunk, 1, sizeof(chunk), f)) > 0) {
    b.append(chunk, r);
    if (b.size() > (64u << 20)) break;
  }
  std::fclose(f);
  if (b.size() < kModelHeader + 4) return fail(SCD_ERR_MODEL, "%s: too short for a model file", path);
  if (std::memcmp(b.data(), kModelMagic, 4) != 0) return fail(SCD_ERR_MODEL, "%s: not a model file", path);
  uint32_t version;
  int32_t Np, n;
  float theta, conf_min;
  std::memcpy(&version, b.data() + 4, 4);
  std::memcpy(&Np, b.data() + 8, 4);
  std::memcpy(&n, b.data() + 12, 4);
  std::memcpy(&theta, b.data() + 16, 4);
  std::memcpy(&conf_min, b.data() + 20, 4);
  if (version != kModelVersion) return fail(SCD_ERR_MODEL, "%s: model file version %u is not %u", path, version, kModelVersion);
  const int expect = scd_mlp_param_count(Np);
  if (expect < 0) return fail(SCD_ERR_MODEL, "%s: Np = %d is not supported", path, Np);
  if (n != expect) return fail(SCD_ERR_MODEL, "%s: %d parameters, %d expected for Np = %d", path, n, expect, Np);
  const size_t want = kModelHeader + 4u * (static_cast<size_t>(n) + 4u * Np) + 4;
  if (b.size() != want) return fail(SCD_ERR_MODEL, "%s: %zu bytes, %zu expected", path, b.size(), want);
  uint32_t hash;
  std::memcpy(&hash, b.data() + want - 4, 4);
  if (hash != fnv1a(reinterpret_cast<const unsigned char*>(b.data()), want - 4))
    return fail(SCD_ERR_MODEL, "%s: checksum mismatch", path);
  std::string arr = b.substr(kModelHeader, want - 4 - kModelHeader);  // aligned copy of the arrays
  const float* h = reinterpret_cast<const float*>(arr.data());
  return scd_model_create(Np, h, h + n, h + n + 2 * Np, theta, conf_min, model);
}

}  // extern "C"

extern "C" {

int scd_fam_ex(const float* x, int Np, int L, int P, const float* win, float* out, const scd_opts* opts) {
  return fam_common(x, Np, L, P, win, out, opts, false);
}

int scd_fam_power_ex(const float* x, int Np, int L, int P, const float* win, float* out, const scd_opts* opts) {
  return fam_common(x, Np, L, P, win, out, opts, true);
}

int scd_fam_cross_ex(const float* x, const float* y, int Np, int L, int P, const float* win, int conjugate, float* out,
                     const scd_opts* opts) {
  if (!y) return fail(SCD_ERR_NULL, "y must be non-NULL");
  return fam_common(x, Np, L, P, win, out, opts, false, y, conjugate != 0);
}

int scd_fam(const float* x, int Np, int L, int P, const float* win, float* out) {
  return scd_fam_ex(x, Np, L, P, win, out, nullptr);
}

int scd_mlp_param_count(int Np) {
  if (!is_pow2(Np) || Np < 16 || Np > 256) return fail(SCD_ERR_SIZE, "Np = %d must be a power of two in [16, 256]", Np);
  return scd::mlp_layout(Np).total;
}

namespace {
// Segment periodograms and the feature reduction of `batch` signals (checked arguments, library lock held).
int features_impl(const float* x, int64_t N, int Np, const float* win, float* feat, int batch, int64_t xs,
                  hipStream_t stream, bool centre) {
  int rc, dev;
  if ((rc = current_device(&dev))) return rc;
  DevState& st = g_dev[dev];
  float2* tabs;
  if ((rc = get_tables(st, 1024, Np, stream, &tabs))) return rc;
  // Segment periodograms of up to kFeatChunk signals per launch.
  constexpr int kFeatChunk = 8;
  const int chunk = batch < kFeatChunk ? batch : kFeatChunk;
  const size_t pb = 4u * 16u * static_cast<size_t>(Np) * 1024u * static_cast<size_t>(chunk);
  void* lrn;
  if ((rc = get_lrn(st, stream, pb, &lrn))) return rc;
  float* P = static_cast<float*>(lrn);
  const float2* xc = reinterpret_cast<const float2*>(x);
  hipError_t e = hipSuccess;
  for (int b = 0; b < batch && e == hipSuccess; b += chunk) {
    const int n = batch - b < chunk ? batch - b : chunk;
    e = scd::launch_features(xc + b * xs, xs, N, Np, n, win, tabs, P, feat + static_cast<size_t>(b) * 2 * Np, stream,
                             centre);
  }
  if (e != hipSuccess) return hip_fail(e, "feature launch");
  return SCD_OK;
}
}  // namespace

int scd_features(const float* x, int64_t N, int Np, const float* win, float* feat, const scd_opts* opts) {
  if (!x || !win || !feat) return fail(SCD_ERR_NULL, "x, win and feat must be non-NULL");
  if (!is_pow2(N) || N < (1 << 14) || N > (1 << 20))
    return fail(SCD_ERR_SIZE, "features need N a power of two in [2^14, 2^20] (got %lld)", static_cast<long long>(N));
  if (!is_pow2(Np) || Np < 16 || Np > 256) return fail(SCD_ERR_SIZE, "Np = %d must be a power of two in [16, 256]", Np);
  Resolved r;
  int rc = resolve(opts, N, 2 * Np, &r);
  if (rc) return rc;
  if (r.work) return fail(SCD_ERR_UNSUPPORTED, "scd_features uses library-owned scratch only");
  std::lock_guard<std::mutex> lk(g_mu);
  const size_t xb = span_bytes(r.batch, r.xs, N);
  if ((rc = check_device_range(x, xb, "x"))) return rc;
  if ((rc = check_device_range(win, 4u * Np, "win"))) return rc;
  if ((rc = check_device_range(feat, 4u * static_cast<size_t>(2 * Np) * r.batch, "feat"))) return rc;
  return features_impl(x, N, Np, win, feat, r.batch, r.xs, r.stream, true);
}

int scd_strip_labels(const float* S, int64_t N, int Np, float* labels, float* ratio, const scd_opts* opts) {
  if (!S || !labels) return fail(SCD_ERR_NULL, "S and labels must be non-NULL");
  if (!is_pow2(N) || N < 1024 || N > (1 << 20)) return fail(SCD_ERR_SIZE, "N must be a power of two in [2^10, 2^20]");
  if (!is_pow2(Np) || Np < 16 || Np > 256) return fail(SCD_ERR_SIZE, "Np must be a power of two in [16, 256]");
  Resolved r;
  int rc = resolve(opts, static_cast<int64_t>(Np) * N, Np, &r);
  if (rc) return rc;
  if (r.xs != static_cast<int64_t>(Np) * N) return fail(SCD_ERR_SIZE, "labels need densely packed SCDs");
  std::lock_guard<std::mutex> lk(g_mu);
  if ((rc = check_device_range(S, 8u * static_cast<size_t>(Np) * N * r.batch, "S"))) return rc;
  if ((rc = check_device_range(labels, 4u * static_cast<size_t>(Np) * r.batch, "labels"))) return rc;
  if (ratio && (rc = check_device_range(ratio, 4u * static_cast<size_t>(Np) * r.batch, "ratio"))) return rc;
  hipError_t e = scd::launch_labels(reinterpret_cast<const float2*>(S), N, Np, r.batch, labels, ratio, r.stream);
  if (e != hipSuccess) return hip_fail(e, "label launch");
  return SCD_OK;
}

int scd_standardize(const float* f, const float* mu, const float* sigma, float* out, int n, int dim, void* stream) {
  if (!f || !mu || !sigma || !out) return fail(SCD_ERR_NULL, "NULL argument");
  if (n < 1 || dim < 1) return fail(SCD_ERR_SIZE, "n and dim must be positive");
  hipError_t e = scd::launch_standardize(f, mu, sigma, out, n, dim, stream ? static_cast<hipStream_t>(stream) : g_stream);
  if (e != hipSuccess) return hip_fail(e, "standardize launch");
  return SCD_OK;
}

int scd_mlp_forward(int Np, int batch, const float* params, const float* x, float* act, float* z, float* scores,
                    void* stream) {
  if (!params || !x || !act || !z || !scores) return fail(SCD_ERR_NULL, "NULL argument");
  if (!is_pow2(Np) || Np < 16 || Np > 256 || batch < 1) return fail(SCD_ERR_SIZE, "bad Np or batch");
  hipError_t e = scd::launch_mlp_forward(Np, batch, params, x, act, z, scores,
                                         stream ? static_cast<hipStream_t>(stream) : g_stream);
  if (e != hipSuccess) return hip_fail(e, "MLP forward launch");
  return SCD_OK;
}

int scd_mlp_backward(int Np, int batch, const float* params, const float* x, const float* act, const float* scores,
                     const float* labels, float* grads, float* scratch, float* dx, void* stream) {
  if (!params || !x || !act || !scores || !labels || !grads || !scratch) return fail(SCD_ERR_NULL, "NULL argument");
  if (!is_pow2(Np) || Np < 16 || Np > 256 || batch < 1) return fail(SCD_ERR_SIZE, "bad Np or batch");
  hipError_t e = scd::launch_mlp_backward(Np, batch, params, x, act, scores, labels, grads, scratch, dx,
                                          stream ? static_cast<hipStream_t>(stream) : g_stream);
  if (e != hipSuccess) return hip_fail(e, "MLP backward launch");
  return SCD_OK;
}

int scd_adam_step(int n, float* params, const float* grads, float* m, float* v, int t, float lr, float beta1,
                  float beta2, float eps, void* stream) {
  if (!params || !grads || !m || !v) return fail(SCD_ERR_NULL, "NULL argument");
  if (n < 1 || t < 1) return fail(SCD_ERR_SIZE, "n and t must be positive");
  hipError_t e = scd::launch_adam(params, grads, m, v, n, t, lr, beta1, beta2, eps,
                                  stream ? static_cast<hipStream_t>(stream) : g_stream);
  if (e != hipSuccess) return hip_fail(e, "Adam launch");
  return SCD_OK;
}

int scd_select(const float* scores, int Np, int batch, float theta, unsigned char* mask, float* conf, void* stream) {
  if (!scores || !mask || !conf) return fail(SCD_ERR_NULL, "NULL argument");
  if (!is_pow2(Np) || Np < 16 || Np > 256 || batch < 1) return fail(SCD_ERR_SIZE, "bad Np or batch");
  hipError_t e = scd::launch_select(scores, Np, batch, theta, mask, conf,
                                    stream ? static_cast<hipStream_t>(stream) : g_stream);
  if (e != hipSuccess) return hip_fail(e, "select launch");
  return SCD_OK;
}

}  // extern "C"

namespace {
// The selector half of the learned form: features, then one kernel chain that standardises them, runs the MLP,
// thresholds the scores, falls back below the confidence floor and writes the device-side selection. Leaves
// the scores at *scores (device, Np floats), the confidence and fallback flag at *conf / *fell and the
// ChanSel at *dsel, all in the library's selector scratch (checked arguments; takes the library lock itself).
// The host-side checks of a learned call's arguments (no device access).
int check_learned_args(const float* x, int64_t N, int Np, const float* win, const scd_selector* selector,
                       const unsigned char* mask) {
  if (!x || !win || !selector || !mask) return fail(SCD_ERR_NULL, "NULL argument");
  if (!selector->params || !selector->mu || !selector->sigma) return fail(SCD_ERR_MODEL, "selector has NULL arrays");
  if (reinterpret_cast<uintptr_t>(selector->params) % 16 != 0)
    return fail(SCD_ERR_MODEL, "selector params must be 16-byte aligned");
  if (selector->Np != Np) return fail(SCD_ERR_MODEL, "selector was trained for Np = %d, not %d", selector->Np, Np);
  if (!is_pow2(N) || N < (1 << 14) || N > (1 << 20))
    return fail(SCD_ERR_SIZE, "the learned form needs N a power of two in [2^14, 2^20]");
  if (!is_pow2(Np) || Np < 16 || Np > 256) return fail(SCD_ERR_SIZE, "Np must be a power of two in [16, 256]");
  return SCD_OK;
}

// The host-side checks of one scd_ssca_batch item (no device access), so that argument errors of any item are
// found before the call enqueues anything.
int check_batch_item(const scd_ssca_item& it, int precision) {
  if (precision < SCD_FP32 || precision > SCD_FP16) return fail(SCD_ERR_SIZE, "unknown precision %d", precision);
  if (it.selector) {
    const int rc = check_learned_args(it.x, it.N, it.Np, it.win, it.selector, it.mask);
    if (rc != SCD_OK) return rc;
    if (!it.out) return fail(SCD_ERR_NULL, "NULL argument");
    if (precision != SCD_FP32 && precision != SCD_SPLIT_BF16)
      return fail(SCD_ERR_UNSUPPORTED, "the learned form runs in FP32 or split-BF16");
    return SCD_OK;
  }
  if (!it.x || !it.win || !it.out) return fail(SCD_ERR_NULL, "input, window and output must be non-NULL");
  if (!is_pow2(it.N) || it.N < 1024 || it.N > (1 << 20))
    return fail(SCD_ERR_SIZE, "N = %lld must be a power of two in [2^10, 2^20]", static_cast<long long>(it.N));
  if (!is_pow2(it.Np) || it.Np < 16 || it.Np > 256)
    return fail(SCD_ERR_SIZE, "Np = %d must be a power of two in [16, 256]", it.Np);
  if (precision != SCD_FP32 && it.Np > 128)
    return fail(SCD_ERR_UNSUPPORTED, "16-bit channelizer precisions support Np <= 128 (got %d)", it.Np);
  return SCD_OK;
}

int learned_select(const float* x, int64_t N, int Np, const float* win, const scd_selector* selector,
                   unsigned char* mask, hipStream_t stream, float** scores, float** conf, int** fell,
                   scd::ChanSel** dsel) {
  int rc;
  if ((rc = check_learned_args(x, N, Np, win, selector, mask))) return rc;
  const scd::MlpLayout L = scd::mlp_layout(Np);
  float* f = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    int dev;
    if ((rc = current_device(&dev))) return rc;
    if ((rc = check_device_range(selector->params, 4u * L.total, "selector params"))) return rc;
    if ((rc = check_device_range(selector->mu, 8u * Np, "selector mu"))) return rc;
    if ((rc = check_device_range(selector->sigma, 8u * Np, "selector sigma"))) return rc;
    if ((rc = check_device_range(mask, static_cast<size_t>(Np), "mask"))) return rc;
    if ((rc = check_device_range(x, 8u * static_cast<size_t>(N), "x"))) return rc;
    if ((rc = check_device_range(win, 4u * Np, "win"))) return rc;
    void* p;
    if ((rc = get_sel(g_dev[dev], stream, 4u * kSelScratchFloats, &p))) return rc;
    f = static_cast<float*>(p);
    // Raw features: the first MLP layer centres the PSD part itself.
    if ((rc = features_impl(x, N, Np, win, f, 1, N, stream, false))) return rc;
  }
  *conf = f + kSelScratchFloats - kSelStructFloats - 2;
  *fell = reinterpret_cast<int*>(*conf + 1);
  *dsel = reinterpret_cast<scd::ChanSel*>(f + kSelScratchFloats - kSelStructFloats);
  // Layout of the selector scratch: features [0, 512), then act: h1 and h2 (256 each) and the Np scores, then
  // the second layer's 4 x 256 partial sums at act + 768 (up to float 2304), then conf, fell and the ChanSel.
  float* act = f + 2 * 256;
  *scores = act + 2 * 256;
  const hipError_t e = scd::launch_select_infer(f, selector->mu, selector->sigma, selector->params, Np,
                                                selector->theta, selector->conf_min, act, mask, *conf, *fell, *dsel,
                                                stream);
  if (e != hipSuccess) return hip_fail(e, "selector");
  return SCD_OK;
}
}  // namespace

extern "C" {

int scd_selector_run(const float* x, int64_t N, int Np, const float* win, const scd_selector* selector, float* scores,
                     unsigned char* mask, float* conf, int* fell_back, const scd_opts* opts) {
  if (!scores) return fail(SCD_ERR_NULL, "NULL argument");
  if (opts && opts->batch > 1) return fail(SCD_ERR_UNSUPPORTED, "scd_selector_run takes one signal per call");
  hipStream_t stream = (opts && opts->stream) ? static_cast<hipStream_t>(opts->stream) : g_stream;
  int rc;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if ((rc = check_device_range(scores, 4u * Np, "scores"))) return rc;
    if (conf && (rc = check_device_range(conf, 4u, "conf"))) return rc;
    if (fell_back && (rc = check_device_range(fell_back, 4u, "fell_back"))) return rc;
  }
  float *dsc, *dconf;
  int* dfell;
  scd::ChanSel* dsel;
  if ((rc = learned_select(x, N, Np, win, selector, mask, stream, &dsc, &dconf, &dfell, &dsel))) return rc;
  hipError_t e = hipMemcpyAsync(scores, dsc, 4u * Np, hipMemcpyDeviceToDevice, stream);
  if (e == hipSuccess && conf) e = hipMemcpyAsync(conf, dconf, 4u, hipMemcpyDeviceToDevice, stream);
  if (e == hipSuccess && fell_back) e = hipMemcpyAsync(fell_back, dfell, 4u, hipMemcpyDeviceToDevice, stream);
  if (e != hipSuccess) return hip_fail(e, "selector result copy");
  return SCD_OK;
}

int scd_ssca_learned(const float* x, int64_t N, int Np, const float* win, const scd_selector* selector, float* out,
                     unsigned char* mask, int* fell_back, const scd_opts* opts) {
  if (!x || !win || !selector || !out || !mask) return fail(SCD_ERR_NULL, "NULL argument");
  if (opts && opts->batch > 1) return fail(SCD_ERR_UNSUPPORTED, "scd_ssca_learned takes one signal per call");
  if (opts && opts->precision != SCD_FP32 && opts->precision != SCD_SPLIT_BF16)
    return fail(SCD_ERR_UNSUPPORTED, "the learned form runs in FP32 or split-BF16");
  hipStream_t stream = (opts && opts->stream) ? static_cast<hipStream_t>(opts->stream) : g_stream;
  int rc;
  float *dsc, *dconf;
  int* dfell;
  scd::ChanSel* dsel;
  if ((rc = learned_select(x, N, Np, win, selector, mask, stream, &dsc, &dconf, &dfell, &dsel))) return rc;
  // The grids cover every subset and strip; the kernels read the selection from dsel and skip the rest.
  const scd::SelArg sel{dsel, Np / 16, Np / 32, Np};
  scd_opts so{};
  if (opts) so = *opts;
  so.batch = 1;
  so.stream = stream;
  if ((rc = ssca_common(SscaPart::kWhole, x, N, Np, win, out, &so, &sel))) return rc;
  if (fell_back) {
    hipError_t e = hipMemcpyAsync(fell_back, dfell, sizeof(int), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "fallback flag read-back");
  }
  return SCD_OK;
}

int scd_ssca_batch(const scd_ssca_item* items, int n, const scd_opts* opts) {
  if (n < 0) return fail(SCD_ERR_SIZE, "n must be at least 0");
  if (n > 0 && !items) return fail(SCD_ERR_NULL, "NULL argument");
  if (opts && opts->batch > 1) return fail(SCD_ERR_SIZE, "each item is one signal: opts->batch must be 0 or 1");
  if (opts && (opts->x_stride != 0 || opts->out_stride != 0))
    return fail(SCD_ERR_UNSUPPORTED, "strides do not apply to scd_ssca_batch items");
  const int prec = opts ? opts->precision : SCD_FP32;
  for (int i = 0; i < n; ++i) {
    const int rc = check_batch_item(items[i], prec);
    if (rc != SCD_OK) {
      const std::string why = g_err;
      return fail(rc, "item %d: %s", i, why.c_str());
    }
  }
  if (n == 0) return SCD_OK;
  std::lock_guard<std::mutex> blk(g_batch_mu);
  hipStream_t stream = (opts && opts->stream) ? static_cast<hipStream_t>(opts->stream) : g_stream;
  scd_opts so{};
  if (opts) so = *opts;
  so.batch = 1;
  // Item i runs on lane i mod kBatchLanes: its selector (if any) and its SSCA in that lane's order, on the lane's
  // own scratch. The lanes start after the work already on the caller's stream, and the caller's stream waits
  // for all of them at the end. A caller workspace is one buffer, so with one the items run in order on the
  // caller's stream, as does a single item.
  const int K = (n > 1 && !(opts && opts->workspace)) ? kBatchLanes : 1;
  hipStream_t lanes[kBatchLanes];
  for (hipStream_t& l : lanes) l = stream;
  BatchPipe* bp = nullptr;
  if (K > 1) {
    std::lock_guard<std::mutex> lk(g_mu);
    int dev, rc;
    if ((rc = current_device(&dev))) return rc;
    BatchPipe& P = g_dev[dev].pipe;
    hipError_t e = hipSuccess;
    for (int j = 0; j < K && e == hipSuccess; ++j) {
      if (!P.lane[j]) e = hipStreamCreateWithFlags(&P.lane[j], hipStreamNonBlocking);
      if (e == hipSuccess && !P.end[j]) e = hipEventCreateWithFlags(&P.end[j], hipEventDisableTiming);
    }
    if (e == hipSuccess && !P.start) e = hipEventCreateWithFlags(&P.start, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(P.start, stream);
    for (int j = 0; j < K && e == hipSuccess; ++j) e = hipStreamWaitEvent(P.lane[j], P.start, 0);
    if (e != hipSuccess) return hip_fail(e, "batch lanes");
    for (int j = 0; j < K; ++j) lanes[j] = P.lane[j];
    bp = &P;
  }
  int rc = SCD_OK, bad = -1;
  for (int i = 0; i < n && rc == SCD_OK; ++i) {
    const scd_ssca_item& it = items[i];
    so.stream = lanes[i % K];
    if (!it.selector) {
      rc = scd_ssca_ex(it.x, it.N, it.Np, it.win, it.out, &so);
    } else {
      float *dsc, *dconf;
      int* dfell;
      scd::ChanSel* dsel;
      rc = learned_select(it.x, it.N, it.Np, it.win, it.selector, it.mask, lanes[i % K], &dsc, &dconf, &dfell,
                          &dsel);
      if (rc == SCD_OK) {
        const scd::SelArg sel{dsel, it.Np / 16, it.Np / 32, it.Np};
        rc = ssca_common(SscaPart::kWhole, it.x, it.N, it.Np, it.win, it.out, &so, &sel);
      }
    }
    if (rc != SCD_OK) bad = i;
  }
  const std::string why = g_err;
  // The caller's stream waits for every lane, also after a failing item (the items before it stay enqueued).
  if (bp) {
    hipError_t e = hipSuccess;
    for (int j = 0; j < K && e == hipSuccess; ++j) {
      e = hipEventRecord(bp->end[j], bp->lane[j]);
      if (e == hipSuccess) e = hipStreamWaitEvent(stream, bp->end[j], 0);
    }
    if (e != hipSuccess && rc == SCD_OK) return hip_fail(e, "batch lanes");
  }
  if (rc != SCD_OK) return fail(rc, "item %d: %s", bad, why.c_str());
  return SCD_OK;
}

void scd_shutdown(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_dev.empty()) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (auto& kv : g_dev) {
    (void)hipSetDevice(kv.first);
    (void)hipDeviceSynchronize();
    for (auto& p : kv.second.plans) (void)hipFree(p.second);
    BatchPipe& P = kv.second.pipe;
    for (int j = 0; j < kBatchLanes; ++j) {
      if (P.lane[j]) (void)hipStreamDestroy(P.lane[j]);
      if (P.end[j]) (void)hipEventDestroy(P.end[j]);
    }
    if (P.start) (void)hipEventDestroy(P.start);
    for (auto& sc : kv.second.streams) {
      if (sc.second.work) (void)hipFree(sc.second.work);
      if (sc.second.aux) (void)hipFree(sc.second.aux);
      if (sc.second.lrn) (void)hipFree(sc.second.lrn);
      if (sc.second.sel) (void)hipFree(sc.second.sel);
    }
  }
  (void)hipSetDevice(cur);
  g_dev.clear();
  (void)hipGetLastError();
}

}  // extern "C"

// ---- the no-allocation SSCA entry point -------------------------------------------------------------------
// Its scratch is a file-scope device array: the FP64-generated tables, then one signal's intermediate. Every GPU
// the library runs on holds its own copy until the process ends. Host code never passes the array's name to a
// kernel: it takes the array's address on each device once (hipGetSymbolAddress, with that device current) and
// uses that pointer.
namespace {
constexpr size_t kNoAllocTabBytes = 256 * ((sizeof(float2) * scd::kTabSize + 255) / 256);
constexpr size_t kNoAllocInterBytes = size_t{64} << 20;
constexpr size_t kNoAllocBytes = kNoAllocTabBytes + kNoAllocInterBytes;
constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
// The device address of this device's scratch (library lock held).
int noalloc_scratch(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(SCD_ERR_UNSUPPORTED, "device %d is beyond the library's limit", dev);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "scratch address");
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
  return SCD_OK;
}
}  // namespace

extern "C" {

size_t scd_ssca_noalloc_limit(void) { return kNoAllocInterBytes; }

int scd_ssca_noalloc(const float* x, int64_t N, int Np, const float* win, float* out, const scd_opts* opts) {
  if (!x || !win || !out) return fail(SCD_ERR_NULL, "input, window and output must be non-NULL");
  if (!is_pow2(N) || N < 1024 || N > (1 << 20))
    return fail(SCD_ERR_SIZE, "N = %lld must be a power of two in [2^10, 2^20]", static_cast<long long>(N));
  if (!is_pow2(Np) || Np < 16 || Np > 256) return fail(SCD_ERR_SIZE, "Np = %d must be a power of two in [16, 256]", Np);
  if (opts && opts->batch > 1) return fail(SCD_ERR_UNSUPPORTED, "scd_ssca_noalloc takes one signal per call");
  if (opts && opts->precision != SCD_FP32) return fail(SCD_ERR_UNSUPPORTED, "scd_ssca_noalloc runs in FP32 only");
  if (opts && (opts->workspace || opts->workspace_bytes))
    return fail(SCD_ERR_UNSUPPORTED, "scd_ssca_noalloc uses its own scratch, not a workspace");
  const int64_t grid = static_cast<int64_t>(Np) * N;
  const size_t inter = N > 1024 ? 8u * static_cast<size_t>(grid) : 0;
  if (inter > kNoAllocInterBytes)
    return fail(SCD_ERR_SIZE, "Np * N * 8 = %zu bytes exceeds the %zu-byte scratch of scd_ssca_noalloc", inter,
                kNoAllocInterBytes);
  const size_t ob = 8u * static_cast<size_t>(grid);
  if (overlaps(out, ob, x, 8u * static_cast<size_t>(N)) || overlaps(out, ob, win, 4u * Np))
    return fail(SCD_ERR_ALIAS, "output overlaps an input");
  const hipStream_t s = (opts && opts->stream) ? static_cast<hipStream_t>(opts->stream) : g_stream;
  std::lock_guard<std::mutex> lk(g_mu);
  int rc, dev;
  if ((rc = check_device_range(x, 8u * static_cast<size_t>(N), "x"))) return rc;
  if ((rc = check_device_range(win, 4u * Np, "win"))) return rc;
  if ((rc = check_device_range(out, ob, "out"))) return rc;
  if ((rc = current_device(&dev))) return rc;
  unsigned char* base;
  if ((rc = noalloc_scratch(dev, &base))) return rc;
  // Tables are regenerated by every call (the scratch keeps whatever the last call on this device left).
  float2* tabs = reinterpret_cast<float2*>(base);
  float2* T = reinterpret_cast<float2*>(base + kNoAllocTabBytes);
  hipError_t e = scd::launch_gen_roots(tabs + scd::kTabTw1024, 1024, 1024, s);
  if (e == hipSuccess) e = scd::launch_gen_roots(tabs + scd::kTabRotLo, 1024, static_cast<int>(N), s);
  if (e == hipSuccess) e = scd::launch_gen_roots(tabs + scd::kTabRoots, Np, Np, s);
  const scd::SelArg sel = scd::selarg_all(Np);
  const float2* xc = reinterpret_cast<const float2*>(x);
  float2* oc = reinterpret_cast<float2*>(out);
  const int n = static_cast<int>(N);
  if (e == hipSuccess) {
    if (inter == 0) {  // N == 1024: the Stage 1 output is the result
      e = scd::launch_ssca_pass1_fp32(xc, n, Np, win, tabs, oc, 1, N, grid, sel, s);
    } else {
      e = scd::launch_ssca_pass1_fp32(xc, n, Np, win, tabs, T, 1, N, grid, sel, s);
      if (e == hipSuccess) e = scd::launch_ssca_pass2(T, n, Np, tabs, oc, 1, grid, grid, sel, s);
    }
  }
  if (e != hipSuccess) return hip_fail(e, "scd_ssca_noalloc launch");
  return SCD_OK;
}

}  // extern "C"
