// gs_exhaustive_noalloc: the exhaustive sum of gauss_sum (method
// GS_EXHAUSTIVE) for callers that cannot allocate device memory.  Every
// intermediate (validation flag, largest weight, reference records, partial
// sums per reference split) lives in one fixed device array of this file, so
// the call makes no hipMalloc, hipFree or allocating library call.  It runs
// the same kernels as the allocating path, in the same configuration, so its
// results are bit-identical to gauss_sum's exhaustive path.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "../../include/gausssum.h"
#include "gs_host.h"
#include "gs_internal.h"

struct gs_ctx : gs::gs_ctx_base {};

using namespace gs;

namespace {

// One array per device, held until the process ends.  In host code its name
// is only a stand-in for the device symbol: host code uses the address that
// hipGetSymbolAddress returns for the current device, never the name.
static __device__ __align__(256) unsigned char scratch[GS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device`, looked up once per device with
// that device current (each device holds its own copy at its own address).
hipError_t scratch_for(int device, unsigned char** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = p;
  }
  *out = static_cast<unsigned char*>(g_scratch_ptr[device]);
  return hipSuccess;
}

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

#define NA_FAIL(ctx, code, msg) \
  do {                          \
    (ctx)->err = (msg);         \
    return (code);              \
  } while (0)

#define NA_HIP(ctx, call)                                                              \
  do {                                                                                 \
    hipError_t _e = (call);                                                            \
    if (_e != hipSuccess) {                                                            \
      (void)hipGetLastError();                                                         \
      (void)hipStreamSynchronize((ctx)->stream);                                       \
      (void)hipGetLastError();                                                         \
      (ctx)->err = std::string("HIP error in ") + #call + ": " + hipGetErrorString(_e); \
      return GS_EDEVICE;                                                               \
    }                                                                                  \
  } while (0)

extern "C" gs_status gs_exhaustive_noalloc(gs_ctx* ctx, const double* queries, int64_t M,
                                           const double* refs, const double* weights, int64_t N,
                                           int32_t D, const double* bandwidths, int32_t n_h,
                                           double* G_out) {
  if (!ctx) return GS_EINVAL;
  ctx->err.clear();
  if (!queries || !refs || !weights || !bandwidths || !G_out)
    NA_FAIL(ctx, GS_EINVAL, "null array pointer");
  if (M < 1 || N < 1 || n_h < 1) NA_FAIL(ctx, GS_EINVAL, "M, N and n_h must be >= 1");
  if (D < 1 || D > kMaxD) NA_FAIL(ctx, GS_EINVAL, "D must be in [1, 64]");
  if (n_h > 4096) NA_FAIL(ctx, GS_EINVAL, "at most 4096 bandwidths per call");
  if (M > INT32_MAX / 2 || N > INT32_MAX / 2) NA_FAIL(ctx, GS_EOVERFLOW, "M and N must be < 2^30");
  if (ctx->device < 0 || ctx->device >= kMaxDevices)
    NA_FAIL(ctx, GS_EINVAL, "device index beyond the devices this entry point serves");
  NA_HIP(ctx, hipSetDevice(ctx->device));
  if (!is_device_pointer(queries) || !is_device_pointer(refs) || !is_device_pointer(weights) ||
      !is_device_pointer(G_out))
    NA_FAIL(ctx, GS_EINVAL, "queries, refs, weights and G_out must be device pointers");
  if (is_device_pointer(bandwidths)) NA_FAIL(ctx, GS_EINVAL, "bandwidths must be a host pointer");
  for (int k = 0; k < n_h; ++k)
    if (!(bandwidths[k] > 0.0) || !std::isfinite(bandwidths[k]))
      NA_FAIL(ctx, GS_EINVAL, "every bandwidth must be finite and > 0");

  // Layout of the scratch array: flags, records, partial sums.
  const size_t rec_bytes = round256((size_t)N * exhaustive_record_stride(D) * sizeof(float));
  const size_t part_bytes = round256(exhaustive_partial_elems_exact(M, N, D, n_h) * sizeof(double));
  const size_t need = 256 + rec_bytes + part_bytes;
  if (need > (size_t)GS_NOALLOC_SCRATCH_BYTES)
    NA_FAIL(ctx, GS_EOVERFLOW,
            "the call needs " + std::to_string(need) + " bytes of scratch; the fixed array holds " +
                std::to_string((size_t)GS_NOALLOC_SCRATCH_BYTES));
  unsigned char* base = nullptr;
  NA_HIP(ctx, scratch_for(ctx->device, &base));
  int* bad = reinterpret_cast<int*>(base);                                   // bytes 0..3
  unsigned long long* wmax = reinterpret_cast<unsigned long long*>(base + 8);  // bytes 8..15
  float* rec = reinterpret_cast<float*>(base + 256);
  double* partial = reinterpret_cast<double*>(base + 256 + rec_bytes);

  hipStream_t st = ctx->stream;
  // The flag and the largest weight start at zero (a fill kernel, no memset).
  NA_HIP(ctx, launch_fill(reinterpret_cast<double*>(base), 2, 0.0, st));
  NA_HIP(ctx, launch_check_finite(queries, M * D, bad, st));
  if (refs != queries) NA_HIP(ctx, launch_check_finite(refs, N * D, bad, st));
  NA_HIP(ctx, launch_check_positive(weights, N, bad, st));
  int bad_h = 0;
  NA_HIP(ctx, hipMemcpyAsync(&bad_h, bad, sizeof(int), hipMemcpyDeviceToHost, st));
  NA_HIP(ctx, hipStreamSynchronize(st));
  if (bad_h & 1) NA_FAIL(ctx, GS_EINVAL, "a coordinate is NaN or infinite");
  if (bad_h & 2) NA_FAIL(ctx, GS_EINVAL, "every weight must be finite and > 0");

  NA_HIP(ctx, launch_exhaustive_records(refs, weights, N, D, rec, wmax, st));
  NA_HIP(ctx, launch_exhaustive(queries, M, rec, N, D, bandwidths, n_h, wmax, partial, G_out, st));
  NA_HIP(ctx, hipStreamSynchronize(st));
  return GS_OK;
}
