// Measured peaks of the device the library runs on: an FP64 matrix-core loop,
// an FP64 vector FMA loop and a plain device copy.  They confirm the nominal
// roofline figures the kernels are compared against.
#include <vector>

#include "common.h"

namespace gw {

typedef double v4d __attribute__((ext_vector_type(4)));

// Eight independent 16x16x4 FP64 MFMA chains per wavefront (2048 flops each per
// instruction); the result is folded into one store so nothing is optimised away.
__global__ void __launch_bounds__(256) k_probe_mfma(int iters, double seed, double* __restrict__ out) {
  const double a = seed + threadIdx.x * 1e-9, b = 1.0 - threadIdx.x * 1e-9;
  v4d c0 = {0, 0, 0, 0}, c1 = c0, c2 = c0, c3 = c0, c4 = c0, c5 = c0, c6 = c0, c7 = c0;
  for (int i = 0; i < iters; ++i) {
    c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c3, 0, 0, 0);
    c4 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c4, 0, 0, 0);
    c5 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c5, 0, 0, 0);
    c6 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c6, 0, 0, 0);
    c7 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c7, 0, 0, 0);
  }
  const v4d s = c0 + c1 + c2 + c3 + c4 + c5 + c6 + c7;
  if (s.x + s.y + s.z + s.w == -1.0) out[blockIdx.x * blockDim.x + threadIdx.x] = s.x;
}

// Eight independent FP64 FMA chains per lane (2 flops each)
__global__ void __launch_bounds__(256) k_probe_fma(int iters, double seed, double* __restrict__ out) {
  double x0 = seed + threadIdx.x * 1e-9, x1 = x0 + 1, x2 = x0 + 2, x3 = x0 + 3, x4 = x0 + 4,
         x5 = x0 + 5, x6 = x0 + 6, x7 = x0 + 7;
  const double m = 0.999999, a = 1e-7;
  for (int i = 0; i < iters; ++i) {
    x0 = fma(x0, m, a);
    x1 = fma(x1, m, a);
    x2 = fma(x2, m, a);
    x3 = fma(x3, m, a);
    x4 = fma(x4, m, a);
    x5 = fma(x5, m, a);
    x6 = fma(x6, m, a);
    x7 = fma(x7, m, a);
  }
  const double s = x0 + x1 + x2 + x3 + x4 + x5 + x6 + x7;
  if (s == -1.0) out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void __launch_bounds__(256) k_probe_copy(const double4* __restrict__ src, size_t n,
                                                    double4* __restrict__ dst) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

}  // namespace gw

using namespace gw;

extern "C" gw_status gw_peak_probe(gw_ctx* c, int kind, double* result) {
  if (!c) return GW_EINVAL;
  c->err.clear();
  if (!result || kind < 0 || kind > 2) return fail(c, GW_EINVAL, "kind must be 0, 1 or 2");
  (void)hipSetDevice(c->device);
  int ncu = 0;
  GW_HIP(c, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device));
  double* out = nullptr;
  void* bufs = nullptr;
  const size_t copy_bytes = (size_t)1 << 30;  // 1 GiB read + 1 GiB written
  if (hipMalloc(reinterpret_cast<void**>(&out), 8 * 1024 * 1024) != hipSuccess)
    return fail(c, GW_ENOMEM, "probe output");
  if (kind == 2 && hipMalloc(&bufs, 2 * copy_bytes) != hipSuccess) {
    (void)hipFree(out);
    return fail(c, GW_ENOMEM, "probe copy buffers");
  }
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  // MFMA: 8 workgroups of 4 wavefronts per CU (eight per SIMD, eight chains each);
  // FMA: 8 workgroups per CU.  About 10 ms per run at the nominal rates.
  const int blocks = kind == 0 ? ncu * 8 : ncu * 8;
  const int iters = kind == 0 ? 5000 : 50000;
  float best = 1e30f;
  for (int rep = 0; rep < 4; ++rep) {
    (void)hipEventRecord(e0, c->stream);
    if (kind == 0)
      hipLaunchKernelGGL(k_probe_mfma, dim3(blocks), dim3(256), 0, c->stream, iters, 0.5, out);
    else if (kind == 1)
      hipLaunchKernelGGL(k_probe_fma, dim3(blocks), dim3(256), 0, c->stream, iters, 0.5, out);
    else
      hipLaunchKernelGGL(k_probe_copy, dim3(ncu * 16), dim3(256), 0, c->stream,
                         static_cast<const double4*>(bufs), copy_bytes / 32,
                         reinterpret_cast<double4*>(static_cast<char*>(bufs) + copy_bytes));
    (void)hipEventRecord(e1, c->stream);
    (void)hipEventSynchronize(e1);
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (rep > 0 && ms < best) best = ms;  // the first run warms up
  }
  const hipError_t le = hipGetLastError();
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(out);
  if (bufs) (void)hipFree(bufs);
  if (le != hipSuccess) return hip_fail(c, le, "probe kernel");
  const double sec = best * 1e-3;
  const double waves = (double)blocks * 4.0;
  if (kind == 0)
    *result = waves * iters * 8.0 * 2048.0 / sec / 1e12;  // TFLOP/s
  else if (kind == 1)
    *result = (double)blocks * 256.0 * iters * 8.0 * 2.0 / sec / 1e12;  // TFLOP/s
  else
    *result = 2.0 * copy_bytes / sec / 1e9;  // GB/s, read + write
  return GW_OK;
}
