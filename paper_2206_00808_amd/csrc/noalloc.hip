// The FP64 chi0 contraction without any allocation, for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid it): its only scratch, the pair weights, lives in a
// fixed device array of this library, and the frequencies travel by value in
// the kernel arguments.
#include <cmath>
#include <mutex>

#include "common.h"

namespace gw {

constexpr size_t kNoAllocScratch = 32u << 20;  // bytes: nfreq * nv * nc doubles at most
constexpr int kNoAllocMaxFreq = 64;
constexpr int kMaxDevices = 64;

// The weights' home on every device that runs this entry point (each device
// holds its own copy). In host code this name is only a handle for
// hipGetSymbolAddress, never an address.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratch];

static std::mutex g_scratch_mu;
static void* g_scratch_dev[kMaxDevices];  // device address of `scratch`, per device

// Address of `scratch` on the context's device, looked up once per device with
// that device current.
static gw_status scratch_address(gw_ctx* c, double** out) {
  if (c->device < 0 || c->device >= kMaxDevices)
    return fail(c, GW_EUNSUPPORTED, "device %d above the scratch table", c->device);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[c->device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(c, e, "hipGetSymbolAddress(scratch)");
    g_scratch_dev[c->device] = p;
  }
  *out = static_cast<double*>(g_scratch_dev[c->device]);
  return GW_OK;
}

struct OmegaArg {
  double w[kNoAllocMaxFreq];
};

// w[f][p] = pref (1/(d - i o_f) + 1/(d + i o_f)) = pref 2 d / (d^2 + o_f^2), d = e_v - e_c
__global__ void k_weights_byval(const double* __restrict__ ev, const double* __restrict__ ec,
                                int nv, int nc, OmegaArg om, int nfreq, double pref,
                                double* __restrict__ w) {
  const int P = nv * nc;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int f = blockIdx.y;
  if (p >= P || f >= nfreq) return;
  const double d = ev[p / nc] - ec[p % nc];
  const double o = om.w[f];
  w[(size_t)f * P + p] = pref * (2.0 * d / (d * d + o * o));
}

}  // namespace gw

using namespace gw;

extern "C" gw_status gw_chi0_accumulate_noalloc(gw_ctx* c, int nv, int nc, int neps,
                                                const void* mtxel, gw_dtype dtype,
                                                const double* ev, const double* ec, int nfreq,
                                                const double* omega, double prefactor,
                                                const double* mhead, int head_index,
                                                double* chi0) {
  if (!c) return GW_EINVAL;
  c->err.clear();
  if (nv < 0 || nc < 0 || neps < 0 || nfreq < 0) return fail(c, GW_EINVAL, "negative size");
  if (dtype != GW_C128 && dtype != GW_C64) return fail(c, GW_EINVAL, "unknown dtype");
  if (nv == 0 || nc == 0 || neps == 0 || nfreq == 0) return GW_OK;
  if (!mtxel || !ev || !ec || !omega || !chi0) return fail(c, GW_EINVAL, "NULL array argument");
  if (!std::isfinite(prefactor)) return fail(c, GW_EINVAL, "non-finite prefactor");
  if (nfreq > kNoAllocMaxFreq)
    return fail(c, GW_EINVAL, "nfreq %d above the %d frequencies this entry point carries", nfreq,
                kNoAllocMaxFreq);
  for (int f = 0; f < nfreq; ++f)
    if (!(omega[f] >= 0.0) || !std::isfinite(omega[f]))
      return fail(c, GW_EINVAL, "omega[%d] must be finite and >= 0", f);
  if (head_index >= neps) return fail(c, GW_EINVAL, "head_index >= neps");
  if ((long long)neps * neps > (1LL << 40)) return fail(c, GW_EINVAL, "neps too large");
  if ((long long)nv * nc > (1LL << 31) / 2) return fail(c, GW_EINVAL, "too many pairs");
  const int P = nv * nc;
  if ((size_t)nfreq * P * sizeof(double) > kNoAllocScratch)
    return fail(c, GW_EINVAL,
                "nfreq * nv * nc = %lld weights exceed the fixed scratch of %zu bytes",
                (long long)nfreq * P, kNoAllocScratch);
  (void)hipSetDevice(c->device);
  double* wts = nullptr;
  gw_status st = scratch_address(c, &wts);
  if (st != GW_OK) return st;
  OmegaArg om{};
  for (int f = 0; f < nfreq; ++f) om.w[f] = omega[f];
  {
    ProfScope ps(c, "chi0_weights");
    hipLaunchKernelGGL(k_weights_byval, dim3((P + 255) / 256, nfreq), dim3(256), 0, c->stream, ev,
                       ec, nv, nc, om, nfreq, prefactor, wts);
    GW_CHECK_LAUNCH(c, "k_weights_byval");
  }
  const bool use_head = mhead != nullptr && head_index >= 0;
  // one pair range: the ordered partial sums of more ranges would need memory
  if ((st = chi0_fp64(c, P, neps, mtxel, dtype, nfreq, wts, use_head ? head_index : -1, chi0, 1,
                      nullptr, /*no_alloc=*/true)) != GW_OK)
    return st;
  if (use_head) return chi0_wings(c, P, neps, mtxel, dtype, mhead, head_index, nfreq, wts, chi0);
  return GW_OK;
}
