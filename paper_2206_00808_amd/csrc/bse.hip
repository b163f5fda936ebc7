// Exchange and direct kernels of the Bethe-Salpeter equation (Tamm-Dancoff form,
// one k-point), from the plane-wave matrix elements the Epsilon path computes.
//
// Sec. II: the spin dependence of K^X and K^D reduces to the spin trace inside
// M_nn'(G), so with v_x the bare Coulomb potential (long-range G = 0 term left
// out by the caller) and W the screened interaction on the eps sphere:
//   K^X_{vc,v'c'} =  sum_G     conj(M_vc(G)) v_x(G) M_v'c'(G),
//   K^D_{vc,v'c'} = -sum_{G,G'} conj(M_cc'(G)) W_GG' M_vv'(G').
// Both are dense contractions and run on the FP64 matrix-core GEMM:
//   K^X = [conj(M_vc) diag(v_x)] [M_vc]^T                       (P x N) (N x P)
//   T   = conj(M_cc) W,  R = T [M_vv]^T,  K^D[(v,c),(v',c')] = -R[(c,c')][(v,v')]
// The operands are widened to double, conjugated and transposed by small
// bandwidth-bound kernels first.
#include "common.h"

namespace gw {

// out[r][g] = conj(m[r][g]) * (scale ? scale[g] : 1), widened to double
template <typename Tin>
__global__ void k_conj_scale(const cpx<Tin>* __restrict__ m, size_t rows, int N,
                             const double* __restrict__ scale, cpx<double>* __restrict__ out) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * (size_t)N) return;
  const cpx<Tin> a = m[e];
  const double s = scale ? scale[e % N] : 1.0;
  out[e] = mk(s * (double)a.x, -s * (double)a.y);
}

// out[g][r] = m[r][g], widened to double; 32 x 32 tiles through LDS, row tiles
// on the grid's x dimension (the row count nv^2 may pass 65535 tiles), G tiles on y
template <typename Tin>
__global__ void __launch_bounds__(256) k_transpose(const cpx<Tin>* __restrict__ m, int rows,
                                                   int N, cpx<double>* __restrict__ out) {
  __shared__ cpx<double> t[32][33];
  const int g0 = blockIdx.y * 32, r0 = blockIdx.x * 32;
  for (int i = threadIdx.y; i < 32; i += 8) {
    const int r = r0 + i, g = g0 + threadIdx.x;
    if (r < rows && g < N) {
      const cpx<Tin> a = m[(size_t)r * N + g];
      t[i][threadIdx.x] = mk((double)a.x, (double)a.y);
    }
  }
  __syncthreads();
  for (int i = threadIdx.y; i < 32; i += 8) {
    const int g = g0 + i, r = r0 + threadIdx.x;
    if (g < N && r < rows) out[(size_t)g * rows + r] = t[threadIdx.x][i];
  }
}

// kd[(v*nc + c)][(u*nc + d)] = -R[(c*nc + d)][(v*nv + u)]
__global__ void k_bse_direct_order(const cpx<double>* __restrict__ R, int nv, int nc,
                                   cpx<double>* __restrict__ kd) {
  const size_t P = (size_t)nv * nc;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= P * P) return;
  const size_t row = e / P, col = e % P;
  const int v = (int)(row / nc), c = (int)(row % nc), u = (int)(col / nc), d = (int)(col % nc);
  const cpx<double> x = R[((size_t)c * nc + d) * ((size_t)nv * nv) + (size_t)v * nv + u];
  kd[e] = mk(-x.x, -x.y);
}

template <typename Tin>
static gw_status bse_run(gw_ctx* c, int nv, int nc, int N, const void* mvc, const void* mcc,
                         const void* mvv, const double* vx, const double* w, double* kx,
                         double* kd) {
  const size_t P = (size_t)nv * nc, C2 = (size_t)nc * nc, V2 = (size_t)nv * nv;
  const size_t nX = P * N, nT = C2 * N, nMv = V2 * N, nR = C2 * V2;
  gw_status st = ws_begin(c, 2 * align_up(nX * 16) + 2 * align_up(nT * 16) +
                                 align_up(nMv * 16) + align_up(nR * 16));
  if (st != GW_OK) return st;
  cpx<double>* X = static_cast<cpx<double>*>(ws_take(c, nX * 16));
  cpx<double>* Mt = static_cast<cpx<double>*>(ws_take(c, nX * 16));
  cpx<double>* Cc = static_cast<cpx<double>*>(ws_take(c, nT * 16));
  cpx<double>* T = static_cast<cpx<double>*>(ws_take(c, nT * 16));
  cpx<double>* MvT = static_cast<cpx<double>*>(ws_take(c, nMv * 16));
  cpx<double>* R = static_cast<cpx<double>*>(ws_take(c, nR * 16));
  const dim3 tb(32, 8);
  {
    ProfScope ps(c, "bse_prep");
    hipLaunchKernelGGL(k_conj_scale<Tin>, dim3((unsigned)((nX + 255) / 256)), dim3(256), 0,
                       c->stream, static_cast<const cpx<Tin>*>(mvc), P, N, vx, X);
    hipLaunchKernelGGL(k_transpose<Tin>, dim3((unsigned)((P + 31) / 32), (N + 31) / 32), tb, 0,
                       c->stream, static_cast<const cpx<Tin>*>(mvc), (int)P, N, Mt);
    hipLaunchKernelGGL(k_conj_scale<Tin>, dim3((unsigned)((nT + 255) / 256)), dim3(256), 0,
                       c->stream, static_cast<const cpx<Tin>*>(mcc), C2, N, nullptr, Cc);
    hipLaunchKernelGGL(k_transpose<Tin>, dim3((unsigned)((V2 + 31) / 32), (N + 31) / 32), tb, 0,
                       c->stream, static_cast<const cpx<Tin>*>(mvv), (int)V2, N, MvT);
    GW_CHECK_LAUNCH(c, "bse operand preparation");
  }
  // K^X = X Mt
  st = zgemm_nn(c, (int)P, (int)P, N, 1.0, reinterpret_cast<const double*>(X), 0, N, 0,
                reinterpret_cast<const double*>(Mt), 0, (int)P, 0, kx, 0, (int)P, 0, 1, nX, nX,
                P * P, 0.0);
  if (st != GW_OK) return st;
  // T = conj(M_cc) W;  R = T M_vv^T
  st = zgemm_nn(c, (int)C2, N, N, 1.0, reinterpret_cast<const double*>(Cc), 0, N, 0, w, 0, N, 0,
                reinterpret_cast<double*>(T), 0, N, 0, 1, nT, (size_t)N * N, nT, 0.0);
  if (st != GW_OK) return st;
  st = zgemm_nn(c, (int)C2, (int)V2, N, 1.0, reinterpret_cast<const double*>(T), 0, N, 0,
                reinterpret_cast<const double*>(MvT), 0, (int)V2, 0, reinterpret_cast<double*>(R),
                0, (int)V2, 0, 1, nT, nMv, nR, 0.0);
  if (st != GW_OK) return st;
  ProfScope ps(c, "bse_order");
  hipLaunchKernelGGL(k_bse_direct_order, dim3((unsigned)((P * P + 255) / 256)), dim3(256), 0,
                     c->stream, R, nv, nc, reinterpret_cast<cpx<double>*>(kd));
  GW_CHECK_LAUNCH(c, "k_bse_direct_order");
  return GW_OK;
}

}  // namespace gw

using namespace gw;

extern "C" gw_status gw_bse_kernel(gw_ctx* c, int nv, int nc, int neps, const void* mvc,
                                   const void* mcc, const void* mvv, gw_dtype dtype,
                                   const double* vx, const double* w, double* kx, double* kd) {
  if (!c) return GW_EINVAL;
  c->err.clear();
  if (nv < 0 || nc < 0 || neps < 0) return fail(c, GW_EINVAL, "negative size");
  if (dtype != GW_C128 && dtype != GW_C64) return fail(c, GW_EINVAL, "unknown dtype");
  if (nv == 0 || nc == 0) return GW_OK;
  if (!kx || !kd) return fail(c, GW_EINVAL, "NULL output");
  if (kx == kd) return fail(c, GW_EINVAL, "kx and kd must differ");
  const long long P = (long long)nv * nc;
  if (P > 46340 || (long long)nc * nc > 46340LL * 46340LL / 4 || neps > 46340)
    return fail(c, GW_EINVAL, "nv*nc above 46340 or neps above 46340");
  if (neps == 0) {
    (void)hipSetDevice(c->device);
    GW_HIP(c, hipMemsetAsync(kx, 0, (size_t)P * P * 16, c->stream));
    GW_HIP(c, hipMemsetAsync(kd, 0, (size_t)P * P * 16, c->stream));
    return GW_OK;
  }
  if (!mvc || !mcc || !mvv || !vx || !w) return fail(c, GW_EINVAL, "NULL array argument");
  const void* outs[2] = {kx, kd};
  const void* ins[5] = {mvc, mcc, mvv, vx, w};
  for (const void* o : outs)
    for (const void* i : ins)
      if (o == i) return fail(c, GW_EINVAL, "an output aliases an input");
  (void)hipSetDevice(c->device);
  if (dtype == GW_C128) return bse_run<double>(c, nv, nc, neps, mvc, mcc, mvv, vx, w, kx, kd);
  return bse_run<float>(c, nv, nc, neps, mvc, mcc, mvv, vx, w, kx, kd);
}
