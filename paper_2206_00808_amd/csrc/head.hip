// Small-q head and wings in double precision.
//
// At a small momentum transfer q0 the G = 0 element M_vc(0) is O(|q0|) while
// v(q0+0) ~ 1/|q0|^2, so the head of eps is sensitive to the relative error of
// M_vc(0).  M_vc(0) is the G = 0 term of the matrix-element definition
// (Sec. II): the overlap sum_s sum_G conj(c_v^s(G)) c_c^s(G) of the periodic
// parts, evaluated here directly in double from the sphere coefficients.  The
// head chi0[h][h] and the wings chi0[h][G'], chi0[G'][h] are then accumulated
// in double from it, whatever the precision of the rest of the contraction.
#include "common.h"

namespace gw {

template <typename Tin>
__global__ void __launch_bounds__(256) k_head_overlap(const cpx<Tin>* __restrict__ cv, int ngv,
                                                      const cpx<Tin>* __restrict__ cc, int ngc,
                                                      int nspinor, int nc,
                                                      const int2* __restrict__ match, int nmatch,
                                                      cpx<double>* __restrict__ mhead) {
  __shared__ double sr[256], si[256];
  const int p = blockIdx.x;
  const int v = p / nc, c = p % nc;
  double ar = 0.0, ai = 0.0;
  for (int s = 0; s < nspinor; ++s) {
    const cpx<Tin>* a = cv + ((size_t)v * nspinor + s) * ngv;
    const cpx<Tin>* b = cc + ((size_t)c * nspinor + s) * ngc;
    for (int m = threadIdx.x; m < nmatch; m += blockDim.x) {
      const int2 ix = match[m];
      const cpx<Tin> x = a[ix.x], y = b[ix.y];
      const double xr = x.x, xi = x.y, yr = y.x, yi = y.y;
      ar += xr * yr + xi * yi;
      ai += xr * yi - xi * yr;
    }
  }
  sr[threadIdx.x] = ar;
  si[threadIdx.x] = ai;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sr[threadIdx.x] += sr[threadIdx.x + s];
      si[threadIdx.x] += si[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) mhead[p] = mk(sr[0], si[0]);
}

gw_status head_overlap(gw_ctx* c, gw_dtype dt, int nspinor, int nv, int ngv, const void* cv,
                       int nc, int ngc, const void* cc, const int* d_match, int nmatch,
                       double* mhead) {
  const int P = nv * nc;
  if (P == 0) return GW_OK;
  ProfScope ps(c, "head_overlap");
  if (dt == GW_C128)
    hipLaunchKernelGGL(k_head_overlap<double>, dim3(P), dim3(256), 0, c->stream,
                       static_cast<const cpx<double>*>(cv), ngv,
                       static_cast<const cpx<double>*>(cc), ngc, nspinor, nc,
                       reinterpret_cast<const int2*>(d_match), nmatch,
                       reinterpret_cast<cpx<double>*>(mhead));
  else
    hipLaunchKernelGGL(k_head_overlap<float>, dim3(P), dim3(256), 0, c->stream,
                       static_cast<const cpx<float>*>(cv), ngv, static_cast<const cpx<float>*>(cc),
                       ngc, nspinor, nc, reinterpret_cast<const int2*>(d_match), nmatch,
                       reinterpret_cast<cpx<double>*>(mhead));
  GW_CHECK_LAUNCH(c, "k_head_overlap");
  return GW_OK;
}

// The head from momentum matrix elements at one k-point (Sec. II, optical
// absorption: the dipole relation with the momentum operator standing in for
// the velocity): M_vc(q, 0) = q.P_vc / (E_v - E_c) to first order in q, with
// P_vc = sum_s sum_G conj(c_v^s(G)) (k+G) c_c^s(G). q.(k+G) = sum_i g_i sq_i + q0k
// with sq_i = 2 pi q_i / a_i and q0k = sum_i k_i sq_i (the host folds the cell
// and k in). One workgroup per pair; the pair sum is reduced in a fixed order.
template <typename Tin>
__global__ void __launch_bounds__(256) k_head_dipole(const cpx<Tin>* __restrict__ cv,
                                                     const cpx<Tin>* __restrict__ cc, int ng,
                                                     int nspinor, int nc,
                                                     const int* __restrict__ g, double sq0,
                                                     double sq1, double sq2, double q0k,
                                                     const double* __restrict__ ev,
                                                     const double* __restrict__ ec,
                                                     cpx<double>* __restrict__ mhead) {
  __shared__ double sr[256], si[256];
  const int p = blockIdx.x;
  const int v = p / nc, c = p % nc;
  double ar = 0.0, ai = 0.0;
  for (int s = 0; s < nspinor; ++s) {
    const cpx<Tin>* a = cv + ((size_t)v * nspinor + s) * ng;
    const cpx<Tin>* b = cc + ((size_t)c * nspinor + s) * ng;
    for (int m = threadIdx.x; m < ng; m += blockDim.x) {
      const double qd = g[3 * m] * sq0 + g[3 * m + 1] * sq1 + g[3 * m + 2] * sq2 + q0k;
      const cpx<Tin> x = a[m], y = b[m];
      const double xr = x.x, xi = x.y, yr = y.x, yi = y.y;
      ar += qd * (xr * yr + xi * yi);
      ai += qd * (xr * yi - xi * yr);
    }
  }
  sr[threadIdx.x] = ar;
  si[threadIdx.x] = ai;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sr[threadIdx.x] += sr[threadIdx.x + s];
      si[threadIdx.x] += si[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double d = ev[v] - ec[c];
    mhead[p] = mk(sr[0] / d, si[0] / d);
  }
}

gw_status head_dipole(gw_ctx* c, gw_dtype dt, int nspinor, int nv, int nc, int ng,
                      const void* cv, const void* cc, const int* d_g, const double sq[3],
                      double q0k, const double* ev, const double* ec, double* mhead) {
  const int P = nv * nc;
  if (P == 0) return GW_OK;
  ProfScope ps(c, "head_dipole");
  if (dt == GW_C128)
    hipLaunchKernelGGL(k_head_dipole<double>, dim3(P), dim3(256), 0, c->stream,
                       static_cast<const cpx<double>*>(cv), static_cast<const cpx<double>*>(cc),
                       ng, nspinor, nc, d_g, sq[0], sq[1], sq[2], q0k, ev, ec,
                       reinterpret_cast<cpx<double>*>(mhead));
  else
    hipLaunchKernelGGL(k_head_dipole<float>, dim3(P), dim3(256), 0, c->stream,
                       static_cast<const cpx<float>*>(cv), static_cast<const cpx<float>*>(cc), ng,
                       nspinor, nc, d_g, sq[0], sq[1], sq[2], q0k, ev, ec,
                       reinterpret_cast<cpx<double>*>(mhead));
  GW_CHECK_LAUNCH(c, "k_head_dipole");
  return GW_OK;
}

// chi0[f][h][j] += sum_p conj(mh_p) w_f(p) X_p(j), X_p(j) = M_p(j) (j != h) or mh_p (j = h);
// chi0[f][j][h] += the conjugate for j != h. A block takes kWingCols columns; its
// kWingSlices thread rows split the pair sum and are added in a fixed order.
constexpr int kWingCols = 32, kWingSlices = 8;
template <typename Tin>
__global__ void __launch_bounds__(kWingCols * kWingSlices) k_wings(
    const cpx<Tin>* __restrict__ M, int P, int neps, const cpx<double>* __restrict__ mh, int h,
    const double* __restrict__ wts, cpx<double>* __restrict__ chi) {
  __shared__ double red[kWingSlices][kWingCols][2];
  const int cl = threadIdx.x % kWingCols, r = threadIdx.x / kWingCols;
  const int j = blockIdx.x * kWingCols + cl;
  const int f = blockIdx.y;
  const double* w = wts + (size_t)f * P;
  double sr = 0.0, si = 0.0;
  if (j < neps) {
    for (int p = r; p < P; p += kWingSlices) {
      const cpx<double> a = mh[p];
      double xr, xi;
      if (j == h) {
        xr = a.x; xi = a.y;
      } else {
        const cpx<Tin> m = M[(size_t)p * neps + j];
        xr = m.x; xi = m.y;
      }
      const double wp = w[p];
      sr += wp * (a.x * xr + a.y * xi);
      si += wp * (a.x * xi - a.y * xr);
    }
  }
  red[r][cl][0] = sr;
  red[r][cl][1] = si;
  __syncthreads();
  if (r != 0 || j >= neps) return;
  for (int q = 1; q < kWingSlices; ++q) {
    sr += red[q][cl][0];
    si += red[q][cl][1];
  }
  cpx<double>* C = chi + (size_t)f * neps * neps;
  cpx<double>* d = C + (size_t)h * neps + j;
  *d = mk(d->x + sr, d->y + si);
  if (j != h) {
    cpx<double>* m = C + (size_t)j * neps + h;
    *m = mk(m->x + sr, m->y - si);
  }
}

gw_status chi0_wings(gw_ctx* c, int P, int neps, const void* mtxel, gw_dtype dt,
                     const double* mhead, int head, int nfreq, const double* wts, double* chi0) {
  ProfScope ps(c, "chi0_wings");
  dim3 g((neps + kWingCols - 1) / kWingCols, nfreq);
  if (dt == GW_C128)
    hipLaunchKernelGGL(k_wings<double>, g, dim3(kWingCols * kWingSlices), 0, c->stream,
                       static_cast<const cpx<double>*>(mtxel), P, neps,
                       reinterpret_cast<const cpx<double>*>(mhead), head, wts,
                       reinterpret_cast<cpx<double>*>(chi0));
  else
    hipLaunchKernelGGL(k_wings<float>, g, dim3(kWingCols * kWingSlices), 0, c->stream,
                       static_cast<const cpx<float>*>(mtxel), P, neps,
                       reinterpret_cast<const cpx<double>*>(mhead), head, wts,
                       reinterpret_cast<cpx<double>*>(chi0));
  GW_CHECK_LAUNCH(c, "k_wings");
  return GW_OK;
}

}  // namespace gw
