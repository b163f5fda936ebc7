// Self-energy with the Hybertsen-Louie generalized plasmon-pole model.
//
// Sec. II splits the diagonal self-energy into a screened-exchange (SX) term
// over occupied states, with eps^-1 at the frequency E - E_n'', and a
// Coulomb-hole (COH) term over all states, an integral over the spectral
// weight of eps^-1.  With the plasmon-pole model the paper uses, each element
// of eps^-1 is one pole,
//   eps^-1_GG'(w) = delta + Omega^2 / (w^2 - wt^2),
//   Omega^2 = wp^2 (q+G).(q+G') / |q+G|^2 rho(G-G') / rho(0),  wp^2 = 4 pi rho(0),
//   wt^2 = Omega^2 / (delta - eps^-1_GG'(0)),
// and with A = Omega^2 / wt, d = E - E_n'':
//   SX  element: delta + Omega^2 / (d^2 - wt^2) = delta + A/2 [1/(d - wt) - 1/(d + wt)]
//   COH element: Omega^2 / (2 wt (d - wt))        = A/2 / (d - wt)
// Sigma_n(E) = -sum_{n'' occ} m^H [SX v] m + sum_{n''} m^H [COH v] m, m = M_{n''n}.
// Modes with |delta - eps^-1| <= 1e-10 or Re wt^2 <= 0 carry no pole (A = 0).
//
// k_sigma_gpp keeps a 16 x 64 tile of (A, wt) in registers (four rows of one
// column per thread) and streams every n'' past it: the work per element and
// energy is one reciprocal (two for occupied n'') and about a dozen FP64
// operations, so the kernel is bound by the vector ALUs, not by memory.
// conj(M(G)) A is formed once per element and n'' and reused for every energy.
// Each thread sums its rows, then its column's v M(G'), over all n'' before a
// single reduction per band.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"

namespace gw {

namespace {
constexpr double kGppDropTol = 1e-10;
constexpr int kTR = 16, kTC = 64, kRows = 4, kChunk = 32;
constexpr int kRB = 4;  // rows sharing one reciprocal (kRows / kRB reciprocals per energy set)
}  // namespace

__global__ void k_gpp_modes(const double* __restrict__ qg, const int* __restrict__ g, int N,
                            const cpx<double>* __restrict__ rho, int n1, int n2, int n3,
                            const cpx<double>* __restrict__ einv, cpx<double>* __restrict__ amp,
                            cpx<double>* __restrict__ wt) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)N * N) return;
  const int i = (int)(e / N), j = (int)(e % N);
  const double rho0 = rho[0].x;
  const double qi0 = qg[3 * i], qi1 = qg[3 * i + 1], qi2 = qg[3 * i + 2];
  const double dot = qi0 * qg[3 * j] + qi1 * qg[3 * j + 1] + qi2 * qg[3 * j + 2];
  const double nrm = qi0 * qi0 + qi1 * qi1 + qi2 * qi2;
  int d0 = (g[3 * i] - g[3 * j]) % n1, d1 = (g[3 * i + 1] - g[3 * j + 1]) % n2,
      d2 = (g[3 * i + 2] - g[3 * j + 2]) % n3;
  d0 += d0 < 0 ? n1 : 0;
  d1 += d1 < 0 ? n2 : 0;
  d2 += d2 < 0 ? n3 : 0;
  const cpx<double> r = rho[((size_t)d0 * n2 + d1) * n3 + d2];
  const double s = 4.0 * M_PI * dot / nrm;  // wp^2 (q+G).(q+G')/|q+G|^2 / rho(0)
  const cpx<double> o2 = mk(s * r.x, s * r.y);
  const cpx<double> x = einv[e];
  const cpx<double> den = mk((i == j ? 1.0 : 0.0) - x.x, -x.y);
  const double dd = den.x * den.x + den.y * den.y;
  cpx<double> a = mk(0.0, 0.0), w = mk(1.0, 0.0);
  if (std::sqrt(dd) > kGppDropTol) {
    // wt^2 = o2 / den
    const cpx<double> w2 = mk((o2.x * den.x + o2.y * den.y) / dd, (o2.y * den.x - o2.x * den.y) / dd);
    if (w2.x > 0.0) {
      // principal square root with Re w2 > 0: re = sqrt((|w2| + Re)/2), im = Im / (2 re)
      const double re = std::sqrt(0.5 * (std::hypot(w2.x, w2.y) + w2.x));
      w = mk(re, w2.y / (2.0 * re));
      const double ww = w.x * w.x + w.y * w.y;
      a = mk((o2.x * w.x + o2.y * w.y) / ww, (o2.y * w.x - o2.x * w.y) / ww);  // o2 / wt
    }
  }
  amp[e] = a;
  wt[e] = w;
}

// 1 / x for x > 0 in double: the hardware reciprocal refined by two Newton
// steps (each squares the relative error), in place of the IEEE division
// sequence, which would dominate the element's cost
__device__ __forceinline__ double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(y, fma(-x, y, 1.0), y);
  return fma(y, fma(-x, y, 1.0), y);
}

template <typename Tin, int NE>
__global__ void __launch_bounds__(256, 3) k_sigma_gpp(
    const cpx<Tin>* __restrict__ m, int nn, int nocc, int nband, int N, int b0,
    const double* __restrict__ en, const double* __restrict__ v,
    const cpx<double>* __restrict__ amp, const cpx<double>* __restrict__ wt,
    const double* __restrict__ energies, int ntc, cpx<double>* __restrict__ part) {
  __shared__ cpx<double> mrow[kChunk][kTR];
  __shared__ cpx<double> wcol[kChunk][kTC];
  __shared__ double red[4][4 * NE];
  const int tile = blockIdx.x, n = b0 + blockIdx.y;
  const int ti = tile / ntc, tj = tile % ntc;
  const int t = threadIdx.x, c = t % kTC, rg = t / kTC;
  const int col = tj * kTC + c;
  const int row0 = ti * kTR + rg * kRows;
  cpx<double> A[kRows], W[kRows];
#pragma unroll
  for (int r = 0; r < kRows; ++r) {
    const int row = row0 + r;
    const bool in = row < N && col < N;
    A[r] = in ? amp[(size_t)row * N + col] : mk(0.0, 0.0);
    W[r] = in ? wt[(size_t)row * N + col] : mk(1.0, 0.0);
  }
  const int diag = (col >= row0 && col < row0 + kRows && col < N) ? col - row0 : -1;
  double WY2[kRows];
#pragma unroll
  for (int r = 0; r < kRows; ++r) WY2[r] = W[r].y * W[r].y;
  double E[NE];
#pragma unroll
  for (int k = 0; k < NE; ++k) E[k] = energies[(size_t)n * NE + k];
  cpx<double> acoh[NE], asx[NE];
#pragma unroll
  for (int k = 0; k < NE; ++k) acoh[k] = asx[k] = mk(0.0, 0.0);

  for (int a0 = 0; a0 < nn; a0 += kChunk) {
    const int na = nn - a0 < kChunk ? nn - a0 : kChunk;
    __syncthreads();
    // stage conj-ready M rows and v M columns of the next n'' chunk
    for (int idx = t; idx < kChunk * (kTR + kTC); idx += 256) {
      const int s = idx / (kTR + kTC), o = idx % (kTR + kTC);
      cpx<double> val = mk(0.0, 0.0);
      if (s < na) {
        const size_t base = ((size_t)(a0 + s) * nband + n) * N;
        if (o < kTR) {
          const int gg = ti * kTR + o;
          if (gg < N) {
            const cpx<Tin> x = m[base + gg];
            val = mk((double)x.x, (double)x.y);
          }
          mrow[s][o] = val;
        } else {
          const int gg = tj * kTC + (o - kTR);
          if (gg < N) {
            const cpx<Tin> x = m[base + gg];
            val = mk(v[gg] * (double)x.x, v[gg] * (double)x.y);
          }
          wcol[s][o - kTR] = val;
        }
      }
    }
    __syncthreads();
    for (int s = 0; s < na; ++s) {
      const int a = a0 + s;
      const double ea = en[a];
      const bool occ = a < nocc;
      const cpx<double> wc = wcol[s][c];
      cpx<double> tc[NE], ts[NE];
#pragma unroll
      for (int k = 0; k < NE; ++k) tc[k] = ts[k] = mk(0.0, 0.0);
      if (!occ && NE <= 3) {
        // empty n'': COH only.  The reciprocals of |d - wt|^2 for kRB rows and every
        // energy come from one hardware reciprocal of their product (prefix
        // products, then back-substitution)
#pragma unroll
        for (int g0 = 0; g0 < kRows; g0 += kRB) {
          double z1[kRB][NE], x[kRB][NE], pre[kRB * NE];
#pragma unroll
          for (int r = 0; r < kRB; ++r)
#pragma unroll
            for (int k = 0; k < NE; ++k) {
              z1[r][k] = (E[k] - ea) - W[g0 + r].x;
              x[r][k] = fma(z1[r][k], z1[r][k], WY2[g0 + r]);
              const int i = r * NE + k;
              pre[i] = i == 0 ? x[0][0] : pre[i - 1] * x[r][k];
            }
          double rr = rcp_nr(pre[kRB * NE - 1]);
#pragma unroll
          for (int r = kRB - 1; r >= 0; --r) {
            const cpx<double> mr = mrow[s][rg * kRows + g0 + r];
            // conj(M(G)) A conj(d - wt) / |d - wt|^2 = A conj(M) / (d - wt); the
            // products of B with Im wt are the same for every energy
            const cpx<double> B = cmulc(mr, A[g0 + r]);
            const double byw = B.y * W[g0 + r].y, bxw = B.x * W[g0 + r].y;
#pragma unroll
            for (int k = NE - 1; k >= 0; --k) {
              const int i = r * NE + k;
              const double inv = i == 0 ? rr : rr * pre[i - 1];
              rr *= x[r][k];
              const cpx<double> b1 = mk(fma(B.x, z1[r][k], -byw), fma(B.y, z1[r][k], bxw));
              tc[k] = mk(fma(inv, b1.x, tc[k].x), fma(inv, b1.y, tc[k].y));
            }
          }
        }
      } else if (!occ) {
        // empty n'', four energies: the NE reciprocals of |d - wt|^2 come from one
        // hardware reciprocal of their product (prefix products, then back-substitution)
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
          const cpx<double> mr = mrow[s][rg * kRows + r];
          // conj(M(G)) A is the same for every energy; A/(d - wt) = A conj(d - wt) / |d - wt|^2
          const cpx<double> B = cmulc(mr, A[r]);
          const double wx = W[r].x, wy = W[r].y, wy2 = wy * wy;
          double z1[NE], x[NE], pre[NE], inv[NE];
#pragma unroll
          for (int k = 0; k < NE; ++k) {
            z1[k] = (E[k] - ea) - wx;
            x[k] = fma(z1[k], z1[k], wy2);
            pre[k] = k == 0 ? x[0] : pre[k - 1] * x[k];
          }
          double rr = rcp_nr(pre[NE - 1]);
#pragma unroll
          for (int k = NE - 1; k > 0; --k) {
            inv[k] = rr * pre[k - 1];
            rr *= x[k];
          }
          inv[0] = rr;
#pragma unroll
          for (int k = 0; k < NE; ++k) {
            // B (z1 + i wy) = B conj(d - wt)
            const cpx<double> b1 = mk(fma(B.x, z1[k], -B.y * wy), fma(B.x, wy, B.y * z1[k]));
            tc[k] = mk(fma(inv[k], b1.x, tc[k].x), fma(inv[k], b1.y, tc[k].y));
          }
        }
      } else {
        // occupied n'': COH and SX, one refined reciprocal per denominator
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
          const cpx<double> mr = mrow[s][rg * kRows + r];
          const cpx<double> B = cmulc(mr, A[r]);
          const double wx = W[r].x, wy = W[r].y;
#pragma unroll
          for (int k = 0; k < NE; ++k) {
            const double d = E[k] - ea;
            const double z1 = d - wx;
            const double y1 = rcp_nr(fma(z1, z1, wy * wy));
            const cpx<double> b1 = mk(fma(B.x, z1, -B.y * wy), fma(B.x, wy, B.y * z1));
            tc[k] = mk(fma(y1, b1.x, tc[k].x), fma(y1, b1.y, tc[k].y));
            const double z2 = d + wx;
            const double y2 = rcp_nr(fma(z2, z2, wy * wy));
            // B conj(d + wt) = B (z2 - i wy)
            const cpx<double> b2 = mk(fma(B.x, z2, B.y * wy), fma(B.y, z2, -B.x * wy));
            cpx<double> f = mk(0.5 * fma(y1, b1.x, -y2 * b2.x), 0.5 * fma(y1, b1.y, -y2 * b2.y));
            if (r == diag) f = f + mk(mr.x, -mr.y);
            ts[k] = ts[k] + f;
          }
        }
      }
#pragma unroll
      for (int k = 0; k < NE; ++k) {
        acoh[k] = acoh[k] + cmul(tc[k], wc);
        asx[k] = asx[k] + cmul(ts[k], wc);
      }
    }
  }
  // one reduction per band: 64-lane butterflies, then the four wavefronts in order
  double vals[4 * NE];
#pragma unroll
  for (int k = 0; k < NE; ++k) {
    vals[4 * k] = acoh[k].x;
    vals[4 * k + 1] = acoh[k].y;
    vals[4 * k + 2] = asx[k].x;
    vals[4 * k + 3] = asx[k].y;
  }
#pragma unroll
  for (int q = 0; q < 4 * NE; ++q)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) vals[q] += __shfl_xor(vals[q], off, 64);
  const int lane = t & 63, wave = t >> 6;
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < 4 * NE; ++q) red[wave][q] = vals[q];
  __syncthreads();
  if (t < 4 * NE) {
    const double sum = ((red[0][t] + red[1][t]) + red[2][t]) + red[3][t];
    reinterpret_cast<double*>(part)[((size_t)blockIdx.y * gridDim.x + tile) * 4 * NE + t] = sum;
  }
}

// sigma_coh[n][k] += pref * 0.5 * sum_tiles coh;  sigma_sx[n][k] -= pref * sum_tiles sx.
// One workgroup per (band, energy): strided partial sums, then a fixed-order tree.
template <int NE>
__global__ void __launch_bounds__(256) k_gpp_reduce(const cpx<double>* __restrict__ part,
                                                    int ntiles, int b0, double pref,
                                                    cpx<double>* __restrict__ sx,
                                                    cpx<double>* __restrict__ coh) {
  __shared__ double red[4][256];
  const int nb = blockIdx.x / NE, k = blockIdx.x % NE, t = threadIdx.x;
  double cr = 0.0, ci = 0.0, sr = 0.0, si = 0.0;
  for (int tl = t; tl < ntiles; tl += 256) {
    const cpx<double>* p = part + ((size_t)nb * ntiles + tl) * 2 * NE;
    cr += p[2 * k].x;
    ci += p[2 * k].y;
    sr += p[2 * k + 1].x;
    si += p[2 * k + 1].y;
  }
  red[0][t] = cr;
  red[1][t] = ci;
  red[2][t] = sr;
  red[3][t] = si;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h)
      for (int q = 0; q < 4; ++q) red[q][t] += red[q][t + h];
    __syncthreads();
  }
  if (t == 0) {
    const size_t o = (size_t)(b0 + nb) * NE + k;
    coh[o] = coh[o] + scal(mk(red[0][0], red[1][0]), 0.5 * pref);
    sx[o] = sx[o] - scal(mk(red[2][0], red[3][0]), pref);
  }
}

template <typename Tin, int NE>
static gw_status sigma_gpp_run(gw_ctx* c, int nn, int nocc, int nband, int N, const void* mtxel,
                               const double* en, const double* vcoul, const double* amp,
                               const double* wt, const double* energies, double pref,
                               double* sx, double* coh) {
  const int ntr = (N + kTR - 1) / kTR, ntc = (N + kTC - 1) / kTC;
  const int ntiles = ntr * ntc;
  const size_t per_band = (size_t)ntiles * 2 * NE * 16;
  // bands per launch: partial sums kept under 256 MiB and the grid's y extent
  int nbc = (int)std::min<size_t>((size_t)nband, std::max<size_t>(1, (256u << 20) / per_band));
  nbc = std::min(nbc, 65535);
  gw_status st = ws_begin(c, align_up(per_band * nbc));
  if (st != GW_OK) return st;
  cpx<double>* part = static_cast<cpx<double>*>(ws_take(c, per_band * nbc));
  for (int b0 = 0; b0 < nband; b0 += nbc) {
    const int nb = std::min(nbc, nband - b0);
    {
      ProfScope ps(c, "sigma_gpp");
      hipLaunchKernelGGL((k_sigma_gpp<Tin, NE>), dim3(ntiles, nb), dim3(256), 0, c->stream,
                         static_cast<const cpx<Tin>*>(mtxel), nn, nocc, nband, N, b0, en, vcoul,
                         reinterpret_cast<const cpx<double>*>(amp),
                         reinterpret_cast<const cpx<double>*>(wt), energies, ntc, part);
      GW_CHECK_LAUNCH(c, "k_sigma_gpp");
    }
    ProfScope ps(c, "sigma_gpp_reduce");
    hipLaunchKernelGGL(k_gpp_reduce<NE>, dim3(nb * NE), dim3(256), 0, c->stream, part, ntiles, b0,
                       pref, reinterpret_cast<cpx<double>*>(sx), reinterpret_cast<cpx<double>*>(coh));
    GW_CHECK_LAUNCH(c, "k_gpp_reduce");
  }
  return GW_OK;
}

template <typename Tin>
static gw_status sigma_gpp_ne(gw_ctx* c, int ne, int nn, int nocc, int nband, int N,
                              const void* mtxel, const double* en, const double* vcoul,
                              const double* amp, const double* wt, const double* energies,
                              double pref, double* sx, double* coh) {
  switch (ne) {
    case 1: return sigma_gpp_run<Tin, 1>(c, nn, nocc, nband, N, mtxel, en, vcoul, amp, wt, energies, pref, sx, coh);
    case 2: return sigma_gpp_run<Tin, 2>(c, nn, nocc, nband, N, mtxel, en, vcoul, amp, wt, energies, pref, sx, coh);
    case 3: return sigma_gpp_run<Tin, 3>(c, nn, nocc, nband, N, mtxel, en, vcoul, amp, wt, energies, pref, sx, coh);
    default: return sigma_gpp_run<Tin, 4>(c, nn, nocc, nband, N, mtxel, en, vcoul, amp, wt, energies, pref, sx, coh);
  }
}

}  // namespace gw

using namespace gw;

extern "C" gw_status gw_gpp_modes(gw_ctx* c, int neps, const int* geps, const double* cell,
                                  const double* qred, const int* box, const double* rho,
                                  const double* epsinv, double* amp, double* wtilde) {
  if (!c) return GW_EINVAL;
  c->err.clear();
  if (neps < 0) return fail(c, GW_EINVAL, "negative size");
  if (neps == 0) return GW_OK;
  if (!geps || !cell || !qred || !box || !rho || !epsinv || !amp || !wtilde)
    return fail(c, GW_EINVAL, "NULL argument");
  if (neps > 46340) return fail(c, GW_EINVAL, "neps above 46340");
  if (amp == wtilde || amp == epsinv || wtilde == epsinv)
    return fail(c, GW_EINVAL, "amp, wtilde and epsinv must be distinct");
  for (int a = 0; a < 3; ++a) {
    if (!(cell[a] > 0.0) || !std::isfinite(cell[a]) || !std::isfinite(qred[a]))
      return fail(c, GW_EINVAL, "cell must be positive and q finite");
    if (box[a] <= 0) return fail(c, GW_EINVAL, "box must be positive");
  }
  std::vector<double> qg((size_t)neps * 3);
  int gmax[3] = {0, 0, 0};
  for (int i = 0; i < neps; ++i) {
    double n2 = 0.0;
    for (int a = 0; a < 3; ++a) {
      const int gi = geps[3 * i + a];
      gmax[a] = std::max(gmax[a], gi < 0 ? -gi : gi);
      qg[3 * i + a] = 2.0 * M_PI * (qred[a] + gi) / cell[a];
      n2 += qg[3 * i + a] * qg[3 * i + a];
    }
    if (!(n2 > 0.0)) return fail(c, GW_EINVAL, "q + G = 0 for eps vector %d", i);
  }
  for (int a = 0; a < 3; ++a)
    if (box[a] <= 2 * gmax[a])
      return fail(c, GW_EINVAL, "box %d along axis %d cannot hold G - G' (max |g| %d)", box[a],
                  a, gmax[a]);
  (void)hipSetDevice(c->device);
  cpx<double> r0;
  GW_HIP(c, hipMemcpyAsync(&r0, rho, sizeof(r0), hipMemcpyDeviceToHost, c->stream));
  GW_HIP(c, hipStreamSynchronize(c->stream));
  if (!(r0.x > 0.0) || !std::isfinite(r0.x)) return fail(c, GW_EINVAL, "rho(0) must be positive");
  const size_t bq = align_up((size_t)neps * 24);
  gw_status st = ws_begin(c, bq + align_up((size_t)neps * 12));
  if (st != GW_OK) return st;
  double* d_qg = static_cast<double*>(ws_take(c, (size_t)neps * 24));
  int* d_g = static_cast<int*>(ws_take(c, (size_t)neps * 12));
  GW_HIP(c, hipMemcpyAsync(d_qg, qg.data(), (size_t)neps * 24, hipMemcpyHostToDevice, c->stream));
  GW_HIP(c, hipMemcpyAsync(d_g, geps, (size_t)neps * 12, hipMemcpyHostToDevice, c->stream));
  const size_t nn = (size_t)neps * neps;
  {
    ProfScope ps(c, "gpp_modes");
    hipLaunchKernelGGL(k_gpp_modes, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, c->stream,
                       d_qg, d_g, neps, reinterpret_cast<const cpx<double>*>(rho), box[0], box[1],
                       box[2], reinterpret_cast<const cpx<double>*>(epsinv),
                       reinterpret_cast<cpx<double>*>(amp), reinterpret_cast<cpx<double>*>(wtilde));
    GW_CHECK_LAUNCH(c, "k_gpp_modes");
  }
  // qg and geps were staged from host memory: finish before returning
  GW_HIP(c, hipStreamSynchronize(c->stream));
  return GW_OK;
}

extern "C" gw_status gw_sigma_gpp(gw_ctx* c, int nn, int nocc, int nband, int neps,
                                  const void* mtxel, gw_dtype dtype, const double* en,
                                  const double* vcoul, const double* amp, const double* wtilde,
                                  int nenergy, const double* energies, double prefactor,
                                  double* sigma_sx, double* sigma_coh) {
  if (!c) return GW_EINVAL;
  c->err.clear();
  if (nn < 0 || nocc < 0 || nband < 0 || neps < 0) return fail(c, GW_EINVAL, "negative size");
  if (nocc > nn) return fail(c, GW_EINVAL, "nocc above nn");
  if (dtype != GW_C128 && dtype != GW_C64) return fail(c, GW_EINVAL, "unknown dtype");
  if (nenergy < 1 || nenergy > 4) return fail(c, GW_EINVAL, "nenergy must be 1 to 4");
  if (!std::isfinite(prefactor)) return fail(c, GW_EINVAL, "non-finite prefactor");
  if (nn == 0 || nband == 0 || neps == 0) return GW_OK;
  if (!mtxel || !en || !vcoul || !amp || !wtilde || !energies || !sigma_sx || !sigma_coh)
    return fail(c, GW_EINVAL, "NULL array argument");
  if (neps > 46340) return fail(c, GW_EINVAL, "neps above 46340");
  if (sigma_sx == sigma_coh) return fail(c, GW_EINVAL, "sigma_sx and sigma_coh must differ");
  (void)hipSetDevice(c->device);
  if (dtype == GW_C128)
    return sigma_gpp_ne<double>(c, nenergy, nn, nocc, nband, neps, mtxel, en, vcoul, amp, wtilde,
                                energies, prefactor, sigma_sx, sigma_coh);
  return sigma_gpp_ne<float>(c, nenergy, nn, nocc, nband, neps, mtxel, en, vcoul, amp, wtilde,
                             energies, prefactor, sigma_sx, sigma_coh);
}
