// chi0 band-pair contraction on the matrix cores (Sec. II, Adler-Wiser
// polarizability at imaginary frequency):
//   chi0_f[i][j] += sum_p conj(M[p][i]) * w_f(p) * M[p][j],
//   w_f(p) = prefactor * (1/(D_p - i w_f) + 1/(D_p + i w_f)),  D_p = e_v - e_c.
// The update is Hermitian, so only tiles ti <= tj are computed; an
// off-diagonal tile is added at (ti,tj) and its conjugate transpose at (tj,ti).
//
// FP64 path: v_mfma_f64_16x16x4_f64, complex via four real products.
// Split-BF16 path: each float x = hi + lo with hi = bf16_rn(x), lo = bf16_rn(x - hi);
// real products use hi*hi + hi*lo + lo*hi on v_mfma_f32_16x16x32_bf16 with
// float accumulation over K-chunks that are flushed into double registers.
#include "tiles.h"

namespace gw {

// ---------------------------------------------------------------- weights
__global__ void k_weights(const double* __restrict__ ev, const double* __restrict__ ec, int nv,
                          int nc, const double* __restrict__ om, int nfreq, double pref,
                          double* __restrict__ w) {
  const int P = nv * nc;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int f = blockIdx.y;
  if (p >= P || f >= nfreq) return;
  const double d = ev[p / nc] - ec[p % nc];
  const double o = om[f];
  // 1/(d - i o) + 1/(d + i o) = 2 d / (d^2 + o^2)
  w[(size_t)f * P + p] = pref * (2.0 * d / (d * d + o * o));
}

gw_status chi0_weights(gw_ctx* c, int nv, int nc, const double* ev, const double* ec, int nfreq,
                       const double* d_omega, double pref, double* wts) {
  const int P = nv * nc;
  ProfScope ps(c, "chi0_weights");
  hipLaunchKernelGGL(k_weights, dim3((P + 255) / 256, nfreq), dim3(256), 0, c->stream, ev, ec, nv,
                     nc, d_omega, nfreq, pref, wts);
  GW_CHECK_LAUNCH(c, "k_weights");
  return GW_OK;
}

// Real-frequency weights with broadening eta > 0, split into two real sets:
// w[f][p] = pref Re b and w[nfreq + f][p] = pref Im b for the bracket
// b = 1/(d - o + i eta) + 1/(d + o + i eta), each term as (x - i eta)/(x^2 + eta^2).
__global__ void k_weights_real(const double* __restrict__ ev, const double* __restrict__ ec,
                               int nv, int nc, const double* __restrict__ om, int nfreq,
                               double eta, double pref, double* __restrict__ w) {
  const int P = nv * nc;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int f = blockIdx.y;
  if (p >= P || f >= nfreq) return;
  const double d = ev[p / nc] - ec[p % nc];
  const double xm = d - om[f], xp = d + om[f];
  const double qm = xm * xm + eta * eta, qp = xp * xp + eta * eta;
  w[(size_t)f * P + p] = pref * (xm / qm + xp / qp);
  w[(size_t)(nfreq + f) * P + p] = -pref * (eta / qm + eta / qp);
}

gw_status chi0_weights_real(gw_ctx* c, int nv, int nc, const double* ev, const double* ec,
                            int nfreq, const double* d_omega, double eta, double pref,
                            double* wts) {
  const int P = nv * nc;
  ProfScope ps(c, "chi0_weights");
  hipLaunchKernelGGL(k_weights_real, dim3((P + 255) / 256, nfreq), dim3(256), 0, c->stream, ev,
                     ec, nv, nc, d_omega, nfreq, eta, pref, wts);
  GW_CHECK_LAUNCH(c, "k_weights_real");
  return GW_OK;
}

// chi0[f] += A[f] + i B[f] for the Hermitian contractions A = h[f], B = h[nfreq + f]
__global__ void k_combine_real(const cpx<double>* __restrict__ h, size_t nn, int nfreq,
                               cpx<double>* __restrict__ chi) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nn) return;
  const size_t f = blockIdx.y;
  const cpx<double> a = h[f * nn + e], b = h[(nfreq + f) * nn + e];
  cpx<double>* o = chi + f * nn + e;
  *o = mk(o->x + (a.x - b.y), o->y + (a.y + b.x));
}

gw_status chi0_combine_real(gw_ctx* c, int neps, int nfreq, const double* h, double* chi0) {
  const size_t nn = (size_t)neps * neps;
  ProfScope ps(c, "chi0_combine");
  hipLaunchKernelGGL(k_combine_real, dim3((unsigned)((nn + 255) / 256), nfreq), dim3(256), 0,
                     c->stream, reinterpret_cast<const cpx<double>*>(h), nn, nfreq,
                     reinterpret_cast<cpx<double>*>(chi0));
  GW_CHECK_LAUNCH(c, "k_combine_real");
  return GW_OK;
}

// ---------------------------------------------------------------- single-q contractions
// Grid (upper-triangle tiles, frequencies, pair ranges). Range 0 adds into chi0;
// range s >= 1 covers pairs [s pc, (s+1) pc) and stores into partial matrix s-1.
// The grid is one-dimensional over (frequency, range, tile), renumbered per
// XCD; the tile order table groups the upper-triangle tiles into 8 x 16 blocks
// of the tile grid, so that the workgroups one XCD runs at a time share the
// operand rows of 8 tile rows and 16 tile columns in its L2.
template <int WM, typename Tin>
__global__ void __launch_bounds__(64 * WM * WM, sizeof(Tin) == 8 ? 3 : 2) k_chi0_f64(const cpx<Tin>* __restrict__ M, int P,
                                                           int neps, const double* __restrict__ wts,
                                                           cpx<double>* __restrict__ chi,
                                                           const int2* __restrict__ order,
                                                           int ntile, int split, int nf,
                                                           int skip_head, int pc,
                                                           cpx<double>* __restrict__ part) {
  const long long lin = xcd_linear(blockIdx.x, (long long)ntile * split * nf);
  if (lin < 0) return;
  int ti, tj;
  if (order) {
    const int2 tt = order[lin % ntile];
    ti = tt.x;
    tj = tt.y;
  } else {  // row-major over the triangle (callers that keep no table)
    int nt = 0;
    while (nt * (nt + 1) / 2 < ntile) ++nt;
    tri_tile((int)(lin % ntile), nt, &ti, &tj);
  }
  const int fs = (int)(lin / ntile), s = fs % split, f = fs / split;
  const int p0 = s * pc, np = min(P, p0 + pc) - p0;
  const size_t nn = (size_t)neps * neps;
  if (s == 0)
    chi0_f64_tile<WM, Tin>(M, np, neps, wts + (size_t)f * P, chi + (size_t)f * nn, ti, tj,
                           skip_head);
  else
    chi0_f64_tile<WM, Tin>(M + (size_t)p0 * neps, np, neps, wts + (size_t)f * P + p0,
                           part + ((size_t)(s - 1) * nf + f) * nn, ti, tj, skip_head, true);
}

// Split the contraction operands once: X_0 = M and X_{1+f} = w_f * M (the
// product taken in float), each component x as hi = bf16_rn(x) and
// lo = bf16_rn(x - hi). Output layout X_o[pb][q][G][32] (see chi0_bf16s_tile),
// zero past P. A block stages 32 pairs x 64 columns of M through LDS, so that
// both the reads of M and the writes are contiguous, and forms every output
// from that one tile (M is read from HBM once); each thread forms 8 values of
// one column per output and writes all four planes of them.
__global__ void __launch_bounds__(256) k_bf16_split(const cpx<float>* __restrict__ M, int P,
                                                    int neps, int nout,
                                                    const double* __restrict__ wts,
                                                    unsigned short* __restrict__ X) {
  __shared__ cpx<float> Ms[BK][64 + 1];
  typedef unsigned short us8 __attribute__((ext_vector_type(8)));
  const int pb = blockIdx.x, Pb = gridDim.x, g0 = blockIdx.y * 64;
  const int tid = threadIdx.x;
  for (int e = tid; e < BK * 64; e += 256) {
    const int k = e / 64, g = e % 64, p = pb * BK + k;
    Ms[k][g] = (p < P && g0 + g < neps) ? M[(size_t)p * neps + g0 + g] : mk(0.f, 0.f);
  }
  __syncthreads();
  const int row = tid / 4, kc = tid % 4, g = g0 + row;
  if (g >= neps) return;
  cpx<float> m[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) m[t] = Ms[kc * 8 + t][row];
  // every output from the one staged tile: M is read once for all of them
  for (int o = 0; o < nout; ++o) {
    us8 v[4];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int p = pb * BK + kc * 8 + t;
      const float wk = (o == 0) ? 1.f : (p < P ? (float)wts[(size_t)(o - 1) * P + p] : 0.f);
      const float xr = wk * m[t].x, xi = wk * m[t].y;
      const unsigned short hr = bf16_rn_bits(xr), hi = bf16_rn_bits(xi);
      v[0][t] = hr;
      v[1][t] = bf16_rn_bits(xr - bf16_to_f(hr));
      v[2][t] = hi;
      v[3][t] = bf16_rn_bits(xi - bf16_to_f(hi));
    }
    unsigned short* Xo = X + (size_t)o * Pb * 4 * neps * BK;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      *reinterpret_cast<us8*>(Xo + (((size_t)pb * 4 + q) * neps + g) * BK + kc * 8) = v[q];
  }
}

// Range s of the pair blocks of frequency f, from the pre-split operands.
template <int WM>
__global__ void __launch_bounds__(64 * WM * WM) k_chi0_bf16s(const unsigned short* __restrict__ X,
                                                             int Pb, int neps,
                                                             cpx<double>* __restrict__ chi, int nt,
                                                             int skip_head, int pbc,
                                                             cpx<double>* __restrict__ part) {
  int ti, tj;
  tri_tile(blockIdx.x, nt, &ti, &tj);
  const int f = blockIdx.y, s = blockIdx.z, nf = gridDim.y;
  const int pb0 = s * pbc, npb = min(Pb, pb0 + pbc) - pb0;
  const size_t nn = (size_t)neps * neps, osz = (size_t)Pb * 4 * neps * BK;
  const unsigned short* XB = X + (size_t)(1 + f) * osz;
  if (s == 0)
    chi0_bf16s_tile<WM>(X, XB, pb0, npb, neps, chi + (size_t)f * nn, ti, tj, skip_head, false);
  else
    chi0_bf16s_tile<WM>(X, XB, pb0, npb, neps, part + ((size_t)(s - 1) * nf + f) * nn, ti, tj,
                        skip_head, true);
}

// The 128 x 128 tiles: grid = the tile order table x ranges x frequencies,
// renumbered per XCD so that each XCD takes a contiguous run of the order, in
// which consecutive tiles form 4 x 8 blocks of the tile grid (the concurrent
// workgroups of an XCD then share the A slabs of 4 tile rows and the B slabs
// of 8 tile columns in its L2). Range s of frequency f adds into chi0 (s = 0)
// or stores into part[s - 1][f].
__global__ void __launch_bounds__(512, 1) k_chi0_bf16w(const unsigned short* __restrict__ X,
                                                       int Pb, int neps,
                                                       const int2* __restrict__ order, int ntile,
                                                       int split, int nf,
                                                       cpx<double>* __restrict__ chi,
                                                       int skip_head, int pbc,
                                                       cpx<double>* __restrict__ part) {
  const long long lin = xcd_linear(blockIdx.x, (long long)ntile * split * nf);
  if (lin < 0) return;
  const int tile = (int)(lin % ntile);
  const int fs = (int)(lin / ntile), s = fs % split, f = fs / split;
  const int2 tt = order[tile];
  const int pb0 = s * pbc, npb = min(Pb, pb0 + pbc) - pb0;
  const size_t nn = (size_t)neps * neps, osz = (size_t)Pb * 4 * neps * BK;
  const unsigned short* XB = X + (size_t)(1 + f) * osz;
  if (s == 0)
    chi0_bf16s_tile_w(X, XB, pb0, npb, neps, chi + (size_t)f * nn, tt.x, tt.y, skip_head, false);
  else
    chi0_bf16s_tile_w(X, XB, pb0, npb, neps, part + ((size_t)(s - 1) * nf + f) * nn, tt.x,
                      tt.y, skip_head, true);
}

// chi0 += part[0] + part[1] + ... (fixed order, so the result does not depend on
// which range finished first)
__global__ void k_chi0_reduce(cpx<double>* __restrict__ chi, const cpx<double>* __restrict__ part,
                              int nparts, size_t total) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  cpx<double> v = chi[e];
  for (int s = 0; s < nparts; ++s) v = v + part[(size_t)s * total + e];
  chi[e] = v;
}

constexpr int kChiWM = 2, kChiTM = 32 * kChiWM;

// pairs summed in float by one workgroup of the 128 x 128 split-BF16 tile
constexpr int kBf16Range = 8192;

// Pair ranges of the 128 x 128 split-BF16 contraction: at least P / 8192 (the
// float accumulation bound), then the count in the next eight that fills the
// last round of workgroups (one per CU) best.
static int chi0_split_w(gw_ctx* c, int P, int neps, int nfreq) {
  const int nt = (neps + WT - 1) / WT;
  const long long b1 = (long long)nt * (nt + 1) / 2 * nfreq;
  const double conc = (double)c->cus;
  auto fill = [&](long long b) {
    const double r = (double)b / conc;
    return r / std::ceil(r);
  };
  const int smin = std::max(1, (P + kBf16Range - 1) / kBf16Range);
  int best = smin;
  double bf = fill(b1 * smin);
  for (int s = smin + 1; s <= smin + 8; ++s) {
    if (P / s < 512) break;  // keep each range long against its epilogue and the extra pass
    const double f = fill(b1 * s);
    if (f > bf + 0.05) { best = s; bf = f; }
  }
  return best;
}

// Upper-triangle tiles (ti <= tj) of an nt x nt tile grid in GR x GC blocks,
// blocks row-major, tiles row-major inside a block; one device table per
// (nt, GR, GC), kept by the context.
static gw_status tile_order(gw_ctx* c, int nt, int GR, int GC, const int2** out) {
  const long long key = ((long long)nt << 16) | (GR << 8) | GC;
  auto it = c->tile_orders.find(key);
  if (it != c->tile_orders.end()) { *out = static_cast<const int2*>(it->second); return GW_OK; }
  std::vector<int2> h;
  for (int bi = 0; bi < nt; bi += GR)
    for (int bj = (bi / GC) * GC; bj < nt; bj += GC)
      for (int i = bi; i < std::min(nt, bi + GR); ++i)
        for (int j = bj; j < std::min(nt, bj + GC); ++j)
          if (i <= j) h.push_back(make_int2(i, j));
  void* d = nullptr;
  GW_HIP(c, hipMalloc(&d, h.size() * sizeof(int2)));
  GW_HIP(c, hipMemcpy(d, h.data(), h.size() * sizeof(int2), hipMemcpyHostToDevice));
  c->tile_orders[key] = d;
  *out = static_cast<const int2*>(d);
  return GW_OK;
}

int chi0_split(gw_ctx* c, int P, int neps, int nfreq, gw_prec prec, gw_dtype dt) {
  if (prec == GW_PREC_SPLITBF16) return chi0_split_w(c, P, neps, nfreq);
  const int nt = (neps + kChiTM - 1) / kChiTM;
  const long long b1 = (long long)nt * (nt + 1) / 2 * nfreq;
  int per_cu = 0;
  hipError_t e;
  if (dt == GW_C128)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_chi0_f64<kChiWM, double>, 64 * kChiWM * kChiWM, 0);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_chi0_f64<kChiWM, float>, 64 * kChiWM * kChiWM, 0);
  if (e != hipSuccess || per_cu < 1) per_cu = 1;
  const double conc = (double)per_cu * c->cus;
  // fraction of the last round of workgroups that does work
  auto fill = [&](long long b) {
    const double r = (double)b / conc;
    return r / std::ceil(r);
  };
  int best = 1;
  double bf = fill(b1);
  for (int s = 2; s <= 4; ++s) {
    if (P / s < 1024) break;  // keep each range long against its epilogue and the extra pass
    const double f = fill(b1 * s);
    if (f > bf + 0.05) { best = s; bf = f; }
  }
  return best;
}

static int range_len(int P, int split) {
  int pc = (P + split - 1) / split;
  return (pc + BK - 1) / BK * BK;  // whole MFMA K steps; the last range is the short one
}

static gw_status chi0_reduce(gw_ctx* c, int neps, int nfreq, double* chi0, int split,
                             const double* part) {
  if (split <= 1) return GW_OK;
  ProfScope ps(c, "chi0_reduce");
  const size_t total = (size_t)nfreq * neps * neps;
  hipLaunchKernelGGL(k_chi0_reduce, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, c->stream,
                     reinterpret_cast<cpx<double>*>(chi0),
                     reinterpret_cast<const cpx<double>*>(part), split - 1, total);
  GW_CHECK_LAUNCH(c, "k_chi0_reduce");
  return GW_OK;
}

gw_status chi0_fp64(gw_ctx* c, int P, int neps, const void* mtxel, gw_dtype dt, int nfreq,
                    const double* wts, int skip_head, double* chi0, int split, double* part,
                    bool no_alloc) {
  const int nt = (neps + kChiTM - 1) / kChiTM;
  const int ntri = nt * (nt + 1) / 2;
  const int pc = range_len(P, split);
  if (split > 1 && (!part || (long long)pc * (split - 1) >= P))
    return fail(c, GW_EINVAL, "chi0 pair split %d of %d pairs is invalid", split, P);
  // the blocked tile order is a device table built on first use; a caller that
  // may not allocate takes the row-major order instead
  const int2* order = nullptr;
  if (!no_alloc) {
    gw_status st = tile_order(c, nt, 8, 16, &order);
    if (st != GW_OK) return st;
  }
  {
    ProfScope ps(c, "chi0_fp64");
    const long long tot = (long long)ntri * split * nfreq;
    const dim3 g((unsigned)(((tot + kXcd - 1) / kXcd) * kXcd));
    auto* pp = reinterpret_cast<cpx<double>*>(part);
    if (dt == GW_C128)
      hipLaunchKernelGGL((k_chi0_f64<kChiWM, double>), g, dim3(64 * kChiWM * kChiWM), 0, c->stream,
                         static_cast<const cpx<double>*>(mtxel), P, neps, wts,
                         reinterpret_cast<cpx<double>*>(chi0), order, ntri, split, nfreq,
                         skip_head, pc, pp);
    else
      hipLaunchKernelGGL((k_chi0_f64<kChiWM, float>), g, dim3(64 * kChiWM * kChiWM), 0, c->stream,
                         static_cast<const cpx<float>*>(mtxel), P, neps, wts,
                         reinterpret_cast<cpx<double>*>(chi0), order, ntri, split, nfreq,
                         skip_head, pc, pp);
    GW_CHECK_LAUNCH(c, "k_chi0_f64");
  }
  return chi0_reduce(c, neps, nfreq, chi0, split, part);
}

size_t bf16_split_bytes(int P, int neps, int nfreq) {
  const size_t Pb = (size_t)(P + BK - 1) / BK;
  return (size_t)(1 + nfreq) * Pb * 4 * neps * BK * sizeof(unsigned short);
}

// X_0 = M and X_{1+f} = w_f M, split into bf16 hi/lo planes (k_bf16_split)
gw_status split_bf16(gw_ctx* c, int P, int neps, const void* mtxel, int nfreq, const double* wts,
                     void* xsplit) {
  if (P <= 0 || neps <= 0) return GW_OK;
  const int Pb = (P + BK - 1) / BK;
  ProfScope ps(c, "bf16_split");
  hipLaunchKernelGGL(k_bf16_split, dim3(Pb, (neps + 63) / 64), dim3(256), 0, c->stream,
                     static_cast<const cpx<float>*>(mtxel), P, neps, 1 + nfreq, wts,
                     static_cast<unsigned short*>(xsplit));
  GW_CHECK_LAUNCH(c, "k_bf16_split");
  return GW_OK;
}

gw_status chi0_splitbf16(gw_ctx* c, int P, int neps, const void* mtxel, int nfreq,
                         const double* wts, int skip_head, double* chi0, int split, double* part,
                         void* xsplit) {
  const int nt = (neps + WT - 1) / WT;
  const int ntile = nt * (nt + 1) / 2;
  const int pc = range_len(P, split), Pb = (P + BK - 1) / BK;
  if (split > 1 && (!part || (long long)pc * (split - 1) >= P))
    return fail(c, GW_EINVAL, "chi0 pair split %d of %d pairs is invalid", split, P);
  if (pc > kBf16Range + BK)
    return fail(c, GW_EINVAL, "chi0 pair range of %d pairs exceeds the float accumulation bound", pc);
  const int2* order = nullptr;
  gw_status st = tile_order(c, nt, 4, 8, &order);
  if (st != GW_OK) return st;
  auto* X = static_cast<unsigned short*>(xsplit);
  if ((st = split_bf16(c, P, neps, mtxel, nfreq, wts, xsplit)) != GW_OK) return st;
  {
    ProfScope ps(c, "chi0_bf16x3");
    const long long tot = (long long)ntile * split * nfreq;
    const unsigned grid = (unsigned)(((tot + kXcd - 1) / kXcd) * kXcd);
    hipLaunchKernelGGL(k_chi0_bf16w, dim3(grid), dim3(512), 0, c->stream, X, Pb, neps, order,
                       ntile, split, nfreq, reinterpret_cast<cpx<double>*>(chi0), skip_head,
                       pc / BK, reinterpret_cast<cpx<double>*>(part));
    GW_CHECK_LAUNCH(c, "k_chi0_bf16w");
  }
  return chi0_reduce(c, neps, nfreq, chi0, split, part);
}

// ---------------------------------------------------------------- generic ZGEMM
// C[i][j] += alpha * sum_k A[i][k] B[k][j], complex double, row-major, batched on z.
__global__ void __launch_bounds__(256) k_zgemm_nn(int m, int n, int kdim, double alpha,
                                                  double beta,
                                                  const cpx<double>* __restrict__ A, int lda,
                                                  long long sA, const cpx<double>* __restrict__ B,
                                                  int ldb, long long sB, cpx<double>* __restrict__ C,
                                                  int ldc, long long sC) {
  zgemm_tile(m, n, kdim, alpha, beta, A + (size_t)blockIdx.z * sA, lda, B + (size_t)blockIdx.z * sB,
             ldb, C + (size_t)blockIdx.z * sC, ldc, blockIdx.y * ZTM, blockIdx.x * ZTM);
}

// Highest complex-element offset (exclusive) one operand touches across the batch.
static size_t span(size_t off, int rows, int cols, int ld, long long stride, int batch) {
  return off + (size_t)(batch - 1) * (size_t)stride + (size_t)(rows - 1) * ld + cols;
}

gw_status zgemm_nn(gw_ctx* c, int m, int n, int k, double alpha, const double* A, size_t offA,
                   int lda, long long sA, const double* B, size_t offB, int ldb, long long sB,
                   double* C, size_t offC, int ldc, long long sC, int batch, size_t extA,
                   size_t extB, size_t extC, double beta) {
  if (beta != 0.0 && beta != 1.0) return fail(c, GW_EINVAL, "zgemm beta must be 0 or 1");
  if (m <= 0 || n <= 0 || k <= 0 || batch <= 0) return GW_OK;
  // every offset, leading dimension and stride is in complex elements; the
  // extents are the complex elements available behind each base pointer
  if (span(offA, m, k, lda, sA, batch) > extA || span(offB, k, n, ldb, sB, batch) > extB ||
      span(offC, m, n, ldc, sC, batch) > extC || lda < k || ldb < n || ldc < n)
    return fail(c, GW_EINVAL, "zgemm operand out of range (m=%d n=%d k=%d batch=%d)", m, n, k,
                batch);
  ProfScope ps(c, "zgemm");
  // the grid's y dimension counts row tiles and is limited to 65535, so taller
  // operands run as several launches over consecutive row ranges
  constexpr int kRowsPerLaunch = 65535 * ZTM;
  for (long long r0 = 0; r0 < m; r0 += kRowsPerLaunch) {
    const int mr = (int)std::min<long long>(kRowsPerLaunch, m - r0);
    dim3 g((n + ZTM - 1) / ZTM, (mr + ZTM - 1) / ZTM, batch);
    hipLaunchKernelGGL(k_zgemm_nn, g, dim3(256), 0, c->stream, mr, n, k, alpha, beta,
                       reinterpret_cast<const cpx<double>*>(A) + offA + (size_t)r0 * lda, lda, sA,
                       reinterpret_cast<const cpx<double>*>(B) + offB, ldb, sB,
                       reinterpret_cast<cpx<double>*>(C) + offC + (size_t)r0 * ldc, ldc, sC);
    GW_CHECK_LAUNCH(c, "k_zgemm_nn");
  }
  return GW_OK;
}

}  // namespace gw
