// Unfolding spinor wavefunctions from one k-point to a symmetry-related one.
//
// Sec. III: an operation {S|tau} (r -> S r + tau) carries the Bloch state at k to
// one at S k.  Its plane-wave coefficients move to the rotated vectors and pick
// up the translation phase, c'(S G) = c(G) e^{-i S G . tau} (the band-independent
// phase e^{-i S k . tau} is dropped), and the two spinor components mix by the
// SU(2) matrix of the rotation part of S (an improper S is inversion times a
// rotation; spin is axial, so inversion leaves it alone).
//
// The host turns S into that 2x2 matrix once per call: S_cart = A S_lat A^-1,
// then the unit quaternion q = (n sin(theta/2), cos(theta/2)) by Markley's
// variant of Shepperd's method (the column of largest norm of the 4x4 matrix
// X = 4 q q^T, no division by sin(theta)), then U = q4 I - i (q1 sx + q2 sy + q3 sz),
// which is exp(-i theta/2 n.sigma) written in q.  It also builds, per output
// vector, the index of its preimage in the input sphere and the phase, so the
// kernel is a gather, a 2x2 complex product and a coalesced store.
#include <cmath>
#include <unordered_map>
#include <vector>

#include "common.h"

namespace gw {

namespace {

// Unit quaternion of a proper rotation (vectors turned by theta about n), with
// the chosen component positive: the positive branch of the double cover.
void quaternion_of(const double r[3][3], double q[4]) {
  const double t = r[0][0] + r[1][1] + r[2][2];
  const double x[4][4] = {
      {1 + 2 * r[0][0] - t, r[0][1] + r[1][0], r[0][2] + r[2][0], r[2][1] - r[1][2]},
      {r[1][0] + r[0][1], 1 + 2 * r[1][1] - t, r[1][2] + r[2][1], r[0][2] - r[2][0]},
      {r[2][0] + r[0][2], r[2][1] + r[1][2], 1 + 2 * r[2][2] - t, r[1][0] - r[0][1]},
      {r[2][1] - r[1][2], r[0][2] - r[2][0], r[1][0] - r[0][1], 1 + t}};
  int best = 0;
  double bn = -1.0;
  for (int j = 0; j < 4; ++j) {
    double s = 0.0;
    for (int i = 0; i < 4; ++i) s += x[i][j] * x[i][j];
    if (s > bn) {
      bn = s;
      best = j;
    }
  }
  // column j is 4 q_j q, and its diagonal entry 4 q_j^2 > 0: dividing by the
  // norm 4 |q_j| leaves q with q_j > 0
  const double inv = 1.0 / std::sqrt(bn);
  for (int i = 0; i < 4; ++i) q[i] = x[i][best] * inv;
}

}  // namespace

// out[b][s][i] = sum_t U[s][t] in[b][t][src[i]] * ph[i]; one thread per output
// vector, BB bands per workgroup so the index and phase are read once per band group
template <typename T, int NS, int BB>
__global__ void __launch_bounds__(256) k_unfold(const cpx<T>* __restrict__ cin, int ng_in,
                                                const int* __restrict__ src,
                                                const cpx<double>* __restrict__ ph, int ng_out,
                                                int nb, cpx<double> u00, cpx<double> u01,
                                                cpx<double> u10, cpx<double> u11,
                                                cpx<T>* __restrict__ cout) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ng_out) return;
  const int j = src[i];
  const cpx<double> p = ph[i];
  const int b0 = blockIdx.y * BB;
  const int b1 = b0 + BB < nb ? b0 + BB : nb;
  for (int b = b0; b < b1; ++b) {
    const cpx<T>* a = cin + (size_t)b * NS * ng_in;
    cpx<T>* o = cout + (size_t)b * NS * ng_out;
    if (NS == 1) {
      const cpx<T> v = a[j];
      const cpx<double> w = cmul(mk((double)v.x, (double)v.y), p);
      o[i] = mk((T)w.x, (T)w.y);
    } else {
      const cpx<T> va = a[j], vb = a[ng_in + j];
      const cpx<double> x0 = cmul(mk((double)va.x, (double)va.y), p);
      const cpx<double> x1 = cmul(mk((double)vb.x, (double)vb.y), p);
      const cpx<double> y0 = cmul(u00, x0) + cmul(u01, x1);
      const cpx<double> y1 = cmul(u10, x0) + cmul(u11, x1);
      o[i] = mk((T)y0.x, (T)y0.y);
      o[ng_out + i] = mk((T)y1.x, (T)y1.y);
    }
  }
}

// out[f][i][j] = (1/nops) sum_S p_S(i) conj(p_S(j)) in[f][idx_S(i)][idx_S(j)]
__global__ void k_chi0_symmetrize(const cpx<double>* __restrict__ in, int N, int nops,
                                  const int* __restrict__ idx, const cpx<double>* __restrict__ ph,
                                  cpx<double>* __restrict__ out) {
  const size_t nn = (size_t)N * N;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nn) return;
  const int i = (int)(e / N), j = (int)(e % N);
  const cpx<double>* x = in + (size_t)blockIdx.y * nn;
  cpx<double> acc = mk(0.0, 0.0);
  for (int s = 0; s < nops; ++s) {
    const int a = idx[(size_t)s * N + i], b = idx[(size_t)s * N + j];
    const cpx<double> pij = cmulc(ph[(size_t)s * N + j], ph[(size_t)s * N + i]);  // p_i conj(p_j)
    acc = acc + cmul(pij, x[(size_t)a * N + b]);
  }
  out[(size_t)blockIdx.y * nn + e] = scal(acc, 1.0 / nops);
}

template <typename T, int NS>
static void launch_unfold(gw_ctx* c, const void* cin, int ng_in, const int* src,
                          const cpx<double>* ph, int ng_out, int nb, const cpx<double> u[4],
                          void* cout) {
  constexpr int BB = 8;
  const dim3 grid((unsigned)((ng_out + 255) / 256), (unsigned)((nb + BB - 1) / BB));
  hipLaunchKernelGGL((k_unfold<T, NS, BB>), grid, dim3(256), 0, c->stream,
                     static_cast<const cpx<T>*>(cin), ng_in, src, ph, ng_out, nb, u[0], u[1],
                     u[2], u[3], static_cast<cpx<T>*>(cout));
}

}  // namespace gw

using namespace gw;

extern "C" gw_status gw_unfold_spinor(gw_ctx* c, int nspinor, int nb, int ng_in, const int* gin,
                                      const void* cin, gw_dtype dtype, int ng_out,
                                      const int* gout, const int* rot, const double* tau,
                                      const int* g0, const double* cell, void* cout) {
  if (!c) return GW_EINVAL;
  c->err.clear();
  if (nspinor != 1 && nspinor != 2) return fail(c, GW_EINVAL, "nspinor must be 1 or 2");
  if (nb < 0 || ng_in < 0 || ng_out < 0) return fail(c, GW_EINVAL, "negative size");
  if (dtype != GW_C128 && dtype != GW_C64) return fail(c, GW_EINVAL, "unknown dtype");
  if (!rot || !tau || !cell) return fail(c, GW_EINVAL, "NULL rot, tau or cell");
  if (nb == 0 || ng_out == 0) return GW_OK;
  if (ng_in == 0) return fail(c, GW_EINVAL, "output vectors but an empty input sphere");
  if (!gin || !cin || !gout || !cout) return fail(c, GW_EINVAL, "NULL array argument");
  if (cin == cout) return fail(c, GW_EINVAL, "cout aliases cin");
  if (nb > 65535 * 8) return fail(c, GW_EINVAL, "nb above 524280");
  for (int i = 0; i < 3; ++i)
    if (!(cell[i] > 0.0) || !std::isfinite(cell[i]) || !std::isfinite(tau[i]))
      return fail(c, GW_EINVAL, "cell must be positive and tau finite");
  // S_cart = A S_lat A^-1 with A = diag(cell): entry (i,j) is a_i S_ij / a_j
  double r[3][3];
  long long m[9];
  for (int i = 0; i < 9; ++i) m[i] = rot[i];
  const long long det = m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6]) +
                        m[2] * (m[3] * m[7] - m[4] * m[6]);
  if (det != 1 && det != -1) return fail(c, GW_EINVAL, "rot has determinant %lld", det);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) r[i][j] = (double)det * cell[i] * rot[3 * i + j] / cell[j];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += r[k][i] * r[k][j];
      if (std::fabs(s - (i == j ? 1.0 : 0.0)) > 1e-9)
        return fail(c, GW_EINVAL, "rot is not a rotation of this orthorhombic lattice");
    }
  // spin rotation of the proper part (r now holds det * S_cart)
  cpx<double> u[4] = {mk(1.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0), mk(1.0, 0.0)};
  if (nspinor == 2) {
    double q[4];
    quaternion_of(r, q);
    u[0] = mk(q[3], -q[2]);
    u[1] = mk(-q[1], -q[0]);
    u[2] = mk(q[1], -q[0]);
    u[3] = mk(q[3], q[2]);
  }
  // preimage index and phase of every output vector: G = G' - G0 relative to S k,
  // preimage S^-1 G = S_lat^T G in integer reciprocal coordinates
  auto key = [](long long x, long long y, long long z) {
    return ((x + (1LL << 20)) << 42) | ((y + (1LL << 20)) << 21) | (z + (1LL << 20));
  };
  std::unordered_map<long long, int> lut;
  lut.reserve((size_t)ng_in * 2);
  for (int i = 0; i < ng_in; ++i) {
    const int* g = gin + 3 * i;
    for (int a = 0; a < 3; ++a)
      if (g[a] < -(1 << 19) || g[a] > (1 << 19))
        return fail(c, GW_EINVAL, "input G component out of range");
    if (!lut.emplace(key(g[0], g[1], g[2]), i).second)
      return fail(c, GW_EINVAL, "duplicate input G (%d %d %d)", g[0], g[1], g[2]);
  }
  const int z0[3] = {0, 0, 0};
  const int* s0 = g0 ? g0 : z0;
  std::vector<int> src((size_t)ng_out);
  std::vector<cpx<double>> ph((size_t)ng_out);
  for (int i = 0; i < ng_out; ++i) {
    const long long gq[3] = {(long long)gout[3 * i] - s0[0], (long long)gout[3 * i + 1] - s0[1],
                             (long long)gout[3 * i + 2] - s0[2]};
    long long gs[3];
    for (int j = 0; j < 3; ++j) gs[j] = gq[0] * m[j] + gq[1] * m[3 + j] + gq[2] * m[6 + j];
    bool in_range = true;
    for (int j = 0; j < 3; ++j) in_range &= gs[j] >= -(1 << 19) && gs[j] <= (1 << 19);
    auto it = in_range ? lut.find(key(gs[0], gs[1], gs[2])) : lut.end();
    if (it == lut.end())
      return fail(c, GW_EINVAL, "output G %d (%d %d %d) has no preimage in the input sphere", i,
                  gout[3 * i], gout[3 * i + 1], gout[3 * i + 2]);
    src[i] = it->second;
    // e^{-2 pi i G.tau} with the argument reduced to [-1/2, 1/2] turns first
    double t = (double)gq[0] * tau[0] + (double)gq[1] * tau[1] + (double)gq[2] * tau[2];
    t -= std::nearbyint(t);
    ph[i] = mk(std::cos(2.0 * M_PI * t), -std::sin(2.0 * M_PI * t));
  }
  (void)hipSetDevice(c->device);
  const size_t bsrc = align_up((size_t)ng_out * sizeof(int));
  gw_status st = ws_begin(c, bsrc + align_up((size_t)ng_out * 16));
  if (st != GW_OK) return st;
  int* d_src = static_cast<int*>(ws_take(c, (size_t)ng_out * sizeof(int)));
  cpx<double>* d_ph = static_cast<cpx<double>*>(ws_take(c, (size_t)ng_out * 16));
  GW_HIP(c, hipMemcpyAsync(d_src, src.data(), (size_t)ng_out * sizeof(int),
                           hipMemcpyHostToDevice, c->stream));
  GW_HIP(c, hipMemcpyAsync(d_ph, ph.data(), (size_t)ng_out * 16, hipMemcpyHostToDevice,
                           c->stream));
  {
    ProfScope ps(c, "unfold");
    if (dtype == GW_C128) {
      if (nspinor == 2) launch_unfold<double, 2>(c, cin, ng_in, d_src, d_ph, ng_out, nb, u, cout);
      else launch_unfold<double, 1>(c, cin, ng_in, d_src, d_ph, ng_out, nb, u, cout);
    } else {
      if (nspinor == 2) launch_unfold<float, 2>(c, cin, ng_in, d_src, d_ph, ng_out, nb, u, cout);
      else launch_unfold<float, 1>(c, cin, ng_in, d_src, d_ph, ng_out, nb, u, cout);
    }
    GW_CHECK_LAUNCH(c, "k_unfold");
  }
  // the index and phase tables live in host vectors: finish before returning
  GW_HIP(c, hipStreamSynchronize(c->stream));
  return GW_OK;
}

extern "C" gw_status gw_chi0_symmetrize(gw_ctx* c, int neps, int nfreq, const int* geps,
                                        const double* qred, int nops, const int* rots,
                                        const double* taus, const double* chi_in,
                                        double* chi_out) {
  if (!c) return GW_EINVAL;
  c->err.clear();
  if (neps < 0 || nfreq < 0 || nops < 0) return fail(c, GW_EINVAL, "negative size");
  if (neps == 0 || nfreq == 0) return GW_OK;
  if (nops == 0 || nops > 96) return fail(c, GW_EINVAL, "nops must be 1 to 96");
  if (!geps || !qred || !rots || !taus || !chi_in || !chi_out)
    return fail(c, GW_EINVAL, "NULL argument");
  if (chi_in == chi_out) return fail(c, GW_EINVAL, "chi_out aliases chi_in");
  if (nfreq > 65535 || neps > 46340) return fail(c, GW_EINVAL, "nfreq or neps too large");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(qred[a])) return fail(c, GW_EINVAL, "q must be finite");
  std::unordered_map<long long, int> lut;
  lut.reserve((size_t)neps * 2);
  auto key = [](long long x, long long y, long long z) {
    return ((x + (1LL << 20)) << 42) | ((y + (1LL << 20)) << 21) | (z + (1LL << 20));
  };
  for (int i = 0; i < neps; ++i) {
    const int* g = geps + 3 * i;
    for (int a = 0; a < 3; ++a)
      if (g[a] < -(1 << 19) || g[a] > (1 << 19)) return fail(c, GW_EINVAL, "G out of range");
    if (!lut.emplace(key(g[0], g[1], g[2]), i).second)
      return fail(c, GW_EINVAL, "duplicate eps G");
  }
  std::vector<int> idx((size_t)nops * neps);
  std::vector<cpx<double>> ph((size_t)nops * neps);
  for (int s = 0; s < nops; ++s) {
    long long m[9];
    for (int i = 0; i < 9; ++i) m[i] = rots[9 * s + i];
    const long long det = m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6]) +
                          m[2] * (m[3] * m[7] - m[4] * m[6]);
    if (det != 1 && det != -1) return fail(c, GW_EINVAL, "operation %d: det %lld", s, det);
    const double* tau = taus + 3 * s;
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(tau[a])) return fail(c, GW_EINVAL, "operation %d: tau not finite", s);
    // S acts on reciprocal integer coordinates as S_lat^-T = adj(S_lat)^T / det;
    // G_S = S q - q must be a reciprocal lattice vector
    long long adj[9];
    adj[0] = m[4] * m[8] - m[5] * m[7];
    adj[1] = m[2] * m[7] - m[1] * m[8];
    adj[2] = m[1] * m[5] - m[2] * m[4];
    adj[3] = m[5] * m[6] - m[3] * m[8];
    adj[4] = m[0] * m[8] - m[2] * m[6];
    adj[5] = m[2] * m[3] - m[0] * m[5];
    adj[6] = m[3] * m[7] - m[4] * m[6];
    adj[7] = m[1] * m[6] - m[0] * m[7];
    adj[8] = m[0] * m[4] - m[1] * m[3];
    long long gsh[3];
    for (int a = 0; a < 3; ++a) {
      // (S_lat^-1)^T q: row a of S_lat^-T is column a of S_lat^-1 = adj / det
      const double sq = (double)(adj[a] * qred[0] + adj[3 + a] * qred[1] + adj[6 + a] * qred[2]) /
                        (double)det;
      const double d = sq - qred[a];
      gsh[a] = (long long)std::llround(d);
      if (std::fabs(d - (double)gsh[a]) > 1e-9)
        return fail(c, GW_EINVAL, "operation %d is not in the little group of q", s);
    }
    for (int i = 0; i < neps; ++i) {
      const long long gq[3] = {geps[3 * i] - gsh[0], geps[3 * i + 1] - gsh[1],
                               geps[3 * i + 2] - gsh[2]};
      // S^-1 (G - G_S) = S_lat^T (G - G_S)
      long long src[3];
      bool ok = true;
      for (int a = 0; a < 3; ++a) {
        src[a] = gq[0] * m[a] + gq[1] * m[3 + a] + gq[2] * m[6 + a];
        ok &= src[a] >= -(1 << 19) && src[a] <= (1 << 19);
      }
      auto it = ok ? lut.find(key(src[0], src[1], src[2])) : lut.end();
      if (it == lut.end())
        return fail(c, GW_EINVAL, "operation %d maps eps G %d outside the sphere", s, i);
      idx[(size_t)s * neps + i] = it->second;
      double t = geps[3 * i] * tau[0] + geps[3 * i + 1] * tau[1] + geps[3 * i + 2] * tau[2];
      t -= std::nearbyint(t);
      ph[(size_t)s * neps + i] = mk(std::cos(2.0 * M_PI * t), -std::sin(2.0 * M_PI * t));
    }
  }
  (void)hipSetDevice(c->device);
  const size_t n_t = (size_t)nops * neps;
  gw_status st = ws_begin(c, align_up(n_t * sizeof(int)) + align_up(n_t * 16));
  if (st != GW_OK) return st;
  int* d_idx = static_cast<int*>(ws_take(c, n_t * sizeof(int)));
  cpx<double>* d_ph = static_cast<cpx<double>*>(ws_take(c, n_t * 16));
  GW_HIP(c, hipMemcpyAsync(d_idx, idx.data(), n_t * sizeof(int), hipMemcpyHostToDevice, c->stream));
  GW_HIP(c, hipMemcpyAsync(d_ph, ph.data(), n_t * 16, hipMemcpyHostToDevice, c->stream));
  const size_t nn = (size_t)neps * neps;
  {
    ProfScope ps(c, "chi0_symmetrize");
    hipLaunchKernelGGL(k_chi0_symmetrize, dim3((unsigned)((nn + 255) / 256), nfreq), dim3(256), 0,
                       c->stream, reinterpret_cast<const cpx<double>*>(chi_in), neps, nops, d_idx,
                       d_ph, reinterpret_cast<cpx<double>*>(chi_out));
    GW_CHECK_LAUNCH(c, "k_chi0_symmetrize");
  }
  // the tables were staged from host vectors: finish before returning
  GW_HIP(c, hipStreamSynchronize(c->stream));
  return GW_OK;
}
