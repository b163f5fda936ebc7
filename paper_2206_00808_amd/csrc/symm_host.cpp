// Host bookkeeping of the symmetry row (Sec. III): the little group of q and
// the orbits of a Monkhorst-Pack grid under it. Plain C++ with exact integer
// arithmetic; no device work and no context, so these entry points can be
// called before any GPU call (and are built and run under the address and
// undefined-behaviour sanitizers by the CPU tests).
#include <cmath>
#include <vector>

#include "../../include/gw.h"

namespace {
// S_lat^-T = adj(S_lat)^T / det for a unimodular integer matrix (row-major)
bool inv_transpose(const int* r, long long out[9]) {
  long long m[9];
  for (int i = 0; i < 9; ++i) m[i] = r[i];
  const long long det = m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6]) +
                        m[2] * (m[3] * m[7] - m[4] * m[6]);
  if (det != 1 && det != -1) return false;
  // adj[i][j] = cofactor[j][i]; (S^-1)^T[i][j] = adj[j][i] / det = cofactor[i][j] / det
  const long long cof[9] = {m[4] * m[8] - m[5] * m[7], m[5] * m[6] - m[3] * m[8],
                            m[3] * m[7] - m[4] * m[6], m[2] * m[7] - m[1] * m[8],
                            m[0] * m[8] - m[2] * m[6], m[1] * m[6] - m[0] * m[7],
                            m[1] * m[5] - m[2] * m[4], m[2] * m[3] - m[0] * m[5],
                            m[0] * m[4] - m[1] * m[3]};
  for (int i = 0; i < 9; ++i) out[i] = cof[i] * det;  // det = +-1, so / det == * det
  return true;
}
}  // namespace

extern "C" gw_status gw_little_group(int nops, const int* rots, const double* qred,
                                     int* in_group, int* gshift) {
  if (nops < 0 || (nops > 0 && (!rots || !qred || !in_group || !gshift))) return GW_EINVAL;
  for (int s = 0; s < nops; ++s) {
    long long t[9];
    if (!inv_transpose(rots + 9 * s, t)) return GW_EINVAL;
    int ok = 1;
    for (int a = 0; a < 3; ++a) {
      const double sq = t[3 * a] * qred[0] + t[3 * a + 1] * qred[1] + t[3 * a + 2] * qred[2];
      const double d = sq - qred[a];
      const double r = std::nearbyint(d);
      gshift[3 * s + a] = (int)r;
      if (std::fabs(d - r) > 1e-9) ok = 0;
    }
    if (!ok) gshift[3 * s] = gshift[3 * s + 1] = gshift[3 * s + 2] = 0;
    in_group[s] = ok;
  }
  return GW_OK;
}

extern "C" gw_status gw_kgrid_orbits(int n1, int n2, int n3, int nops, const int* rots, int* rep,
                                     int* op, int* g0, int* weight, int* nirr) {
  if (n1 <= 0 || n2 <= 0 || n3 <= 0 || nops <= 0 || !rots || !rep || !op || !g0 || !weight ||
      !nirr)
    return GW_EINVAL;
  const long long n[3] = {n1, n2, n3};
  const long long npts = n[0] * n[1] * n[2];
  if (npts > (1LL << 26)) return GW_EINVAL;
  auto gcd = [](long long a, long long b) {
    while (b) {
      const long long t = a % b;
      a = b;
      b = t;
    }
    return a;
  };
  long long L = n[0];
  for (int a = 1; a < 3; ++a) L = L / gcd(L, n[a]) * n[a];
  std::vector<long long> t((size_t)nops * 9);
  for (int s = 0; s < nops; ++s)
    if (!inv_transpose(rots + 9 * s, t.data() + 9 * s)) return GW_EINVAL;
  for (long long i = 0; i < npts; ++i) {
    rep[i] = -1;
    weight[i] = 0;
  }
  int count = 0;
  for (long long i = 0; i < npts; ++i) {
    if (rep[i] >= 0) continue;
    const long long ii[3] = {i / (n[1] * n[2]), (i / n[2]) % n[1], i % n[2]};
    ++count;
    for (int s = 0; s < nops; ++s) {
      const long long* m = t.data() + 9 * s;
      // (S k)_a = sum_b m[a][b] i_b / n_b = x / L with L = lcm(n); in units of 1/n_a
      // that is x n_a / L, which must be an integer for the grid to be closed
      long long cellv[3], pos[3];
      for (int a = 0; a < 3; ++a) {
        long long x = 0;
        for (int b = 0; b < 3; ++b) x += m[3 * a + b] * ii[b] * (L / n[b]);
        if ((x * n[a]) % L != 0) return GW_EINVAL;
        const long long acc = x * n[a] / L;
        // floor division: S k = cellv + pos / n with 0 <= pos < n
        cellv[a] = acc >= 0 ? acc / n[a] : -((-acc + n[a] - 1) / n[a]);
        pos[a] = acc - cellv[a] * n[a];
      }
      const long long j = (pos[0] * n[1] + pos[1]) * n[2] + pos[2];
      if (rep[j] < 0) {
        rep[j] = (int)i;
        op[j] = s;
        for (int a = 0; a < 3; ++a) g0[3 * j + a] = (int)cellv[a];
        weight[i] += 1;
      }
    }
  }
  *nirr = count;
  return GW_OK;
}
