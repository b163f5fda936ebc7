// Driver for the symmetry row's host bookkeeping (gw_little_group,
// gw_kgrid_orbits) built with the address and undefined-behaviour sanitizers:
// every call of the CPU tests' cases plus the error paths, with the orbit
// invariants checked here. Prints "ok" and exits 0 when every check holds.
#include <cstdio>
#include <vector>

#include "../../include/gw.h"

namespace {
struct Mat {
  int m[9];
};
Mat mul(const Mat& a, const Mat& b) {
  Mat c{};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) c.m[3 * i + j] += a.m[3 * i + k] * b.m[3 * k + j];
  return c;
}
bool same(const Mat& a, const Mat& b) {
  for (int i = 0; i < 9; ++i)
    if (a.m[i] != b.m[i]) return false;
  return true;
}
// the 4/mmm point group in a tetragonal lattice basis, by closure of its generators
std::vector<Mat> group_4mmm() {
  const Mat gen[3] = {{{0, -1, 0, 1, 0, 0, 0, 0, 1}},     // C4 about z
                      {{1, 0, 0, 0, -1, 0, 0, 0, -1}},    // C2 about x
                      {{-1, 0, 0, 0, -1, 0, 0, 0, -1}}};  // inversion
  std::vector<Mat> g = {{{1, 0, 0, 0, 1, 0, 0, 0, 1}}};
  for (size_t i = 0; i < g.size(); ++i)
    for (const Mat& s : gen) {
      const Mat p = mul(g[i], s);
      bool found = false;
      for (const Mat& h : g) found = found || same(h, p);
      if (!found) g.push_back(p);
    }
  return g;
}
int failures = 0;
void check(bool ok, const char* what) {
  if (!ok) {
    std::printf("FAILED: %s\n", what);
    ++failures;
  }
}
}  // namespace

int main() {
  const std::vector<Mat> g = group_4mmm();
  check(g.size() == 16, "4/mmm has 16 operations");
  std::vector<int> rots;
  for (const Mat& s : g) rots.insert(rots.end(), s.m, s.m + 9);
  const double qs[5][3] = {{0, 0, 1.0 / 3}, {0.25, 0, 0}, {0.1, 0.2, 0.3}, {0.5, 0.5, 0.5}, {0, 0, 0}};
  const int grids[4][3] = {{3, 3, 3}, {4, 4, 2}, {6, 6, 4}, {4, 4, 4}};
  for (const auto& q : qs) {
    std::vector<int> in(g.size()), shift(3 * g.size());
    check(gw_little_group((int)g.size(), rots.data(), q, in.data(), shift.data()) == GW_OK,
          "little group of a valid q");
    check(in[0] == 1, "the identity is in every little group");
    std::vector<int> little;
    for (size_t s = 0; s < g.size(); ++s)
      if (in[s]) little.insert(little.end(), rots.begin() + 9 * s, rots.begin() + 9 * s + 9);
    const int nl = (int)little.size() / 9;
    for (const auto& n : grids) {
      const int npts = n[0] * n[1] * n[2];
      std::vector<int> rep(npts), op(npts), g0(3 * npts), w(npts);
      int nirr = -1;
      const gw_status st = gw_kgrid_orbits(n[0], n[1], n[2], nl, little.data(), rep.data(),
                                           op.data(), g0.data(), w.data(), &nirr);
      if (st != GW_OK) continue;  // a grid the little group does not map onto itself
      long long total = 0;
      int reps = 0;
      for (int i = 0; i < npts; ++i) {
        check(rep[i] >= 0 && rep[i] < npts, "representative on the grid");
        check(rep[rep[i]] == rep[i], "a representative represents itself");
        check((w[i] > 0) == (rep[i] == i), "weight only on representatives");
        check(op[i] >= 0 && op[i] < nl, "operation index in range");
        total += w[i];
        reps += w[i] > 0;
      }
      check(total == npts, "weights add up to the grid");
      check(nirr == reps, "irreducible count");
    }
  }
  // error paths
  const int bad[9] = {1, 1, 0, 0, 1, 1, 1, 0, 1};  // determinant 2
  int in1 = 0, sh1[3] = {0, 0, 0};
  const double q0[3] = {0, 0, 0};
  check(gw_little_group(1, bad, q0, &in1, sh1) == GW_EINVAL, "non-unimodular operation");
  check(gw_little_group(1, nullptr, q0, &in1, sh1) == GW_EINVAL, "null rotations");
  check(gw_little_group(0, nullptr, nullptr, nullptr, nullptr) == GW_OK, "empty group");
  std::vector<int> rep(24), op(24), g0(72), w(24);
  int nirr = 0;
  check(gw_kgrid_orbits(4, 3, 2, (int)g.size(), rots.data(), rep.data(), op.data(), g0.data(),
                        w.data(), &nirr) == GW_EINVAL,
        "C4 does not map a 4 x 3 x 2 grid onto itself");
  check(gw_kgrid_orbits(0, 2, 2, (int)g.size(), rots.data(), rep.data(), op.data(), g0.data(),
                        w.data(), &nirr) == GW_EINVAL,
        "empty grid");
  check(gw_kgrid_orbits(2, 2, 2, 1, rots.data(), nullptr, op.data(), g0.data(), w.data(),
                        &nirr) == GW_EINVAL,
        "null output");
  if (failures) return 1;
  std::printf("ok\n");
  return 0;
}
