// Spinor matrix elements on boxes with large planes (e.g. 60 x 60 x 160, the
// layered-cell workload), Sec. II, Eq. (matrix_el):
//   rho_vc(r) = sum_s conj(u_v^s(r)) u_c^s(r),
//   M_vc(G)   = (1/N) sum_j rho_vc(r_j) exp(+2 pi i g.j/n),  G on the eps sphere.
//
// The transform is taken x first, then y, on the xy-plane of each z, and
// along z last. One workgroup owns one z and CT conduction bands and walks
// every valence band of the launch:
//   - the conduction xy-planes are built on chip from compact z-transformed
//     slabs (k_band_zc: [c][s][z][jy][jx], the conduction sphere's (x, y)
//     extent only) and stay in registers for the whole valence loop;
//   - the valence xy-planes at that z ([v][s][z][y][x]) are read from the
//     caches: with the grid numbered z-major and renumbered per XCD, the
//     workgroups of one XCD share a z, and all valence planes of one z fit its
//     L2 (3.2 MB in float, 6.4 MB in double for 56 bands);
//   - the spin-summed product, the x transform (keeping |g_x| <= g_eps,x) and
//     the y transform (keeping |g_y| <= g_eps,y) leave (2 g_x + 1)(2 g_y + 1)
//     values per pair and z, of which those in the (x, y) columns that hold
//     eps-sphere points are written to T[pair][z][column];
//   - k_pair_zp transforms T along z, keeps |g_z| <= g_eps,z, scales by 1/N
//     and scatters onto the eps sphere.
// The yz-plane of such a box (9,600 points) would not fit on chip beside a
// valence stream, and the valence yz-planes of one x (17 MB in double) would
// not fit an L2; the xy-plane (3,600 points) does both.
#include <algorithm>

#include "common.h"
#include "regfft.h"

namespace gw {

namespace {

constexpr int kZThreads = 128;

// lanes per pencil in the pair kernel: A lanes of B values each (n = A B).
// Many lanes with few values keep the registers per lane low (the conduction
// planes and the next valence band stay resident); the second factor is then
// evaluated only at the kept frequencies (kept_out).
constexpr int xy_split(int n) { return n == 60 ? 15 : n == 16 ? 4 : split_n1(n); }

template <typename T, int N1, int N2>
struct XyShape {
  static constexpr int A1 = xy_split(N1), B1 = N1 / A1, L1 = pow2_at_least(A1);
  static constexpr int NTH = ((N2 * L1 + 63) / 64) * 64;  // one lane group per row y
  // exchange row pitch: in double, rows 4 (mod 16) entries apart put the 16
  // (row, column) chunks that a wavefront's Horner reads touch at once on
  // distinct LDS banks (columns are A1 entries apart)
  static constexpr int XP = sizeof(T) == 8 ? ((N1 + 1 + 11) / 16) * 16 + 4 : N1 + 1;
  static constexpr int A2 = xy_split(N2), B2 = N2 / A2, L2 = pow2_at_least(A2);
  static_assert(64 % L1 == 0 && 64 % L2 == 0, "a pencil must sit in one wavefront");
  static_assert(NTH <= 1024, "block too large");
};

// One kept output of the second factor of a two-factor transform of length
// N = A B: for the signed frequency f (k = f mod N = k2 + B k1),
//   X(k) = sum_{t < A} W_A^(t k1) line[(k2 A + t) es],
// where line holds the twiddled first-factor results of the pencil. Evaluated
// by Horner's rule in w = W_A^(k1) = W_N^(B k1), read from the length-N table.
template <typename T, int A, int B>
__device__ __forceinline__ cpx<T> kept_out(const cpx<T>* line, int es, int f,
                                           const cpx<T>* twN) {
  constexpr int N = A * B;
  const int k = f < 0 ? f + N : f;
  const int k2 = k % B, k1 = k / B;
  const cpx<T> w = twN[(B * k1) % N];
  const cpx<T>* p = line + k2 * A * es;
  cpx<T> x = p[(A - 1) * es];
  // x <- x w + p[t], four fused multiply-adds per step
#pragma unroll
  for (int t = A - 2; t >= 0; --t) {
    const cpx<T> q = p[t * es];
    x = mk(fma(x.x, w.x, fma(-x.y, w.y, q.x)), fma(x.x, w.y, fma(x.y, w.x, q.y)));
  }
  return x;
}

// kept_out split into the per-lane part that does not change from pencil to
// pencil (the first-factor column and the roots) and the sum itself. For A a
// multiple of 3 the sum runs as three interleaved Horner chains in w^3 over
// t = r (mod 3), joined by two steps in w:
//   X = sum_r w^r sum_b (w^3)^b line[(r + 3 b) es],
// the same number of complex multiply-adds as one chain but a third of its
// dependent length, so the LDS reads of one chain overlap the others' FMAs.
template <typename T>
struct KeptPlan {
  cpx<T> w, w3;
  int off;  // k2 A: first entry of the column in the line, in entries
};
template <typename T, int A, int B>
__device__ __forceinline__ KeptPlan<T> kept_plan(int f, const cpx<T>* twN) {
  constexpr int N = A * B;
  const int k = f < 0 ? f + N : f;
  const int k1 = k / B;
  KeptPlan<T> pl;
  pl.off = (k % B) * A;
  pl.w = twN[(B * k1) % N];
  pl.w3 = twN[(3 * B * k1) % N];
  return pl;
}
template <typename T>
__device__ __forceinline__ cpx<T> horner_step(cpx<T> x, cpx<T> w, cpx<T> q) {
  return mk(fma(x.x, w.x, fma(-x.y, w.y, q.x)), fma(x.x, w.y, fma(x.y, w.x, q.y)));
}
template <typename T, int A>
__device__ __forceinline__ cpx<T> kept_eval(const cpx<T>* line, int es, const KeptPlan<T>& pl) {
  const cpx<T>* p = line + pl.off * es;
  if constexpr (A % 3 == 0 && A > 3) {
    constexpr int L = A / 3;
    cpx<T> x0 = p[(3 * (L - 1)) * es], x1 = p[(3 * (L - 1) + 1) * es],
           x2 = p[(3 * (L - 1) + 2) * es];
#pragma unroll
    for (int b = L - 2; b >= 0; --b) {
      x0 = horner_step(x0, pl.w3, p[(3 * b) * es]);
      x1 = horner_step(x1, pl.w3, p[(3 * b + 1) * es]);
      x2 = horner_step(x2, pl.w3, p[(3 * b + 2) * es]);
    }
    return horner_step(horner_step(x2, pl.w, x1), pl.w, x0);
  } else {
    cpx<T> x = p[(A - 1) * es];
#pragma unroll
    for (int t = A - 2; t >= 0; --t) x = horner_step(x, pl.w, p[t * es]);
    return x;
  }
}

// sum_s conj(v_s) c_s over NS spinor components, as fused multiply-adds
template <typename T, int NS>
__device__ __forceinline__ cpx<T> spin_dot(const cpx<T> (&v)[NS], const cpx<T> (&c)[NS]) {
  T re = v[0].x * c[0].x, im = v[0].x * c[0].y;
  re = fma(v[0].y, c[0].y, re);
  im = fma(-v[0].y, c[0].x, im);
#pragma unroll
  for (int s = 1; s < NS; ++s) {
    re = fma(v[s].x, c[s].x, fma(v[s].y, c[s].y, re));
    im = fma(v[s].x, c[s].y, fma(-v[s].y, c[s].x, im));
  }
  return mk(re, im);
}

// conduction planes per workgroup and valence bands per y pass
template <typename T> struct XyTile;
template <> struct XyTile<double> { static constexpr int CT = 1, VB = 4; };
template <> struct XyTile<float> { static constexpr int CT = 2, VB = 2; };

__device__ __forceinline__ int mod_pos(int a, int n) {
  const int r = a % n;
  return r < 0 ? r + n : r;
}

}  // namespace

// ---------------------------------------------------------------- conduction slabs
// z transform of every compact (jx, jy) column of one band-spin's sphere:
// out[bs][z][jy * ex + jx] = sum_gz c(gx, gy, gz) exp(+2 pi i gz z / N3).
// A lanes per column hold B values each (index n = t + A m): a B-point DFT in
// registers, the twiddle, one exchange through the column's LDS row, and
// A-point DFTs; every output is written.
template <typename T, int N3>
__global__ void __launch_bounds__(kZThreads) k_band_zc(const cpx<T>* __restrict__ coef, int ng,
                                                       const int* __restrict__ cube, int ex,
                                                       int ey, int ez, int gz,
                                                       const cpx<T>* __restrict__ twz,
                                                       cpx<T>* __restrict__ out) {
  constexpr int A = split_n1(N3), B = N3 / A, L = pow2_at_least(A), CPB = kZThreads / L;
  __shared__ cpx<T> X[CPB][N3 + 1];
  __shared__ cpx<T> tw[N3];
  const int bs = blockIdx.y, tid = threadIdx.x;
  for (int i = tid; i < N3; i += kZThreads) tw[i] = twz[i];
  __syncthreads();
  const int ncol = ex * ey;
  const int cq = tid / L, t = tid % L;
  const int col = blockIdx.x * CPB + cq;
  if (col >= ncol || t >= A) return;
  const int jy = col / ex, jx = col - jy * ex;
  const cpx<T>* cf = coef + (size_t)bs * ng;
  const int* cz = cube + ((size_t)jx * ey + jy) * ez;
  cpx<T> a[B];
#pragma unroll
  for (int m = 0; m < B; ++m) {
    const int n = t + A * m;
    const int g = 2 * n <= N3 ? n : n - N3;
    int idx = -1;
    if (g >= -gz && g <= gz) idx = cz[g + gz];
    a[m] = idx >= 0 ? cf[idx] : mk<T>(0, 0);
  }
  reg_dft<T, B>(a);
#pragma unroll
  for (int k2 = 1; k2 < B; ++k2) a[k2] = cmul(a[k2], tw[t * k2]);
  cpx<T>* Xr = X[cq];
#pragma unroll
  for (int k2 = 0; k2 < B; ++k2) Xr[k2 * A + t] = a[k2];
  // the column's lanes share a wavefront, whose LDS accesses complete in order
  __builtin_amdgcn_wave_barrier();
  cpx<T>* o = out + (size_t)bs * N3 * ncol + col;
#pragma unroll
  for (int s = 0; s < (B + A - 1) / A; ++s) {
    const int k2 = t + A * s;
    if (k2 < B) {
      cpx<T> u[A];
#pragma unroll
      for (int n = 0; n < A; ++n) u[n] = Xr[k2 * A + n];
      reg_dft<T, A>(u);
#pragma unroll
      for (int k1 = 0; k1 < A; ++k1) o[(size_t)(k2 + B * k1) * ncol] = u[k1];
    }
  }
}

// ---------------------------------------------------------------- valence layout
// u[bs][x][y][z] -> w[bs][z][y][x], 32 x 32 (x, z) tiles through LDS for each
// (bs, y); grid (z tiles, x tiles, bs * n2).
template <typename T>
__global__ void __launch_bounds__(256) k_to_zyx(const cpx<T>* __restrict__ u, int n1, int n2,
                                                int n3, cpx<T>* __restrict__ w) {
  __shared__ cpx<T> tile[32][33];
  const int z0 = blockIdx.x * 32, x0 = blockIdx.y * 32;
  const size_t bsy = blockIdx.z;
  const size_t bs = bsy / n2;
  const int y = (int)(bsy % n2);
  const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
  for (int r = ty; r < 32; r += 8) {
    const int x = x0 + r, z = z0 + tx;
    if (x < n1 && z < n3) tile[r][tx] = u[((bs * n1 + x) * n2 + y) * n3 + z];
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int z = z0 + r, x = x0 + tx;
    if (x < n1 && z < n3) w[((bs * n3 + z) * n2 + y) * n1 + x] = tile[tx][r];
  }
}

// ---------------------------------------------------------------- pair planes
// Workgroup (z, conduction group cg): conduction bands c0 + cg*CT + ct, every
// valence band v0 .. v0 + nvt - 1. Lane group y (L1 lanes, A1 of them active)
// owns row y of the xy-plane; lane t holds x = t + A1 m, m < B1.
//
// Conduction build, per band and spin: the compact slab Q[jy][jx] at z goes to
// LDS; its y transform Yw[y][jx] = sum_gy Q W_N2^(gy y) is a direct sum (the
// slab has few columns); then for x = t + A1 m,
//   C[t + A1 m] = sum_r exp(+2 pi i r m / B1) b_r,
//   b_r = sum_{gx = r mod B1} Yw[y][gx] W_N1^(gx t),
// a B1-point DFT of per-lane sums, which leaves the plane in the layout the
// valence rows are read in.
//
// Valence loop, VB bands per y pass: the lane's row slice of both spins is
// loaded, the product with each conduction plane is formed in registers, and
// its x transform is the two-factor scheme: B1-point DFTs in registers, the
// twiddle W_N1^(t k2), an exchange through the row's own LDS line (the row's
// lanes share a wavefront), A1-point DFTs; kept outputs go to Xk[j][ct][y][jkx].
// After a block barrier, the y transforms of the VB * CT * (2 gx + 1) kept
// columns run the same way with A2 lanes per column and write
// T[pair][z][jky][jkx], pair = (c - c0) * nvt + (v - v0).
template <typename T, int NS, int N1, int N2>
__global__ void __launch_bounds__((XyShape<T, N1, N2>::NTH), 1) k_pair_xy(
    const cpx<T>* __restrict__ uvz, const cpx<T>* __restrict__ tcz, int exw, int eyw, int gxw,
    int gyw, int v0, int nvt, int c0, int nct, int n3, int gx, int gy,
    const cpx<T>* __restrict__ twx, const cpx<T>* __restrict__ twy,
    const int* __restrict__ disk, int ndisk, cpx<T>* __restrict__ tout) {
  using S = XyShape<T, N1, N2>;
  constexpr int CT = XyTile<T>::CT, VB = XyTile<T>::VB;
  constexpr int NP = N1 * N2;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* tw1 = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* tw2 = tw1 + N1;
  cpx<T>* Xr0 = tw2 + N2;              // N2 exchange rows of pitch XP
  cpx<T>* R = Xr0 + N2 * S::XP;        // build: Q, Yw; valence loop: Xk
  static_assert(XyTile<T>::CT <= 2, "the y pass splits columns over at most two planes");
  const int ekx = 2 * gx + 1, eky = 2 * gy + 1, XKP = ekx | 1;
  const unsigned ekx_magic = ekx > 1 ? 0xffffffffu / (unsigned)ekx + 1u : 0u;
  const int ncg = (nct + CT - 1) / CT;
  const long long lin = xcd_linear(blockIdx.x, (long long)n3 * ncg);
  if (lin < 0) return;
  const int z = (int)(lin / ncg), cg = (int)(lin % ncg);
  const int tid = threadIdx.x;
  const int y = tid / S::L1, t = tid % S::L1;
  const bool act = y < N2 && t < S::A1;
  for (int i = tid; i < N1; i += S::NTH) tw1[i] = twx[i];
  for (int i = tid; i < N2; i += S::NTH) tw2[i] = twy[i];
  const int ncw = exw * eyw, YP = exw | 1;
  // FP32: the column table of T in LDS after R (build: ncw + N2 (exw | 1)
  // entries; valence loop: VB CT N2 XKP), read once per kept output of the y
  // pass (1% of the C3 plane pass). FP64 reads it from global memory: the LDS
  // copy's pointer costs the 128-register kernel two more spilled registers,
  // which cost more than the loads save.
  constexpr bool kDkLds = sizeof(T) == 4;
  const int rlen = max(ncw + N2 * YP, VB * CT * N2 * XKP);
  int* Dk = reinterpret_cast<int*>(R + rlen);
  if constexpr (kDkLds)
    for (int i = tid; i < ekx * eky; i += S::NTH) Dk[i] = disk[i];
  cpx<T>* Q = R;
  cpx<T>* Yw = R + ncw;

  // ---- conduction planes, built from their compact slabs
  cpx<T> cr[CT][S::B1][NS];
#pragma unroll
  for (int ct = 0; ct < CT; ++ct) {
    const int cl = cg * CT + ct;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (cl < nct) {
        const cpx<T>* src = tcz + (((size_t)(c0 + cl) * NS + s) * n3 + z) * ncw;
        for (int i = tid; i < ncw; i += S::NTH) Q[i] = src[i];
      }
      lds_sync();  // Q in place (and the twiddles, the first time)
      if (cl < nct) {
        // y transform of the slab's columns, split as n2 = A2 B2 like the
        // pencils: for output y = t + A2 m, b_r = sum_{g_y = r mod B2} Q(g_y)
        // W_n2^(g_y t) and one B2-point DFT gives the B2 outputs of item (jx, t)
        for (int o = tid; o < exw * S::A2; o += S::NTH) {
          const int jx = o / S::A2, t2 = o - jx * S::A2;
          cpx<T> b[S::B2];
#pragma unroll
          for (int r = 0; r < S::B2; ++r) {
            b[r] = mk<T>(0, 0);
            for (int g = -gyw + mod_pos(r + gyw, S::B2); g <= gyw; g += S::B2)
              b[r] = b[r] + cmul(Q[(g + gyw) * exw + jx], tw2[mod_pos(g * t2, N2)]);
          }
          reg_dft<T, S::B2>(b);
#pragma unroll
          for (int m = 0; m < S::B2; ++m) Yw[(t2 + S::A2 * m) * YP + jx] = b[m];
        }
      }
      lds_sync();  // Yw complete
      if (act) {
        cpx<T> b[S::B1];
#pragma unroll
        for (int r = 0; r < S::B1; ++r) {
          b[r] = mk<T>(0, 0);
          if (cl < nct) {
            // gx = r (mod B1), from the smallest such gx >= -gxw
            for (int g = -gxw + mod_pos(r + gxw, S::B1); g <= gxw; g += S::B1)
              b[r] = b[r] + cmul(Yw[y * YP + g + gxw], tw1[mod_pos(g * t, N1)]);
          }
        }
        reg_dft<T, S::B1>(b);
#pragma unroll
        for (int m = 0; m < S::B1; ++m) cr[ct][m][s] = b[m];
      }
      lds_sync();  // Q and Yw consumed before the next slab
    }
  }

  // ---- valence loop; the next band's row slice is loaded while the current
  // band is transformed (barriers order LDS only, so the loads stay in flight)
  cpx<T>* Xr = Xr0 + (act ? y : 0) * S::XP;
  cpx<T>* Xk = R;
  const size_t vstride = (size_t)n3 * NP;  // one spinor component of one band
  const int nvalid = min(CT, nct - cg * CT);
  const cpx<T>* pv0 = uvz + (size_t)z * NP + (size_t)(act ? y : 0) * N1 + (act ? t : 0);
  // one row-slice buffer: each band's slice is consumed by the products before
  // the next band's loads are issued into the same registers
  // the lane's first kept x and y frequencies (more only when an eps sphere is
  // wider than a lane group: 2 g + 1 > 16)
  const KeptPlan<T> xplan = kept_plan<T, S::A1, S::B1>(t - gx, tw1);
  const int tt = tid % S::L2;
  cpx<T> vn[S::B1][NS];
  auto fetch = [&](int vl) {
    const cpx<T>* pv = pv0 + (size_t)(v0 + vl) * NS * vstride;
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int m = 0; m < S::B1; ++m) vn[m][s] = pv[s * vstride + S::A1 * m];
  };
  if (act) fetch(0);
  for (int g0 = 0; g0 < nvt; g0 += VB) {
    const int nb = min(VB, nvt - g0);
    for (int j = 0; j < nb; ++j) {
      if (act) {
        // products of the band's row slice with every conduction plane
        cpx<T> pa[CT][S::B1];
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
          for (int m = 0; m < S::B1; ++m) pa[ct][m] = spin_dot<T, NS>(vn[m], cr[ct][m]);
        // the last band fetches itself again (unconditional loads keep the
        // buffer in one set of registers). The empty asm statements pin the
        // products ahead of the loads: the loads then reuse the registers the
        // products just consumed, instead of a second set that is copied back
        // (and waited for) at the end of every iteration
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
          for (int m = 0; m < S::B1; ++m) asm volatile("" ::"v"(pa[ct][m].x), "v"(pa[ct][m].y));
        asm volatile("" ::: "memory");
        fetch(min(g0 + j + 1, nvt - 1));
        // x transforms, kept outputs to Xk. The lane index is made opaque
        // here so that the twiddle addresses t k2 are recomputed (one integer
        // multiply each) rather than held across the loop, where they would be
        // spilled and their reloads would wait on the prefetch just issued
        int tq = t;
        asm volatile("" : "+v"(tq));
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
          if (ct < nvalid) {
            cpx<T>* a = pa[ct];
            reg_dft<T, S::B1>(a);
            // tw[0] = 1 exactly, so lane 0 multiplies by one without rounding
#pragma unroll
            for (int k2 = 1; k2 < S::B1; ++k2) a[k2] = cmul(a[k2], tw1[tq * k2]);
#pragma unroll
            for (int k2 = 0; k2 < S::B1; ++k2) Xr[k2 * S::A1 + t] = a[k2];
            // the row's lanes share a wavefront, whose LDS accesses complete in order
            __builtin_amdgcn_wave_barrier();
            cpx<T>* xk = Xk + ((size_t)(j * CT + ct) * N2 + y) * XKP;
            if (t < ekx) xk[t] = kept_eval<T, S::A1>(Xr, 1, xplan);
            for (int jk = t + S::L1; jk < ekx; jk += S::L1)
              xk[jk] = kept_out<T, S::A1, S::B1>(Xr, 1, jk - gx, tw1);
            // the next product's exchange writes follow these reads in order
            __builtin_amdgcn_wave_barrier();
          }
        }
      }
    }
    lds_sync();  // every kept x column of the group is in Xk
    // y transforms of the kept columns (j, ct, jkx): A2 lanes of B2 values per
    // column, the first factor in registers (written back in place, twiddled),
    // the second at the kept y frequencies only
    const int pp = tid / S::L2;
    const KeptPlan<T> yplan = kept_plan<T, S::A2, S::B2>(tt - gy, tw2);
    const int tot = nb * nvalid * ekx;
    for (int q0 = 0; q0 < tot; q0 += S::NTH / S::L2) {
      const int q = q0 + pp;
      if (q < tot) {
        // q / ekx by multiply-high (exact for q ekx < 2^32; the magic number
        // of ekx = 1 would be 2^32)
        const int jc = ekx == 1 ? q : (int)__umulhi((unsigned)q, ekx_magic), jk = q - jc * ekx;
        const int j = nvalid == 1 ? jc : jc >> 1, ct = jc - j * nvalid;
        cpx<T>* col = Xk + (size_t)(j * CT + ct) * N2 * XKP + jk;
        if (tt < S::A2) {
          cpx<T> a[S::B2];
#pragma unroll
          for (int m = 0; m < S::B2; ++m) a[m] = col[(tt + S::A2 * m) * XKP];
          reg_dft<T, S::B2>(a);
#pragma unroll
          for (int k2 = 1; k2 < S::B2; ++k2) a[k2] = cmul(a[k2], tw2[tt * k2]);
#pragma unroll
          for (int k2 = 0; k2 < S::B2; ++k2) col[(k2 * S::A2 + tt) * XKP] = a[k2];
        }
        __builtin_amdgcn_wave_barrier();
        // only the (x, y) columns that hold eps-sphere points are kept
        const size_t pl = (size_t)(cg * CT + ct) * nvt + g0 + j;
        cpx<T>* dst = tout + (pl * n3 + z) * (size_t)ndisk;
        if (tt < eky) {
          const cpx<T> val = kept_eval<T, S::A2>(col, XKP, yplan);
          const int d = kDkLds ? Dk[tt * ekx + jk] : disk[tt * ekx + jk];
          if (d >= 0) dst[d] = val;
        }
        for (int jky = tt + S::L2; jky < eky; jky += S::L2) {
          const cpx<T> val = kept_out<T, S::A2, S::B2>(col, XKP, jky - gy, tw2);
          const int d = kDkLds ? Dk[jky * ekx + jk] : disk[jky * ekx + jk];
          if (d >= 0) dst[d] = val;
        }
      }
    }
    lds_sync();  // Xk consumed before the next group writes it
  }
}

// ---------------------------------------------------------------- z pass
// For each pair and (jkx, jky) column of T (those holding eps-sphere points,
// listed after the column map in disk), the z transform with A lanes
// of B values, keeping |g_z| <= gz, scaled by 1/N and scattered onto the eps
// sphere through its compact cube map emap[jx][jy][jz].
template <typename T, int N3>
__global__ void __launch_bounds__(kZThreads) k_pair_zp(
    const cpx<T>* __restrict__ tin, int ekx, int eky, int ekz, int gz,
    const int* __restrict__ emap, const int* __restrict__ disk, int ndisk,
    const cpx<T>* __restrict__ twz, T invN, int v0, int nvt, int c0, int nc_total, int neps,
    int npairs, cpx<T>* __restrict__ M) {
  constexpr int A = split_n1(N3), B = N3 / A, L = pow2_at_least(A), CPB = kZThreads / L;
  __shared__ cpx<T> X[CPB][N3 + 1];
  __shared__ cpx<T> tw[N3];
  // all column blocks of a pair on one XCD: its scattered stores into the
  // pair's row of M then fill whole lines in that XCD's L2 before write-back
  const int ncol = ndisk, nbx = (ncol + CPB - 1) / CPB;
  const long long lin = xcd_linear(blockIdx.x, (long long)nbx * npairs);
  if (lin < 0) return;
  const int pr = (int)(lin / nbx), bx = (int)(lin - (long long)pr * nbx), tid = threadIdx.x;
  for (int i = tid; i < N3; i += kZThreads) tw[i] = twz[i];
  __syncthreads();
  const int cq = tid / L, t = tid % L;
  const int col = bx * CPB + cq;
  if (col >= ncol || t >= A) return;
  const cpx<T>* src = tin + (size_t)pr * N3 * ncol + col;
  cpx<T> a[B];
#pragma unroll
  for (int m = 0; m < B; ++m) a[m] = src[(size_t)(t + A * m) * ncol];
  reg_dft<T, B>(a);
#pragma unroll
  for (int k2 = 1; k2 < B; ++k2) a[k2] = cmul(a[k2], tw[t * k2]);
  cpx<T>* Xr = X[cq];
#pragma unroll
  for (int k2 = 0; k2 < B; ++k2) Xr[k2 * A + t] = a[k2];
  __builtin_amdgcn_wave_barrier();
  const int v = v0 + pr % nvt, c = c0 + pr / nvt;
  cpx<T>* dst = M + ((size_t)v * nc_total + c) * neps;
  const int cxy = disk[ekx * eky + col];  // jky * ekx + jkx of this column
  const int jky = cxy / ekx, jkx = cxy - jky * ekx;
  const int* em = emap + ((size_t)jkx * eky + jky) * ekz;
#pragma unroll
  for (int s = 0; s < (B + A - 1) / A; ++s) {
    const int k2 = t + A * s;
    if (k2 < B) {
      cpx<T> u[A];
#pragma unroll
      for (int n = 0; n < A; ++n) u[n] = Xr[k2 * A + n];
      reg_dft<T, A>(u);
#pragma unroll
      for (int k1 = 0; k1 < A; ++k1) {
        const int jz = kept(k2 + B * k1, N3, gz);
        if (jz >= 0) {
          const int idx = em[jz];
          if (idx >= 0) dst[idx] = scal(u[k1], invN);
        }
      }
    }
  }
}

// ---------------------------------------------------------------- launchers
// (n1, n2) xy-plane shapes and z lengths built for this path
#define GW_XY_SHAPES(X) X(60, 60) X(16, 16)
#define GW_XY_ZLEN(X) X(160) X(40)

bool pair_xy_shape(const int box[3]) {
  bool plane = false, zlen = false;
#define X(A, B) if (box[0] == A && box[1] == B) plane = true;
  GW_XY_SHAPES(X)
#undef X
#define X(N) if (box[2] == N) zlen = true;
  GW_XY_ZLEN(X)
#undef X
  return plane && zlen;
}

size_t band_zc_bytes(const int box[3], const SphereMap* sm, int nbs, size_t elem) {
  return (size_t)nbs * box[2] * sm->ext[0] * sm->ext[1] * elem;
}

size_t pair_xy_scratch_bytes(const int box[3], const SphereMap* em, int npairs, size_t elem) {
  return (size_t)npairs * box[2] * em->ndisk * elem;
}

template <typename K>
static hipError_t allow_lds_xy(K kernel, size_t bytes) {
  if (bytes <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <typename T>
gw_status band_zc(gw_ctx* c, const int box[3], int nbs, int ng, const void* coef,
                  const SphereMap* sm, void* out) {
  const void* twz;
  gw_status st;
  if ((st = twiddle_table(c, box[2], sizeof(T) == 8, &twz)) != GW_OK) return st;
  const int ncol = sm->ext[0] * sm->ext[1];
  ProfScope ps(c, "band_zc");
  bool done = false;
#define X(N)                                                                                  \
  if (!done && box[2] == N) {                                                                 \
    done = true;                                                                              \
    constexpr int CPB = kZThreads / pow2_at_least(split_n1(N));                               \
    for (int b0 = 0; b0 < nbs; b0 += 65535) {                                                 \
      const int nb = std::min(65535, nbs - b0);                                               \
      hipLaunchKernelGGL((k_band_zc<T, N>), dim3((ncol + CPB - 1) / CPB, nb), dim3(kZThreads), \
                         0, c->stream, static_cast<const cpx<T>*>(coef) + (size_t)b0 * ng, ng, \
                         sm->d_cube, sm->ext[0], sm->ext[1], sm->ext[2], sm->gmax[2],         \
                         static_cast<const cpx<T>*>(twz),                                     \
                         static_cast<cpx<T>*>(out) + (size_t)b0 * N * ncol);                   \
    }                                                                                         \
  }
  GW_XY_ZLEN(X)
#undef X
  if (!done) return fail(c, GW_EUNSUPPORTED, "no z-slab kernel for n3 = %d", box[2]);
  GW_CHECK_LAUNCH(c, "k_band_zc");
  return GW_OK;
}

template <typename T>
gw_status grid_to_zyx(gw_ctx* c, const int box[3], int nbs, const void* u, void* w) {
  const int n1 = box[0], n2 = box[1], n3 = box[2];
  ProfScope ps(c, "band_zyx");
  const int per = std::max(1, 65535 / n2);  // band-spins per launch (grid z <= 65535)
  for (int b0 = 0; b0 < nbs; b0 += per) {
    const int nb = std::min(per, nbs - b0);
    const size_t off = (size_t)b0 * n1 * n2 * n3;
    hipLaunchKernelGGL(k_to_zyx<T>, dim3((n3 + 31) / 32, (n1 + 31) / 32, nb * n2), dim3(256), 0,
                       c->stream, static_cast<const cpx<T>*>(u) + off, n1, n2, n3,
                       static_cast<cpx<T>*>(w) + off);
  }
  GW_CHECK_LAUNCH(c, "k_to_zyx");
  return GW_OK;
}

template <typename T>
gw_status pair_to_eps_xy(gw_ctx* c, const int box[3], int nspinor, const void* uvz,
                         const void* tcz, const SphereMap* sc, int v0, int nvt, int c0, int nct,
                         int nc_total, const SphereMap* em, void* mtxel, void* scratch) {
  const int n1 = box[0], n2 = box[1], n3 = box[2];
  const void *twx, *twy, *twz;
  const bool dbl = sizeof(T) == 8;
  gw_status st;
  if ((st = twiddle_table(c, n1, dbl, &twx)) != GW_OK) return st;
  if ((st = twiddle_table(c, n2, dbl, &twy)) != GW_OK) return st;
  if ((st = twiddle_table(c, n3, dbl, &twz)) != GW_OK) return st;
  if (nvt <= 0 || nct <= 0) return GW_OK;
  const int gx = em->gmax[0], gy = em->gmax[1];
  const int ekx = em->ext[0], eky = em->ext[1];
  cpx<T>* tbuf = static_cast<cpx<T>*>(scratch);
  bool done = false;
  {
    ProfScope ps(c, "pair_plane");
#define X(A, B)                                                                                 \
  if (!done && n1 == A && n2 == B) {                                                            \
    done = true;                                                                                \
    using S = XyShape<T, A, B>;                                                                 \
    constexpr int CT = XyTile<T>::CT, VB = XyTile<T>::VB;                                       \
    const int ncw = sc->ext[0] * sc->ext[1];                                                    \
    const size_t build = (size_t)ncw + (size_t)B * (sc->ext[0] | 1);                            \
    const size_t xk = (size_t)VB * CT * B * (ekx | 1);                                          \
    const size_t lds = ((size_t)A + B + (size_t)B * S::XP + std::max(build, xk)) * sizeof(cpx<T>) + \
                       (size_t)ekx * eky * sizeof(int);                                           \
    const int ncg = (nct + CT - 1) / CT;                                                        \
    const long long tot = (long long)n3 * ncg;                                                  \
    const unsigned grid = (unsigned)(((tot + kXcd - 1) / kXcd) * kXcd);                         \
    if (nspinor == 2) {                                                                         \
      if (!c->capturing) GW_HIP(c, allow_lds_xy(k_pair_xy<T, 2, A, B>, lds));                   \
      hipLaunchKernelGGL((k_pair_xy<T, 2, A, B>), dim3(grid), dim3(S::NTH), lds, c->stream,     \
                         static_cast<const cpx<T>*>(uvz), static_cast<const cpx<T>*>(tcz),       \
                         sc->ext[0], sc->ext[1], sc->gmax[0], sc->gmax[1], v0, nvt, c0, nct, n3, \
                         gx, gy, static_cast<const cpx<T>*>(twx),                               \
                         static_cast<const cpx<T>*>(twy), em->d_disk, em->ndisk, tbuf);          \
    } else {                                                                                    \
      if (!c->capturing) GW_HIP(c, allow_lds_xy(k_pair_xy<T, 1, A, B>, lds));                   \
      hipLaunchKernelGGL((k_pair_xy<T, 1, A, B>), dim3(grid), dim3(S::NTH), lds, c->stream,     \
                         static_cast<const cpx<T>*>(uvz), static_cast<const cpx<T>*>(tcz),       \
                         sc->ext[0], sc->ext[1], sc->gmax[0], sc->gmax[1], v0, nvt, c0, nct, n3, \
                         gx, gy, static_cast<const cpx<T>*>(twx),                               \
                         static_cast<const cpx<T>*>(twy), em->d_disk, em->ndisk, tbuf);          \
    }                                                                                           \
  }
    GW_XY_SHAPES(X)
#undef X
    if (!done) return fail(c, GW_EUNSUPPORTED, "no xy-plane kernel for %d x %d", n1, n2);
    GW_CHECK_LAUNCH(c, "k_pair_xy");
  }
  {
    ProfScope ps(c, "pair_xpass");
    const T invN = (T)(1.0 / ((double)n1 * n2 * n3));
    const int npairs = nvt * nct;
    done = false;
#define X(N)                                                                                   \
  if (!done && n3 == N) {                                                                      \
    done = true;                                                                               \
    constexpr int CPB = kZThreads / pow2_at_least(split_n1(N));                                \
    const long long tot = (long long)((em->ndisk + CPB - 1) / CPB) * npairs;                   \
    const unsigned grid = (unsigned)(((tot + kXcd - 1) / kXcd) * kXcd);                        \
    hipLaunchKernelGGL((k_pair_zp<T, N>), dim3(grid), dim3(kZThreads), 0, c->stream, tbuf,     \
                       ekx, eky, em->ext[2], em->gmax[2], em->d_cube, em->d_disk, em->ndisk,    \
                       static_cast<const cpx<T>*>(twz), invN, v0, nvt, c0, nc_total, em->n,    \
                       npairs, static_cast<cpx<T>*>(mtxel));                                   \
  }
    GW_XY_ZLEN(X)
#undef X
    if (!done) return fail(c, GW_EUNSUPPORTED, "no z-pass kernel for n3 = %d", n3);
    GW_CHECK_LAUNCH(c, "k_pair_zp");
  }
  return GW_OK;
}

template gw_status band_zc<double>(gw_ctx*, const int*, int, int, const void*, const SphereMap*,
                                   void*);
template gw_status band_zc<float>(gw_ctx*, const int*, int, int, const void*, const SphereMap*,
                                  void*);
template gw_status grid_to_zyx<double>(gw_ctx*, const int*, int, const void*, void*);
template gw_status grid_to_zyx<float>(gw_ctx*, const int*, int, const void*, void*);
template gw_status pair_to_eps_xy<double>(gw_ctx*, const int*, int, const void*, const void*,
                                          const SphereMap*, int, int, int, int, int,
                                          const SphereMap*, void*, void*);
template gw_status pair_to_eps_xy<float>(gw_ctx*, const int*, int, const void*, const void*,
                                         const SphereMap*, int, int, int, int, int,
                                         const SphereMap*, void*, void*);

}  // namespace gw
