// eps^-1 in a reduced basis of static eigenvectors.
//
// Sec. IV (Bi2Se3, full frequency) keeps 200 eigenvectors of the static
// dielectric matrix, about a tenth of the spectrum, and treats every frequency
// in that basis.  With V = diag(v) and the Hermitian epst(w) = I - V^1/2 chi0(w) V^1/2
// (eps is similar to it), U the eigenvectors of epst(0) with the nb largest
// eigenvalues and epst_B(w) = U^H epst(w) U:
//   epst^-1(w) ~= I + U (epst_B(w)^-1 - I) U^H,   eps^-1 = V^1/2 epst^-1 V^-1/2.
//
// The eigenvectors come from a Jacobi method on the GPU, repeated in sweeps
// until the off-diagonal Frobenius norm is below 1e-14 of the matrix's, one
// sweep captured into a HIP graph and replayed:
//   - N >= 128: block Jacobi. 32 x 32 sub-problems (pairs of 16-row blocks) are
//     diagonalised in LDS (k_bj_solve), and their unitaries update the block
//     rows and columns of A and the eigenvector rows on the matrix cores
//     (k_bj_mix), in round-robin rounds over block pairs;
//   - N < 128: N - 1 rounds of N/2 disjoint plane rotations, each round one
//     kernel that forms its rotations and rewrites the two rows of J^H A J and
//     of the eigenvector rows of every pair in LDS (k_jac_round_pp).
// The projections and the small inverses run on the FP64 GEMM and the
// library's Hermitian inverse (Gauss-Jordan with its checks).
#include <cmath>
#include <vector>

#include "common.h"

namespace gw {

namespace {
struct JacRot {
  int p, q, skip, pad;
  double c, s, er, ei;  // J = [[c, s], [-s e^{-i phi}, c e^{-i phi}]], e^{i phi} = er + i ei
};
}  // namespace

__global__ void k_lr_epst(const cpx<double>* __restrict__ chi, const double* __restrict__ v,
                          int N, cpx<double>* __restrict__ E) {
  const size_t nn = (size_t)N * N;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nn) return;
  const int i = (int)(e / N), j = (int)(e % N);
  const double s = sqrt(v[i]) * sqrt(v[j]);
  const cpx<double> x = chi[(size_t)blockIdx.y * nn + e];
  E[(size_t)blockIdx.y * nn + e] = mk((i == j ? 1.0 : 0.0) - s * x.x, -s * x.y);
}

// The whole round in one kernel, reading A_in and writing A_out (the two buffers
// alternate between rounds): every workgroup first forms the rotation of every
// pair of the round from A_in into LDS (so no separate parameter kernel and no
// grid-wide wait), then rewrites its own pair's two rows as k_jac_round does.
__global__ void __launch_bounds__(256) k_jac_round_pp(const cpx<double>* __restrict__ Ain,
                                                      cpx<double>* __restrict__ Aout,
                                                      cpx<double>* __restrict__ Vt, int N, int m,
                                                      int r) {
  extern __shared__ char smem[];
  JacRot* rot = reinterpret_cast<JacRot*>(smem);
  int* pairof = reinterpret_cast<int*>(rot + m / 2);
  cpx<double>* bp = reinterpret_cast<cpx<double>*>(pairof + ((N + 3) & ~3));
  cpx<double>* bq = bp + N;
  for (int k = threadIdx.x; k < m / 2; k += blockDim.x) {
    int p, q;
    if (k == 0) {
      p = r;
      q = m - 1;
    } else {
      p = (r + k) % (m - 1);
      q = (r - k + (m - 1)) % (m - 1);
    }
    if (p > q) {
      const int t = p;
      p = q;
      q = t;
    }
    JacRot o;
    o.p = p;
    o.q = q;
    o.pad = 0;
    o.skip = 1;
    o.c = 1.0;
    o.s = 0.0;
    o.er = 1.0;
    o.ei = 0.0;
    if (q < N) {
      const cpx<double> b = Ain[(size_t)p * N + q];
      const double ab = hypot(b.x, b.y);
      if (ab > 0.0) {
        const double a = Ain[(size_t)p * N + p].x, d = Ain[(size_t)q * N + q].x;
        const double tau = (d - a) / (2.0 * ab);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        o.c = 1.0 / sqrt(1.0 + t * t);
        o.s = t * o.c;
        o.er = b.x / ab;
        o.ei = b.y / ab;
        o.skip = 0;
      }
    }
    rot[k] = o;
    if (p < N) pairof[p] = k;
    if (q < N) pairof[q] = k;
  }
  __syncthreads();
  const JacRot o = rot[blockIdx.x];
  const bool hasq = o.q < N;
  const cpx<double> e = mk(o.er, o.ei), ec = mk(o.er, -o.ei);
  for (int j = threadIdx.x; j < N; j += blockDim.x) {
    const cpx<double> ap = Ain[(size_t)o.p * N + j];
    const cpx<double> aq = hasq ? Ain[(size_t)o.q * N + j] : mk(0.0, 0.0);
    if (o.skip) {
      bp[j] = ap;
      bq[j] = aq;
    } else {
      const cpx<double> eq = cmul(e, aq);
      bp[j] = scal(ap, o.c) - scal(eq, o.s);
      bq[j] = scal(ap, o.s) + scal(eq, o.c);
      const cpx<double> vp = Vt[(size_t)o.p * N + j], vq = Vt[(size_t)o.q * N + j];
      const cpx<double> ev = cmul(ec, vq);
      Vt[(size_t)o.p * N + j] = scal(vp, o.c) - scal(ev, o.s);
      Vt[(size_t)o.q * N + j] = scal(vp, o.s) + scal(ev, o.c);
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < N; j += blockDim.x) {
    const JacRot w = rot[pairof[j]];
    cpx<double> np = bp[j], nq = bq[j];
    if (!w.skip) {
      const cpx<double> wc = mk(w.er, -w.ei);
      if (j == w.p) {
        np = scal(bp[w.p], w.c) - scal(cmul(wc, bp[w.q]), w.s);
        nq = scal(bq[w.p], w.c) - scal(cmul(wc, bq[w.q]), w.s);
      } else {
        np = scal(bp[w.p], w.s) + scal(cmul(wc, bp[w.q]), w.c);
        nq = scal(bq[w.p], w.s) + scal(cmul(wc, bq[w.q]), w.c);
      }
    }
    Aout[(size_t)o.p * N + j] = np;
    if (hasq) Aout[(size_t)o.q * N + j] = nq;
  }
}

__global__ void k_lr_copy(const cpx<double>* __restrict__ src, size_t n, cpx<double>* __restrict__ dst) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) dst[e] = src[e];
}

typedef double v4f64 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------- block Jacobi
// For larger N the rotations act on pairs of 16-wide blocks: a round pairs the
// nblk blocks in round-robin order; each pair's 32 x 32 Hermitian sub-matrix is
// diagonalised in LDS by a few inner sweeps of the same scalar rotations, and the
// accumulated 32 x 32 unitaries then update A in one pass: the tile on the rows
// of pair P and the columns of pair Q becomes W_P^H A W_Q, and the eigenvector
// rows of pair P become W_P^T Vt.
// The matrix is padded to a multiple of 32 with zero rows and columns, which no
// rotation ever touches (their off-diagonal entries stay 0).
constexpr int kBJ = 16;           // block width
constexpr int kBJ2 = 2 * kBJ;     // sub-problem size
constexpr int kBJInner = 1;       // inner sweeps per round

__device__ __forceinline__ void bj_pair(int nblk, int r, int k, int* I, int* J) {
  int a, b;
  if (k == 0) {
    a = r;
    b = nblk - 1;
  } else {
    a = (r + k) % (nblk - 1);
    b = (r - k + (nblk - 1)) % (nblk - 1);
  }
  *I = a < b ? a : b;
  *J = a < b ? b : a;
}

// Qt[k] (32 x 32, rows = columns of W) for pair k of round r
// Reciprocal and reciprocal square root from the hardware estimates refined by
// two Newton steps (about one ulp); finite, positive, normal arguments only.
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ double rsq_nr(double x) {
  double r = __builtin_amdgcn_rsq(x);
  r = fma(0.5 * r, fma(-x * r, r, 1.0), r);
  return fma(0.5 * r, fma(-x * r, r, 1.0), r);
}

__global__ void __launch_bounds__(512) k_bj_solve(const cpx<double>* __restrict__ A, int Np,
                                                  int nblk, int r, cpx<double>* __restrict__ Qt) {
  __shared__ cpx<double> S[kBJ2][kBJ2 + 1];
  __shared__ cpx<double> W[kBJ2][kBJ2 + 1];  // W^T: row x = column x of W
  __shared__ JacRot prm[kBJ];
  int I, J;
  bj_pair(nblk, r, blockIdx.x, &I, &J);
  const int t = threadIdx.x;
  for (int e = t; e < kBJ2 * kBJ2; e += blockDim.x) {
    const int x = e / kBJ2, y = e % kBJ2;
    const int gx = (x < kBJ ? I * kBJ + x : J * kBJ + x - kBJ);
    const int gy = (y < kBJ ? I * kBJ + y : J * kBJ + y - kBJ);
    S[x][y] = A[(size_t)gx * Np + gy];
    W[x][y] = mk(x == y ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  for (int sweep = 0; sweep < kBJInner; ++sweep)
    for (int rr = 0; rr < kBJ2 - 1; ++rr) {
      if (t < kBJ) {
        int p, q;
        if (t == 0) {
          p = rr;
          q = kBJ2 - 1;
        } else {
          p = (rr + t) % (kBJ2 - 1);
          q = (rr - t + (kBJ2 - 1)) % (kBJ2 - 1);
        }
        if (p > q) {
          const int tmp = p;
          p = q;
          q = tmp;
        }
        JacRot o;
        o.p = p;
        o.q = q;
        o.pad = 0;
        o.skip = 1;
        o.c = 1.0;
        o.s = 0.0;
        o.er = 1.0;
        o.ei = 0.0;
        const cpx<double> b = S[p][q];
        const double n2 = b.x * b.x + b.y * b.y;
        // below 1e-300 the entry is far under the convergence threshold; skipping
        // it also keeps the reciprocal square root away from subnormal input
        if (n2 > 1e-300) {
          const double a = S[p][p].x, d = S[q][q].x;
          // 1/|b|; squares past 1e300 (|b| above 1e150) take the IEEE route
          const double rab = n2 < 1e300 ? rsq_nr(n2) : 1.0 / hypot(b.x, b.y);
          const double tau = 0.5 * (d - a) * rab;
          const double at = fabs(tau);
          // tt = sign(tau) / (|tau| + sqrt(1 + tau^2)), the smaller root
          double tt;
          if (at < 1e100) {
            const double u = fma(tau, tau, 1.0);
            tt = rcp_nr(at + u * rsq_nr(u));
          } else {
            tt = 0.5 * rcp_nr(at);
          }
          if (tau < 0.0) tt = -tt;
          o.c = rsq_nr(fma(tt, tt, 1.0));
          o.s = tt * o.c;
          o.er = b.x * rab;
          o.ei = b.y * rab;
          o.skip = 0;
        }
        prm[t] = o;
      }
      __syncthreads();
      // rows of S (J^H S) and of W^T (J^T W^T), one (pair, column) per work item
      for (int e = t; e < kBJ * kBJ2; e += blockDim.x) {
        const JacRot o = prm[e / kBJ2];
        const int j = e % kBJ2;
        if (o.skip) continue;
        const cpx<double> ev = mk(o.er, o.ei), ec = mk(o.er, -o.ei);
        const cpx<double> ap = S[o.p][j], aq = S[o.q][j];
        const cpx<double> eq = cmul(ev, aq);
        S[o.p][j] = scal(ap, o.c) - scal(eq, o.s);
        S[o.q][j] = scal(ap, o.s) + scal(eq, o.c);
        const cpx<double> wp = W[o.p][j], wq = W[o.q][j];
        const cpx<double> ew = cmul(ec, wq);
        W[o.p][j] = scal(wp, o.c) - scal(ew, o.s);
        W[o.q][j] = scal(wp, o.s) + scal(ew, o.c);
      }
      __syncthreads();
      // columns of S (S J), one (pair, row) per work item
      for (int e = t; e < kBJ * kBJ2; e += blockDim.x) {
        const JacRot o = prm[e / kBJ2];
        const int i = e % kBJ2;
        if (o.skip) continue;
        const cpx<double> ec = mk(o.er, -o.ei);
        const cpx<double> ap = S[i][o.p], aq = S[i][o.q];
        const cpx<double> eq = cmul(ec, aq);
        S[i][o.p] = scal(ap, o.c) - scal(eq, o.s);
        S[i][o.q] = scal(ap, o.s) + scal(eq, o.c);
      }
      __syncthreads();
    }
  cpx<double>* out = Qt + (size_t)blockIdx.x * kBJ2 * kBJ2;
  for (int e = t; e < kBJ2 * kBJ2; e += blockDim.x) out[e] = W[e / kBJ2][e % kBJ2];
}

// One round's update of A and of the eigenvector rows in a single pass, in place:
//   - blockIdx.y < npairs: the 32 x 32 tile of A on the rows of pair P =
//     blockIdx.x and the columns of pair Q = blockIdx.y becomes W_P^H A[P][Q] W_Q
//     (every tile belongs to one workgroup, which reads it before writing it);
//   - blockIdx.y >= npairs: 32 columns of the eigenvector rows of pair P become
//     W_P^T V[P][cols].
// Qt holds W transposed per pair: Qt[x][y] = W[y][x].
__global__ void __launch_bounds__(256) k_bj_mix(cpx<double>* __restrict__ A,
                                                cpx<double>* __restrict__ Vt, int Np, int nblk,
                                                int r, const cpx<double>* __restrict__ Qt) {
  __shared__ cpx<double> wp[kBJ2][kBJ2 + 1];
  __shared__ cpx<double> wq[kBJ2][kBJ2 + 1];  // wq[y][z] = W_Q[y][z]
  __shared__ cpx<double> a[kBJ2][kBJ2 + 1];
  const int npairs = nblk / 2, t = threadIdx.x;
  const bool vpart = (int)blockIdx.y >= npairs;
  int I, J, I2 = 0, J2 = 0;
  bj_pair(nblk, r, blockIdx.x, &I, &J);
  const cpx<double>* qp = Qt + (size_t)blockIdx.x * kBJ2 * kBJ2;
  for (int e = t; e < kBJ2 * kBJ2; e += blockDim.x) wp[e / kBJ2][e % kBJ2] = qp[e];
  if (!vpart) {
    bj_pair(nblk, r, blockIdx.y, &I2, &J2);
    const cpx<double>* qq = Qt + (size_t)blockIdx.y * kBJ2 * kBJ2;
    for (int e = t; e < kBJ2 * kBJ2; e += blockDim.x) wq[e % kBJ2][e / kBJ2] = qq[e];
  }
  const int c0 = vpart ? ((int)blockIdx.y - npairs) * kBJ2 : 0;
  auto grow = [](int x, int i, int j) { return x < kBJ ? i * kBJ + x : j * kBJ + x - kBJ; };
  auto gcol = [&](int z) { return vpart ? c0 + z : grow(z, I2, J2); };
  cpx<double>* M = vpart ? Vt : A;
  for (int e = t; e < kBJ2 * kBJ2; e += blockDim.x) {
    const int y = e / kBJ2, z = e % kBJ2;
    a[y][z] = M[(size_t)grow(y, I, J) * Np + gcol(z)];
  }
  __syncthreads();
  // Both 32 x 32 complex products run on the FP64 matrix cores: each wavefront
  // owns one 16 x 16 quadrant, three real v_mfma_f64_16x16x4_f64 products per
  // complex one (Re = t1 - t2, Im = t3 - t1 - t2), operand fragments read from
  // LDS (A operand: row l16, k lk; B operand: k lk, column l16; result element
  // e of a lane at row lk + 4e, column l16).
  const int lane = t & 63, wave = t >> 6, l16 = lane & 15, lk = lane >> 4;
  const int xq = (wave >> 1) * 16, zq = (wave & 1) * 16;
  const double sgn = vpart ? 1.0 : -1.0;  // W^T for the eigenvector rows, W^H for A
  v4f64 t1 = {0, 0, 0, 0}, t2 = t1, t3 = t1;
  for (int k0 = 0; k0 < kBJ2; k0 += 4) {
    const cpx<double> fa = wp[xq + l16][k0 + lk], fb = a[k0 + lk][zq + l16];
    const double ar = fa.x, ai = sgn * fa.y;
    t1 = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, fb.x, t1, 0, 0, 0);
    t2 = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, fb.y, t2, 0, 0, 0);
    t3 = __builtin_amdgcn_mfma_f64_16x16x4f64(ar + ai, fb.x + fb.y, t3, 0, 0, 0);
  }
  if (vpart) {
#pragma unroll
    for (int e = 0; e < 4; ++e)
      Vt[(size_t)grow(xq + lk + 4 * e, I, J) * Np + c0 + zq + l16] =
          mk(t1[e] - t2[e], (t3[e] - t1[e]) - t2[e]);
    return;
  }
  __syncthreads();  // every fragment read of the tile is done
#pragma unroll
  for (int e = 0; e < 4; ++e) a[xq + lk + 4 * e][zq + l16] = mk(t1[e] - t2[e], (t3[e] - t1[e]) - t2[e]);
  __syncthreads();
  t1 = (v4f64){0, 0, 0, 0};
  t2 = t1;
  t3 = t1;
  for (int k0 = 0; k0 < kBJ2; k0 += 4) {
    const cpx<double> fa = a[xq + l16][k0 + lk], fb = wq[k0 + lk][zq + l16];
    t1 = __builtin_amdgcn_mfma_f64_16x16x4f64(fa.x, fb.x, t1, 0, 0, 0);
    t2 = __builtin_amdgcn_mfma_f64_16x16x4f64(fa.y, fb.y, t2, 0, 0, 0);
    t3 = __builtin_amdgcn_mfma_f64_16x16x4f64(fa.x + fa.y, fb.x + fb.y, t3, 0, 0, 0);
  }
#pragma unroll
  for (int e = 0; e < 4; ++e)
    A[(size_t)grow(xq + lk + 4 * e, I, J) * Np + grow(zq + l16, I2, J2)] =
        mk(t1[e] - t2[e], (t3[e] - t1[e]) - t2[e]);
}

// zero-padded copy: dst (Np x Np) from src (N x N)
__global__ void k_bj_pad(const cpx<double>* __restrict__ src, int N, int Np,
                         cpx<double>* __restrict__ dst) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)Np * Np) return;
  const int i = (int)(e / Np), j = (int)(e % Np);
  dst[e] = (i < N && j < N) ? src[(size_t)i * N + j] : mk(0.0, 0.0);
}

// rank among the first N diagonal entries of the padded matrix (descending, ties by index)
__global__ void k_bj_rank(const cpx<double>* __restrict__ A, int Np, int N, int* __restrict__ rank,
                          double* __restrict__ lam_out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double li = A[(size_t)i * Np + i].x;
  int r = 0;
  for (int j = 0; j < N; ++j) {
    const double lj = A[(size_t)j * Np + j].x;
    r += (lj > li || (lj == li && j < i)) ? 1 : 0;
  }
  rank[i] = r;
  if (lam_out) lam_out[N - 1 - r] = li;
}

__global__ void k_bj_select(const cpx<double>* __restrict__ Vt, int Np, const int* __restrict__ rank,
                            int N, int nb, cpx<double>* __restrict__ U,
                            cpx<double>* __restrict__ Uh) {
  const int i = blockIdx.x;
  const int r = rank[i];
  if (r >= nb) return;
  for (int g = threadIdx.x; g < N; g += blockDim.x) {
    const cpx<double> x = Vt[(size_t)i * Np + g];
    U[(size_t)g * nb + r] = x;
    Uh[(size_t)r * N + g] = mk(x.x, -x.y);
  }
}

// Frobenius norms as (scale, ssq) with norm = scale * sqrt(ssq), the scaled
// sum of squares of LAPACK's lassq: no square is formed of an unscaled entry,
// so entries up to the double range neither overflow nor lose their smallest
// companions to underflow.
struct ScaledSsq {
  double scale, ssq;
};
__host__ __device__ __forceinline__ void ssq_add(ScaledSsq& a, double x) {
  const double ax = fabs(x);
  if (ax == 0.0) return;
  if (a.scale < ax) {
    const double r = a.scale / ax;
    a.ssq = fma(a.ssq * r, r, 1.0);
    a.scale = ax;
  } else {
    const double r = ax / a.scale;
    a.ssq = fma(r, r, a.ssq);
  }
}
__host__ __device__ __forceinline__ ScaledSsq ssq_merge(ScaledSsq a, ScaledSsq b) {
  if (a.scale < b.scale) {
    const ScaledSsq t = a;
    a = b;
    b = t;
  }
  if (b.scale == 0.0) return a;
  const double r = b.scale / a.scale;
  a.ssq = fma(b.ssq * r, r, a.ssq);
  return a;
}
// Non-finite entries are flagged on their own: a NaN compares false in ssq_add
// and would drop out of the sums.
constexpr int kNormParts = 1024;          // blocks of the norm reduction, at most
constexpr size_t kNormPartBytes = (size_t)kNormParts * 5 * sizeof(double);

// per block: (scale, ssq) off the diagonal and over all entries, and a
// non-finite flag, in a fixed order
__global__ void __launch_bounds__(256) k_lr_norms(const cpx<double>* __restrict__ A, int N,
                                                  double* __restrict__ part) {
  __shared__ ScaledSsq so[256], sa[256];
  __shared__ int bad[256];
  const size_t nn = (size_t)N * N;
  ScaledSsq off{0.0, 0.0}, all{0.0, 0.0};
  int nf = 0;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < nn; e += (size_t)gridDim.x * 256) {
    const cpx<double> x = A[e];
    nf |= !(isfinite(x.x) && isfinite(x.y));
    ssq_add(all, x.x);
    ssq_add(all, x.y);
    if (e / N != e % N) {
      ssq_add(off, x.x);
      ssq_add(off, x.y);
    }
  }
  so[threadIdx.x] = off;
  sa[threadIdx.x] = all;
  bad[threadIdx.x] = nf;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      so[threadIdx.x] = ssq_merge(so[threadIdx.x], so[threadIdx.x + h]);
      sa[threadIdx.x] = ssq_merge(sa[threadIdx.x], sa[threadIdx.x + h]);
      bad[threadIdx.x] |= bad[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double* o = part + 5 * (size_t)blockIdx.x;
    o[0] = so[0].scale;
    o[1] = so[0].ssq;
    o[2] = sa[0].scale;
    o[3] = sa[0].ssq;
    o[4] = bad[0] ? 1.0 : 0.0;
  }
}

// Jacobi convergence from the per-block norms, tracked over the sweeps.
// Converged when the off-diagonal norm is at most 1e-14 of the whole, or when
// it has reached the rounding floor of the sweeps themselves: each sweep
// rounds every entry about N times, which leaves an off-diagonal norm of order
// eps sqrt(N) of the whole that no further sweep removes (about 1.4e-14 at
// N = 4000). That floor is taken as reached once the norm is below 1e-11 of
// the whole and a sweep no longer halves it. A non-finite entry is an error.
struct JacobiTrack {
  double prev = -1.0;  // off-diagonal / whole after the previous sweep
  // 1 converged, 0 not yet, -1 a non-finite entry
  int update(const std::vector<double>& hp, int nblocks) {
    ScaledSsq so{0.0, 0.0}, sa{0.0, 0.0};
    for (int b = 0; b < nblocks; ++b) {
      const double* p = hp.data() + 5 * (size_t)b;
      if (p[4] != 0.0) return -1;
      so = ssq_merge(so, ScaledSsq{p[0], p[1]});
      sa = ssq_merge(sa, ScaledSsq{p[2], p[3]});
    }
    if (!std::isfinite(sa.scale) || !std::isfinite(sa.ssq)) return -1;
    const double all = sa.scale * std::sqrt(sa.ssq);
    const double rel = all > 0.0 ? so.scale * std::sqrt(so.ssq) / all : 0.0;
    const bool floor = prev >= 0.0 && rel <= 1e-11 && rel > 0.5 * prev;
    prev = rel;
    return (rel <= 1e-14 || floor) ? 1 : 0;
  }
};

// rank of eigenvalue i in descending order (ties by index); eigenvalues ascending out
__global__ void k_lr_rank(const cpx<double>* __restrict__ A, int N, int* __restrict__ rank,
                          double* __restrict__ lam_out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double li = A[(size_t)i * N + i].x;
  int r = 0;
  for (int j = 0; j < N; ++j) {
    const double lj = A[(size_t)j * N + j].x;
    r += (lj > li || (lj == li && j < i)) ? 1 : 0;
  }
  rank[i] = r;
  if (lam_out) lam_out[N - 1 - r] = li;
}

// U[g][rank i] = Vt[i][g] and Uh[rank i][g] = conj(Vt[i][g]) for the nb leading i
__global__ void k_lr_select(const cpx<double>* __restrict__ Vt, const int* __restrict__ rank,
                            int N, int nb, cpx<double>* __restrict__ U,
                            cpx<double>* __restrict__ Uh) {
  const int i = blockIdx.x;
  const int r = rank[i];
  if (r >= nb) return;
  for (int g = threadIdx.x; g < N; g += blockDim.x) {
    const cpx<double> x = Vt[(size_t)i * N + g];
    U[(size_t)g * nb + r] = x;
    Uh[(size_t)r * N + g] = mk(x.x, -x.y);
  }
}

// x[f] <- sign * x[f] + add * I   (nb x nb blocks)
__global__ void k_lr_shift(cpx<double>* __restrict__ x, int nb, double sign, double add) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t bb = (size_t)nb * nb;
  if (e >= bb) return;
  cpx<double>* y = x + (size_t)blockIdx.y * bb + e;
  const bool diag = (e / nb) == (e % nb);
  *y = mk(sign * y->x + (diag ? add : 0.0), sign * y->y);
}

__global__ void k_lr_fill(cpx<double>* __restrict__ out, int N, double* __restrict__ ones,
                          int nb) {
  const size_t nn = (size_t)N * N;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nn) out[(size_t)blockIdx.y * nn + e] = mk((e / N) == (e % N) ? 1.0 : 0.0, 0.0);
  if (blockIdx.x == 0 && blockIdx.y == 0)
    for (int k = threadIdx.x; k < nb; k += blockDim.x) ones[k] = 1.0;
}

__global__ void k_lr_unscale(cpx<double>* __restrict__ out, const double* __restrict__ v, int N) {
  const size_t nn = (size_t)N * N;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nn) return;
  const int i = (int)(e / N), j = (int)(e % N);
  cpx<double>* y = out + (size_t)blockIdx.y * nn + e;
  *y = scal(*y, sqrt(v[i]) / sqrt(v[j]));
}

// X[p][g] = M[p][g] sqrt(v[g]), widened to double
template <typename Tin>
__global__ void k_proj_prep(const cpx<Tin>* __restrict__ m, size_t rows, int N,
                            const double* __restrict__ v, cpx<double>* __restrict__ x) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * (size_t)N) return;
  const cpx<Tin> a = m[e];
  const double s = sqrt(v[e % N]);
  x[e] = mk(s * (double)a.x, s * (double)a.y);
}

// Uh[r][g] = conj(U[g][r])
__global__ void k_lr_conjt(const cpx<double>* __restrict__ U, int N, int nb,
                           cpx<double>* __restrict__ Uh) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)N * nb) return;
  const int g = (int)(e / nb), r = (int)(e % nb);
  const cpx<double> x = U[e];
  Uh[(size_t)r * N + g] = mk(x.x, -x.y);
}

// Eigenvectors of the Hermitian A (destroyed) by cyclic Jacobi; U[g][r] and
// Uh[r][g] receive the eigenvectors of the nb largest eigenvalues in descending
// order, lam (may be NULL) all eigenvalues ascending.
// Block-Jacobi form of jacobi_basis for larger N (own padded buffers).
static gw_status jacobi_basis_block(gw_ctx* c, int N, int nb, const cpx<double>* A,
                                    cpx<double>* U, cpx<double>* Uh, double* lam) {
  const int Np = (N + kBJ2 - 1) / kBJ2 * kBJ2;
  const int nblk = Np / kBJ, npairs = nblk / 2;
  const size_t nnp = (size_t)Np * Np;
  const size_t bytes = 2 * align_up(nnp * 16) + align_up((size_t)npairs * kBJ2 * kBJ2 * 16) +
                       align_up(kNormPartBytes) + align_up((size_t)N * 4) + 1024;
  char* base = nullptr;
  if (hipMalloc(reinterpret_cast<void**>(&base), bytes) != hipSuccess)
    return fail(c, GW_ENOMEM, "block-Jacobi buffers of %zu bytes", bytes);
  struct Free {
    char* p;
    gw_ctx* c;
    ~Free() {
      (void)hipStreamSynchronize(c->stream);
      (void)hipFree(p);
    }
  } guard{base, c};
  size_t off = 0;
  auto take = [&](size_t b) {
    char* p = base + off;
    off += align_up(b);
    return p;
  };
  auto* Ap = reinterpret_cast<cpx<double>*>(take(nnp * 16));
  auto* Vp = reinterpret_cast<cpx<double>*>(take(nnp * 16));
  auto* Qt = reinterpret_cast<cpx<double>*>(take((size_t)npairs * kBJ2 * kBJ2 * 16));
  auto* part = reinterpret_cast<double*>(take(kNormPartBytes));
  auto* rank = reinterpret_cast<int*>(take((size_t)N * 4));
  const unsigned gnp = (unsigned)((nnp + 255) / 256);
  {
    ProfScope ps(c, "lowrank_prep");
    hipLaunchKernelGGL(k_bj_pad, dim3(gnp), dim3(256), 0, c->stream, A, N, Np, Ap);
    hipLaunchKernelGGL(k_lr_fill, dim3(gnp, 1), dim3(256), 0, c->stream, Vp, Np, part, 0);
    GW_CHECK_LAUNCH(c, "block-Jacobi preparation");
  }
  struct SweepGraph {
    hipStream_t cap = nullptr;
    hipGraph_t g = nullptr;
    hipGraphExec_t exec = nullptr;
    ~SweepGraph() {
      if (exec) (void)hipGraphExecDestroy(exec);
      if (g) (void)hipGraphDestroy(g);
      if (cap) (void)hipStreamDestroy(cap);
    }
  } sg;
  GW_HIP(c, hipStreamCreateWithFlags(&sg.cap, hipStreamNonBlocking));
  GW_HIP(c, hipStreamBeginCapture(sg.cap, hipStreamCaptureModeThreadLocal));
  for (int r = 0; r < nblk - 1; ++r) {
    hipLaunchKernelGGL(k_bj_solve, dim3(npairs), dim3(512), 0, sg.cap, Ap, Np, nblk, r, Qt);
    hipLaunchKernelGGL(k_bj_mix, dim3(npairs, 2 * npairs), dim3(256), 0, sg.cap, Ap, Vp, Np, nblk,
                       r, Qt);
  }
  {
    const hipError_t le = hipGetLastError();
    const hipError_t ce = hipStreamEndCapture(sg.cap, &sg.g);
    if (le != hipSuccess) return hip_fail(c, le, "block-Jacobi sweep capture");
    if (ce != hipSuccess) return hip_fail(c, ce, "hipStreamEndCapture");
  }
  GW_HIP(c, hipGraphInstantiate(&sg.exec, sg.g, nullptr, nullptr, 0));
  const int nrb = (int)std::min<size_t>(kNormParts, (nnp + 255) / 256);
  std::vector<double> hp(5 * (size_t)nrb);
  bool done = false;
  JacobiTrack track;
  for (int sweep = 0; sweep < 40 && !done; ++sweep) {
    {
      ProfScope ps(c, "jacobi_sweep");
      GW_HIP(c, hipGraphLaunch(sg.exec, c->stream));
    }
    hipLaunchKernelGGL(k_lr_norms, dim3(nrb), dim3(256), 0, c->stream, Ap, Np, part);
    GW_CHECK_LAUNCH(c, "k_lr_norms");
    GW_HIP(c, hipMemcpyAsync(hp.data(), part, hp.size() * 8, hipMemcpyDeviceToHost, c->stream));
    GW_HIP(c, hipStreamSynchronize(c->stream));
    const int cv = track.update(hp, nrb);
    if (cv < 0) return fail(c, GW_EINVAL, "non-finite entries in epst(0)");
    done = cv > 0;
  }
  if (!done) return fail(c, GW_EINVAL, "block-Jacobi eigen-decomposition did not converge (off-diagonal norm %.3g of the whole after 40 sweeps)", track.prev);
  ProfScope ps(c, "lowrank_basis");
  hipLaunchKernelGGL(k_bj_rank, dim3((N + 255) / 256), dim3(256), 0, c->stream, Ap, Np, N, rank,
                     lam);
  hipLaunchKernelGGL(k_bj_select, dim3(N), dim3(256), 0, c->stream, Vp, Np, rank, N, nb, U, Uh);
  GW_CHECK_LAUNCH(c, "block-Jacobi basis");
  return GW_OK;
}

constexpr int kBlockJacobiMin = 128;  // from this N on, block Jacobi

// A2 and Vt (N x N) are used only below kBlockJacobiMin (null otherwise)
static gw_status jacobi_basis(gw_ctx* c, int N, int nb, cpx<double>* A, cpx<double>* A2,
                              cpx<double>* Vt, double* part, int* rank, cpx<double>* U,
                              cpx<double>* Uh, double* lam) {
  if (N >= kBlockJacobiMin) return jacobi_basis_block(c, N, nb, A, U, Uh, lam);
  static_assert(kBlockJacobiMin <= 1024, "the one-kernel rounds keep two rows in LDS");
  const size_t nn = (size_t)N * N;
  const int m = N + (N & 1);
  {
    ProfScope ps(c, "lowrank_prep");
    double* dummy_ones = part;  // k_lr_fill's ones output is unused here (nb = 0)
    hipLaunchKernelGGL(k_lr_fill, dim3((unsigned)((nn + 255) / 256), 1), dim3(256), 0, c->stream,
                       Vt, N, dummy_ones, 0);
    GW_CHECK_LAUNCH(c, "k_lr_fill");
  }
  // cyclic Jacobi on epst(0): one sweep (2 (m - 1) small launches) is captured
  // once into a graph on a private stream and replayed until converged
  const int nblk = (int)std::min<size_t>(kNormParts, (nn + 255) / 256);
  std::vector<double> hp(5 * (size_t)nblk);
  struct SweepGraph {
    hipStream_t cap = nullptr;
    hipGraph_t g = nullptr;
    hipGraphExec_t exec = nullptr;
    ~SweepGraph() {
      if (exec) (void)hipGraphExecDestroy(exec);
      if (g) (void)hipGraphDestroy(g);
      if (cap) (void)hipStreamDestroy(cap);
    }
  } sg;
  GW_HIP(c, hipStreamCreateWithFlags(&sg.cap, hipStreamNonBlocking));
  GW_HIP(c, hipStreamBeginCapture(sg.cap, hipStreamCaptureModeThreadLocal));
  // one kernel per round: every pair's rotation and the two rows fit in LDS
  // (under 8 KiB below N = 128); rounds alternate A -> A2 -> A ..., and an odd
  // number of rounds ends with a copy back
  const size_t lds_pp = (size_t)(m / 2) * sizeof(JacRot) + (size_t)((N + 3) & ~3) * 4 +
                        (size_t)2 * N * 16;
  for (int r = 0; r < m - 1; ++r) {
    const bool even = (r & 1) == 0;
    hipLaunchKernelGGL(k_jac_round_pp, dim3(m / 2), dim3(256), lds_pp, sg.cap, even ? A : A2,
                       even ? A2 : A, Vt, N, m, r);
  }
  if ((m - 1) & 1)
    hipLaunchKernelGGL(k_lr_copy, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, sg.cap, A2,
                       nn, A);
  {
    const hipError_t le = hipGetLastError();
    const hipError_t ce = hipStreamEndCapture(sg.cap, &sg.g);
    if (le != hipSuccess) return hip_fail(c, le, "jacobi sweep capture");
    if (ce != hipSuccess) return hip_fail(c, ce, "hipStreamEndCapture");
  }
  GW_HIP(c, hipGraphInstantiate(&sg.exec, sg.g, nullptr, nullptr, 0));
  bool done = false;
  JacobiTrack track;
  for (int sweep = 0; sweep < 40 && !done; ++sweep) {
    {
      ProfScope ps(c, "jacobi_sweep");
      GW_HIP(c, hipGraphLaunch(sg.exec, c->stream));
    }
    hipLaunchKernelGGL(k_lr_norms, dim3(nblk), dim3(256), 0, c->stream, A, N, part);
    GW_CHECK_LAUNCH(c, "k_lr_norms");
    GW_HIP(c, hipMemcpyAsync(hp.data(), part, hp.size() * 8, hipMemcpyDeviceToHost, c->stream));
    GW_HIP(c, hipStreamSynchronize(c->stream));
    const int cv = track.update(hp, nblk);
    if (cv < 0) return fail(c, GW_EINVAL, "non-finite entries in epst(0)");
    done = cv > 0;
  }
  if (!done) return fail(c, GW_EINVAL, "Jacobi eigen-decomposition of epst(0) did not converge (off-diagonal norm %.3g of the whole after 40 sweeps)", track.prev);
  {
    ProfScope ps(c, "lowrank_basis");
    hipLaunchKernelGGL(k_lr_rank, dim3((N + 255) / 256), dim3(256), 0, c->stream, A, N, rank, lam);
    hipLaunchKernelGGL(k_lr_select, dim3(N), dim3(256), 0, c->stream, Vt, rank, N, nb, U, Uh);
    GW_CHECK_LAUNCH(c, "low-rank basis");
  }
  return GW_OK;
}

// Given chi_B[f] (nb x nb, the projected V^1/2 chi0 V^1/2) and the basis U (N x nb)
// with Uh = U^H: epsinv[f] (pre-filled with I) += U ((I - chi_B)^-1 - I) U^H, then
// eps^-1 = V^1/2 epst^-1 V^-1/2.  chiB is kept; Bi, Y are scratch.
static gw_status lowrank_apply(gw_ctx* c, int N, int nb, int nfreq, cpx<double>* chiB,
                               cpx<double>* Bi, const double* ones, const cpx<double>* U,
                               const cpx<double>* Uh, cpx<double>* Y, const double* vcoul,
                               double* epsinv) {
  const size_t nn = (size_t)N * N, nub = (size_t)N * nb, bb = (size_t)nb * nb;
  const long long snn = (long long)nn, snb = (long long)nub, sbb = (long long)bb;
  const unsigned gnn = (unsigned)((nn + 255) / 256);
  gw_status st = epsinv_run(c, nb, nfreq, reinterpret_cast<const double*>(chiB), ones,
                            reinterpret_cast<double*>(Bi));
  if (st != GW_OK) return st;
  {
    ProfScope ps(c, "lowrank_small");
    hipLaunchKernelGGL(k_lr_shift, dim3((unsigned)((bb + 255) / 256), nfreq), dim3(256), 0,
                       c->stream, Bi, nb, 1.0, -1.0);
    GW_CHECK_LAUNCH(c, "k_lr_shift");
  }
  // Y_f = U (B_f^-1 - I);  out_f = I + Y_f U^H
  st = zgemm_nn(c, N, nb, nb, 1.0, reinterpret_cast<const double*>(U), 0, nb, 0,
                reinterpret_cast<const double*>(Bi), 0, nb, sbb, reinterpret_cast<double*>(Y), 0,
                nb, snb, nfreq, nub, nfreq * bb, nfreq * nub, 0.0);
  if (st != GW_OK) return st;
  st = zgemm_nn(c, N, N, nb, 1.0, reinterpret_cast<const double*>(Y), 0, nb, snb,
                reinterpret_cast<const double*>(Uh), 0, N, 0, epsinv, 0, N, snn, nfreq,
                nfreq * nub, nub, nfreq * nn, 1.0);
  if (st != GW_OK) return st;
  ProfScope ps(c, "lowrank_unscale");
  hipLaunchKernelGGL(k_lr_unscale, dim3(gnn, nfreq), dim3(256), 0, c->stream,
                     reinterpret_cast<cpx<double>*>(epsinv), vcoul, N);
  GW_CHECK_LAUNCH(c, "k_lr_unscale");
  return GW_OK;
}

static gw_status lowrank_run(gw_ctx* c, int N, int nfreq, const double* chi0,
                             const double* vcoul, int nb, double* epsinv, double* lam,
                             char* base) {
  const size_t nn = (size_t)N * N, nub = (size_t)N * nb, bb = (size_t)nb * nb;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base + off;
    off += align_up(bytes);
    return p;
  };
  const bool small = N < kBlockJacobiMin;
  auto* E = reinterpret_cast<cpx<double>*>(take(nfreq * nn * 16));
  auto* A = reinterpret_cast<cpx<double>*>(take(nn * 16));
  auto* A2 = small ? reinterpret_cast<cpx<double>*>(take(nn * 16)) : nullptr;
  auto* Vt = small ? reinterpret_cast<cpx<double>*>(take(nn * 16)) : nullptr;
  auto* U = reinterpret_cast<cpx<double>*>(take(nub * 16));
  auto* Uh = reinterpret_cast<cpx<double>*>(take(nub * 16));
  auto* Y = reinterpret_cast<cpx<double>*>(take(nfreq * nub * 16));
  auto* B = reinterpret_cast<cpx<double>*>(take(nfreq * bb * 16));
  auto* Bi = reinterpret_cast<cpx<double>*>(take(nfreq * bb * 16));
  auto* part = reinterpret_cast<double*>(take(kNormPartBytes));
  auto* rank = reinterpret_cast<int*>(take((size_t)N * 4));
  auto* ones = reinterpret_cast<double*>(take((size_t)nb * 8));
  const unsigned gnn = (unsigned)((nn + 255) / 256);
  {
    ProfScope ps(c, "lowrank_prep");
    hipLaunchKernelGGL(k_lr_epst, dim3(gnn, nfreq), dim3(256), 0, c->stream,
                       reinterpret_cast<const cpx<double>*>(chi0), vcoul, N, E);
    GW_HIP(c, hipMemcpyAsync(A, E, nn * 16, hipMemcpyDeviceToDevice, c->stream));
    // the identity that the final products accumulate onto, and ones
    hipLaunchKernelGGL(k_lr_fill, dim3(gnn, nfreq), dim3(256), 0, c->stream,
                       reinterpret_cast<cpx<double>*>(epsinv), N, ones, nb);
    GW_CHECK_LAUNCH(c, "low-rank preparation");
  }
  gw_status st = jacobi_basis(c, N, nb, A, A2, Vt, part, rank, U, Uh, lam);
  if (st != GW_OK) return st;
  const long long snn = (long long)nn, snb = (long long)nub, sbb = (long long)bb;
  // Y_f = E_f U;  B_f = U^H Y_f
  st = zgemm_nn(c, N, nb, N, 1.0, reinterpret_cast<const double*>(E), 0, N, snn,
                reinterpret_cast<const double*>(U), 0, nb, 0, reinterpret_cast<double*>(Y), 0, nb,
                snb, nfreq, nfreq * nn, nub, nfreq * nub, 0.0);
  if (st != GW_OK) return st;
  st = zgemm_nn(c, nb, nb, N, 1.0, reinterpret_cast<const double*>(Uh), 0, N, 0,
                reinterpret_cast<const double*>(Y), 0, nb, snb, reinterpret_cast<double*>(B), 0,
                nb, sbb, nfreq, nub, nfreq * nub, nfreq * bb, 0.0);
  if (st != GW_OK) return st;
  // chi_B = I - B_f, then the reduced-basis inverse
  {
    ProfScope ps(c, "lowrank_small");
    hipLaunchKernelGGL(k_lr_shift, dim3((unsigned)((bb + 255) / 256), nfreq), dim3(256), 0,
                       c->stream, B, nb, -1.0, 1.0);
    GW_CHECK_LAUNCH(c, "k_lr_shift");
  }
  return lowrank_apply(c, N, nb, nfreq, B, Bi, ones, U, Uh, Y, vcoul, epsinv);
}

}  // namespace gw

using namespace gw;

extern "C" gw_status gw_epsinv_lowrank(gw_ctx* c, int neps, int nfreq, const double* chi0,
                                       const double* vcoul, int nb, double* epsinv,
                                       double* eigenvalues) {
  if (!c) return GW_EINVAL;
  c->err.clear();
  if (neps < 0 || nfreq < 0) return fail(c, GW_EINVAL, "negative size");
  if (neps == 0 || nfreq == 0) return GW_OK;
  if (nb < 1 || nb > neps) return fail(c, GW_EINVAL, "nb must be 1 to neps");
  if (!chi0 || !vcoul || !epsinv) return fail(c, GW_EINVAL, "NULL array argument");
  if (chi0 == epsinv) return fail(c, GW_EINVAL, "epsinv aliases chi0");
  if (neps > 8192 || nfreq > 65535) return fail(c, GW_EINVAL, "neps above 8192 or nfreq too large");
  (void)hipSetDevice(c->device);
  // v > 0 is required for V^1/2: checked on a host copy
  std::vector<double> hv((size_t)neps);
  GW_HIP(c, hipMemcpyAsync(hv.data(), vcoul, (size_t)neps * 8, hipMemcpyDeviceToHost, c->stream));
  GW_HIP(c, hipStreamSynchronize(c->stream));
  for (double x : hv)
    if (!(x > 0.0) || !std::isfinite(x)) return fail(c, GW_EINVAL, "vcoul must be positive");
  const size_t nn = (size_t)neps * neps, nub = (size_t)neps * nb, bb = (size_t)nb * nb;
  const int nsq = neps < kBlockJacobiMin ? 3 : 1;  // A, and A2 and Vt for plane rotations
  const size_t bytes = align_up(nfreq * nn * 16) + nsq * align_up(nn * 16) +
                       2 * align_up(nub * 16) + align_up(nfreq * nub * 16) +
                       2 * align_up(nfreq * bb * 16) + align_up(kNormPartBytes) +
                       align_up((size_t)neps * 4) + align_up((size_t)nb * 8) + 4096;
  // its own buffers: the small inverse below uses the context workspace
  void* base = nullptr;
  hipError_t e = hipMalloc(&base, bytes);
  if (e != hipSuccess) return fail(c, GW_ENOMEM, "low-rank buffers of %zu bytes", bytes);
  gw_status st = lowrank_run(c, neps, nfreq, chi0, vcoul, nb, epsinv, eigenvalues,
                             static_cast<char*>(base));
  hipError_t e2 = hipStreamSynchronize(c->stream);
  (void)hipFree(base);
  if (st != GW_OK) return st;
  if (e2 != hipSuccess) return hip_fail(c, e2, "hipStreamSynchronize");
  return GW_OK;
}

static gw_status check_v_positive(gw_ctx* c, const double* vcoul, int n) {
  std::vector<double> hv((size_t)n);
  GW_HIP(c, hipMemcpyAsync(hv.data(), vcoul, (size_t)n * 8, hipMemcpyDeviceToHost, c->stream));
  GW_HIP(c, hipStreamSynchronize(c->stream));
  for (double x : hv)
    if (!(x > 0.0) || !std::isfinite(x)) return fail(c, GW_EINVAL, "vcoul must be positive");
  return GW_OK;
}

extern "C" gw_status gw_lowrank_basis(gw_ctx* c, int neps, const double* chi0_static,
                                      const double* vcoul, int nb, double* basis,
                                      double* eigenvalues) {
  if (!c) return GW_EINVAL;
  c->err.clear();
  if (neps < 1 || nb < 1 || nb > neps) return fail(c, GW_EINVAL, "need 1 <= nb <= neps");
  if (neps > 8192) return fail(c, GW_EINVAL, "neps above 8192");
  if (!chi0_static || !vcoul || !basis) return fail(c, GW_EINVAL, "NULL array argument");
  (void)hipSetDevice(c->device);
  gw_status st = check_v_positive(c, vcoul, neps);
  if (st != GW_OK) return st;
  const size_t nn = (size_t)neps * neps, nub = (size_t)neps * nb;
  const bool small = neps < kBlockJacobiMin;
  const size_t bytes = (small ? 3 : 1) * align_up(nn * 16) + align_up(nub * 16) +
                       align_up(kNormPartBytes) + align_up((size_t)neps * 4) + 4096;
  char* base = nullptr;
  if (hipMalloc(reinterpret_cast<void**>(&base), bytes) != hipSuccess)
    return fail(c, GW_ENOMEM, "basis buffers of %zu bytes", bytes);
  size_t off = 0;
  auto take = [&](size_t b) {
    char* p = base + off;
    off += align_up(b);
    return p;
  };
  auto* A = reinterpret_cast<cpx<double>*>(take(nn * 16));
  auto* A2 = small ? reinterpret_cast<cpx<double>*>(take(nn * 16)) : nullptr;
  auto* Vt = small ? reinterpret_cast<cpx<double>*>(take(nn * 16)) : nullptr;
  auto* Uh = reinterpret_cast<cpx<double>*>(take(nub * 16));
  auto* part = reinterpret_cast<double*>(take(kNormPartBytes));
  auto* rank = reinterpret_cast<int*>(take((size_t)neps * 4));
  {
    ProfScope ps(c, "lowrank_prep");
    hipLaunchKernelGGL(k_lr_epst, dim3((unsigned)((nn + 255) / 256), 1), dim3(256), 0, c->stream,
                       reinterpret_cast<const cpx<double>*>(chi0_static), vcoul, neps, A);
    st = hipGetLastError() == hipSuccess ? GW_OK : GW_EDEVICE;
  }
  if (st == GW_OK)
    st = jacobi_basis(c, neps, nb, A, A2, Vt, part, rank,
                      reinterpret_cast<cpx<double>*>(basis), Uh, eigenvalues);
  const hipError_t e2 = hipStreamSynchronize(c->stream);
  (void)hipFree(base);
  if (st != GW_OK) return st == GW_EDEVICE ? fail(c, st, "k_lr_epst launch") : st;
  if (e2 != hipSuccess) return hip_fail(c, e2, "hipStreamSynchronize");
  return GW_OK;
}

extern "C" gw_status gw_mtxel_project(gw_ctx* c, int npairs, int neps, const void* mtxel,
                                      gw_dtype dtype, const double* vcoul, int nb,
                                      const double* basis, double* out) {
  if (!c) return GW_EINVAL;
  c->err.clear();
  if (npairs < 0 || neps < 1 || nb < 1 || nb > neps) return fail(c, GW_EINVAL, "bad sizes");
  if (dtype != GW_C128 && dtype != GW_C64) return fail(c, GW_EINVAL, "unknown dtype");
  if (npairs == 0) return GW_OK;
  if (!mtxel || !vcoul || !basis || !out) return fail(c, GW_EINVAL, "NULL array argument");
  if (out == mtxel || out == basis) return fail(c, GW_EINVAL, "out aliases an input");
  (void)hipSetDevice(c->device);
  const size_t nx = (size_t)npairs * neps;
  gw_status st = ws_begin(c, align_up(nx * 16));
  if (st != GW_OK) return st;
  auto* X = static_cast<cpx<double>*>(ws_take(c, nx * 16));
  {
    ProfScope ps(c, "mtxel_project_prep");
    if (dtype == GW_C128)
      hipLaunchKernelGGL(k_proj_prep<double>, dim3((unsigned)((nx + 255) / 256)), dim3(256), 0,
                         c->stream, static_cast<const cpx<double>*>(mtxel), (size_t)npairs, neps,
                         vcoul, X);
    else
      hipLaunchKernelGGL(k_proj_prep<float>, dim3((unsigned)((nx + 255) / 256)), dim3(256), 0,
                         c->stream, static_cast<const cpx<float>*>(mtxel), (size_t)npairs, neps,
                         vcoul, X);
    GW_CHECK_LAUNCH(c, "k_proj_prep");
  }
  // out = X U  (npairs x nb)
  return zgemm_nn(c, npairs, nb, neps, 1.0, reinterpret_cast<const double*>(X), 0, neps, 0, basis,
                  0, nb, 0, out, 0, nb, 0, 1, nx, (size_t)neps * nb, (size_t)npairs * nb, 0.0);
}

extern "C" gw_status gw_epsinv_from_basis(gw_ctx* c, int neps, int nb, int nfreq,
                                          const double* chi_b, const double* vcoul,
                                          const double* basis, double* epsinv) {
  if (!c) return GW_EINVAL;
  c->err.clear();
  if (neps < 1 || nb < 1 || nb > neps || nfreq < 0) return fail(c, GW_EINVAL, "bad sizes");
  if (nfreq == 0) return GW_OK;
  if (!chi_b || !vcoul || !basis || !epsinv) return fail(c, GW_EINVAL, "NULL array argument");
  if (epsinv == chi_b || epsinv == basis) return fail(c, GW_EINVAL, "epsinv aliases an input");
  if (neps > 46340 || nfreq > 65535) return fail(c, GW_EINVAL, "neps or nfreq too large");
  (void)hipSetDevice(c->device);
  gw_status st = check_v_positive(c, vcoul, neps);
  if (st != GW_OK) return st;
  const size_t nn = (size_t)neps * neps, nub = (size_t)neps * nb, bb = (size_t)nb * nb;
  // own buffers: the small inverse uses the context workspace
  const size_t bytes = align_up(nub * 16) + align_up(nfreq * bb * 16) * 2 +
                       align_up(nfreq * nub * 16) + align_up((size_t)nb * 8) + 4096;
  char* base = nullptr;
  if (hipMalloc(reinterpret_cast<void**>(&base), bytes) != hipSuccess)
    return fail(c, GW_ENOMEM, "buffers of %zu bytes", bytes);
  size_t off = 0;
  auto take = [&](size_t b) {
    char* p = base + off;
    off += align_up(b);
    return p;
  };
  auto* Uh = reinterpret_cast<cpx<double>*>(take(nub * 16));
  auto* chiB = reinterpret_cast<cpx<double>*>(take(nfreq * bb * 16));
  auto* Bi = reinterpret_cast<cpx<double>*>(take(nfreq * bb * 16));
  auto* Y = reinterpret_cast<cpx<double>*>(take(nfreq * nub * 16));
  auto* ones = reinterpret_cast<double*>(take((size_t)nb * 8));
  st = GW_OK;
  {
    ProfScope ps(c, "lowrank_prep");
    hipLaunchKernelGGL(k_lr_conjt, dim3((unsigned)((nub + 255) / 256)), dim3(256), 0, c->stream,
                       reinterpret_cast<const cpx<double>*>(basis), neps, nb, Uh);
    hipLaunchKernelGGL(k_lr_fill, dim3((unsigned)((nn + 255) / 256), nfreq), dim3(256), 0,
                       c->stream, reinterpret_cast<cpx<double>*>(epsinv), neps, ones, nb);
    if (hipMemcpyAsync(chiB, chi_b, nfreq * bb * 16, hipMemcpyDeviceToDevice, c->stream) !=
            hipSuccess ||
        hipGetLastError() != hipSuccess)
      st = fail(c, GW_EDEVICE, "low-rank preparation");
  }
  if (st == GW_OK)
    st = lowrank_apply(c, neps, nb, nfreq, chiB, Bi, ones,
                       reinterpret_cast<const cpx<double>*>(basis), Uh, Y, vcoul, epsinv);
  const hipError_t e2 = hipStreamSynchronize(c->stream);
  (void)hipFree(base);
  if (st != GW_OK) return st;
  if (e2 != hipSuccess) return hip_fail(c, e2, "hipStreamSynchronize");
  return GW_OK;
}
