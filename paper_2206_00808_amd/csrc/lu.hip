// eps = I - diag(v) chi0 and its inverse in double (Sec. II, dielectric matrix;
// the Performance section names this inversion as a large part of Epsilon).
//
// Default path: on the static and imaginary-frequency axis chi0 is Hermitian
// negative semidefinite, so with S = diag(sqrt(v)) (v > 0)
//   eps = S (I - S chi0 S) S^-1 = S epst S^-1,  epst Hermitian positive definite
// (every eigenvalue >= 1).  epst is inverted in place by blocked Gauss-Jordan
// elimination without pivoting (stable for a positive-definite matrix), whose
// work is one rank-nb GEMM update of the whole matrix per block, and then
// eps^-1 = S epst^-1 S^-1.  Each diagonal pivot is checked to be real and
// positive (>= 1/2, since epst >= I); if any is not (or some v <= 0), the result
// is discarded and the general path below runs instead.
//
// General path: right-looking blocked LU with partial pivoting (PA = LU), every
// frequency in the same launches (grid.z / grid.y = frequency):
//   panel  : one 1024-thread workgroup factors the N x nb column panel
//            (pivot = largest |re|+|im|, lowest row on ties)
//   laswp  : the panel's row interchanges applied to the other columns
//   trsm   : U12 = L11^-1 A12
//   update : A22 -= L21 U12 on the FP64 matrix cores
// then eps^-1 = U^-1 L^-1 P by blocked forward/back substitution on P*I.
#include "common.h"
#include "tiles.h"

namespace gw {

constexpr int NB = 32;  // block width of the factorisation and the substitutions

__global__ void k_eps_build(const cpx<double>* __restrict__ chi, const double* __restrict__ v,
                            cpx<double>* __restrict__ A, int N) {
  const size_t nn = (size_t)N * N;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nn) return;
  const size_t off = (size_t)blockIdx.y * nn + idx;
  const int i = (int)(idx / N), j = (int)(idx % N);
  const cpx<double> x = chi[off];
  A[off] = mk((i == j ? 1.0 : 0.0) - v[i] * x.x, -v[i] * x.y);
}

__global__ void __launch_bounds__(1024) k_lu_panel(cpx<double>* __restrict__ A, int N, int k,
                                                   int nbk, int* __restrict__ ipiv,
                                                   int* __restrict__ flag) {
  __shared__ double sv[1024];
  __shared__ int si[1024];
  __shared__ cpx<double> prow[NB];
  const int tid = threadIdx.x, nt = blockDim.x;
  A += (size_t)blockIdx.x * N * N;
  ipiv += (size_t)blockIdx.x * N;
  for (int jj = 0; jj < nbk; ++jj) {
    const int j = k + jj;
    double best = -1.0;
    int bi = N;
    for (int i = j + tid; i < N; i += nt) {
      const cpx<double> a = A[(size_t)i * N + j];
      const double m = fabs(a.x) + fabs(a.y);
      if (m > best) { best = m; bi = i; }
    }
    sv[tid] = best;
    si[tid] = bi;
    __syncthreads();
    for (int s = nt / 2; s > 0; s >>= 1) {
      if (tid < s) {
        const double o = sv[tid + s];
        const int oi = si[tid + s];
        if (o > sv[tid] || (o == sv[tid] && oi < si[tid])) { sv[tid] = o; si[tid] = oi; }
      }
      __syncthreads();
    }
    const double pm = sv[0];
    const int p = (si[0] < N) ? si[0] : j;  // no finite candidate: keep the diagonal
    if (tid == 0) {
      ipiv[j] = p;
      if (!(pm > 0.0)) flag[0] = 1;
    }
    if (p != j) {
      for (int c = tid; c < nbk; c += nt) {
        const cpx<double> t = A[(size_t)j * N + k + c];
        A[(size_t)j * N + k + c] = A[(size_t)p * N + k + c];
        A[(size_t)p * N + k + c] = t;
      }
    }
    __syncthreads();
    for (int c = tid; c < nbk; c += nt) prow[c] = A[(size_t)j * N + k + c];
    __syncthreads();
    if (pm > 0.0) {
      const cpx<double> piv = prow[jj];
      const double den = piv.x * piv.x + piv.y * piv.y;
      const cpx<double> inv = mk(piv.x / den, -piv.y / den);
      for (int i = j + 1 + tid; i < N; i += nt) {
        cpx<double>* row = A + (size_t)i * N + k;
        const cpx<double> l = cmul(row[jj], inv);
        row[jj] = l;
        for (int c = jj + 1; c < nbk; ++c) row[c] = row[c] - cmul(l, prow[c]);
      }
    }
    __syncthreads();
  }
}

__global__ void k_lu_laswp(cpx<double>* __restrict__ A, int N, int k, int nbk,
                           const int* __restrict__ ipiv) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N || (c >= k && c < k + nbk)) return;
  A += (size_t)blockIdx.y * N * N;
  ipiv += (size_t)blockIdx.y * N;
  for (int s = k; s < k + nbk; ++s) {
    const int p = ipiv[s];
    if (p != s) {
      const cpx<double> t = A[(size_t)s * N + c];
      A[(size_t)s * N + c] = A[(size_t)p * N + c];
      A[(size_t)p * N + c] = t;
    }
  }
}

// Solve T X = B in place on rows kb..kb+nbk of X for columns c0..c0+ncols, where
// T is the nbk x nbk diagonal block of the LU factors: unit lower (UPPER=false)
// or non-unit upper (UPPER=true).  One thread per right-hand-side column.
template <bool UPPER>
__global__ void __launch_bounds__(256) k_trsm_block(const cpx<double>* __restrict__ LU, int N,
                                                   int kb, int nbk, cpx<double>* __restrict__ X,
                                                   int c0, int ncols) {
  __shared__ cpx<double> T[NB][NB + 1];
  __shared__ cpx<double> dinv[NB];
  LU += (size_t)blockIdx.y * N * N;
  X += (size_t)blockIdx.y * N * N;
  for (int e = threadIdx.x; e < nbk * nbk; e += blockDim.x) {
    const int r = e / nbk, cc = e % nbk;
    T[r][cc] = LU[(size_t)(kb + r) * N + kb + cc];
  }
  __syncthreads();
  if (UPPER && threadIdx.x < nbk) {
    const cpx<double> d = T[threadIdx.x][threadIdx.x];
    const double den = d.x * d.x + d.y * d.y;
    dinv[threadIdx.x] = mk(d.x / den, -d.y / den);
  }
  __syncthreads();
  const int cidx = blockIdx.x * blockDim.x + threadIdx.x;
  if (cidx >= ncols) return;
  const int col = c0 + cidx;
  cpx<double> x[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i)
    x[i] = (i < nbk) ? X[(size_t)(kb + i) * N + col] : mk<double>(0, 0);
  if (!UPPER) {
#pragma unroll
    for (int i = 1; i < NB; ++i) {
      if (i < nbk) {
        cpx<double> s = x[i];
#pragma unroll
        for (int t = 0; t < i; ++t) s = s - cmul(T[i][t], x[t]);
        x[i] = s;
      }
    }
  } else {
#pragma unroll
    for (int i = NB - 1; i >= 0; --i) {
      if (i < nbk) {
        cpx<double> s = x[i];
#pragma unroll
        for (int t = i + 1; t < NB; ++t)
          if (t < nbk) s = s - cmul(T[i][t], x[t]);
        x[i] = cmul(s, dinv[i]);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < NB; ++i)
    if (i < nbk) X[(size_t)(kb + i) * N + col] = x[i];
}

// Row s of P*I is e_perm[s], perm = identity after the interchanges s <-> ipiv[s].
__global__ void __launch_bounds__(256) k_perm_build(const int* __restrict__ ipiv, int N,
                                                    int* __restrict__ perm) {
  extern __shared__ int sp[];
  const int f = blockIdx.x;
  ipiv += (size_t)f * N;
  perm += (size_t)f * N;
  for (int i = threadIdx.x; i < N; i += blockDim.x) sp[i] = i;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int s = 0; s < N; ++s) {
      const int p = ipiv[s];
      const int t = sp[s];
      sp[s] = sp[p];
      sp[p] = t;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < N; i += blockDim.x) perm[i] = sp[i];
}

__global__ void k_perm_identity(const int* __restrict__ perm, int N, cpx<double>* __restrict__ Y) {
  const size_t nn = (size_t)N * N;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nn) return;
  const int s = (int)(e / N), j = (int)(e % N);
  Y[(size_t)blockIdx.y * nn + e] = mk(j == perm[(size_t)blockIdx.y * N + s] ? 1.0 : 0.0, 0.0);
}


// ---------------------------------------------------------------- Gauss-Jordan path
constexpr int GB = 64;  // Gauss-Jordan block width

__global__ void k_fill_int(int* p, int n, int v) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = v;
}


// epst = I - S chi0 S with S = diag(sqrt(v)), one 32x32 tile per workgroup
// (grid: tiles x tiles x nfreq). flag[1] = 1 if some v <= 0 or non-finite;
// flag[4] = 1 if some chi0 entry is not finite;
// flag[3] = 1 if chi0 is not Hermitian: |chi_ij - conj(chi_ji)| above
// kHermRel (|chi_ij| + |chi_ji|) for some pair, checked against the mirror
// tile staged through LDS. The Gauss-Jordan pivot test alone cannot tell a
// Hermitian positive-definite epst from a non-Hermitian one whose pivots
// happen to look the same.
constexpr double kHermRel = 1e-12;
constexpr int ET = 32;
__global__ void __launch_bounds__(256) k_epst_build(const cpx<double>* __restrict__ chi,
                                                    const double* __restrict__ v,
                                                    cpx<double>* __restrict__ A, int N,
                                                    int* __restrict__ flag) {
  __shared__ cpx<double> mir[ET][ET + 1];
  const size_t nn = (size_t)N * N;
  const int ti = blockIdx.y, tj = blockIdx.x;
  chi += (size_t)blockIdx.z * nn;
  A += (size_t)blockIdx.z * nn;
  const int c = threadIdx.x % ET, r0 = threadIdx.x / ET;  // 8 rows per pass
  // mirror tile (tj, ti), read row-wise and stored transposed
  for (int r = r0; r < ET; r += 256 / ET) {
    const int i = tj * ET + r, j = ti * ET + c;
    if (i < N && j < N) mir[c][r] = chi[(size_t)i * N + j];
  }
  __syncthreads();
  bool bad = false, nonfinite = false;
  for (int r = r0; r < ET; r += 256 / ET) {
    const int i = ti * ET + r, j = tj * ET + c;
    if (i >= N || j >= N) continue;
    const double vi = v[i], vj = v[j];
    if (j == 0 && (!(vi > 0.0) || !(vi < INFINITY))) flag[1] = 1;
    const cpx<double> x = chi[(size_t)i * N + j];
    const cpx<double> y = mir[r][c];  // chi[j][i]
    const double dr = x.x - y.x, di = x.y + y.y;
    const double lim = kHermRel * (fabs(x.x) + fabs(x.y) + fabs(y.x) + fabs(y.y));
    nonfinite = nonfinite || !(fabs(x.x) < INFINITY && fabs(x.y) < INFINITY);
    bad = bad || !(fabs(dr) <= lim && fabs(di) <= lim);
    const double s = sqrt(vi) * sqrt(vj);
    A[(size_t)i * N + j] = mk((i == j ? 1.0 : 0.0) - s * x.x, -s * x.y);
  }
  if (bad) flag[3] = 1;
  if (nonfinite) flag[4] = 1;
}

// Inverse of the diagonal block D = A[K][K] (nbk <= GB = 64) by Gauss-Jordan
// without pivoting, register resident (gj_invert_64); the block of frequency f
// is src[f * sstride + i * ld + j] and its inverse goes to Dw[f]. A pivot that
// is not real and >= 1/2 sets flag[2].
__global__ void __launch_bounds__(1024) k_gj_diag(const cpx<double>* __restrict__ src, int ld,
                                                  size_t sstride, int nbk,
                                                  cpx<double>* __restrict__ Dw,
                                                  int* __restrict__ flag) {
  static_assert(GB == 64, "gj_invert_64 holds a 64x64 block");
  __shared__ cpx<double> rowb[2][GB], colb[2][GB];
  const int f = blockIdx.x;
  src += (size_t)f * sstride;
  Dw += (size_t)f * GB * GB;
  const int tid = threadIdx.x, ti = tid / 32, tj = tid % 32;
  cpx<double> d[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int i = ti + 32 * a, j = tj + 32 * b;
      d[a][b] = (i < nbk && j < nbk) ? src[(size_t)i * ld + j] : mk(i == j ? 1.0 : 0.0, 0.0);
    }
  if (gj_invert_64<32>(d, nbk, rowb, colb)) flag[2] = 1;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int i = ti + 32 * a, j = tj + 32 * b;
      if (i < nbk && j < nbk) Dw[i * GB + j] = d[a][b];
    }
}

// The one launch between the row panel and the rank update of step K (block
// k, width nbk):
//   - row block of the previous step (kp, nbp; none when nbp is 0) <- Rp outside
//     its columns and Dp inside, its Gauss-Jordan value;
//   - Cb[i][t] = A[i][k+t], the rows of the previous block taking those values;
//   - R[t][k+j] = delta_tj + D[t][j]; with R in the K columns set this way,
//     A[:,K] - Cb R leaves -Cb D in the column block, its Gauss-Jordan value.
// No entry is both read and written: the previous block's rows are taken from
// Rp and Dp.
__global__ void k_gj_step(cpx<double>* __restrict__ A, int N, int k, int nbk,
                          cpx<double>* __restrict__ Cb, cpx<double>* __restrict__ R,
                          const cpx<double>* __restrict__ D, int kp, int nbp,
                          const cpx<double>* __restrict__ Rp, const cpx<double>* __restrict__ Dp) {
  const size_t f = blockIdx.y;
  A += f * (size_t)N * N;
  Cb += f * (size_t)N * GB;
  R += f * (size_t)GB * N;
  Rp += f * (size_t)GB * N;
  D += f * (size_t)GB * GB;
  Dp += f * (size_t)GB * GB;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  auto fixed = [&](int t, int j) {
    return (j >= kp && j < kp + nbp) ? Dp[t * GB + (j - kp)] : Rp[(size_t)t * N + j];
  };
  if (e < nbp * N) {
    const int t = e / N, j = e % N;
    A[(size_t)(kp + t) * N + j] = fixed(t, j);
  }
  if (e < N * nbk) {
    const int i = e / nbk, t = e % nbk;
    Cb[(size_t)i * GB + t] = (i >= kp && i < kp + nbp) ? fixed(i - kp, k + t)
                                                       : A[(size_t)i * N + k + t];
  }
  if (e < nbk * nbk) {
    const int t = e / nbk, j = e % nbk;
    const cpx<double> dv = D[t * GB + j];
    R[(size_t)t * N + k + j] = mk(dv.x + (t == j ? 1.0 : 0.0), dv.y);
  }
}

// Row block K <- R outside the K columns and Dinv inside.
__global__ void k_gj_fix(cpx<double>* __restrict__ A, int N, int k, int nbk,
                         const cpx<double>* __restrict__ R, const cpx<double>* __restrict__ Dw) {
  const size_t f = blockIdx.y;
  A += f * (size_t)N * N;
  R += f * (size_t)GB * N;
  Dw += f * (size_t)GB * GB;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nbk * N) return;
  const int t = e / N, j = e % N;
  A[(size_t)(k + t) * N + j] = (j >= k && j < k + nbk) ? Dw[t * GB + (j - k)] : R[(size_t)t * N + j];
}

// The rank-nbk update A -= Cb R of every row and column (one matrix per
// frequency), the bulk of each Gauss-Jordan step, with the next step's
// diagonal inverse in the same launch.
//   - Update tiles: with K at most GB the product per output is short and the C
//     tile streams through once, so there is no LDS staging and no barrier.
//     Each wavefront computes a 32x32 block (2x2 v_mfma_f64_16x16x4_f64, three
//     real products per complex one) with its fragments loaded straight from
//     Cb (N x GB) and R (GB x N), which stay in L2; the next four K are loaded
//     while the current ones feed the matrix cores. C is read in the epilogue;
//     three workgroups per CU cover that latency with the other wavefronts'
//     products. From N = 2048 the operands pass through LDS instead
//     (gj_update_tile_lds), which loads each fragment once per workgroup.
//     Tiles of 64x64 are numbered frequency, row band, column band and
//     renumbered per XCD, so one XCD's L2 holds the panels of its tiles.
//   - Look-ahead (nb2 > 0): the first nfreq workgroups each form the next
//     diagonal block Dn = A[K'][K'] - Cb[K'] R[:, K'] with the same tile code,
//     invert it in registers (gj_invert_64, 16x16 threads holding 4x4 entries)
//     and write the inverse to Dw. The update skips tile (K', K'): that block
//     is only ever read into values that a later step overwrites (the next
//     panel's K' columns and row block K', which the step after rewrites from
//     R and Dinv), so no workgroup writes what another reads.
constexpr int UT = 64;  // workgroup tile (2x2 wavefronts of 32x32)

// A -= product on a wavefront's 32x32 block at (ia, ja): Re = t1 - t2, Im = t3 -
// t1 - t2 (f64 16x16x4 D layout: row lk + 4r, column l16). The 8 entries of
// each row block are loaded (at clamped, always valid addresses) before any is
// stored, so the loads are in flight together: with a load, a wait and a store
// per entry, each of the 16 entries cost a full memory round trip.
__device__ __forceinline__ void gj_epilogue(const d4 (&t1)[2][2], const d4 (&t2)[2][2],
                                            const d4 (&t3)[2][2], cpx<double>* A, int N, int ia,
                                            int ja) {
  const int lane = threadIdx.x & 63, l16 = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    cpx<double> v[2][4];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = min(ia + a * 16 + lk + 4 * r, N - 1), j = min(ja + b * 16 + l16, N - 1);
        v[b][r] = A[(size_t)i * N + j];
      }
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = ia + a * 16 + lk + 4 * r, j = ja + b * 16 + l16;
        if (i < N && j < N)
          A[(size_t)i * N + j] = mk(v[b][r].x - (t1[a][b][r] - t2[a][b][r]),
                                    v[b][r].y - ((t3[a][b][r] - t1[a][b][r]) - t2[a][b][r]));
      }
  }
}

// A -= Cb R on the 64x64 tile at (i0, j0) (rows and columns below N) with the
// operands staged in LDS: Cb[i0 .. i0 + 63][K] and R[K][j0 .. j0 + 63] pass in
// chunks of 8 K through two 16 KiB buffers, loaded by global_load_lds, so each
// fragment comes from L2 once per workgroup, where the 2x2 wavefronts loading
// their fragments directly fetch each twice.
//   - Cb chunk [64 rows][8 k of 16 B]: k stored at slot k ^ (row & 7). A
//     fragment read (16 rows, one k per group of 16 lanes) then takes as many
//     LDS cycles as a contiguous 1 KiB read, by the bank-conflict counter;
//     (row & 7) ^ ((row >> 3) & 1) took twice as many. R chunk [8 k][64
//     columns]: a fragment read is 256 contiguous bytes per k.
//   - K past kdim is read clamped and zeroed at the fragment (stale panel
//     entries may hold anything); rows and columns past N are clamped and
//     feed outputs that are not stored.
//   - Products as in gj_update_tile: 2x2 v_mfma_f64_16x16x4_f64 blocks per
//     wavefront, three real products per complex one, A read in the epilogue.
__device__ __forceinline__ void gj_update_tile_lds(const cpx<double>* __restrict__ Cb,
                                                   const cpx<double>* __restrict__ R,
                                                   cpx<double>* A, int N, int kdim, int i0,
                                                   int j0) {
  __shared__ __align__(16) cpx<double> Cs0[UT * 8], Rs0[8 * UT], Cs1[UT * 8], Rs1[8 * UT];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, lk = lane >> 4;
  const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
  d4 t1[2][2], t2[2][2], t3[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      t1[a][b] = (d4){0, 0, 0, 0};
      t2[a][b] = (d4){0, 0, 0, 0};
      t3[a][b] = (d4){0, 0, 0, 0};
    }
  // chunk at K offset kc: 16 row blocks of 1 KiB (8 of Cb, 8 rows each; 8 of
  // R, one k each), 4 per wavefront
  auto issue = [&](cpx<double>* Cs, cpx<double>* Rs, int kc) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int idx = wave * 4 + u;
      const int row = (idx & 7) * 8 + (lane >> 3);
      const int kb = (lane & 7) ^ (lane >> 3);  // row & 7 = lane >> 3
      const cpx<double>* sa = Cb + (size_t)min(i0 + row, N - 1) * GB + min(kc + kb, kdim - 1);
      const cpx<double>* sr = R + (size_t)min(kc + (idx & 7), kdim - 1) * N + min(j0 + lane, N - 1);
      if (idx < 8)
        __builtin_amdgcn_global_load_lds((const void*)sa, (lds_void*)(Cs + idx * 64), 16, 0, 0);
      else
        __builtin_amdgcn_global_load_lds((const void*)sr, (lds_void*)(Rs + (idx - 8) * 64), 16,
                                         0, 0);
    }
  };
  auto compute = [&](const cpx<double>* Cs, const cpx<double>* Rs, int kc) {
#pragma unroll
    for (int kk = 0; kk < 8; kk += 4) {
      const int k = kk + lk;
      const bool ok = kc + k < kdim;
      cpx<double> fa[2], fb[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int row = wi + a * 16 + l16;
        const cpx<double> v = Cs[row * 8 + (k ^ (l16 & 7))];
        fa[a] = ok ? v : mk(0.0, 0.0);
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const cpx<double> v = Rs[k * UT + wj + b * 16 + l16];
        fb[b] = ok ? v : mk(0.0, 0.0);
      }
      double sa[2], sb[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) sa[a] = fa[a].x + fa[a].y;
#pragma unroll
      for (int b = 0; b < 2; ++b) sb[b] = fb[b].x + fb[b].y;
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          t1[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a].x, fb[b].x, t1[a][b], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          t2[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a].y, fb[b].y, t2[a][b], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          t3[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(sa[a], sb[b], t3[a][b], 0, 0, 0);
    }
  };
  const int nch = (kdim + 7) / 8;
  issue(Cs0, Rs0, 0);
  __syncthreads();  // (its fence waits for the loads)
  for (int c = 0; c < nch; c += 2) {
    if (c + 1 < nch) issue(Cs1, Rs1, (c + 1) * 8);
    compute(Cs0, Rs0, c * 8);
    __syncthreads();
    if (c + 1 < nch) {
      if (c + 2 < nch) issue(Cs0, Rs0, (c + 2) * 8);
      compute(Cs1, Rs1, (c + 1) * 8);
      __syncthreads();
    }
  }
  gj_epilogue(t1, t2, t3, A, N, i0 + wi, j0 + wj);
}

template <bool kLds>
__global__ void __launch_bounds__(256, 3) k_gj_update(cpx<double>* __restrict__ A, int N,
                                                      int kdim, const cpx<double>* __restrict__ Cb,
                                                      const cpx<double>* __restrict__ R,
                                                      int nfreq, int k2, int nb2,
                                                      cpx<double>* __restrict__ Dn,
                                                      cpx<double>* __restrict__ Dw,
                                                      int* __restrict__ flag) {
  const int nt = (N + UT - 1) / UT;
  const int wave = threadIdx.x >> 6;
  const int ndiag = nb2 > 0 ? nfreq : 0;
  if ((int)blockIdx.x < ndiag) {
    static_assert(GB == 64 && UT == GB, "the look-ahead block is one 64x64 tile");
    __shared__ cpx<double> rowb[2][GB], colb[2][GB];
    const int f = blockIdx.x;
    A += (size_t)f * N * N;
    Dn += (size_t)f * GB * GB;
    Dw += (size_t)f * GB * GB;
    gj_update_tile(Cb + (size_t)f * N * GB, GB, R + (size_t)f * GB * N, A, N, kdim,
                   k2 + (wave >> 1) * 32, k2 + (wave & 1) * 32, k2 + nb2, Dn, GB, k2);
    __syncthreads();  // Dn complete and visible to the workgroup
    constexpr int TG = 16, TE = GB / TG;
    const int ti = threadIdx.x / TG, tj = threadIdx.x % TG;
    cpx<double> d[TE][TE];
#pragma unroll
    for (int a = 0; a < TE; ++a)
#pragma unroll
      for (int b = 0; b < TE; ++b) {
        const int i = ti + TG * a, j = tj + TG * b;
        d[a][b] = (i < nb2 && j < nb2) ? Dn[i * GB + j] : mk(i == j ? 1.0 : 0.0, 0.0);
      }
    if (gj_invert_64<TG>(d, nb2, rowb, colb)) flag[2] = 1;
#pragma unroll
    for (int a = 0; a < TE; ++a)
#pragma unroll
      for (int b = 0; b < TE; ++b) {
        const int i = ti + TG * a, j = tj + TG * b;
        if (i < nb2 && j < nb2) Dw[i * GB + j] = d[a][b];
      }
    return;
  }
  const long long lin = xcd_linear(blockIdx.x - ndiag, (long long)nt * nt * nfreq);
  if (lin < 0) return;
  const int f = (int)(lin / ((long long)nt * nt));
  const int rem = (int)(lin % ((long long)nt * nt));
  const int ti = rem / nt, tj = rem % nt;
  if (nb2 > 0 && ti == k2 / UT && tj == k2 / UT) return;
  A += (size_t)f * N * N;
  if constexpr (kLds)
    gj_update_tile_lds(Cb + (size_t)f * N * GB, R + (size_t)f * GB * N, A, N, kdim, ti * UT,
                       tj * UT);
  else
    gj_update_tile(Cb + (size_t)f * N * GB, GB, R + (size_t)f * GB * N, A, N, kdim,
                   ti * UT + (wave >> 1) * 32, tj * UT + (wave & 1) * 32, N, A, N, 0);
}

// ---------------------------------------------------------------- consumers of eps^-1
// W[f][G][G'] = eps^-1[f][G][G'] v(q+G')
__global__ void k_screened_w(const cpx<double>* __restrict__ einv, const double* __restrict__ v,
                             int N, cpx<double>* __restrict__ w) {
  const size_t nn = (size_t)N * N;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nn) return;
  const size_t off = (size_t)blockIdx.y * nn + e;
  w[off] = scal(einv[off], v[e % N]);
}

// X[p][G] = conj(M[p][G]) in double (the left factor of the SX quadratic form)
template <typename Tin>
__global__ void k_conj_widen(const cpx<Tin>* __restrict__ m, size_t n, cpx<double>* __restrict__ x) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const cpx<Tin> a = m[e];
  x[e] = mk((double)a.x, -(double)a.y);
}

// sigma[n] += -pref sum_{n''} sum_G' U[(n'',n)][G'] v(G') M[(n'',n)][G'], U = conj(M) eps^-1;
// one workgroup per band n, the occupied bands and G' summed in a fixed order
template <typename Tin>
__global__ void __launch_bounds__(256) k_sx_reduce(const cpx<double>* __restrict__ U,
                                                   const cpx<Tin>* __restrict__ m,
                                                   const double* __restrict__ v, int nocc,
                                                   int nband, int N, double pref,
                                                   cpx<double>* __restrict__ sigma) {
  __shared__ double sr[256], si[256];
  const int n = blockIdx.x;
  double ar = 0.0, ai = 0.0;
  for (int o = 0; o < nocc; ++o) {
    const size_t row = ((size_t)o * nband + n) * N;
    for (int g = threadIdx.x; g < N; g += blockDim.x) {
      const cpx<double> u = U[row + g];
      const cpx<Tin> b = m[row + g];
      const double br = v[g] * (double)b.x, bi = v[g] * (double)b.y;
      ar += u.x * br - u.y * bi;
      ai += u.x * bi + u.y * br;
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
  if (threadIdx.x == 0) sigma[n] = mk(sigma[n].x - pref * sr[0], sigma[n].y - pref * si[0]);
}

gw_status screened_w(gw_ctx* c, int N, int nfreq, const double* epsinv, const double* vcoul,
                     double* w) {
  const size_t nn = (size_t)N * N;
  ProfScope ps(c, "screened_w");
  hipLaunchKernelGGL(k_screened_w, dim3((unsigned)((nn + 255) / 256), nfreq), dim3(256), 0,
                     c->stream, reinterpret_cast<const cpx<double>*>(epsinv), vcoul, N,
                     reinterpret_cast<cpx<double>*>(w));
  GW_CHECK_LAUNCH(c, "k_screened_w");
  return GW_OK;
}

gw_status sigma_sx_static(gw_ctx* c, int nocc, int nband, int N, const void* mtxel, gw_dtype dt,
                          const double* epsinv, const double* vcoul, double prefactor,
                          double* sigma) {
  const int P = nocc * nband;
  const size_t np = (size_t)P * N;
  gw_status st = ws_begin(c, 2 * align_up(np * 16));
  if (st != GW_OK) return st;
  cpx<double>* X = static_cast<cpx<double>*>(ws_take(c, np * 16));
  double* U = static_cast<double*>(ws_take(c, np * 16));
  {
    ProfScope ps(c, "sx_conj");
    if (dt == GW_C128)
      hipLaunchKernelGGL(k_conj_widen<double>, dim3((unsigned)((np + 255) / 256)), dim3(256), 0,
                         c->stream, static_cast<const cpx<double>*>(mtxel), np, X);
    else
      hipLaunchKernelGGL(k_conj_widen<float>, dim3((unsigned)((np + 255) / 256)), dim3(256), 0,
                         c->stream, static_cast<const cpx<float>*>(mtxel), np, X);
    GW_CHECK_LAUNCH(c, "k_conj_widen");
  }
  // U = conj(M) eps^-1 on the matrix cores
  st = zgemm_nn(c, P, N, N, 1.0, reinterpret_cast<const double*>(X), 0, N, 0, epsinv, 0, N, 0, U,
                0, N, 0, 1, np, (size_t)N * N, np, 0.0);
  if (st != GW_OK) return st;
  ProfScope ps(c, "sx_reduce");
  if (dt == GW_C128)
    hipLaunchKernelGGL(k_sx_reduce<double>, dim3(nband), dim3(256), 0, c->stream,
                       reinterpret_cast<const cpx<double>*>(U),
                       static_cast<const cpx<double>*>(mtxel), vcoul, nocc, nband, N, prefactor,
                       reinterpret_cast<cpx<double>*>(sigma));
  else
    hipLaunchKernelGGL(k_sx_reduce<float>, dim3(nband), dim3(256), 0, c->stream,
                       reinterpret_cast<const cpx<double>*>(U),
                       static_cast<const cpx<float>*>(mtxel), vcoul, nocc, nband, N, prefactor,
                       reinterpret_cast<cpx<double>*>(sigma));
  GW_CHECK_LAUNCH(c, "k_sx_reduce");
  return GW_OK;
}

// eps^-1 = S epst^-1 S^-1, in place.
__global__ void k_unscale(cpx<double>* __restrict__ A, const double* __restrict__ v, int N) {
  const size_t nn = (size_t)N * N;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nn) return;
  const int i = (int)(idx / N), j = (int)(idx % N);
  const double s = sqrt(v[i]) / sqrt(v[j]);
  cpx<double>* a = A + (size_t)blockIdx.y * nn + idx;
  *a = scal(*a, s);
}

gw_status epsinv_pivoted_one(gw_ctx* c, int N, int nfreq, const double* chi0,
                             const double* vcoul, double* epsinv) {
  const size_t nn = (size_t)N * N;
  const size_t bytes = align_up(nfreq * nn * 16) + 2 * align_up((size_t)nfreq * N * 4);
  gw_status st = ws_begin(c, bytes);
  if (st != GW_OK) return st;
  cpx<double>* LU = static_cast<cpx<double>*>(ws_take(c, nfreq * nn * 16));
  int* ipiv = static_cast<int*>(ws_take(c, (size_t)nfreq * N * 4));
  int* perm = static_cast<int*>(ws_take(c, (size_t)nfreq * N * 4));
  cpx<double>* Y = reinterpret_cast<cpx<double>*>(epsinv);
  {
    ProfScope ps(c, "flags_clear");
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, c->stream, c->d_flag, 16, 0);
    GW_CHECK_LAUNCH(c, "k_fill_int");
  }
  {
    ProfScope ps(c, "eps_build");
    hipLaunchKernelGGL(k_eps_build, dim3((unsigned)((nn + 255) / 256), nfreq), dim3(256), 0,
                       c->stream, reinterpret_cast<const cpx<double>*>(chi0), vcoul, LU, N);
    GW_CHECK_LAUNCH(c, "k_eps_build");
  }
  const long long s2 = (long long)nn;  // batch stride in complex elements
  const size_t ext = (size_t)nfreq * nn;  // complex elements in LU and in epsinv
  double* LUd = reinterpret_cast<double*>(LU);
  for (int k = 0; k < N; k += NB) {
    const int nbk = std::min(NB, N - k);
    {
      ProfScope ps(c, "lu_panel");
      hipLaunchKernelGGL(k_lu_panel, dim3(nfreq), dim3(1024), 0, c->stream, LU, N, k, nbk, ipiv,
                         c->d_flag);
      GW_CHECK_LAUNCH(c, "k_lu_panel");
    }
    {
      ProfScope ps(c, "lu_laswp");
      hipLaunchKernelGGL(k_lu_laswp, dim3((N + 255) / 256, nfreq), dim3(256), 0, c->stream, LU,
                         N, k, nbk, ipiv);
      GW_CHECK_LAUNCH(c, "k_lu_laswp");
    }
    const int rest = N - k - nbk;
    if (rest > 0) {
      {
        ProfScope ps(c, "lu_trsm");
        hipLaunchKernelGGL(k_trsm_block<false>, dim3((rest + 255) / 256, nfreq), dim3(256), 0,
                           c->stream, LU, N, k, nbk, LU, k + nbk, rest);
        GW_CHECK_LAUNCH(c, "k_trsm_block");
      }
      st = zgemm_nn(c, rest, rest, nbk, -1.0, LUd, (size_t)(k + nbk) * N + k, N, s2, LUd,
                    (size_t)k * N + k + nbk, N, s2, LUd, (size_t)(k + nbk) * N + k + nbk, N, s2,
                    nfreq, ext, ext, ext);
      if (st != GW_OK) return st;
    }
  }
  {
    ProfScope ps(c, "inv_perm");
    hipLaunchKernelGGL(k_perm_build, dim3(nfreq), dim3(256), (size_t)N * 4, c->stream, ipiv, N,
                       perm);
    GW_CHECK_LAUNCH(c, "k_perm_build");
    hipLaunchKernelGGL(k_perm_identity, dim3((unsigned)((nn + 255) / 256), nfreq), dim3(256), 0,
                       c->stream, perm, N, Y);
    GW_CHECK_LAUNCH(c, "k_perm_identity");
  }
  // forward: L Y = P I
  for (int kb = 0; kb < N; kb += NB) {
    const int nbk = std::min(NB, N - kb);
    {
      ProfScope ps(c, "inv_trsm_lower");
      hipLaunchKernelGGL(k_trsm_block<false>, dim3((N + 255) / 256, nfreq), dim3(256), 0,
                         c->stream, LU, N, kb, nbk, Y, 0, N);
      GW_CHECK_LAUNCH(c, "k_trsm_block");
    }
    const int below = N - kb - nbk;
    if (below > 0) {
      st = zgemm_nn(c, below, N, nbk, -1.0, LUd, (size_t)(kb + nbk) * N + kb, N, s2, epsinv,
                    (size_t)kb * N, N, s2, epsinv, (size_t)(kb + nbk) * N, N, s2, nfreq, ext, ext,
                    ext);
      if (st != GW_OK) return st;
    }
  }
  // back: U X = Y
  const int nblk = (N + NB - 1) / NB;
  for (int b = nblk - 1; b >= 0; --b) {
    const int kb = b * NB;
    const int nbk = std::min(NB, N - kb);
    {
      ProfScope ps(c, "inv_trsm_upper");
      hipLaunchKernelGGL(k_trsm_block<true>, dim3((N + 255) / 256, nfreq), dim3(256), 0,
                         c->stream, LU, N, kb, nbk, Y, 0, N);
      GW_CHECK_LAUNCH(c, "k_trsm_block");
    }
    if (kb > 0) {
      st = zgemm_nn(c, kb, N, nbk, -1.0, LUd, (size_t)kb, N, s2, epsinv, (size_t)kb * N, N, s2,
                    epsinv, 0, N, s2, nfreq, ext, ext, ext);
      if (st != GW_OK) return st;
    }
  }
  int flag = 0;
  GW_HIP(c, hipMemcpyAsync(&flag, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  GW_HIP(c, hipStreamSynchronize(c->stream));
  if (flag) return fail(c, GW_ESINGULAR, "eps has a zero pivot (singular dielectric matrix)");
  return GW_OK;
}

static gw_status epsinv_gauss_jordan(gw_ctx* c, int N, int nfreq, const double* chi0,
                                     const double* vcoul, double* epsinv) {
  const size_t nn = (size_t)N * N;
  const size_t nR = (size_t)nfreq * GB * N, nC = (size_t)nfreq * N * GB, nD = (size_t)nfreq * GB * GB;
  gw_status st = ws_begin(c, 2 * align_up(nR * 16) + align_up(nC * 16) + 3 * align_up(nD * 16));
  if (st != GW_OK) return st;
  cpx<double>* Rw[2] = {static_cast<cpx<double>*>(ws_take(c, nR * 16)),
                        static_cast<cpx<double>*>(ws_take(c, nR * 16))};
  cpx<double>* Cb = static_cast<cpx<double>*>(ws_take(c, nC * 16));
  cpx<double>* Dw[2] = {static_cast<cpx<double>*>(ws_take(c, nD * 16)),
                        static_cast<cpx<double>*>(ws_take(c, nD * 16))};
  cpx<double>* Dn = static_cast<cpx<double>*>(ws_take(c, nD * 16));
  cpx<double>* A = reinterpret_cast<cpx<double>*>(epsinv);
  const double* Ad = epsinv;
  {
    ProfScope ps(c, "flags_clear");
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, c->stream, c->d_flag, 16, 0);
    GW_CHECK_LAUNCH(c, "k_fill_int");
  }
  {
    ProfScope ps(c, "eps_build");
    const unsigned nt = (unsigned)((N + ET - 1) / ET);
    hipLaunchKernelGGL(k_epst_build, dim3(nt, nt, nfreq), dim3(256), 0, c->stream,
                       reinterpret_cast<const cpx<double>*>(chi0), vcoul, A, N, c->d_flag);
    GW_CHECK_LAUNCH(c, "k_epst_build");
  }
  {
    ProfScope ps(c, "gj_diag");
    hipLaunchKernelGGL(k_gj_diag, dim3(nfreq), dim3(1024), 0, c->stream, A, N, nn,
                       std::min(GB, N), Dw[0], c->d_flag);
    GW_CHECK_LAUNCH(c, "k_gj_diag");
  }
  const size_t ext = (size_t)nfreq * nn;
  // Per step K: the row panel R = Dinv A[K][:], one small kernel, and the rank
  // update, whose launch also forms and inverts the next diagonal block (the
  // look-ahead) on its first workgroups. The panels R and the diagonal inverses
  // alternate between two buffers by step parity.
  int kp = 0, nbp = 0;
  for (int k = 0, s = 0; k < N; k += GB, ++s) {
    const int nbk = std::min(GB, N - k);
    cpx<double>* D = Dw[s & 1];
    cpx<double>* R = Rw[s & 1];
    // R = Dinv A[K][:] (rows nbk.. of R are never read)
    st = zgemm_nn(c, nbk, N, nbk, 1.0, reinterpret_cast<const double*>(D), 0, GB, GB * GB, Ad,
                  (size_t)k * N, N, (long long)nn, reinterpret_cast<double*>(R), 0, N,
                  (long long)GB * N, nfreq, nD, ext, nR, 0.0);
    if (st != GW_OK) return st;
    {
      ProfScope ps(c, "gj_small");
      hipLaunchKernelGGL(k_gj_step, dim3((N * GB + 255) / 256, nfreq), dim3(256), 0, c->stream,
                         A, N, k, nbk, Cb, R, D, kp, nbp, Rw[(s + 1) & 1], Dw[(s + 1) & 1]);
      GW_CHECK_LAUNCH(c, "k_gj_step");
    }
    // A -= Cb R over the whole matrix: every row outside K is final, including
    // its K columns; row block K is rewritten by the next step's small kernel
    const int k2 = k + GB, nb2 = std::max(0, std::min(GB, N - k2));
    {
      ProfScope ps(c, "gj_update");
      const int nt = (N + UT - 1) / UT;
      const long long tiles = (long long)nt * nt * nfreq;
      const long long grid = (nb2 > 0 ? nfreq : 0) + ((tiles + kXcd - 1) / kXcd) * kXcd;
      // operands staged in LDS from N = 2048 (C3, N = 4000: 8.8 vs 9.7 ms per step);
      // below, fragments straight from L2 (C2, N = 1000: 1.68 vs 1.84 ms)
      if (N >= 2048)
        hipLaunchKernelGGL(k_gj_update<true>, dim3((unsigned)grid), dim3(256), 0, c->stream, A,
                           N, nbk, Cb, R, nfreq, k2, nb2, Dn, Dw[(s + 1) & 1], c->d_flag);
      else
        hipLaunchKernelGGL(k_gj_update<false>, dim3((unsigned)grid), dim3(256), 0, c->stream, A,
                           N, nbk, Cb, R, nfreq, k2, nb2, Dn, Dw[(s + 1) & 1], c->d_flag);
      GW_CHECK_LAUNCH(c, "k_gj_update");
    }
    kp = k;
    nbp = nbk;
  }
  {
    ProfScope ps(c, "gj_small");
    const int s_last = (N + GB - 1) / GB - 1;
    hipLaunchKernelGGL(k_gj_fix, dim3((N * nbp + 255) / 256, nfreq), dim3(256), 0, c->stream,
                       A, N, kp, nbp, Rw[s_last & 1], Dw[s_last & 1]);
    GW_CHECK_LAUNCH(c, "k_gj_fix");
  }
  {
    ProfScope ps(c, "eps_unscale");
    hipLaunchKernelGGL(k_unscale, dim3((unsigned)((nn + 255) / 256), nfreq), dim3(256), 0,
                       c->stream, A, vcoul, N);
    GW_CHECK_LAUNCH(c, "k_unscale");
  }
  return GW_OK;
}

// rmax[f] = max_ij |R_f[i][j] - delta_ij| (|re| + |im|), one workgroup per
// frequency; a non-finite entry makes the result non-finite
__global__ void __launch_bounds__(1024) k_resid_max(const cpx<double>* __restrict__ R, int N,
                                                    double* __restrict__ rmax) {
  __shared__ double sm[1024];
  const size_t nn = (size_t)N * N;
  R += (size_t)blockIdx.x * nn;
  double m = 0.0;
  for (size_t e = threadIdx.x; e < nn; e += blockDim.x) {
    const int i = (int)(e / N), j = (int)(e % N);
    const cpx<double> r = R[e];
    const double a = fabs(r.x - (i == j ? 1.0 : 0.0)) + fabs(r.y);
    m = (a > m || a != a) ? a : m;
  }
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      const double o = sm[threadIdx.x + s];
      if (o > sm[threadIdx.x] || o != o) sm[threadIdx.x] = o;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) rmax[blockIdx.x] = sm[0];
}

// Whether X solves eps X = I for every frequency to max_ij |(eps X - I)_ij| <=
// kVerifyRel / N, with eps = I - diag(v) chi0 formed again. Since X - eps^-1 =
// eps^-1 (eps X - I), that bounds the relative error of X in the infinity norm
// by N max_ij |.| <= kVerifyRel.
constexpr double kVerifyRel = 1e-10;
static gw_status epsinv_verified(gw_ctx* c, int N, int nfreq, const double* chi0,
                                 const double* vcoul, const double* X, bool* ok) {
  const size_t nn = (size_t)N * N, ext = (size_t)nfreq * nn;
  gw_status st = ws_begin(c, 2 * align_up(ext * 16) + align_up((size_t)nfreq * 8));
  if (st != GW_OK) return st;
  cpx<double>* E = static_cast<cpx<double>*>(ws_take(c, ext * 16));
  double* R = static_cast<double*>(ws_take(c, ext * 16));
  double* d_rmax = static_cast<double*>(ws_take(c, (size_t)nfreq * 8));
  {
    ProfScope ps(c, "eps_build");
    hipLaunchKernelGGL(k_eps_build, dim3((unsigned)((nn + 255) / 256), nfreq), dim3(256), 0,
                       c->stream, reinterpret_cast<const cpx<double>*>(chi0), vcoul, E, N);
    GW_CHECK_LAUNCH(c, "k_eps_build");
  }
  st = zgemm_nn(c, N, N, N, 1.0, reinterpret_cast<const double*>(E), 0, N, (long long)nn, X, 0, N,
                (long long)nn, R, 0, N, (long long)nn, nfreq, ext, ext, ext, 0.0);
  if (st != GW_OK) return st;
  {
    ProfScope ps(c, "eps_verify");
    hipLaunchKernelGGL(k_resid_max, dim3(nfreq), dim3(1024), 0, c->stream,
                       reinterpret_cast<const cpx<double>*>(R), N, d_rmax);
    GW_CHECK_LAUNCH(c, "k_resid_max");
  }
  std::vector<double> rmax(nfreq);
  GW_HIP(c, hipMemcpyAsync(rmax.data(), d_rmax, (size_t)nfreq * 8, hipMemcpyDeviceToHost,
                           c->stream));
  GW_HIP(c, hipStreamSynchronize(c->stream));
  *ok = true;
  for (double r : rmax) *ok = *ok && r <= kVerifyRel / N;
  return GW_OK;
}

gw_status epsinv_run(gw_ctx* c, int N, int nfreq, const double* chi0, const double* vcoul,
                     double* epsinv) {
  gw_status st = epsinv_gauss_jordan(c, N, nfreq, chi0, vcoul, epsinv);
  if (st != GW_OK) return st;
  int flags[5] = {0, 0, 0, 0, 0};
  GW_HIP(c, hipMemcpyAsync(flags, c->d_flag, sizeof flags, hipMemcpyDeviceToHost, c->stream));
  GW_HIP(c, hipStreamSynchronize(c->stream));
  if (flags[4]) return fail(c, GW_EINVAL, "chi0 holds a non-finite entry");
  // some v <= 0: the symmetric form eps~ does not exist; general LU
  if (flags[1]) return epsinv_pivoted_one(c, N, nfreq, chi0, vcoul, epsinv);
  if (!flags[2] && !flags[3]) return GW_OK;
  // chi0 not Hermitian (as on the real frequency axis), or a pivot not of the
  // Hermitian positive-definite kind: Gauss-Jordan without pivoting carries no
  // stability guarantee there, so its result is kept only if it solves
  // eps X = I to within kVerifyRel / N per entry; otherwise general LU with
  // partial pivoting
  bool ok = false;
  if ((st = epsinv_verified(c, N, nfreq, chi0, vcoul, epsinv, &ok)) != GW_OK) return st;
  if (ok) return GW_OK;
  return epsinv_pivoted_one(c, N, nfreq, chi0, vcoul, epsinv);
}

}  // namespace gw
