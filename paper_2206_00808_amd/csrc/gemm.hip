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
#include "common.h"

namespace gw {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

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

// upper-triangle tile index -> (ti, tj), ti <= tj, row-major over the triangle
__device__ __forceinline__ void tri_tile(int idx, int nt, int* ti, int* tj) {
  int r = 0, start = 0;
  while (start + (nt - r) <= idx) { start += nt - r; ++r; }
  *ti = r;
  *tj = r + (idx - start);
}

// ---------------------------------------------------------------- FP64 chi0
constexpr int TM = 64;   // tile edge (complex elements)
constexpr int KT = 16;   // K step (pairs)
constexpr int LP = TM + 1;  // LDS pitch

template <typename Tin>
__device__ __forceinline__ cpx<double> load_widen(const cpx<Tin>* p) {
  cpx<Tin> v = *p;
  return mk<double>((double)v.x, (double)v.y);
}

// 64x64 output tile per workgroup (4 waves of 32x32), K-step of 16 pairs.
// Planar re/im LDS tiles padded so each quarter-wave row group lands on its own
// half of the banks; the next K-tile is fetched into registers while the
// matrix cores work on the current one.
constexpr int PT = TM + 16;

template <typename Tin>
__global__ void __launch_bounds__(256) k_chi0_f64(const cpx<Tin>* __restrict__ M, int P, int neps,
                                                  const double* __restrict__ wts,
                                                  cpx<double>* __restrict__ chi, int nt,
                                                  int skip_head) {
  __shared__ double Ar[KT][PT], Ai[KT][PT], Br[KT][PT], Bi[KT][PT];
  int ti, tj;
  tri_tile(blockIdx.x, nt, &ti, &tj);
  const int f = blockIdx.y;
  const double* w = wts + (size_t)f * P;
  const int i0 = ti * TM, j0 = tj * TM;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int l16 = lane & 15, lk = lane >> 4;
  constexpr int NE = (KT * TM) / 256;
  d4 cr[2][2], ci[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      cr[a][b] = (d4){0, 0, 0, 0};
      ci[a][b] = (d4){0, 0, 0, 0};
    }
  // raw loads from clamped (always valid) addresses; masking and the weight
  // are applied at the LDS store so the prefetch never waits on its own loads
  cpx<Tin> ra[NE], rb[NE];
  double rw[NE];
  auto gload = [&](int p0) {
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const int idx = tid + e * 256;
      const int kk = idx / TM, ii = idx % TM;
      const int p = min(p0 + kk, P - 1);
      ra[e] = M[(size_t)p * neps + min(i0 + ii, neps - 1)];
      rb[e] = M[(size_t)p * neps + min(j0 + ii, neps - 1)];
      rw[e] = w[p];
    }
  };
  gload(0);
  for (int p0 = 0; p0 < P; p0 += KT) {
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const int idx = tid + e * 256;
      const int kk = idx / TM, ii = idx % TM;
      const bool pk = p0 + kk < P;
      const double ma = (pk && i0 + ii < neps) ? 1.0 : 0.0;
      const double mb = (pk && j0 + ii < neps) ? rw[e] : 0.0;
      Ar[kk][ii] = ma * (double)ra[e].x; Ai[kk][ii] = ma * (double)ra[e].y;
      Br[kk][ii] = mb * (double)rb[e].x; Bi[kk][ii] = mb * (double)rb[e].y;
    }
    __syncthreads();
    if (p0 + KT < P) gload(p0 + KT);
#pragma unroll
    for (int s = 0; s < KT / 4; ++s) {
      const int kk = s * 4 + lk;
      double ar[2], ai[2], br[2], bi[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        ar[a] = Ar[kk][wr * 32 + a * 16 + l16];
        ai[a] = Ai[kk][wr * 32 + a * 16 + l16];
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        br[b] = Br[kk][wc * 32 + b * 16 + l16];
        bi[b] = Bi[kk][wc * 32 + b * 16 + l16];
      }
      // conj(a) * b = (ar br + ai bi) + i (ar bi - ai br); the four products are
      // issued round-robin over the eight accumulators so that no MFMA waits on
      // the one just issued
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          cr[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[a], br[b], cr[a][b], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          ci[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[a], bi[b], ci[a][b], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          cr[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[a], bi[b], cr[a][b], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          ci[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai[a], br[b], ci[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
  cpx<double>* C = chi + (size_t)f * neps * neps;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wr * 32 + a * 16 + lk + 4 * r;  // f64 16x16x4 D layout
        const int j = j0 + wc * 32 + b * 16 + l16;
        if (i >= neps || j >= neps) continue;
        if (skip_head >= 0 && (i == skip_head || j == skip_head)) continue;
        const double re = cr[a][b][r], im = ci[a][b][r];
        cpx<double>* d = C + (size_t)i * neps + j;
        *d = mk(d->x + re, d->y + im);
        if (ti != tj) {
          cpx<double>* m = C + (size_t)j * neps + i;
          *m = mk(m->x + re, m->y - im);
        }
      }
}

gw_status chi0_fp64(gw_ctx* c, int P, int neps, const void* mtxel, gw_dtype dt, int nfreq,
                    const double* wts, int skip_head, double* chi0) {
  const int nt = (neps + TM - 1) / TM;
  const int ntri = nt * (nt + 1) / 2;
  ProfScope ps(c, "chi0_fp64");
  if (dt == GW_C128)
    hipLaunchKernelGGL(k_chi0_f64<double>, dim3(ntri, nfreq), dim3(256), 0, c->stream,
                       static_cast<const cpx<double>*>(mtxel), P, neps, wts,
                       reinterpret_cast<cpx<double>*>(chi0), nt, skip_head);
  else
    hipLaunchKernelGGL(k_chi0_f64<float>, dim3(ntri, nfreq), dim3(256), 0, c->stream,
                       static_cast<const cpx<float>*>(mtxel), P, neps, wts,
                       reinterpret_cast<cpx<double>*>(chi0), nt, skip_head);
  GW_CHECK_LAUNCH(c, "k_chi0_f64");
  return GW_OK;
}

// ---------------------------------------------------------------- generic ZGEMM
// C[i][j] += alpha * sum_k A[i][k] B[k][j], complex double, row-major, batched on z.
__global__ void __launch_bounds__(256) k_zgemm_nn(int m, int n, int kdim, double alpha,
                                                  const cpx<double>* __restrict__ A, int lda,
                                                  long long sA, const cpx<double>* __restrict__ B,
                                                  int ldb, long long sB, cpx<double>* __restrict__ C,
                                                  int ldc, long long sC) {
  __shared__ cpx<double> As[KT][LP];
  __shared__ cpx<double> Bs[KT][LP];
  const int i0 = blockIdx.y * TM, j0 = blockIdx.x * TM;
  A += (size_t)blockIdx.z * sA;
  B += (size_t)blockIdx.z * sB;
  C += (size_t)blockIdx.z * sC;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int l16 = lane & 15, lk = lane >> 4;
  d4 cr[2][2], ci[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      cr[a][b] = (d4){0, 0, 0, 0};
      ci[a][b] = (d4){0, 0, 0, 0};
    }
  for (int k0 = 0; k0 < kdim; k0 += KT) {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < (KT * TM) / 256; ++e) {
      const int idx = tid + e * 256;
      // A tile: TM rows x KT columns, k fastest for coalescing
      const int ai = idx / KT, ak = idx % KT;
      cpx<double> a = mk<double>(0, 0);
      if (i0 + ai < m && k0 + ak < kdim) a = A[(size_t)(i0 + ai) * lda + k0 + ak];
      As[ak][ai] = a;
      const int bk = idx / TM, bj = idx % TM;
      cpx<double> b = mk<double>(0, 0);
      if (k0 + bk < kdim && j0 + bj < n) b = B[(size_t)(k0 + bk) * ldb + j0 + bj];
      Bs[bk][bj] = b;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < KT / 4; ++s) {
      const int kk = s * 4 + lk;
      cpx<double> av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = As[kk][wr * 32 + a * 16 + l16];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = Bs[kk][wc * 32 + b * 16 + l16];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          // a * b = (ar br - ai bi) + i (ar bi + ai br)
          cr[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a].x, bv[b].x, cr[a][b], 0, 0, 0);
          cr[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-av[a].y, bv[b].y, cr[a][b], 0, 0, 0);
          ci[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a].x, bv[b].y, ci[a][b], 0, 0, 0);
          ci[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a].y, bv[b].x, ci[a][b], 0, 0, 0);
        }
    }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wr * 32 + a * 16 + lk + 4 * r;  // f64 16x16x4 D layout
        const int j = j0 + wc * 32 + b * 16 + l16;
        if (i >= m || j >= n) continue;
        cpx<double>* d = C + (size_t)i * ldc + j;
        *d = mk(d->x + alpha * cr[a][b][r], d->y + alpha * ci[a][b][r]);
      }
}

// Highest complex-element offset (exclusive) one operand touches across the batch.
static size_t span(size_t off, int rows, int cols, int ld, long long stride, int batch) {
  return off + (size_t)(batch - 1) * (size_t)stride + (size_t)(rows - 1) * ld + cols;
}

gw_status zgemm_nn(gw_ctx* c, int m, int n, int k, double alpha, const double* A, size_t offA,
                   int lda, long long sA, const double* B, size_t offB, int ldb, long long sB,
                   double* C, size_t offC, int ldc, long long sC, int batch, size_t extA,
                   size_t extB, size_t extC) {
  if (m <= 0 || n <= 0 || k <= 0 || batch <= 0) return GW_OK;
  // every offset, leading dimension and stride is in complex elements; the
  // extents are the complex elements available behind each base pointer
  if (span(offA, m, k, lda, sA, batch) > extA || span(offB, k, n, ldb, sB, batch) > extB ||
      span(offC, m, n, ldc, sC, batch) > extC || lda < k || ldb < n || ldc < n)
    return fail(c, GW_EINVAL, "zgemm operand out of range (m=%d n=%d k=%d batch=%d)", m, n, k,
                batch);
  ProfScope ps(c, "zgemm_update");
  dim3 g((n + TM - 1) / TM, (m + TM - 1) / TM, batch);
  hipLaunchKernelGGL(k_zgemm_nn, g, dim3(256), 0, c->stream, m, n, k, alpha,
                     reinterpret_cast<const cpx<double>*>(A) + offA, lda, sA,
                     reinterpret_cast<const cpx<double>*>(B) + offB, ldb, sB,
                     reinterpret_cast<cpx<double>*>(C) + offC, ldc, sC);
  GW_CHECK_LAUNCH(c, "k_zgemm_nn");
  return GW_OK;
}

// ---------------------------------------------------------------- split-BF16 chi0
// bf16 round-to-nearest-even from the IEEE-754 binary32 bit pattern (finite inputs).
__device__ __forceinline__ unsigned short bf16_rn_bits(float x) {
  unsigned int u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(unsigned short h) {
  return __uint_as_float(((unsigned int)h) << 16);
}

constexpr int BK = 32;          // K step (pairs) = one 16x16x32 MFMA
constexpr int BKP = BK + 8;     // LDS pitch in bf16 (16-byte aligned rows)
constexpr int KFLUSH = 512;     // pairs accumulated in float before the double flush

// LDS arrays [4 parts: re_hi, re_lo, im_hi, im_lo][TM rows][BKP]
__global__ void __launch_bounds__(256) k_chi0_bf16x3(const cpx<float>* __restrict__ M, int P,
                                                     int neps, const double* __restrict__ wts,
                                                     cpx<double>* __restrict__ chi, int nt,
                                                     int skip_head) {
  __shared__ __align__(16) unsigned short As[4][TM][BKP];
  __shared__ __align__(16) unsigned short Bs[4][TM][BKP];
  int ti, tj;
  tri_tile(blockIdx.x, nt, &ti, &tj);
  const int f = blockIdx.y;
  const double* w = wts + (size_t)f * P;
  const int i0 = ti * TM, j0 = tj * TM;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int l16 = lane & 15, lk = lane >> 4;
  double dr[2][2][4], di[2][2][4];
  f4 cr[2][2], ci[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      cr[a][b] = (f4){0, 0, 0, 0};
      ci[a][b] = (f4){0, 0, 0, 0};
#pragma unroll
      for (int r = 0; r < 4; ++r) dr[a][b][r] = di[a][b][r] = 0.0;
    }
  int since_flush = 0;
  constexpr int NE = (BK * TM) / 256;
  // raw prefetch of the next K-tile (clamped addresses); split at the LDS store
  cpx<float> ra[NE], rb[NE];
  double rw[NE];
  auto gload = [&](int p0) {
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const int idx = tid + e * 256;
      const int kk = idx / TM, ii = idx % TM;
      const int p = min(p0 + kk, P - 1);
      ra[e] = M[(size_t)p * neps + min(i0 + ii, neps - 1)];
      rb[e] = M[(size_t)p * neps + min(j0 + ii, neps - 1)];
      rw[e] = w[p];
    }
  };
  gload(0);
  for (int p0 = 0; p0 < P; p0 += BK) {
    // stage: BK pairs x TM columns of A (=M) and B (=w*M), split into hi/lo
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const int idx = tid + e * 256;
      const int kk = idx / TM, ii = idx % TM;
      const bool pk = p0 + kk < P;
      const float ma = (pk && i0 + ii < neps) ? 1.f : 0.f;
      const float wf = (pk && j0 + ii < neps) ? (float)rw[e] : 0.f;
      const float ar = ma * ra[e].x, ai = ma * ra[e].y;
      const float br = wf * rb[e].x, bi = wf * rb[e].y;
      unsigned short h;
      h = bf16_rn_bits(ar); As[0][ii][kk] = h; As[1][ii][kk] = bf16_rn_bits(ar - bf16_to_f(h));
      h = bf16_rn_bits(ai); As[2][ii][kk] = h; As[3][ii][kk] = bf16_rn_bits(ai - bf16_to_f(h));
      h = bf16_rn_bits(br); Bs[0][ii][kk] = h; Bs[1][ii][kk] = bf16_rn_bits(br - bf16_to_f(h));
      h = bf16_rn_bits(bi); Bs[2][ii][kk] = h; Bs[3][ii][kk] = bf16_rn_bits(bi - bf16_to_f(h));
    }
    __syncthreads();
    if (p0 + BK < P) gload(p0 + BK);
    bf8 a[2][4], b[2][4];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[x][q] = *reinterpret_cast<const bf8*>(&As[q][wr * 32 + x * 16 + l16][lk * 8]);
        b[x][q] = *reinterpret_cast<const bf8*>(&Bs[q][wc * 32 + x * 16 + l16][lk * 8]);
      }
    // the fragments are in registers: the tile may be restaged after this point
    __syncthreads();
    // -ai as the A operand of the ai*br terms (sign bit of every bf16 lane)
    bf8 na[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        typedef unsigned short us8 __attribute__((ext_vector_type(8)));
        us8 t = __builtin_bit_cast(us8, a[x][2 + q]);
        t ^= (us8)(0x8000);
        na[x][q] = __builtin_bit_cast(bf8, t);
      }
    // Re += ar*br + ai*bi, Im += ar*bi - ai*br, each real product as
    // hi*hi + hi*lo + lo*hi; terms outermost so consecutive MFMAs go to
    // different accumulators
#define GW_MF(ACC, A, B)                                                              \
  _Pragma("unroll") for (int x = 0; x < 2; ++x) _Pragma("unroll") for (int y = 0; y < 2; ++y) \
      ACC[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B, ACC[x][y], 0, 0, 0);
    GW_MF(cr, a[x][0], b[y][0])
    GW_MF(ci, a[x][0], b[y][2])
    GW_MF(cr, a[x][0], b[y][1])
    GW_MF(ci, a[x][0], b[y][3])
    GW_MF(cr, a[x][1], b[y][0])
    GW_MF(ci, a[x][1], b[y][2])
    GW_MF(cr, a[x][2], b[y][2])
    GW_MF(ci, na[x][0], b[y][0])
    GW_MF(cr, a[x][2], b[y][3])
    GW_MF(ci, na[x][0], b[y][1])
    GW_MF(cr, a[x][3], b[y][2])
    GW_MF(ci, na[x][1], b[y][0])
#undef GW_MF
    since_flush += BK;
    if (since_flush >= KFLUSH || p0 + BK >= P) {
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            dr[x][y][r] += (double)cr[x][y][r];
            di[x][y][r] += (double)ci[x][y][r];
          }
          cr[x][y] = (f4){0, 0, 0, 0};
          ci[x][y] = (f4){0, 0, 0, 0};
        }
      since_flush = 0;
    }
  }
  cpx<double>* C = chi + (size_t)f * neps * neps;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wr * 32 + x * 16 + lk * 4 + r;
        const int j = j0 + wc * 32 + y * 16 + l16;
        if (i >= neps || j >= neps) continue;
        if (skip_head >= 0 && (i == skip_head || j == skip_head)) continue;
        const double re = dr[x][y][r], im = di[x][y][r];
        cpx<double>* d = C + (size_t)i * neps + j;
        *d = mk(d->x + re, d->y + im);
        if (ti != tj) {
          cpx<double>* m = C + (size_t)j * neps + i;
          *m = mk(m->x + re, m->y - im);
        }
      }
}

gw_status chi0_splitbf16(gw_ctx* c, int P, int neps, const void* mtxel, int nfreq,
                         const double* wts, int skip_head, double* chi0) {
  const int nt = (neps + TM - 1) / TM;
  const int ntri = nt * (nt + 1) / 2;
  ProfScope ps(c, "chi0_bf16x3");
  hipLaunchKernelGGL(k_chi0_bf16x3, dim3(ntri, nfreq), dim3(256), 0, c->stream,
                     static_cast<const cpx<float>*>(mtxel), P, neps, wts,
                     reinterpret_cast<cpx<double>*>(chi0), nt, skip_head);
  GW_CHECK_LAUNCH(c, "k_chi0_bf16x3");
  return GW_OK;
}

}  // namespace gw
