// Learned closure of the truncated conduction-band sum.
//
// A small network predicts chi0_full - chi0_trunc for one (q, omega = 0) matrix
// from per-(G <= G') features; chi0_trunc plus the Hermitised prediction is the
// corrected matrix, and the full band sum remains the fallback and the
// reference for its error.  The nearest idea in the paper is the static remainder used for
// the Coulomb-hole sum over empty states (Computational Details).
//
//   features  |q+G|, |q+G'|, (q+G).(q+G')/10, Re chi_t/s, Im chi_t/s, 10 gap, 2 emax
//             (zero-padded to 32), s = max_G |chi_t[G][G]|, rows = upper triangle
//   network   depth hidden layers of `width` with SiLU, then a linear output;
//             products on v_mfma_f32_16x16x32_bf16 (bf16 operands rounded to
//             nearest even from float, float accumulation), float master weights
//   training  MSE over the real outputs, backpropagation by the same GEMM
//             kernel with transposed operands, Adam with bias correction
//   fallback  a double-precision blocked Cholesky of -chi_out; if it meets a
//             pivot that is not positive, the full sum is returned instead
#include <cmath>
#include <cstring>

#include "tiles.h"

namespace gw {

constexpr int CL_KPAD = 32;  // input features padded to one MFMA K-step
constexpr int CL_OPAD = 32;  // outputs padded (the real ones first, the rest kept zero)
constexpr int CL_RT = 64;    // row tile
constexpr int CL_NFEAT = 7;
constexpr int CL_NOUT = 2;
constexpr uint32_t CL_MAGIC = 0x4C4D5747u;  // "GWML"

__device__ __forceinline__ float silu_f(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float dsilu_f(float z) {
  const float s = 1.0f / (1.0f + __expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

// row r of the upper triangle (row major) -> (i, j), i <= j < N
__device__ __forceinline__ void tri_rc(long long r, int N, int* oi, int* oj) {
  const double b = 2.0 * N + 1.0;
  long long i = (long long)floor((b - sqrt(b * b - 8.0 * (double)r)) * 0.5);
  auto off = [&](long long k) { return k * (2LL * N - k + 1) / 2; };
  if (i < 0) i = 0;
  while (i > 0 && off(i) > r) --i;
  while (off(i + 1) <= r) ++i;
  *oi = (int)i;
  *oj = (int)(i + (r - off(i)));
}

__global__ void k_cl_scale(const cpx<double>* __restrict__ chi, int N, double* __restrict__ s) {
  __shared__ double red[256];
  double m = 0.0;
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    const cpx<double> d = chi[(size_t)i * N + i];
    m = fmax(m, sqrt(d.x * d.x + d.y * d.y));
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int k = blockDim.x / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + k]);
    __syncthreads();
  }
  if (threadIdx.x == 0) s[0] = red[0] > 0.0 ? red[0] : 1.0;
}

// X[r][0..31] and (when full != NULL) T[r][0..1]; rows >= n zero.
__global__ void k_cl_features(const double* __restrict__ qg, const cpx<double>* __restrict__ chi,
                              const cpx<double>* __restrict__ full, int N, long long n,
                              long long npad, double gap, double emax,
                              const double* __restrict__ sc, float* __restrict__ X,
                              float* __restrict__ T) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= npad) return;
  float* x = X + r * CL_KPAD;
  for (int k = 0; k < CL_KPAD; ++k) x[k] = 0.f;
  if (T) { T[r * 2] = 0.f; T[r * 2 + 1] = 0.f; }
  if (r >= n) return;
  int i, j;
  tri_rc(r, N, &i, &j);
  const double s = sc[0];
  const double* a = qg + 3 * (size_t)i;
  const double* b = qg + 3 * (size_t)j;
  const cpx<double> c = chi[(size_t)i * N + j];
  x[0] = (float)sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
  x[1] = (float)sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
  x[2] = (float)((a[0] * b[0] + a[1] * b[1] + a[2] * b[2]) / 10.0);
  x[3] = (float)(c.x / s);
  x[4] = (float)(c.y / s);
  x[5] = (float)(10.0 * gap);
  x[6] = (float)(2.0 * emax);
  if (T) {
    const cpx<double> f = full[(size_t)i * N + j];
    T[r * 2] = (float)((f.x - c.x) / s);
    T[r * 2 + 1] = (float)((f.y - c.y) / s);
  }
}

// ------------------------------------------------------------------ bf16 GEMM
// C[M][N] = sum_k A(m,k) B(k,n) with A(m,k) = TA ? A[k*lda+m] : A[m*lda+k] and
// B(k,n) = TB ? B[n*ldb+k] : B[k*ldb+n]; float in, bf16 (RNE) operands, float
// accumulation.  grid.z splits K into chunks of kchunk (EPI_STORE writes the
// partial of split z at C + z*cstride).
enum { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_SILU = 2, EPI_DSILU = 3 };

template <bool TA, bool TB, int EPI>
__global__ void __launch_bounds__(256) k_bgemm(int M, int N, int K, const float* __restrict__ A,
                                               int lda, const float* __restrict__ B, int ldb,
                                               float* __restrict__ C, int ldc,
                                               const float* __restrict__ bias,
                                               float* __restrict__ Zout,
                                               const float* __restrict__ Zin, int kchunk,
                                               long long cstride) {
  __shared__ __align__(16) unsigned short As[64][BKP];
  __shared__ __align__(16) unsigned short Bs[64][BKP];
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int kb = blockIdx.z * kchunk, ke = min(K, kb + kchunk);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int l16 = lane & 15, lk = lane >> 4;
  f4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = (f4){0, 0, 0, 0};
  for (int k0 = kb; k0 < ke; k0 += 32) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int idx = tid + e * 256;
      int m, k;
      if (TA) { k = idx / 64; m = idx % 64; } else { m = idx / 32; k = idx % 32; }
      float a = 0.f;
      if (m0 + m < M && k0 + k < ke)
        a = TA ? A[(size_t)(k0 + k) * lda + m0 + m] : A[(size_t)(m0 + m) * lda + k0 + k];
      As[m][k] = bf16_rn_bits(a);
      int n, kk;
      if (TB) { n = idx / 32; kk = idx % 32; } else { kk = idx / 64; n = idx % 64; }
      float b = 0.f;
      if (n0 + n < N && k0 + kk < ke)
        b = TB ? B[(size_t)(n0 + n) * ldb + k0 + kk] : B[(size_t)(k0 + kk) * ldb + n0 + n];
      Bs[n][kk] = bf16_rn_bits(b);
    }
    __syncthreads();
    bf8 a[2], b[2];
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      a[x] = *reinterpret_cast<const bf8*>(&As[wr * 32 + x * 16 + l16][lk * 8]);
      b[x] = *reinterpret_cast<const bf8*>(&Bs[wc * 32 + x * 16 + l16][lk * 8]);
    }
    __syncthreads();
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
        acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[x], b[y], acc[x][y], 0, 0, 0);
  }
  float* Cz = C + (size_t)blockIdx.z * cstride;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = m0 + wr * 32 + x * 16 + lk * 4 + r;
        const int j = n0 + wc * 32 + y * 16 + l16;
        if (i >= M || j >= N) continue;
        const size_t o = (size_t)i * ldc + j;
        const float v = acc[x][y][r];
        if (EPI == EPI_STORE) Cz[o] = v;
        else if (EPI == EPI_BIAS) C[o] = v + bias[j];
        else if (EPI == EPI_BIAS_SILU) {
          const float z = v + bias[j];
          Zout[o] = z;
          C[o] = silu_f(z);
        } else {
          C[o] = v * dsilu_f(Zin[o]);
        }
      }
}

// sum of `splits` partials of length n
__global__ void k_sum_splits(const float* __restrict__ part, int splits, size_t n,
                             float* __restrict__ out) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.f;
  for (int z = 0; z < splits; ++z) s += part[(size_t)z * n + i];
  out[i] = s;
}

// column sums of X[rows][cols] in row chunks: part[chunk][col]
__global__ void k_colsum(const float* __restrict__ X, long long rows, int cols, long long rchunk,
                         float* __restrict__ part) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  const long long r0 = (long long)blockIdx.y * rchunk, r1 = min(rows, r0 + rchunk);
  float s = 0.f;
  for (long long r = r0; r < r1; ++r) s += X[r * cols + c];
  part[(size_t)blockIdx.y * cols + c] = s;
}

// dY = 2 (Y - T) / (n nout) on the real outputs; per-block partial sums of (Y-T)^2
__global__ void k_cl_dy(const float* __restrict__ Y, const float* __restrict__ T, long long n,
                        long long npad, float* __restrict__ dY, double* __restrict__ part) {
  __shared__ double red[256];
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double s = 0.0;
  if (r < npad) {
    for (int o = 0; o < CL_OPAD; ++o) dY[r * CL_OPAD + o] = 0.f;
    if (r < n) {
      const double scale = 2.0 / ((double)n * CL_NOUT);
      for (int o = 0; o < CL_NOUT; ++o) {
        const float d = Y[r * CL_OPAD + o] - T[r * 2 + o];
        dY[r * CL_OPAD + o] = (float)(scale * d);
        s += (double)d * d;
      }
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = blockDim.x / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_sum_f64(const double* __restrict__ part, int n, double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = blockDim.x / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, size_t n, float lr, float b1, float b2, float eps,
                       float bc1, float bc2) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// out = chi_t + s * Hermitise(Y): (i<=j) gets y, (j,i) its conjugate, diagonal real
__global__ void k_cl_apply(const cpx<double>* __restrict__ chi, const float* __restrict__ Y, int N,
                           long long n, const double* __restrict__ sc,
                           cpx<double>* __restrict__ out) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  int i, j;
  tri_rc(r, N, &i, &j);
  const double s = sc[0];
  const double yr = s * (double)Y[r * CL_OPAD], yi = s * (double)Y[r * CL_OPAD + 1];
  const cpx<double> c = chi[(size_t)i * N + j];
  if (i == j) {
    out[(size_t)i * N + i] = mk(c.x + yr, c.y);
  } else {
    out[(size_t)i * N + j] = mk(c.x + yr, c.y + yi);
    const cpx<double> d = chi[(size_t)j * N + i];
    out[(size_t)j * N + i] = mk(d.x + yr, d.y - yi);
  }
}

// ------------------------------------------------------------------ Cholesky check
// A = -chi (lower Cholesky, right-looking, blocks of 32).  flag = 1 on a pivot
// that is not positive.
constexpr int CB = 32;

__global__ void k_set_i32(int* p, int v) { *p = v; }

__global__ void k_chol_neg(const cpx<double>* __restrict__ chi, cpx<double>* __restrict__ A,
                           size_t nn) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nn) A[i] = mk(-chi[i].x, -chi[i].y);
}

// factor the diagonal block in LDS; store L11 and W = L11^-H (upper) in Lw
__global__ void __launch_bounds__(1024) k_chol_diag(cpx<double>* __restrict__ A, int N, int k,
                                                    cpx<double>* __restrict__ Lw,
                                                    int* __restrict__ flag) {
  __shared__ cpx<double> L[CB][CB + 1];
  __shared__ cpx<double> Wi[CB][CB + 1];
  __shared__ double dpiv;
  const int nbk = min(CB, N - k);
  const int tid = threadIdx.x, i = tid / CB, j = tid % CB;
  if (i < nbk && j < nbk) L[i][j] = A[(size_t)(k + i) * N + k + j];
  __syncthreads();
  for (int t = 0; t < nbk; ++t) {
    if (tid == 0) {
      const double d = L[t][t].x;
      if (!(d > 0.0) || !(d < INFINITY)) { flag[0] = 1; dpiv = 1.0; } else dpiv = sqrt(d);
    }
    __syncthreads();
    const double p = dpiv;
    // column t below the pivot: l_it = a_it / p
    if (j == t && i > t && i < nbk) L[i][t] = scal(L[i][t], 1.0 / p);
    if (tid == 0) L[t][t] = mk(p, 0.0);
    __syncthreads();
    // trailing: a_ij -= l_it conj(l_jt), i >= j > t
    if (i > t && j > t && i < nbk && j <= i) L[i][j] = L[i][j] - cmulc(L[j][t], L[i][t]);
    __syncthreads();
  }
  // W = L^-1 (lower) by forward substitution on the identity, one column per thread
  if (tid < nbk) {
    const int c = tid;
    for (int r = 0; r < nbk; ++r) {
      cpx<double> s = mk(r == c ? 1.0 : 0.0, 0.0);
      for (int u = c; u < r; ++u) s = s - cmul(L[r][u], Wi[u][c]);
      Wi[r][c] = r >= c ? cmul(s, mk(1.0 / L[r][r].x, 0.0)) : mk(0.0, 0.0);
    }
  }
  __syncthreads();
  if (i < nbk && j < nbk) {
    A[(size_t)(k + i) * N + k + j] = j <= i ? L[i][j] : mk(0.0, 0.0);
    Lw[i * CB + j] = Wi[i][j];  // L11^-1, lower
  }
}

// rows below the block: L21 = A21 L11^-H, i.e. l_i = a_i (L11^-1)^H; also R = L21^H
__global__ void k_chol_panel(cpx<double>* __restrict__ A, int N, int k,
                             const cpx<double>* __restrict__ Lw, cpx<double>* __restrict__ R) {
  const int nbk = min(CB, N - k);
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int rows = N - k - nbk;
  if (e >= rows * nbk) return;
  const int i = k + nbk + e / nbk, t = e % nbk;
  // sum_u a_iu conj(W[t][u]), W = L11^-1 lower
  cpx<double> s = mk(0.0, 0.0);
  for (int u = 0; u <= t; ++u) s = s + cmul(A[(size_t)i * N + k + u], mk(Lw[t * CB + u].x, -Lw[t * CB + u].y));
  // written to R first: the row of A is still being read by the other t of this row
  R[(size_t)t * N + i] = mk(s.x, -s.y);
}

__global__ void k_chol_store(cpx<double>* __restrict__ A, int N, int k,
                             const cpx<double>* __restrict__ R) {
  const int nbk = min(CB, N - k);
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int rows = N - k - nbk;
  if (e >= rows * nbk) return;
  const int i = k + nbk + e / nbk, t = e % nbk;
  const cpx<double> r = R[(size_t)t * N + i];
  A[(size_t)i * N + k + t] = mk(r.x, -r.y);
}

__global__ void __launch_bounds__(256) k_chol_update(cpx<double>* __restrict__ A, int N, int k,
                                                     const cpx<double>* __restrict__ R) {
  const int nbk = min(CB, N - k);
  const int s = k + nbk, rest = N - s;
  const int i0 = blockIdx.y * ZTM, j0 = blockIdx.x * ZTM;
  if (i0 >= rest || j0 >= rest) return;
  // A22 -= L21 L21^H, L21 = A[s:, k:k+nbk] (ld N), L21^H = R[:, s:] (ld N)
  zgemm_tile(rest, rest, nbk, -1.0, 1.0, A + (size_t)s * N + k, N, R + s, N, A + (size_t)s * N + s, N,
             i0, j0);
}

}  // namespace gw

// ------------------------------------------------------------------ network object
struct gw_mlp {
  gw_ctx* ctx = nullptr;
  int nin = 0, width = 0, depth = 0, nout = 0;
  std::vector<int> din, dout;          // per linear layer (padded)
  std::vector<size_t> woff, boff;      // offsets (floats) into the flat parameter arrays
  size_t count = 0;
  float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  long long step = 0;
  bool ready = false;                  // trained or loaded
  double tol = 1e-4;                   // INFER with chi0_full: largest accepted rel_F
  char* act = nullptr;                 // activations and scratch
  size_t act_cap = 0;
};

namespace gw {

void mlp_free(gw_mlp* n) {
  if (n->p) (void)hipFree(n->p);
  if (n->act) (void)hipFree(n->act);
  delete n;
}

static uint64_t splitmix64(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <bool TA, bool TB, int EPI>
static gw_status bgemm(gw_ctx* c, int M, int N, int K, const float* A, int lda, const float* B,
                       int ldb, float* C, int ldc, const float* bias, float* Zout,
                       const float* Zin, int splits, long long cstride, const char* name) {
  const int kchunk = ((K + splits - 1) / splits + 31) / 32 * 32;
  dim3 g((N + 63) / 64, (M + 63) / 64, splits);
  ProfScope ps(c, name);
  hipLaunchKernelGGL((k_bgemm<TA, TB, EPI>), g, dim3(256), 0, c->stream, M, N, K, A, lda, B, ldb,
                     C, ldc, bias, Zout, Zin, kchunk, cstride);
  GW_CHECK_LAUNCH(c, "k_bgemm");
  return GW_OK;
}

// activation layout (floats): X[npad][KPAD]; Z_l, H_l [npad][width] for l < depth;
// Y, dY [npad][OPAD]; dZa, dZb [npad][width]; T [npad][2]; split partials; loss partials
struct ClBufs {
  float *X, *Y, *dY, *dZa, *dZb, *T, *part, *bpart;
  std::vector<float*> Z, H;
  double *lpart, *loss, *scale, *rpart, *rsum;
  cpx<double>* chol;
  cpx<double>* R;
  cpx<double>* Lw;
};

static constexpr int kSplits = 32;
static constexpr int kRowChunks = 64;
static constexpr int kRelBlocks = 256;  // workgroups of the fixed-order rel_F reduction

static gw_status cl_buffers(gw_mlp* net, int N, long long npad, ClBufs* b) {
  gw_ctx* c = net->ctx;
  const size_t w = net->width;
  std::vector<std::pair<void**, size_t>> parts;
  b->Z.assign(net->depth, nullptr);
  b->H.assign(net->depth, nullptr);
  parts.push_back({reinterpret_cast<void**>(&b->X), (size_t)npad * CL_KPAD * 4});
  for (int l = 0; l < net->depth; ++l) {
    parts.push_back({reinterpret_cast<void**>(&b->Z[l]), (size_t)npad * w * 4});
    parts.push_back({reinterpret_cast<void**>(&b->H[l]), (size_t)npad * w * 4});
  }
  parts.push_back({reinterpret_cast<void**>(&b->Y), (size_t)npad * CL_OPAD * 4});
  parts.push_back({reinterpret_cast<void**>(&b->dY), (size_t)npad * CL_OPAD * 4});
  parts.push_back({reinterpret_cast<void**>(&b->dZa), (size_t)npad * w * 4});
  parts.push_back({reinterpret_cast<void**>(&b->dZb), (size_t)npad * w * 4});
  parts.push_back({reinterpret_cast<void**>(&b->T), (size_t)npad * 2 * 4});
  parts.push_back({reinterpret_cast<void**>(&b->part), (size_t)kSplits * w * w * 4});
  parts.push_back({reinterpret_cast<void**>(&b->bpart), (size_t)kRowChunks * w * 4});
  parts.push_back({reinterpret_cast<void**>(&b->lpart), (size_t)((npad + 255) / 256) * 8});
  parts.push_back({reinterpret_cast<void**>(&b->loss), 8});
  parts.push_back({reinterpret_cast<void**>(&b->scale), 8});
  parts.push_back({reinterpret_cast<void**>(&b->rpart), 2 * kRelBlocks * 8});
  parts.push_back({reinterpret_cast<void**>(&b->rsum), 2 * 8});
  parts.push_back({reinterpret_cast<void**>(&b->chol), (size_t)N * N * 16});
  parts.push_back({reinterpret_cast<void**>(&b->R), (size_t)CB * N * 16});
  parts.push_back({reinterpret_cast<void**>(&b->Lw), (size_t)CB * CB * 16});
  size_t total = 0;
  for (auto& p : parts) total += align_up(p.second);
  if (total > net->act_cap) {
    if (net->act) {
      GW_HIP(c, hipStreamSynchronize(c->stream));
      (void)hipFree(net->act);
      net->act = nullptr;
      net->act_cap = 0;
    }
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, total);
    if (e != hipSuccess) return fail(c, GW_ENOMEM, "closure workspace of %zu bytes", total);
    net->act = static_cast<char*>(q);
    net->act_cap = total;
  }
  size_t off = 0;
  for (auto& p : parts) {
    *p.first = net->act + off;
    off += align_up(p.second);
  }
  return GW_OK;
}

static gw_status cl_forward(gw_mlp* net, long long npad, ClBufs& b) {
  gw_ctx* c = net->ctx;
  gw_status st;
  const float* h = b.X;
  int ld = CL_KPAD;
  for (int l = 0; l < net->depth; ++l) {
    st = bgemm<false, true, EPI_BIAS_SILU>(c, (int)npad, net->dout[l], net->din[l], h, ld,
                                          net->p + net->woff[l], net->din[l], b.H[l],
                                          net->dout[l], net->p + net->boff[l], b.Z[l], nullptr, 1,
                                          0, "closure_fwd");
    if (st != GW_OK) return st;
    h = b.H[l];
    ld = net->dout[l];
  }
  const int L = net->depth;
  return bgemm<false, true, EPI_BIAS>(c, (int)npad, net->dout[L], net->din[L], h, ld,
                                      net->p + net->woff[L], net->din[L], b.Y, CL_OPAD,
                                      net->p + net->boff[L], nullptr, nullptr, 1, 0, "closure_fwd");
}

// gradients of the loss already expressed in dY into net->g
static gw_status cl_backward(gw_mlp* net, long long npad, ClBufs& b) {
  gw_ctx* c = net->ctx;
  gw_status st;
  const int L = net->depth;
  float* dz = b.dY;        // gradient w.r.t. the current layer's output (pre-activation)
  int ldz = CL_OPAD;
  for (int l = L; l >= 0; --l) {
    const int din = net->din[l], dout = net->dout[l];
    const float* hin = l == 0 ? b.X : b.H[l - 1];
    // dW_l = dz^T hin  (split over rows)
    st = bgemm<true, false, EPI_STORE>(c, dout, din, (int)npad, dz, ldz, hin, din, b.part, din,
                                       nullptr, nullptr, nullptr, kSplits,
                                       (long long)dout * din, "closure_wgrad");
    if (st != GW_OK) return st;
    {
      ProfScope ps(c, "closure_reduce");
      const size_t n = (size_t)dout * din;
      hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream,
                         b.part, kSplits, n, net->g + net->woff[l]);
      GW_CHECK_LAUNCH(c, "k_sum_splits");
      const long long rchunk = (npad + kRowChunks - 1) / kRowChunks;
      hipLaunchKernelGGL(k_colsum, dim3((dout + 255) / 256, kRowChunks), dim3(256), 0, c->stream,
                         dz, npad, dout, rchunk, b.bpart);
      GW_CHECK_LAUNCH(c, "k_colsum");
      hipLaunchKernelGGL(k_sum_splits, dim3((dout + 255) / 256), dim3(256), 0, c->stream, b.bpart,
                         kRowChunks, (size_t)dout, net->g + net->boff[l]);
      GW_CHECK_LAUNCH(c, "k_sum_splits");
    }
    if (l == 0) break;
    // d(pre-activation of layer l-1) = (dz W_l) * SiLU'(Z_{l-1})
    float* nd = (dz == b.dZa) ? b.dZb : b.dZa;
    st = bgemm<false, false, EPI_DSILU>(c, (int)npad, din, dout, dz, ldz, net->p + net->woff[l],
                                        din, nd, din, nullptr, nullptr, b.Z[l - 1], 1, 0,
                                        "closure_bwd");
    if (st != GW_OK) return st;
    dz = nd;
    ldz = din;
  }
  return GW_OK;
}

// Per workgroup, in a fixed order: the sums of |a - b|^2 and of |b|^2 over
// the elements i = blockIdx.x * 256 + threadIdx.x + k * gridDim.x * 256, into
// part[blockIdx.x] and part[gridDim.x + blockIdx.x].
__global__ void __launch_bounds__(256) k_relf_part(const cpx<double>* __restrict__ a,
                                                   const cpx<double>* __restrict__ b, size_t n,
                                                   double* __restrict__ part) {
  __shared__ double sd[256], sr[256];
  double d = 0.0, r = 0.0;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    const cpx<double> x = a[i], y = b[i];
    const double ex = x.x - y.x, ey = x.y - y.y;
    d += ex * ex + ey * ey;
    r += y.x * y.x + y.y * y.y;
  }
  sd[threadIdx.x] = d;
  sr[threadIdx.x] = r;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) {
      sd[threadIdx.x] += sd[threadIdx.x + k];
      sr[threadIdx.x] += sr[threadIdx.x + k];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x] = sd[0];
    part[gridDim.x + blockIdx.x] = sr[0];
  }
}

// rel_F(a, b) = ||a - b||_F / ||b||_F over N x N complex doubles, reduced on the
// device in a fixed order (the same inputs give the same bits); synchronises.
static gw_status cl_rel_f(gw_ctx* c, int N, const double* a, const double* b, ClBufs& bf,
                          double* rel) {
  const size_t nn = (size_t)N * N;
  {
    ProfScope ps(c, "closure_judge");
    hipLaunchKernelGGL(k_relf_part, dim3(kRelBlocks), dim3(256), 0, c->stream,
                       reinterpret_cast<const cpx<double>*>(a),
                       reinterpret_cast<const cpx<double>*>(b), nn, bf.rpart);
    GW_CHECK_LAUNCH(c, "k_relf_part");
    hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(256), 0, c->stream, bf.rpart, kRelBlocks, bf.rsum);
    GW_CHECK_LAUNCH(c, "k_sum_f64");
    hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(256), 0, c->stream, bf.rpart + kRelBlocks,
                       kRelBlocks, bf.rsum + 1);
    GW_CHECK_LAUNCH(c, "k_sum_f64");
  }
  double h[2] = {0.0, 0.0};
  GW_HIP(c, hipMemcpyAsync(h, bf.rsum, sizeof h, hipMemcpyDeviceToHost, c->stream));
  GW_HIP(c, hipStreamSynchronize(c->stream));
  *rel = h[1] > 0.0 ? std::sqrt(h[0] / h[1]) : (h[0] > 0.0 ? INFINITY : 0.0);
  return GW_OK;
}

static gw_status cl_cholesky_fails(gw_ctx* c, int N, const double* chi, ClBufs& b, bool* fails) {
  const size_t nn = (size_t)N * N;
  {
    ProfScope ps(c, "closure_chol");
    hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(1), 0, c->stream, c->d_flag + 2, 0);
    GW_CHECK_LAUNCH(c, "k_set_i32");
    hipLaunchKernelGGL(k_chol_neg, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, c->stream,
                       reinterpret_cast<const cpx<double>*>(chi), b.chol, nn);
    GW_CHECK_LAUNCH(c, "k_chol_neg");
    for (int k = 0; k < N; k += CB) {
      const int nbk = std::min(CB, N - k), rest = N - k - nbk;
      hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(1024), 0, c->stream, b.chol, N, k, b.Lw,
                         c->d_flag + 2);
      GW_CHECK_LAUNCH(c, "k_chol_diag");
      if (rest <= 0) break;
      hipLaunchKernelGGL(k_chol_panel, dim3((rest * nbk + 255) / 256), dim3(256), 0, c->stream,
                         b.chol, N, k, b.Lw, b.R);
      GW_CHECK_LAUNCH(c, "k_chol_panel");
      hipLaunchKernelGGL(k_chol_store, dim3((rest * nbk + 255) / 256), dim3(256), 0, c->stream,
                         b.chol, N, k, b.R);
      GW_CHECK_LAUNCH(c, "k_chol_store");
      const int t = (rest + ZTM - 1) / ZTM;
      hipLaunchKernelGGL(k_chol_update, dim3(t, t), dim3(256), 0, c->stream, b.chol, N, k, b.R);
      GW_CHECK_LAUNCH(c, "k_chol_update");
    }
  }
  int flag = 0;
  GW_HIP(c, hipMemcpyAsync(&flag, c->d_flag + 2, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  GW_HIP(c, hipStreamSynchronize(c->stream));
  *fails = flag != 0;
  return GW_OK;
}

}  // namespace gw

using namespace gw;

extern "C" {

gw_status gw_mlp_create(gw_ctx* c, gw_mlp** out, int nin, int width, int depth, int nout,
                        uint64_t seed) {
  if (!c || !out) return GW_EINVAL;
  *out = nullptr;
  c->err.clear();
  if (nin < 1 || nin > CL_KPAD || nout < 1 || nout > CL_OPAD || width < 64 || width % 64 ||
      width > 4096 || depth < 1 || depth > 8)
    return fail(c, GW_EINVAL, "network shape: 1<=nin<=32, 1<=nout<=32, width a multiple of 64 "
                              "(<=4096), 1<=depth<=8");
  gw_mlp* n = new gw_mlp();
  n->ctx = c;
  n->nin = nin;
  n->width = width;
  n->depth = depth;
  n->nout = nout;
  for (int l = 0; l <= depth; ++l) {
    n->din.push_back(l == 0 ? CL_KPAD : width);
    n->dout.push_back(l == depth ? CL_OPAD : width);
  }
  for (int l = 0; l <= depth; ++l) {
    n->woff.push_back(n->count);
    n->count += (size_t)n->din[l] * n->dout[l];
    n->boff.push_back(n->count);
    n->count += n->dout[l];
  }
  // Glorot-uniform weights on the real fan-in/fan-out (splitmix64 uniforms);
  // padded rows and columns and every bias start (and stay) at zero
  std::vector<float> h(n->count, 0.f);
  uint64_t s = seed;
  for (int l = 0; l <= depth; ++l) {
    const int ri = l == 0 ? nin : width, ro = l == depth ? nout : width;
    const double lim = std::sqrt(6.0 / (ri + ro));
    for (int o = 0; o < ro; ++o)
      for (int i = 0; i < ri; ++i) {
        const double u = (double)(splitmix64(s) >> 11) * (1.0 / 9007199254740992.0);
        h[n->woff[l] + (size_t)o * n->din[l] + i] = (float)((2.0 * u - 1.0) * lim);
      }
  }
  void* mem = nullptr;
  if (hipMalloc(&mem, 4 * n->count * sizeof(float)) != hipSuccess) {
    delete n;
    return fail(c, GW_ENOMEM, "network parameters");
  }
  n->p = static_cast<float*>(mem);
  n->g = n->p + n->count;
  n->m = n->g + n->count;
  n->v = n->m + n->count;
  hipError_t e = hipMemcpy(n->p, h.data(), n->count * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(n->g, 0, 3 * n->count * 4);
  if (e != hipSuccess) {
    (void)hipFree(mem);
    delete n;
    return hip_fail(c, e, "network init");
  }
  c->mlps.insert(n);
  *out = n;
  return GW_OK;
}

gw_status gw_mlp_set_tolerance(gw_mlp* n, double tol) {
  if (!n) return GW_EINVAL;
  if (!(tol >= 0.0) || !std::isfinite(tol))
    return fail(n->ctx, GW_EINVAL, "the closure tolerance must be finite and >= 0");
  n->tol = tol;
  return GW_OK;
}

gw_status gw_mlp_destroy(gw_mlp* n) {
  if (!n) return GW_EINVAL;
  (void)hipStreamSynchronize(n->ctx->stream);
  n->ctx->mlps.erase(n);
  gw::mlp_free(n);
  return GW_OK;
}

// layout: u32 magic, u32 version, i32 nin, width, depth, nout, kpad, opad,
//         i64 step, i64 count, then float params[count], m[count], v[count]
gw_status gw_mlp_save(const gw_mlp* n, void* buf, size_t* nbytes) {
  if (!n || !nbytes) return GW_EINVAL;
  const size_t need = 48 + 3 * n->count * 4;
  if (!buf) { *nbytes = need; return GW_OK; }
  if (*nbytes < need) return fail(n->ctx, GW_EINVAL, "buffer of %zu bytes, %zu needed", *nbytes, need);
  char* b = static_cast<char*>(buf);
  uint32_t hdr[2] = {CL_MAGIC, 1};
  int32_t dims[6] = {n->nin, n->width, n->depth, n->nout, CL_KPAD, CL_OPAD};
  int64_t tail[2] = {n->step, (int64_t)n->count};
  std::memcpy(b, hdr, 8);
  std::memcpy(b + 8, dims, 24);
  std::memcpy(b + 32, tail, 16);
  hipError_t e = hipStreamSynchronize(n->ctx->stream);
  if (e == hipSuccess) e = hipMemcpy(b + 48, n->p, n->count * 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(b + 48 + n->count * 4, n->m, n->count * 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(b + 48 + 2 * n->count * 4, n->v, n->count * 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(n->ctx, e, "gw_mlp_save");
  *nbytes = need;
  return GW_OK;
}

gw_status gw_mlp_load(gw_mlp* n, const void* buf, size_t nbytes) {
  if (!n || !buf) return GW_EINVAL;
  const char* b = static_cast<const char*>(buf);
  if (nbytes < 48) return fail(n->ctx, GW_EINVAL, "buffer too short");
  uint32_t hdr[2];
  int32_t dims[6];
  int64_t tail[2];
  std::memcpy(hdr, b, 8);
  std::memcpy(dims, b + 8, 24);
  std::memcpy(tail, b + 32, 16);
  if (hdr[0] != CL_MAGIC || hdr[1] != 1) return fail(n->ctx, GW_EINVAL, "not a saved network");
  if (dims[0] != n->nin || dims[1] != n->width || dims[2] != n->depth || dims[3] != n->nout ||
      dims[4] != CL_KPAD || dims[5] != CL_OPAD || tail[1] != (int64_t)n->count)
    return fail(n->ctx, GW_EINVAL, "saved network has another shape");
  if (nbytes < 48 + 3 * n->count * 4) return fail(n->ctx, GW_EINVAL, "buffer too short");
  hipError_t e = hipStreamSynchronize(n->ctx->stream);
  if (e == hipSuccess) e = hipMemcpy(n->p, b + 48, n->count * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(n->m, b + 48 + n->count * 4, n->count * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(n->v, b + 48 + 2 * n->count * 4, n->count * 4, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(n->ctx, e, "gw_mlp_load");
  n->step = tail[0];
  n->ready = true;
  return GW_OK;
}

gw_status gw_chi0_closure(gw_ctx* c, gw_mlp* net, int mode, int N, const double* qG,
                          const double* chi0_trunc, double gap, double emax,
                          const double* chi0_full, float lr, float* loss, double* chi0_out) {
  if (!c) return GW_EINVAL;
  c->err.clear();
  if (mode != GW_CLOSURE_INFER && mode != GW_CLOSURE_TRAIN_STEP && mode != GW_CLOSURE_FULL_FALLBACK)
    return fail(c, GW_EINVAL, "unknown closure mode");
  if (N <= 0 || N > 16384) return fail(c, GW_EINVAL, "neps must be in 1..16384");
  (void)hipSetDevice(c->device);
  const size_t nn = (size_t)N * N;
  if (mode == GW_CLOSURE_FULL_FALLBACK) {
    if (!chi0_full || !chi0_out) return fail(c, GW_EINVAL, "FULL_FALLBACK needs chi0_full and chi0_out");
    GW_HIP(c, hipMemcpyAsync(chi0_out, chi0_full, nn * 16, hipMemcpyDeviceToDevice, c->stream));
    return GW_OK;
  }
  if (!net || net->ctx != c) return fail(c, GW_EINVAL, "network missing or from another context");
  if (net->nin != CL_NFEAT || net->nout != CL_NOUT)
    return fail(c, GW_EINVAL, "the closure network maps %d features to %d outputs", CL_NFEAT, CL_NOUT);
  if (!qG || !chi0_trunc) return fail(c, GW_EINVAL, "NULL qG or chi0_trunc");
  if (mode == GW_CLOSURE_TRAIN_STEP && !chi0_full) return fail(c, GW_EINVAL, "training needs chi0_full");
  if (mode == GW_CLOSURE_INFER && !chi0_out) return fail(c, GW_EINVAL, "INFER needs chi0_out");
  if (mode == GW_CLOSURE_INFER && !net->ready)
    return fail(c, GW_ENOTTRAINED, "the network has not been trained or loaded");
  if (!(lr >= 0.f) && mode == GW_CLOSURE_TRAIN_STEP) return fail(c, GW_EINVAL, "negative learning rate");
  const long long n = (long long)N * (N + 1) / 2;
  const long long npad = (n + CL_RT - 1) / CL_RT * CL_RT;
  ClBufs b;
  gw_status st = cl_buffers(net, N, npad, &b);
  if (st != GW_OK) return st;
  const cpx<double>* ct = reinterpret_cast<const cpx<double>*>(chi0_trunc);
  const cpx<double>* cf = reinterpret_cast<const cpx<double>*>(chi0_full);
  {
    ProfScope ps(c, "closure_features");
    hipLaunchKernelGGL(k_cl_scale, dim3(1), dim3(256), 0, c->stream, ct, N, b.scale);
    GW_CHECK_LAUNCH(c, "k_cl_scale");
    hipLaunchKernelGGL(k_cl_features, dim3((unsigned)((npad + 255) / 256)), dim3(256), 0,
                       c->stream, qG, ct, mode == GW_CLOSURE_TRAIN_STEP ? cf : nullptr, N, n, npad,
                       gap, emax, b.scale, b.X, mode == GW_CLOSURE_TRAIN_STEP ? b.T : nullptr);
    GW_CHECK_LAUNCH(c, "k_cl_features");
  }
  if ((st = cl_forward(net, npad, b)) != GW_OK) return st;
  if (mode == GW_CLOSURE_TRAIN_STEP) {
    const int nblk = (int)((npad + 255) / 256);
    {
      ProfScope ps(c, "closure_loss");
      hipLaunchKernelGGL(k_cl_dy, dim3(nblk), dim3(256), 0, c->stream, b.Y, b.T, n, npad, b.dY,
                         b.lpart);
      GW_CHECK_LAUNCH(c, "k_cl_dy");
      hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(256), 0, c->stream, b.lpart, nblk, b.loss);
      GW_CHECK_LAUNCH(c, "k_sum_f64");
    }
    if ((st = cl_backward(net, npad, b)) != GW_OK) return st;
    net->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float bc1 = 1.f - std::pow(b1, (float)net->step), bc2 = 1.f - std::pow(b2, (float)net->step);
    {
      ProfScope ps(c, "closure_adam");
      hipLaunchKernelGGL(k_adam, dim3((unsigned)((net->count + 255) / 256)), dim3(256), 0,
                         c->stream, net->p, net->g, net->m, net->v, net->count, lr, b1, b2, 1e-8f,
                         bc1, bc2);
      GW_CHECK_LAUNCH(c, "k_adam");
    }
    net->ready = true;
    if (loss) {
      double l = 0.0;
      GW_HIP(c, hipMemcpyAsync(&l, b.loss, 8, hipMemcpyDeviceToHost, c->stream));
      GW_HIP(c, hipStreamSynchronize(c->stream));
      *loss = (float)(l / ((double)n * CL_NOUT));
    }
    return GW_OK;
  }
  // INFER
  {
    ProfScope ps(c, "closure_apply");
    hipLaunchKernelGGL(k_cl_apply, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, ct,
                       b.Y, N, n, b.scale, reinterpret_cast<cpx<double>*>(chi0_out));
    GW_CHECK_LAUNCH(c, "k_cl_apply");
  }
  if (chi0_full) {
    // the full sum judges the prediction: it is kept only if it is within the
    // network's tolerance of the full sum and negative semidefinite
    double rel = 0.0;
    if ((st = cl_rel_f(c, N, chi0_out, chi0_full, b, &rel)) != GW_OK) return st;
    bool fails = !(rel <= net->tol);
    if (!fails && (st = cl_cholesky_fails(c, N, chi0_out, b, &fails)) != GW_OK) return st;
    if (fails) {
      GW_HIP(c, hipMemcpyAsync(chi0_out, chi0_full, nn * 16, hipMemcpyDeviceToDevice, c->stream));
      return GW_EFALLBACK;
    }
  }
  return GW_OK;
}

}  // extern "C"
