// FFT stage of the spinor matrix elements (Sec. II, Eq. (matrix_el)).
//
//   band_to_grid : sphere coefficients -> periodic spinor components on the grid
//                  u(r_j) = sum_G c(G) exp(+2 pi i g.j/n)            (input-pruned 3D FFT)
//   pair_to_eps  : rho_vc = sum_s conj(u_v^s) u_c^s, then
//                  M_vc(G) = (1/N) sum_j rho_vc(r_j) exp(+2 pi i g.j/n)  on the eps sphere
//                  (output-pruned 3D FFT; the spin sum is fused into the product)
//
// Layout: u[band][spin][x][y][z] (z fastest).  Each 3D transform is split into
// an x-pass over pencils of the compact (y,z) cube and a plane pass that does
// the y and z transforms of one x-plane inside LDS, so a plane crosses HBM once.
// Pruning keeps only the |g_i| <= gmax_i rows/columns of the transforms whose
// input (band) or output (pair) is confined to a sphere.
#include "common.h"
#include "regfft.h"

#include <cmath>

namespace gw {

// ---------------------------------------------------------------- host tables
FftPlan make_fft_plan(int n) {
  FftPlan p{};
  p.n = n;
  p.npass = 0;
  int m = n;
  while (m % 4 == 0) { p.radix[p.npass++] = 4; m /= 4; }
  while (m % 2 == 0) { p.radix[p.npass++] = 2; m /= 2; }
  while (m % 3 == 0) { p.radix[p.npass++] = 3; m /= 3; }
  while (m % 5 == 0) { p.radix[p.npass++] = 5; m /= 5; }
  if (m != 1) p.npass = -1;
  return p;
}

// exp(+2 pi i m / n) in double with the argument reduced to [0, pi/4] by exact
// integer quadrant/octant folding, so every entry is within ~1 ulp.
static void unit_root(int m, int n, double* c, double* s) {
  m %= n;
  if (m < 0) m += n;
  long long q = (4LL * m) / n;            // quadrant
  long long rem = 4LL * m - q * n;        // angle within quadrant = (pi/2) rem / n
  double cc, ss;
  if (2 * rem <= n) {
    double a = (M_PI / 2.0) * (double)rem / (double)n;
    cc = std::cos(a); ss = std::sin(a);
  } else {
    double a = (M_PI / 2.0) * (double)(n - rem) / (double)n;
    cc = std::sin(a); ss = std::cos(a);
  }
  switch (q) {
    case 0: *c = cc; *s = ss; break;
    case 1: *c = -ss; *s = cc; break;
    case 2: *c = -cc; *s = -ss; break;
    default: *c = ss; *s = -cc; break;
  }
}

gw_status twiddle_table(gw_ctx* c, int n, bool dbl, const void** out) {
  auto key = std::make_pair(n, dbl ? 1 : 0);
  auto it = c->twiddles.find(key);
  if (it != c->twiddles.end()) { *out = it->second; return GW_OK; }
  std::vector<double> h(2 * (size_t)n);
  for (int m = 0; m < n; ++m) unit_root(m, n, &h[2 * m], &h[2 * m + 1]);
  void* d = nullptr;
  size_t bytes = (size_t)n * (dbl ? 16 : 8);
  GW_HIP(c, hipMalloc(&d, bytes));
  if (dbl) {
    GW_HIP(c, hipMemcpy(d, h.data(), bytes, hipMemcpyHostToDevice));
  } else {
    std::vector<float> f(2 * (size_t)n);
    for (size_t i = 0; i < f.size(); ++i) f[i] = (float)h[i];
    GW_HIP(c, hipMemcpy(d, f.data(), bytes, hipMemcpyHostToDevice));
  }
  c->twiddles[key] = d;
  *out = d;
  return GW_OK;
}

// ---------------------------------------------------------------- radix kernels
// y_k = sum_j a_j exp(+2 pi i j k / R), R fixed at compile time so the
// butterfly stays in registers.
template <typename T, int R>
__device__ __forceinline__ void dft(cpx<T>* a) {
  if constexpr (R == 4) {
    cpx<T> t0 = a[0] + a[2], t1 = a[0] - a[2];
    cpx<T> t2 = a[1] + a[3], t3 = mul_i(a[1] - a[3]);
    a[0] = t0 + t2; a[2] = t0 - t2;
    a[1] = t1 + t3; a[3] = t1 - t3;
  } else if constexpr (R == 2) {
    cpx<T> t = a[0];
    a[0] = t + a[1]; a[1] = t - a[1];
  } else if constexpr (R == 3) {
    const T h = (T)0.86602540378443864676;  // sin(2 pi / 3)
    cpx<T> t1 = a[1] + a[2];
    cpx<T> t2 = a[0] - scal(t1, (T)0.5);
    cpx<T> t3 = scal(mul_i(a[1] - a[2]), h);
    a[0] = a[0] + t1;
    a[1] = t2 + t3;
    a[2] = t2 - t3;
  } else {  // R == 5
    const T c1 = (T)0.30901699437494742410, s1 = (T)0.95105651629515357212;   // 2 pi / 5
    const T c2 = (T)-0.80901699437494742410, s2 = (T)0.58778525229247312917;  // 4 pi / 5
    cpx<T> t1 = a[1] + a[4], t2 = a[2] + a[3];
    cpx<T> t3 = a[1] - a[4], t4 = a[2] - a[3];
    cpx<T> b1 = a[0] + scal(t1, c1) + scal(t2, c2);
    cpx<T> b2 = a[0] + scal(t1, c2) + scal(t2, c1);
    cpx<T> d1 = mul_i(scal(t3, s1) + scal(t4, s2));
    cpx<T> d2 = mul_i(scal(t3, s2) - scal(t4, s1));
    a[0] = a[0] + t1 + t2;
    a[1] = b1 + d1; a[4] = b1 - d1;
    a[2] = b2 + d2; a[3] = b2 - d2;
  }
}

// One Stockham pass of radix R over `npen` pencils (element i of pencil b at
// buf[off(b) + i*es]); Ns = product of the radices already applied.  Every
// butterfly of a group of whole pencils is read into registers before any is
// written, so the pass runs in place.  Ends with a barrier.
template <typename T, int R, int MAXB, typename Off>
__device__ __forceinline__ void stockham_pass(cpx<T>* buf, int npen, int es, Off off, int n,
                                              int Ns, const cpx<T>* __restrict__ tw) {
  constexpr int nt = 256;  // every FFT kernel runs 256-thread workgroups
  const int nq = n / R;
  const int tws = n / (Ns * R);
  int gp = (nt * MAXB) / nq;
  if (gp < 1) gp = 1;
  for (int p0 = 0; p0 < npen; p0 += gp) {
    const int pend = min(npen, p0 + gp);
    const int tbeg = p0 * nq, tend = pend * nq;
    cpx<T> v[MAXB][R];
#pragma unroll
    for (int u = 0; u < MAXB; ++u) {
      const int t = tbeg + u * nt + (int)threadIdx.x;
      if (t < tend) {
        const int b = t / nq, j = t - b * nq;
        const int o = off(b);
        const int k = j % Ns;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          cpx<T> a = buf[o + (j + r * nq) * es];
          if (r != 0 && k != 0) a = cmul(a, tw[r * k * tws]);
          v[u][r] = a;
        }
        dft<T, R>(v[u]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < MAXB; ++u) {
      const int t = tbeg + u * nt + (int)threadIdx.x;
      if (t < tend) {
        const int b = t / nq, j = t - b * nq;
        const int o = off(b);
        const int k = j % Ns;
        const int d = (j / Ns) * Ns * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) buf[o + (d + r * Ns) * es] = v[u][r];
      }
    }
    __syncthreads();
  }
}

// Batched in-LDS transform y_k = sum_j x_j exp(+2 pi i jk/n) of `npen` pencils.
template <typename T, int MAXB, typename Off>
__device__ void lds_fft(cpx<T>* buf, int npen, int es, Off off, const FftPlan& pl,
                        const cpx<T>* __restrict__ tw) {
  int Ns = 1;
  for (int s = 0; s < pl.npass; ++s) {
    const int R = pl.radix[s];
    if (R == 4) stockham_pass<T, 4, MAXB>(buf, npen, es, off, pl.n, Ns, tw);
    else if (R == 2) stockham_pass<T, 2, MAXB>(buf, npen, es, off, pl.n, Ns, tw);
    else if (R == 3) stockham_pass<T, 3, MAXB>(buf, npen, es, off, pl.n, Ns, tw);
    else stockham_pass<T, 5, MAXB>(buf, npen, es, off, pl.n, Ns, tw);
    Ns *= R;
  }
}

// Compile-time radix plan (same order as make_fft_plan) for pencil lengths
// known when the kernel is built: every divisor in the pass index math is then a
// constant.
constexpr int cx_npass(int n) {
  int c = 0;
  while (n % 4 == 0) { n /= 4; ++c; }
  while (n % 2 == 0) { n /= 2; ++c; }
  while (n % 3 == 0) { n /= 3; ++c; }
  while (n % 5 == 0) { n /= 5; ++c; }
  return n == 1 ? c : -1;
}
constexpr int cx_radix(int n, int s) {
  int c = 0;
  while (n % 4 == 0) { n /= 4; if (c++ == s) return 4; }
  while (n % 2 == 0) { n /= 2; if (c++ == s) return 2; }
  while (n % 3 == 0) { n /= 3; if (c++ == s) return 3; }
  while (n % 5 == 0) { n /= 5; if (c++ == s) return 5; }
  return 0;
}

template <typename T, int N, int S, int NSC, int MAXB, typename Off>
__device__ __forceinline__ void fft_ct(cpx<T>* buf, int npen, int es, Off off,
                                       const cpx<T>* __restrict__ tw) {
  if constexpr (S < cx_npass(N)) {
    constexpr int R = cx_radix(N, S);
    stockham_pass<T, R, MAXB>(buf, npen, es, off, N, NSC, tw);
    fft_ct<T, N, S + 1, NSC * R, MAXB>(buf, npen, es, off, tw);
  }
}

// N > 0: length fixed at build time; N == 0: the runtime plan.
template <typename T, int N, int MAXB, typename Off>
__device__ __forceinline__ void fft_any(cpx<T>* buf, int npen, int es, Off off,
                                        const FftPlan& pl, const cpx<T>* __restrict__ tw) {
  if constexpr (N > 0) {
    static_assert(cx_npass(N) > 0, "length must factor into 2, 3, 5");
    fft_ct<T, N, 0, 1, MAXB>(buf, npen, es, off, tw);
  } else {
    lds_fft<T, MAXB>(buf, npen, es, off, pl, tw);
  }
}

constexpr int kThreads = 256;
constexpr int kMaxB = 4;

__device__ __forceinline__ int wrap(int g, int n) { return g < 0 ? g + n : g; }

// The pair kernels' logical order (xcd_linear) is x-plane major, so one XCD
// walks a few x-planes and keeps their valence planes resident in its L2 while
// the conduction planes stream through once.

// ---------------------------------------------------------------- band transforms
// Each kernel takes its pencil lengths as template arguments (0 = runtime).

// x-pass from the sphere: for each compact column (jy,jz) gather the |gx|<=gmax
// coefficients, transform along x, write T1[bs][x][col].
template <typename T, int N1>
__global__ void __launch_bounds__(kThreads) k_band_x(
    const cpx<T>* __restrict__ coef, int ng, const int* __restrict__ cube, int ex, int ey,
    int ez, int gx, int n1_rt, int ncol, int CH, FftPlan pl, const cpx<T>* __restrict__ tw,
    cpx<T>* __restrict__ out) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  const int n1 = N1 ? N1 : n1_rt;
  const int bs = blockIdx.y;
  const int col0 = blockIdx.x * CH;
  const int nch = min(CH, ncol - col0);
  const cpx<T>* cf = coef + (size_t)bs * ng;
  for (int i = threadIdx.x; i < n1 * CH; i += kThreads) lds[i] = mk<T>(0, 0);
  __syncthreads();
  for (int i = threadIdx.x; i < ex * nch; i += kThreads) {
    const int jx = i / nch, cl = i - jx * nch;
    const int col = col0 + cl;
    const int jy = col / ez, jz = col - jy * ez;
    const int idx = cube[(jx * ey + jy) * ez + jz];
    if (idx >= 0) lds[wrap(jx - gx, n1) * CH + cl] = cf[idx];
  }
  __syncthreads();
  fft_any<T, N1, kMaxB>(lds, nch, CH, [](int b) { return b; }, pl, tw);
  cpx<T>* o = out + (size_t)bs * n1 * ncol;
  for (int i = threadIdx.x; i < n1 * nch; i += kThreads) {
    const int x = i / nch, cl = i - x * nch;
    o[(size_t)x * ncol + col0 + cl] = lds[x * CH + cl];
  }
}

__host__ __device__ constexpr int plane_pitch(int n3) { return (n3 % 2 == 0) ? n3 + 1 : n3; }

// plane pass: expand the compact (y,z) plane of one x, transform along y on the
// occupied z columns, then along z on every row; write the full plane.
template <typename T, int N2, int N3>
__global__ void __launch_bounds__(kThreads) k_band_plane(
    const cpx<T>* __restrict__ t1, int ey, int ez, int gy, int gz, int n1, int n2_rt, int n3_rt,
    FftPlan ply, FftPlan plz, const cpx<T>* __restrict__ twy, const cpx<T>* __restrict__ twz,
    cpx<T>* __restrict__ u) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* pl = reinterpret_cast<cpx<T>*>(smem_raw);
  const int n2 = N2 ? N2 : n2_rt, n3 = N3 ? N3 : n3_rt;
  const int P = plane_pitch(n3);
  const int x = blockIdx.x, bs = blockIdx.y;
  const int ncol = ey * ez;
  for (int i = threadIdx.x; i < n2 * P; i += kThreads) pl[i] = mk<T>(0, 0);
  __syncthreads();
  const cpx<T>* src = t1 + ((size_t)bs * n1 + x) * ncol;
  for (int i = threadIdx.x; i < ncol; i += kThreads) {
    const int jy = i / ez, jz = i - jy * ez;
    pl[wrap(jy - gy, n2) * P + wrap(jz - gz, n3)] = src[i];
  }
  __syncthreads();
  fft_any<T, N2, kMaxB>(pl, ez, P, [=](int b) { return wrap(b - gz, n3); }, ply, twy);
  fft_any<T, N3, kMaxB>(pl, n2, 1, [=](int b) { return b * P; }, plz, twz);
  cpx<T>* dst = u + ((size_t)bs * n1 + x) * (size_t)n2 * n3;
  for (int i = threadIdx.x; i < n2 * n3; i += kThreads) {
    const int y = i / n3, z = i - y * n3;
    dst[i] = pl[y * P + z];
  }
}

// ---------------------------------------------------------------- pair transforms
// plane pass: spin-summed product of one x-plane, z transform (keep |gz|<=gmax),
// y transform of the kept columns (keep |gy|<=gmax), write T2[pair][x][jy][jz].
template <typename T, int NS, int N2, int N3>
__global__ void __launch_bounds__(kThreads) k_pair_plane(
    const cpx<T>* __restrict__ uv, const cpx<T>* __restrict__ uc, int v0, int nvt, int c0,
    int n1, int n2_rt, int n3_rt, int ey, int ez, int gy, int gz, FftPlan ply, FftPlan plz,
    const cpx<T>* __restrict__ twy, const cpx<T>* __restrict__ twz, cpx<T>* __restrict__ t2,
    int npairs) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* pl = reinterpret_cast<cpx<T>*>(smem_raw);
  const int n2 = N2 ? N2 : n2_rt, n3 = N3 ? N3 : n3_rt;
  const int P = plane_pitch(n3);
  const long long lin = xcd_linear(blockIdx.x, (long long)n1 * npairs);
  if (lin < 0) return;
  const int x = (int)(lin / npairs), pr = (int)(lin % npairs);
  const int v = v0 + pr % nvt, c = c0 + pr / nvt;
  const size_t nb = (size_t)n1 * n2 * n3, np = (size_t)n2 * n3;
  const cpx<T>* pv = uv + (size_t)v * NS * nb + (size_t)x * np;
  const cpx<T>* pc = uc + (size_t)c * NS * nb + (size_t)x * np;
  for (int i = threadIdx.x; i < (int)np; i += kThreads) {
    cpx<T> acc = cmulc(pv[i], pc[i]);
    if (NS == 2) acc = acc + cmulc(pv[nb + i], pc[nb + i]);
    const int y = i / n3, z = i - y * n3;
    pl[y * P + z] = acc;
  }
  __syncthreads();
  fft_any<T, N3, kMaxB>(pl, n2, 1, [=](int b) { return b * P; }, plz, twz);
  fft_any<T, N2, kMaxB>(pl, ez, P, [=](int b) { return wrap(b - gz, n3); }, ply, twy);
  const int ncol = ey * ez;
  cpx<T>* dst = t2 + ((size_t)pr * n1 + x) * ncol;
  for (int i = threadIdx.x; i < ncol; i += kThreads) {
    const int jy = i / ez, jz = i - jy * ez;
    dst[i] = pl[wrap(jy - gy, n2) * P + wrap(jz - gz, n3)];
  }
}

// x-pass + eps gather: transform the kept (jy,jz) columns along x, keep the
// |gx|<=gmax outputs that lie on the eps sphere, scale by 1/N.
template <typename T, int N1>
__global__ void __launch_bounds__(kThreads) k_pair_x(
    const cpx<T>* __restrict__ t2, int n1_rt, int ncol, int CH, int ex, int ey, int ez, int gx,
    const int* __restrict__ emap, FftPlan plx, const cpx<T>* __restrict__ twx, T invN, int v0,
    int nvt, int c0, int nct_total, int neps, cpx<T>* __restrict__ M) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* lds = reinterpret_cast<cpx<T>*>(smem_raw);
  const int n1 = N1 ? N1 : n1_rt;
  const int col0 = blockIdx.x * CH, pr = blockIdx.y;
  const int nch = min(CH, ncol - col0);
  const cpx<T>* src = t2 + (size_t)pr * n1 * ncol;
  for (int i = threadIdx.x; i < n1 * nch; i += kThreads) {
    const int x = i / nch, cl = i - x * nch;
    lds[x * CH + cl] = src[(size_t)x * ncol + col0 + cl];
  }
  __syncthreads();
  fft_any<T, N1, kMaxB>(lds, nch, CH, [](int b) { return b; }, plx, twx);
  const int v = v0 + pr % nvt, c = c0 + pr / nvt;
  cpx<T>* dst = M + ((size_t)v * nct_total + c) * neps;
  for (int i = threadIdx.x; i < ex * nch; i += kThreads) {
    const int jx = i / nch, cl = i - jx * nch;
    const int col = col0 + cl;
    const int jy = col / ez, jz = col - jy * ez;
    const int idx = emap[(jx * ey + jy) * ez + jz];
    if (idx >= 0) dst[idx] = scal(lds[wrap(jx - gx, n1) * CH + cl], invN);
  }
}

// ---------------------------------------------------------------- two-factor plane kernels
// A pencil of length N = A*B is transformed by A threads holding B elements
// each (element t + A*m in thread t): a B-point DFT in registers, the twiddle
// exp(+2 pi i t k2 / N), one exchange through LDS, and A-point DFTs in
// registers over the B columns (thread t takes k2 = t, t+A, ...).  Output
// k = k2 + B*k1.  One LDS round trip per transform instead of one per radix.


template <int N>
__host__ __device__ constexpr int ex_pitch() { return N + 1; }

// pair plane: product, z transform keeping |gz| <= g, y transform keeping |gy| <= g
template <typename T, int NS, int N2, int N3>
__global__ void __launch_bounds__(kThreads) k_pair_plane_rf(
    const cpx<T>* __restrict__ uv, const cpx<T>* __restrict__ uc, int v0, int nvt, int c0,
    int n1, int ey, int ez, int gy, int gz, const cpx<T>* __restrict__ twy,
    const cpx<T>* __restrict__ twz, cpx<T>* __restrict__ t2, int npairs) {
  constexpr int A3 = split_n1(N3), B3 = N3 / A3, RZ = kThreads / A3, EP3 = ex_pitch<N3>();
  constexpr int A2 = split_n1(N2), B2 = N2 / A2, RY = kThreads / A2, EP2 = ex_pitch<N2>();
  constexpr int ER3 = RZ < N2 ? RZ : N2, ER2 = RY < N3 ? RY : N3;
  constexpr int ESZ = (ER3 * EP3 > ER2 * EP2) ? ER3 * EP3 : ER2 * EP2;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* E = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* Zb = E + ESZ;
  const int ZP = ez | 1;
  const long long lin = xcd_linear(blockIdx.x, (long long)n1 * npairs);
  if (lin < 0) return;
  const int x = (int)(lin / npairs), pr = (int)(lin % npairs);
  const int v = v0 + pr % nvt, c = c0 + pr / nvt;
  const size_t nb = (size_t)n1 * N2 * N3, np = (size_t)N2 * N3;
  const cpx<T>* pv = uv + (size_t)v * NS * nb + (size_t)x * np;
  const cpx<T>* pc = uc + (size_t)c * NS * nb + (size_t)x * np;
  const int tid = threadIdx.x;
  // ---- z transforms of the rows
  {
    const int rr = tid / A3, t = tid % A3;
    for (int y0 = 0; y0 < N2; y0 += RZ) {
      const int y = y0 + rr;
      const bool act = y < N2;
      cpx<T> a[B3];
      if (act) {
#pragma unroll
        for (int m = 0; m < B3; ++m) {
          const size_t o = (size_t)y * N3 + t + A3 * m;
          cpx<T> r = cmulc(pv[o], pc[o]);
          if (NS == 2) r = r + cmulc(pv[nb + o], pc[nb + o]);
          a[m] = r;
        }
        reg_dft<T, B3>(a);
#pragma unroll
        for (int k2 = 1; k2 < B3; ++k2)
          if (t) a[k2] = cmul(a[k2], twz[t * k2]);
#pragma unroll
        for (int k2 = 0; k2 < B3; ++k2) E[rr * EP3 + k2 * A3 + t] = a[k2];
      }
      __syncthreads();
      if (act) {
#pragma unroll
        for (int s = 0; s < (B3 + A3 - 1) / A3; ++s) {
          const int k2 = t + A3 * s;
          if (k2 < B3) {
            cpx<T> u[A3];
#pragma unroll
            for (int n = 0; n < A3; ++n) u[n] = E[rr * EP3 + k2 * A3 + n];
            reg_dft<T, A3>(u);
#pragma unroll
            for (int k1 = 0; k1 < A3; ++k1) {
              const int jz = kept(k2 + B3 * k1, N3, gz);
              if (jz >= 0) Zb[y * ZP + jz] = u[k1];
            }
          }
        }
      }
      __syncthreads();
    }
  }
  // ---- y transforms of the kept columns
  {
    const int pp = tid / A2, t = tid % A2;
    const int ncol = ey * ez;
    cpx<T>* dst = t2 + ((size_t)pr * n1 + x) * ncol;
    for (int p0 = 0; p0 < ez; p0 += RY) {
      const int jz = p0 + pp;
      const bool act = jz < ez;
      cpx<T> a[B2];
      if (act) {
#pragma unroll
        for (int m = 0; m < B2; ++m) a[m] = Zb[(t + A2 * m) * ZP + jz];
        reg_dft<T, B2>(a);
#pragma unroll
        for (int k2 = 1; k2 < B2; ++k2)
          if (t) a[k2] = cmul(a[k2], twy[t * k2]);
#pragma unroll
        for (int k2 = 0; k2 < B2; ++k2) E[pp * EP2 + k2 * A2 + t] = a[k2];
      }
      __syncthreads();
      if (act) {
#pragma unroll
        for (int s = 0; s < (B2 + A2 - 1) / A2; ++s) {
          const int k2 = t + A2 * s;
          if (k2 < B2) {
            cpx<T> u[A2];
#pragma unroll
            for (int n = 0; n < A2; ++n) u[n] = E[pp * EP2 + k2 * A2 + n];
            reg_dft<T, A2>(u);
#pragma unroll
            for (int k1 = 0; k1 < A2; ++k1) {
              const int jy = kept(k2 + B2 * k1, N2, gy);
              if (jy >= 0) dst[jy * ez + jz] = u[k1];
            }
          }
        }
      }
      __syncthreads();
    }
  }
}

// band plane: compact (y,z) input, y transform on the occupied columns, z
// transform of every row, full plane written
template <typename T, int N2, int N3>
__global__ void __launch_bounds__(kThreads) k_band_plane_rf(
    const cpx<T>* __restrict__ t1, int ey, int ez, int gy, int gz, int n1,
    const cpx<T>* __restrict__ twy, const cpx<T>* __restrict__ twz, cpx<T>* __restrict__ u) {
  constexpr int A3 = split_n1(N3), B3 = N3 / A3, RZ = kThreads / A3, EP3 = ex_pitch<N3>();
  constexpr int A2 = split_n1(N2), B2 = N2 / A2, RY = kThreads / A2, EP2 = ex_pitch<N2>();
  constexpr int ER3 = RZ < N2 ? RZ : N2, ER2 = RY < N3 ? RY : N3;
  constexpr int ESZ = (ER3 * EP3 > ER2 * EP2) ? ER3 * EP3 : ER2 * EP2;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* E = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* Zb = E + ESZ;
  const int ZP = ez | 1;
  const int x = blockIdx.x, bs = blockIdx.y;
  const int ncol = ey * ez;
  const cpx<T>* src = t1 + ((size_t)bs * n1 + x) * ncol;
  const int tid = threadIdx.x;
  // ---- y transforms of the occupied columns (input rows |gy| <= g only)
  {
    const int pp = tid / A2, t = tid % A2;
    for (int p0 = 0; p0 < ez; p0 += RY) {
      const int jz = p0 + pp;
      const bool act = jz < ez;
      cpx<T> a[B2];
      if (act) {
#pragma unroll
        for (int m = 0; m < B2; ++m) {
          const int jy = kept(t + A2 * m, N2, gy);
          a[m] = jy >= 0 ? src[jy * ez + jz] : mk<T>(0, 0);
        }
        reg_dft<T, B2>(a);
#pragma unroll
        for (int k2 = 1; k2 < B2; ++k2)
          if (t) a[k2] = cmul(a[k2], twy[t * k2]);
#pragma unroll
        for (int k2 = 0; k2 < B2; ++k2) E[pp * EP2 + k2 * A2 + t] = a[k2];
      }
      __syncthreads();
      if (act) {
#pragma unroll
        for (int s = 0; s < (B2 + A2 - 1) / A2; ++s) {
          const int k2 = t + A2 * s;
          if (k2 < B2) {
            cpx<T> w[A2];
#pragma unroll
            for (int n = 0; n < A2; ++n) w[n] = E[pp * EP2 + k2 * A2 + n];
            reg_dft<T, A2>(w);
#pragma unroll
            for (int k1 = 0; k1 < A2; ++k1) Zb[(k2 + B2 * k1) * ZP + jz] = w[k1];
          }
        }
      }
      __syncthreads();
    }
  }
  // ---- z transforms of every row (input columns |gz| <= g only)
  {
    const int rr = tid / A3, t = tid % A3;
    cpx<T>* dst = u + ((size_t)bs * n1 + x) * (size_t)N2 * N3;
    for (int y0 = 0; y0 < N2; y0 += RZ) {
      const int y = y0 + rr;
      const bool act = y < N2;
      cpx<T> a[B3];
      if (act) {
#pragma unroll
        for (int m = 0; m < B3; ++m) {
          const int jz = kept(t + A3 * m, N3, gz);
          a[m] = jz >= 0 ? Zb[y * ZP + jz] : mk<T>(0, 0);
        }
        reg_dft<T, B3>(a);
#pragma unroll
        for (int k2 = 1; k2 < B3; ++k2)
          if (t) a[k2] = cmul(a[k2], twz[t * k2]);
#pragma unroll
        for (int k2 = 0; k2 < B3; ++k2) E[rr * EP3 + k2 * A3 + t] = a[k2];
      }
      __syncthreads();
      if (act) {
#pragma unroll
        for (int s = 0; s < (B3 + A3 - 1) / A3; ++s) {
          const int k2 = t + A3 * s;
          if (k2 < B3) {
            cpx<T> w[A3];
#pragma unroll
            for (int n = 0; n < A3; ++n) w[n] = E[rr * EP3 + k2 * A3 + n];
            reg_dft<T, A3>(w);
#pragma unroll
            for (int k1 = 0; k1 < A3; ++k1) dst[(size_t)y * N3 + k2 + B3 * k1] = w[k1];
          }
        }
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------- conduction-stationary pair planes
// One block owns the x-plane of one conduction band and walks every valence
// band of the launch.
//   - The conduction plane (all spinor components) stays in registers.
//   - The next valence plane is fetched while the current one is transformed.
//   - VB valence bands share one y pass, so that its columns fill the block.
// Each pair costs one plane load from the caches instead of two. The output
// layout is the one k_pair_plane_rf writes. Barriers order LDS only, so the
// prefetch stays in flight across them; the twiddles live in LDS for the
// same reason (a global load issued after the prefetch would wait for it).

constexpr int cs_split(int n) { return n == 48 ? 8 : split_n1(n); }

// Offset of entry k within a row of an LDS plane. LAYOUT 1 (8-byte entries, 4
// lanes per row, row pitch 60 for length 48) puts one pad entry after every 4,
// so that the z pass's accesses (4 consecutive entries of 8 rows, or entries 4
// apart) fall in distinct banks (64 banks of 4 bytes); LAYOUT 0 is plain rows.
template <int LAYOUT>
__device__ __forceinline__ int zoff(int k) {
  return LAYOUT == 1 ? k + (k >> 2) : k;
}

// Full x-plane of one band and spinor component, built in LDS from its slab of
// the compact (y,z) cube that k_band_x writes (src[jy * ezw + jz], |g| <= gyw,
// gzw). It takes the y transforms of the occupied z columns (into Zw, pitch
// ZWP), then the z transforms of every row (into P, pitch PP). A2/A3 lanes per
// pencil, all in one wavefront: each exchange goes through the pencil's own LDS
// line, with every read of a stage finished before its writes.
template <typename T, int N2, int N3, int A2, int A3, int NTH, int LAYOUT>
__device__ __forceinline__ void build_plane(const cpx<T>* __restrict__ src, int ezw, int gyw,
                                            int gzw, const cpx<T>* tw2, const cpx<T>* tw3,
                                            cpx<T>* Zw, int ZWP, cpx<T>* P, int PP, int tid) {
  constexpr int B2 = N2 / A2, L2 = pow2_at_least(A2), R2 = NTH / L2, NR2 = (B2 + A2 - 1) / A2;
  constexpr int B3 = N3 / A3, L3 = pow2_at_least(A3), R3 = NTH / L3, NR3 = (B3 + A3 - 1) / A3;
  static_assert(64 % L2 == 0 && 64 % L3 == 0, "a pencil must sit in one wavefront");
  {
    const int pp = tid / L2, t = tid % L2;
    for (int q0 = 0; q0 < ezw; q0 += R2) {
      const int jz = q0 + pp;
      if (jz < ezw && t < A2) {
        cpx<T> a[B2];
#pragma unroll
        for (int m = 0; m < B2; ++m) {
          const int jy = kept(t + A2 * m, N2, gyw);
          a[m] = jy >= 0 ? src[jy * ezw + jz] : mk<T>(0, 0);
        }
        reg_dft<T, B2>(a);
#pragma unroll
        for (int k2 = 1; k2 < B2; ++k2) a[k2] = cmul(a[k2], tw2[t * k2]);
        cpx<T>* col = Zw + jz;
#pragma unroll
        for (int k2 = 0; k2 < B2; ++k2) col[(k2 * A2 + t) * ZWP] = a[k2];
        __builtin_amdgcn_wave_barrier();
        cpx<T> o[NR2][A2];
#pragma unroll
        for (int r = 0; r < NR2; ++r) {
          const int k2 = t + A2 * r;
          if (k2 < B2) {
#pragma unroll
            for (int n = 0; n < A2; ++n) o[r][n] = col[(k2 * A2 + n) * ZWP];
            reg_dft<T, A2>(o[r]);
          }
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int r = 0; r < NR2; ++r) {
          const int k2 = t + A2 * r;
          if (k2 < B2) {
#pragma unroll
            for (int k1 = 0; k1 < A2; ++k1) col[(k2 + B2 * k1) * ZWP] = o[r][k1];
          }
        }
      }
    }
  }
  lds_sync();
  {
    const int rr = tid / L3, t = tid % L3;
    for (int y0 = 0; y0 < N2; y0 += R3) {
      const int y = y0 + rr;
      if (y < N2 && t < A3) {
        cpx<T> a[B3];
#pragma unroll
        for (int m = 0; m < B3; ++m) {
          const int jz = kept(t + A3 * m, N3, gzw);
          a[m] = jz >= 0 ? Zw[y * ZWP + jz] : mk<T>(0, 0);
        }
        reg_dft<T, B3>(a);
#pragma unroll
        for (int k2 = 1; k2 < B3; ++k2) a[k2] = cmul(a[k2], tw3[t * k2]);
        cpx<T>* row = P + y * PP;
#pragma unroll
        for (int k2 = 0; k2 < B3; ++k2) row[zoff<LAYOUT>(k2 * A3 + t)] = a[k2];
        __builtin_amdgcn_wave_barrier();
        cpx<T> o[NR3][A3];
#pragma unroll
        for (int r = 0; r < NR3; ++r) {
          const int k2 = t + A3 * r;
          if (k2 < B3) {
#pragma unroll
            for (int n = 0; n < A3; ++n) o[r][n] = row[zoff<LAYOUT>(k2 * A3 + n)];
            reg_dft<T, A3>(o[r]);
          }
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int r = 0; r < NR3; ++r) {
          const int k2 = t + A3 * r;
          if (k2 < B3) {
#pragma unroll
            for (int k1 = 0; k1 < A3; ++k1) row[zoff<LAYOUT>(k2 + B3 * k1)] = o[r][k1];
          }
        }
      }
    }
  }
  lds_sync();
}

template <int N2, int N3>
struct CsShape {
  static constexpr int NP = N2 * N3;                        // plane elements
  static constexpr int NI = (NP + kThreads - 1) / kThreads;  // per thread
  static constexpr int PP = N3 + 1;                          // product row pitch
  // z pass: A3 lanes (padded to L3, a power of two) per row, B3 values each
  // 8 lanes x 6 values for length 48 keeps the FP64 instance within 256 VGPRs
  static constexpr int A3 = cs_split(N3), B3 = N3 / A3, L3 = pow2_at_least(A3), R3 = kThreads / L3;
  static constexpr int A2 = cs_split(N2), B2 = N2 / A2, L2 = pow2_at_least(A2), R2 = kThreads / L2;
  static constexpr int VB = 4;  // valence bands per y pass
  static_assert(64 % L3 == 0 && 64 % L2 == 0, "a row or column must sit in one wavefront");
};

// LDS elements: twiddles (N3 + N2), product plane, and a region that holds the
// VB kept-column slabs of the valence loop and, before it, the y-transformed
// columns of the conduction plane being built
template <int N2, int N3>
static size_t cs_lds_elems(int ez, int ezw) {
  using S = CsShape<N2, N3>;
  const size_t slabs = std::max((size_t)S::VB * N2 * (ez | 1), (size_t)N2 * (ezw | 1));
  return (size_t)N3 + N2 + (size_t)N2 * S::PP + slabs;
}

template <typename T, int NS, int N2, int N3>
__global__ void __launch_bounds__(kThreads, 2) k_pair_cs(
    const cpx<T>* __restrict__ uv, const cpx<T>* __restrict__ tc, int ezw, int gyw, int gzw,
    int ncw, int v0, int nvt, int c0, int nct, int n1, int ey, int ez, int gy, int gz,
    const cpx<T>* __restrict__ twy, const cpx<T>* __restrict__ twz, cpx<T>* __restrict__ t2) {
  using S = CsShape<N2, N3>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* tw3 = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* tw2 = tw3 + N3;
  cpx<T>* P = tw2 + N2;
  cpx<T>* Zb = P + N2 * S::PP;
  const int ZP = ez | 1, zslab = N2 * ZP, ncol = ey * ez;
  const long long lin = xcd_linear(blockIdx.x, (long long)n1 * nct);
  if (lin < 0) return;
  const int x = (int)(lin / nct), cl = (int)(lin % nct);
  const size_t nb = (size_t)n1 * S::NP;
  const int tid = threadIdx.x;
  for (int i = tid; i < N3; i += kThreads) tw3[i] = twz[i];
  for (int i = tid; i < N2; i += kThreads) tw2[i] = twy[i];

  cpx<T> cr[NS][S::NI], vr[NS][S::NI];
  auto fetch_v = [&](int vl) {
    const cpx<T>* pv = uv + (size_t)(v0 + vl) * NS * nb + (size_t)x * S::NP;
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int i = 0; i < S::NI; ++i) {
        const int e = tid + kThreads * i;
        vr[s][i] = (S::NP % kThreads == 0 || e < S::NP) ? pv[s * nb + e] : mk<T>(0, 0);
      }
  };
  fetch_v(0);
  lds_sync();  // twiddles in place
  // the conduction plane (every spinor component), built from its compact slab
  // and kept in registers in the flat layout
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const cpx<T>* src = tc + (((size_t)(c0 + cl) * NS + s) * n1 + x) * ncw;
    build_plane<T, N2, N3, S::A2, S::A3, kThreads, 0>(src, ezw, gyw, gzw, tw2, tw3, Zb, ezw | 1,
                                                      P, S::PP, tid);
#pragma unroll
    for (int i = 0; i < S::NI; ++i) {
      const int e = tid + kThreads * i;
      cr[s][i] = (S::NP % kThreads == 0 || e < S::NP) ? P[(e / N3) * S::PP + e % N3] : mk<T>(0, 0);
    }
  }

  for (int g0 = 0; g0 < nvt; g0 += S::VB) {
    const int nbv = min(S::VB, nvt - g0);
    for (int j = 0; j < nbv; ++j) {
      const int vl = g0 + j;
      lds_sync();  // the previous z pass (or the plane build) has read P
      // spinor-summed product conj(psi_v) psi_c of this plane
#pragma unroll
      for (int i = 0; i < S::NI; ++i) {
        const int e = tid + kThreads * i;
        cpx<T> r = cmulc(vr[0][i], cr[0][i]);
        if (NS == 2) r = r + cmulc(vr[1][i], cr[1][i]);
        if (S::NP % kThreads == 0 || e < S::NP) P[(e / N3) * S::PP + e % N3] = r;
      }
      if (vl + 1 < nvt) fetch_v(vl + 1);
      lds_sync();
      // z transforms of the rows; the kept |gz| <= g entries go to slab j
      cpx<T>* Z = Zb + j * zslab;
      const int rr = tid / S::L3, t = tid % S::L3;
      for (int y0 = 0; y0 < N2; y0 += S::R3) {
        const int y = y0 + rr;
        if (y < N2 && t < S::A3) {
          cpx<T>* row = P + y * S::PP;
          cpx<T> a[S::B3];
#pragma unroll
          for (int m = 0; m < S::B3; ++m) a[m] = row[t + S::A3 * m];
          reg_dft<T, S::B3>(a);
          // tw[0] = 1 exactly, so lane 0 multiplies by one without rounding
#pragma unroll
          for (int k2 = 1; k2 < S::B3; ++k2) a[k2] = cmul(a[k2], tw3[t * k2]);
          // each lane rewrites the row entries it read; the row's lanes share a
          // wavefront, whose LDS accesses complete in order
#pragma unroll
          for (int k2 = 0; k2 < S::B3; ++k2) row[k2 * S::A3 + t] = a[k2];
          __builtin_amdgcn_wave_barrier();
#pragma unroll
          for (int s = 0; s < (S::B3 + S::A3 - 1) / S::A3; ++s) {
            const int k2 = t + S::A3 * s;
            if (k2 < S::B3) {
              cpx<T> u[S::A3];
#pragma unroll
              for (int n = 0; n < S::A3; ++n) u[n] = row[k2 * S::A3 + n];
              reg_dft<T, S::A3>(u);
#pragma unroll
              for (int k1 = 0; k1 < S::A3; ++k1) {
                const int jz = kept(k2 + S::B3 * k1, N3, gz);
                if (jz >= 0) Z[y * ZP + jz] = u[k1];
              }
            }
          }
        }
      }
    }
    lds_sync();  // every slab of the group is complete
    // y transforms of the kept columns of the group's valence bands
    const int pp = tid / S::L2, t = tid % S::L2;
    const int tot = nbv * ez;
    for (int q0 = 0; q0 < tot; q0 += S::R2) {
      const int q = q0 + pp;
      if (q < tot && t < S::A2) {
        const int j = q / ez, jz = q % ez;
        cpx<T>* col = Zb + j * zslab + jz;
        cpx<T> a[S::B2];
#pragma unroll
        for (int m = 0; m < S::B2; ++m) a[m] = col[(t + S::A2 * m) * ZP];
        reg_dft<T, S::B2>(a);
#pragma unroll
        for (int k2 = 1; k2 < S::B2; ++k2) a[k2] = cmul(a[k2], tw2[t * k2]);
#pragma unroll
        for (int k2 = 0; k2 < S::B2; ++k2) col[(k2 * S::A2 + t) * ZP] = a[k2];
        __builtin_amdgcn_wave_barrier();
        cpx<T>* dst = t2 + ((size_t)(cl * nvt + g0 + j) * n1 + x) * ncol;
#pragma unroll
        for (int s = 0; s < (S::B2 + S::A2 - 1) / S::A2; ++s) {
          const int k2 = t + S::A2 * s;
          if (k2 < S::B2) {
            cpx<T> u[S::A2];
#pragma unroll
            for (int n = 0; n < S::A2; ++n) u[n] = col[(k2 * S::A2 + n) * ZP];
            reg_dft<T, S::A2>(u);
#pragma unroll
            for (int k1 = 0; k1 < S::A2; ++k1) {
              const int jy = kept(k2 + S::B2 * k1, N2, gy);
              if (jy >= 0) dst[jy * ez + jz] = u[k1];
            }
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------- row-resident pair planes
// Like k_pair_cs, one block owns the x-plane of one conduction band and walks
// the valence bands, but every row of the plane belongs to one group of lanes
// inside one wavefront.
//   - Those lanes load their row slice of both bands straight from memory and
//     form the spinor product in registers.
//   - They exchange the row through LDS for the second factor of the z
//     transform without a block barrier: a wavefront's LDS accesses complete
//     in order.
// Block barriers remain only around the y pass, which runs once per group of
// vb valence bands. There is no register prefetch: at three wavefronts per SIMD,
// the other block covers the load latency. This is the FP32 kernel; in FP64
// the conduction row plus its working set leave too few wavefronts, and
// k_pair_cs is faster.


template <typename T, int N2, int N3>
struct RrShape {
  static constexpr int A3 = split_n1(N3), B3 = N3 / A3, L3 = pow2_at_least(A3);
  static constexpr int A2 = split_n1(N2), B2 = N2 / A2, L2 = pow2_at_least(A2);
  static constexpr int NTH = N2 * L3;  // threads: one lane group per row
  static constexpr int LAYOUT = N3 == 48 && A3 == 4 ? 1 : 0;  // exchange row layout (zoff)
  static constexpr int PP = LAYOUT ? N3 + N3 / 4 : N3 + 1;     // exchange row pitch
  static constexpr int CPP = NTH / L2; // y columns per pass
  static_assert(64 % L3 == 0 && 64 % L2 == 0, "a row or column must sit in one wavefront");
  static_assert(NTH <= 1024 && NTH % 64 == 0, "block must be whole wavefronts");
};

// LDS elements: twiddles, exchange plane, and a region for the vb kept-column
// slabs (before the valence loop: the conduction plane's y-transformed columns)
template <typename T, int N2, int N3>
static size_t rr_lds_elems(int ez, int vb, int ezw) {
  using S = RrShape<T, N2, N3>;
  const size_t slabs = std::max((size_t)vb * N2 * (ez | 1), (size_t)N2 * (ezw | 1));
  return (size_t)N3 + N2 + (size_t)N2 * S::PP + slabs;
}

// valence bands per y pass: fill the pass's columns, keep LDS within half a CU
template <typename T, int N2, int N3>
static int rr_group(int ez, int ezw) {
  using S = RrShape<T, N2, N3>;
  int vb = std::max(1, std::min(8, S::CPP / std::max(1, ez)));
  while (vb > 1 && rr_lds_elems<T, N2, N3>(ez, vb, ezw) * sizeof(cpx<T>) > 80 * 1024) --vb;
  return vb;
}

template <typename T, int NS, int N2, int N3>
__global__ void __launch_bounds__((RrShape<T, N2, N3>::NTH), 3) k_pair_rr(
    const cpx<T>* __restrict__ uv, const cpx<T>* __restrict__ tc, int ezw, int gyw, int gzw,
    int ncw, int v0, int nvt, int c0, int nct, int n1, int ey, int ez, int gy, int gz, int vb,
    const cpx<T>* __restrict__ twy, const cpx<T>* __restrict__ twz, cpx<T>* __restrict__ t2) {
  using S = RrShape<T, N2, N3>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  cpx<T>* tw3 = reinterpret_cast<cpx<T>*>(smem_raw);
  cpx<T>* tw2 = tw3 + N3;
  cpx<T>* X = tw2 + N2;
  cpx<T>* Zb = X + N2 * S::PP;
  const int ZP = ez | 1, zslab = N2 * ZP, ncol = ey * ez;
  const long long lin = xcd_linear(blockIdx.x, (long long)n1 * nct);
  if (lin < 0) return;
  const int x = (int)(lin / nct), cl = (int)(lin % nct);
  const int tid = threadIdx.x;
  for (int i = tid; i < N3; i += S::NTH) tw3[i] = twz[i];
  for (int i = tid; i < N2; i += S::NTH) tw2[i] = twy[i];
  const int y = tid / S::L3, t = tid % S::L3;
  const bool act = t < S::A3;
  cpx<T>* Xr = X + y * S::PP;
  const size_t nb = (size_t)n1 * N2 * N3;
  const size_t roff = ((size_t)x * N2 + y) * N3 + t;

  cpx<T> cr[NS][S::B3], vr[NS][S::B3];
  auto fetch_v = [&](int vl) {
    const cpx<T>* pv = uv + (size_t)(v0 + vl) * NS * nb + roff;
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int m = 0; m < S::B3; ++m) vr[s][m] = pv[s * nb + S::A3 * m];
  };
  lds_sync();  // twiddles in place
  // the conduction plane, built from its compact slab; the z pass of the build
  // leaves row y with the lanes that own it here
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const cpx<T>* src = tc + (((size_t)(c0 + cl) * NS + s) * n1 + x) * ncw;
    build_plane<T, N2, N3, S::A2, S::A3, S::NTH, S::LAYOUT>(src, ezw, gyw, gzw, tw2, tw3, Zb,
                                                           ezw | 1, X,
                                                 S::PP, tid);
    if (act) {
#pragma unroll
      for (int m = 0; m < S::B3; ++m) cr[s][m] = Xr[zoff<S::LAYOUT>(t + S::A3 * m)];
    }
  }

  for (int g0 = 0; g0 < nvt; g0 += vb) {
    const int nbv = min(vb, nvt - g0);
    for (int j = 0; j < nbv; ++j) {
      const int vl = g0 + j;
      if (act) {
        fetch_v(vl);
        // spinor-summed product conj(psi_v) psi_c on the lane's row slice
        cpx<T> a[S::B3];
#pragma unroll
        for (int m = 0; m < S::B3; ++m) {
          a[m] = cmulc(vr[0][m], cr[0][m]);
          if (NS == 2) a[m] = a[m] + cmulc(vr[1][m], cr[1][m]);
        }
        reg_dft<T, S::B3>(a);
        // tw[0] = 1 exactly, so lane 0 multiplies by one without rounding
#pragma unroll
        for (int k2 = 1; k2 < S::B3; ++k2) a[k2] = cmul(a[k2], tw3[t * k2]);
#pragma unroll
        for (int k2 = 0; k2 < S::B3; ++k2) Xr[zoff<S::LAYOUT>(k2 * S::A3 + t)] = a[k2];
      }
      __builtin_amdgcn_wave_barrier();
      if (act) {
        cpx<T>* Z = Zb + j * zslab + y * ZP;
#pragma unroll
        for (int s = 0; s < (S::B3 + S::A3 - 1) / S::A3; ++s) {
          const int k2 = t + S::A3 * s;
          if (k2 < S::B3) {
            cpx<T> u[S::A3];
#pragma unroll
            for (int n = 0; n < S::A3; ++n) u[n] = Xr[zoff<S::LAYOUT>(k2 * S::A3 + n)];
            reg_dft<T, S::A3>(u);
#pragma unroll
            for (int k1 = 0; k1 < S::A3; ++k1) {
              const int jz = kept(k2 + S::B3 * k1, N3, gz);
              if (jz >= 0) Z[jz] = u[k1];
            }
          }
        }
      }
      // the next band's exchange writes follow these reads in the same wavefront
      __builtin_amdgcn_wave_barrier();
    }
    lds_sync();  // every slab of the group is complete
    const int pp = tid / S::L2, tt = tid % S::L2;
    const int tot = nbv * ez;
    for (int q0 = 0; q0 < tot; q0 += S::CPP) {
      const int q = q0 + pp;
      if (q < tot && tt < S::A2) {
        const int j = q / ez, jz = q % ez;
        cpx<T>* col = Zb + j * zslab + jz;
        cpx<T> a[S::B2];
#pragma unroll
        for (int m = 0; m < S::B2; ++m) a[m] = col[(tt + S::A2 * m) * ZP];
        reg_dft<T, S::B2>(a);
#pragma unroll
        for (int k2 = 1; k2 < S::B2; ++k2) a[k2] = cmul(a[k2], tw2[tt * k2]);
#pragma unroll
        for (int k2 = 0; k2 < S::B2; ++k2) col[(k2 * S::A2 + tt) * ZP] = a[k2];
        __builtin_amdgcn_wave_barrier();
        cpx<T>* dst = t2 + ((size_t)(cl * nvt + g0 + j) * n1 + x) * ncol;
#pragma unroll
        for (int s = 0; s < (S::B2 + S::A2 - 1) / S::A2; ++s) {
          const int k2 = tt + S::A2 * s;
          if (k2 < S::B2) {
            cpx<T> u[S::A2];
#pragma unroll
            for (int n = 0; n < S::A2; ++n) u[n] = col[(k2 * S::A2 + n) * ZP];
            reg_dft<T, S::A2>(u);
#pragma unroll
            for (int k1 = 0; k1 < S::A2; ++k1) {
              const int jy = kept(k2 + S::B2 * k1, N2, gy);
              if (jy >= 0) dst[jy * ez + jz] = u[k1];
            }
          }
        }
      }
    }
    lds_sync();  // the group's slabs are consumed before the next z pass
  }
}

// ---------------------------------------------------------------- pair x pass, register resident
// The x pencils of one pair's kept (y, z) columns: A lanes per column each hold
// B values (x = t + A m), B-point DFT in registers, twiddle, exchange through
// the column's LDS row inside the wavefront, A-point DFTs. Only the kept
// |gx| <= g outputs are written, scaled by 1/N and scattered to the sphere.
template <typename T, int N1>
struct XpShape {
  static constexpr int A = split_n1(N1), B = N1 / A, L = pow2_at_least(A), CPB = kThreads / L;
  static_assert(64 % L == 0, "a column must sit in one wavefront");
};

template <typename T, int N1>
__global__ void __launch_bounds__(kThreads) k_pair_x_rf(
    const cpx<T>* __restrict__ t2, int ncol, int ey, int ez, int gx,
    const int* __restrict__ emap, const cpx<T>* __restrict__ twx, T invN, int v0, int nvt,
    int c0, int nct_total, int neps, int npairs, cpx<T>* __restrict__ M) {
  using S = XpShape<T, N1>;
  __shared__ cpx<T> X[S::CPB][N1 + 1];
  __shared__ cpx<T> tw[N1];
  // all column blocks of a pair on one XCD: its scattered stores into the
  // pair's row of M then fill whole lines in that XCD's L2 before write-back
  const int nbx = (ncol + S::CPB - 1) / S::CPB;
  const long long lin = xcd_linear(blockIdx.x, (long long)nbx * npairs);
  if (lin < 0) return;
  const int pr = (int)(lin / nbx), bx = (int)(lin - (long long)pr * nbx), tid = threadIdx.x;
  for (int i = tid; i < N1; i += kThreads) tw[i] = twx[i];
  __syncthreads();
  const int cq = tid / S::L, t = tid % S::L;
  const int col = bx * S::CPB + cq;
  if (col >= ncol || t >= S::A) return;
  const cpx<T>* src = t2 + (size_t)pr * N1 * ncol + col;
  cpx<T> a[S::B];
#pragma unroll
  for (int m = 0; m < S::B; ++m) a[m] = src[(size_t)(t + S::A * m) * ncol];
  reg_dft<T, S::B>(a);
  // tw[0] = 1 exactly, so lane 0 multiplies by one without rounding
#pragma unroll
  for (int k2 = 1; k2 < S::B; ++k2) a[k2] = cmul(a[k2], tw[t * k2]);
  cpx<T>* Xr = X[cq];
#pragma unroll
  for (int k2 = 0; k2 < S::B; ++k2) Xr[k2 * S::A + t] = a[k2];
  // the column's lanes share a wavefront, whose LDS accesses complete in order
  __builtin_amdgcn_wave_barrier();
  const int v = v0 + pr % nvt, c = c0 + pr / nvt;
  cpx<T>* dst = M + ((size_t)v * nct_total + c) * neps;
  const int jy = col / ez, jz = col - jy * ez;
#pragma unroll
  for (int s = 0; s < (S::B + S::A - 1) / S::A; ++s) {
    const int k2 = t + S::A * s;
    if (k2 < S::B) {
      cpx<T> u[S::A];
#pragma unroll
      for (int n = 0; n < S::A; ++n) u[n] = Xr[k2 * S::A + n];
      reg_dft<T, S::A>(u);
#pragma unroll
      for (int k1 = 0; k1 < S::A; ++k1) {
        const int jx = kept(k2 + S::B * k1, N1, gx);
        if (jx >= 0) {
          const int idx = emap[(jx * ey + jy) * ez + jz];
          if (idx >= 0) dst[idx] = scal(u[k1], invN);
        }
      }
    }
  }
}

template <int N2, int N3>
static size_t rf_lds_elems(int ez) {
  constexpr int A3 = split_n1(N3), RZ = kThreads / A3, EP3 = N3 + 1;
  constexpr int A2 = split_n1(N2), RY = kThreads / A2, EP2 = N2 + 1;
  constexpr int ER3 = RZ < N2 ? RZ : N2, ER2 = RY < N3 ? RY : N3;
  constexpr int ESZ = (ER3 * EP3 > ER2 * EP2) ? ER3 * EP3 : ER2 * EP2;
  return (size_t)ESZ + (size_t)N2 * (ez | 1);
}

// Pencil lengths (x) and plane shapes (y, z) built with constant lengths; any
// other box factoring into 2, 3, 5 runs the same kernels with runtime lengths.
#define GW_X_LENGTHS(X) X(16) X(20) X(24) X(30) X(32) X(48) X(60)
#define GW_PLANE_SHAPES(X) X(16, 16) X(24, 30) X(32, 32) X(48, 48) X(60, 160)
// plane shapes of the conduction-stationary pair kernels (k_pair_cs in FP64, k_pair_rr in FP32)
#define GW_CS_SHAPES(X) X(16, 16) X(24, 30) X(32, 32) X(48, 48)

// ---------------------------------------------------------------- launchers

template <typename T>
static int col_chunk(int n1) {
  // keep the x-pass tile (n1 x CH) at <= 48 KiB
  int ch = (48 * 1024) / (n1 * (int)sizeof(cpx<T>));
  if (ch > 128) ch = 128;
  if (ch < 1) ch = 1;
  return ch;
}

template <typename K>
static hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

size_t band_scratch_bytes(const int box[3], const SphereMap* sm, int nbs, size_t elem) {
  return (size_t)nbs * box[0] * sm->ext[1] * sm->ext[2] * elem;
}

size_t pair_scratch_bytes(const int box[3], const SphereMap* em, int npairs, size_t elem) {
  return (size_t)npairs * box[0] * em->ext[1] * em->ext[2] * elem;
}

// kernel selection by box shape
template <typename T>
static decltype(&k_band_x<T, 0>) pick_band_x(int n1) {
#define X(N) if (n1 == N) return &k_band_x<T, N>;
  GW_X_LENGTHS(X)
#undef X
  return &k_band_x<T, 0>;
}
template <typename T>
static decltype(&k_pair_x<T, 0>) pick_pair_x(int n1) {
#define X(N) if (n1 == N) return &k_pair_x<T, N>;
  GW_X_LENGTHS(X)
#undef X
  return &k_pair_x<T, 0>;
}
template <typename T>
static decltype(&k_band_plane<T, 0, 0>) pick_band_plane(int n2, int n3) {
#define X(A, B) if (n2 == A && n3 == B) return &k_band_plane<T, A, B>;
  GW_PLANE_SHAPES(X)
#undef X
  return &k_band_plane<T, 0, 0>;
}
template <typename T, int NS>
static decltype(&k_pair_plane<T, NS, 0, 0>) pick_pair_plane(int n2, int n3) {
#define X(A, B) if (n2 == A && n3 == B) return &k_pair_plane<T, NS, A, B>;
  GW_PLANE_SHAPES(X)
#undef X
  return &k_pair_plane<T, NS, 0, 0>;
}

template <typename T>
gw_status band_to_grid(gw_ctx* c, const int box[3], int nbs, int ng, const void* coef,
                       const SphereMap* sm, void* u_out, void* scratch, size_t scratch_bytes) {
  const int n1 = box[0], n2 = box[1], n3 = box[2];
  FftPlan px = make_fft_plan(n1), py = make_fft_plan(n2), pz = make_fft_plan(n3);
  const void *twx, *twy, *twz;
  const bool dbl = sizeof(T) == 8;
  gw_status st;
  if ((st = twiddle_table(c, n1, dbl, &twx)) != GW_OK) return st;
  if ((st = twiddle_table(c, n2, dbl, &twy)) != GW_OK) return st;
  if ((st = twiddle_table(c, n3, dbl, &twz)) != GW_OK) return st;
  const int ncol = sm->ext[1] * sm->ext[2];
  const size_t per = (size_t)n1 * ncol * sizeof(cpx<T>);
  int chunk = (int)(scratch_bytes / per);
  if (chunk < 1) return fail(c, GW_ENOMEM, "band scratch too small");
  if (chunk > 65535) chunk = 65535;
  const int CH = col_chunk<T>(n1);
  const size_t lds_x = (size_t)n1 * CH * sizeof(cpx<T>);
  const int P = plane_pitch(n3);
  const size_t lds_p = (size_t)n2 * P * sizeof(cpx<T>);
  auto kx = pick_band_x<T>(n1);
  auto kp = pick_band_plane<T>(n2, n3);
  if (!c->capturing) {
    GW_HIP(c, allow_lds(kx, lds_x));
    GW_HIP(c, allow_lds(kp, lds_p));
  }
  bool rf = false;
#define X(A, B) if (n2 == A && n3 == B) rf = true;
  GW_PLANE_SHAPES(X)
#undef X
  const cpx<T>* cf = static_cast<const cpx<T>*>(coef);
  cpx<T>* u = static_cast<cpx<T>*>(u_out);
  cpx<T>* t1 = static_cast<cpx<T>*>(scratch);
  for (int b0 = 0; b0 < nbs; b0 += chunk) {
    const int nb = std::min(chunk, nbs - b0);
    {
      ProfScope ps(c, "band_xpass");
      dim3 g((ncol + CH - 1) / CH, nb);
      hipLaunchKernelGGL(kx, g, dim3(kThreads), lds_x, c->stream, cf + (size_t)b0 * ng, ng,
                         sm->d_cube, sm->ext[0], sm->ext[1], sm->ext[2], sm->gmax[0], n1, ncol,
                         CH, px, static_cast<const cpx<T>*>(twx), t1);
      GW_CHECK_LAUNCH(c, "k_band_x");
    }
    {
      ProfScope ps(c, "band_plane");
      dim3 g(n1, nb);
      cpx<T>* ub = u + (size_t)b0 * n1 * n2 * n3;
      const cpx<T>* ty = static_cast<const cpx<T>*>(twy);
      const cpx<T>* tz = static_cast<const cpx<T>*>(twz);
      if (rf) {
#define X(A, B)                                                                           \
  if (n2 == A && n3 == B) {                                                               \
    const size_t lds = rf_lds_elems<A, B>(sm->ext[2]) * sizeof(cpx<T>);                   \
    if (!c->capturing) GW_HIP(c, allow_lds(k_band_plane_rf<T, A, B>, lds));               \
    hipLaunchKernelGGL((k_band_plane_rf<T, A, B>), g, dim3(kThreads), lds, c->stream, t1, \
                       sm->ext[1], sm->ext[2], sm->gmax[1], sm->gmax[2], n1, ty, tz, ub); \
  }
        GW_PLANE_SHAPES(X)
#undef X
      } else {
        hipLaunchKernelGGL(kp, g, dim3(kThreads), lds_p, c->stream, t1, sm->ext[1], sm->ext[2],
                           sm->gmax[1], sm->gmax[2], n1, n2, n3, py, pz, ty, tz, ub);
      }
      GW_CHECK_LAUNCH(c, "k_band_plane");
    }
  }
  return GW_OK;
}

bool pair_compact_shape(const int box[3]) {
  bool yes = false;
#define X(A, B) if (box[1] == A && box[2] == B) yes = true;
  GW_CS_SHAPES(X)
#undef X
  return yes;
}

size_t band_compact_bytes(const int box[3], const SphereMap* sm, int nbs, size_t elem) {
  return (size_t)nbs * box[0] * sm->ext[1] * sm->ext[2] * elem;
}

// x transform only: out[bs][x][jy][jz] on the band's compact (y,z) cube, for the
// pair kernels that build each conduction plane themselves
template <typename T>
gw_status band_compact(gw_ctx* c, const int box[3], int nbs, int ng, const void* coef,
                       const SphereMap* sm, void* out) {
  const int n1 = box[0];
  FftPlan px = make_fft_plan(n1);
  const void* twx;
  gw_status st;
  if ((st = twiddle_table(c, n1, sizeof(T) == 8, &twx)) != GW_OK) return st;
  const int ncol = sm->ext[1] * sm->ext[2];
  const int CH = col_chunk<T>(n1);
  const size_t lds_x = (size_t)n1 * CH * sizeof(cpx<T>);
  auto kx = pick_band_x<T>(n1);
  if (!c->capturing) GW_HIP(c, allow_lds(kx, lds_x));
  const cpx<T>* cf = static_cast<const cpx<T>*>(coef);
  cpx<T>* o = static_cast<cpx<T>*>(out);
  ProfScope ps(c, "band_xpass");
  for (int b0 = 0; b0 < nbs; b0 += 65535) {
    const int nb = std::min(65535, nbs - b0);
    dim3 g((ncol + CH - 1) / CH, nb);
    hipLaunchKernelGGL(kx, g, dim3(kThreads), lds_x, c->stream, cf + (size_t)b0 * ng, ng,
                       sm->d_cube, sm->ext[0], sm->ext[1], sm->ext[2], sm->gmax[0], n1, ncol, CH,
                       px, static_cast<const cpx<T>*>(twx), o + (size_t)b0 * n1 * ncol);
    GW_CHECK_LAUNCH(c, "k_band_x");
  }
  return GW_OK;
}

template <typename T>
gw_status pair_to_eps(gw_ctx* c, const int box[3], int nspinor, const void* uv, const void* uc,
                      const void* tc, const SphereMap* sc, int v0, int nvt, int c0, int nct,
                      int nc_total, const SphereMap* em, void* mtxel, void* scratch) {
  const int n1 = box[0], n2 = box[1], n3 = box[2];
  FftPlan px = make_fft_plan(n1), py = make_fft_plan(n2), pz = make_fft_plan(n3);
  const void *twx, *twy, *twz;
  const bool dbl = sizeof(T) == 8;
  gw_status st;
  if ((st = twiddle_table(c, n1, dbl, &twx)) != GW_OK) return st;
  if ((st = twiddle_table(c, n2, dbl, &twy)) != GW_OK) return st;
  if ((st = twiddle_table(c, n3, dbl, &twz)) != GW_OK) return st;
  const int npairs = nvt * nct;
  const int P = plane_pitch(n3);
  const size_t lds_p = (size_t)n2 * P * sizeof(cpx<T>);
  const int ncol = em->ext[1] * em->ext[2];
  const int CH = col_chunk<T>(n1);
  const size_t lds_x = (size_t)n1 * CH * sizeof(cpx<T>);
  cpx<T>* t2 = static_cast<cpx<T>*>(scratch);
  auto kp = nspinor == 2 ? pick_pair_plane<T, 2>(n2, n3) : pick_pair_plane<T, 1>(n2, n3);
  auto kx = pick_pair_x<T>(n1);
  if (!c->capturing) {
    GW_HIP(c, allow_lds(kp, lds_p));
    GW_HIP(c, allow_lds(kx, lds_x));
  }
  {
    ProfScope ps(c, "pair_plane");
    const long long tot = (long long)n1 * npairs;
    dim3 g((unsigned)(((tot + kXcd - 1) / kXcd) * kXcd));
    const cpx<T>* pu = static_cast<const cpx<T>*>(uv);
    const cpx<T>* pc = static_cast<const cpx<T>*>(uc);
    const cpx<T>* ty = static_cast<const cpx<T>*>(twy);
    const cpx<T>* tz = static_cast<const cpx<T>*>(twz);
    bool rf = false;
    if (tc && nvt > 0 && nct > 0) {
      const unsigned gcs = (unsigned)((((long long)n1 * nct + kXcd - 1) / kXcd) * kXcd);
      const cpx<T>* ptc = static_cast<const cpx<T>*>(tc);
      const int ncw = sc->ext[1] * sc->ext[2];
      if constexpr (sizeof(T) == 8) {
#define X(A, B)                                                                               \
  if (!rf && n2 == A && n3 == B) {                                                            \
    rf = true;                                                                                \
    const size_t lds = cs_lds_elems<A, B>(em->ext[2], sc->ext[2]) * sizeof(cpx<T>);           \
    if (nspinor == 2) {                                                                       \
      if (!c->capturing) GW_HIP(c, allow_lds(k_pair_cs<T, 2, A, B>, lds));                    \
      hipLaunchKernelGGL((k_pair_cs<T, 2, A, B>), dim3(gcs), dim3(kThreads), lds, c->stream,  \
                         pu, ptc, sc->ext[2], sc->gmax[1], sc->gmax[2], ncw, v0, nvt, c0, nct, \
                         n1, em->ext[1], em->ext[2], em->gmax[1],                             \
                         em->gmax[2], ty, tz, t2);                                            \
    } else {                                                                                  \
      if (!c->capturing) GW_HIP(c, allow_lds(k_pair_cs<T, 1, A, B>, lds));                    \
      hipLaunchKernelGGL((k_pair_cs<T, 1, A, B>), dim3(gcs), dim3(kThreads), lds, c->stream,  \
                         pu, ptc, sc->ext[2], sc->gmax[1], sc->gmax[2], ncw, v0, nvt, c0, nct, \
                         n1, em->ext[1], em->ext[2], em->gmax[1],                             \
                         em->gmax[2], ty, tz, t2);                                            \
    }                                                                                         \
  }
        GW_CS_SHAPES(X)
#undef X
      } else {
#define X(A, B)                                                                               \
  if (!rf && n2 == A && n3 == B) {                                                            \
    rf = true;                                                                                \
    const int vb = rr_group<T, A, B>(em->ext[2], sc->ext[2]);                                 \
    const size_t lds = rr_lds_elems<T, A, B>(em->ext[2], vb, sc->ext[2]) * sizeof(cpx<T>);    \
    const dim3 blk(RrShape<T, A, B>::NTH);                                                    \
    if (nspinor == 2) {                                                                       \
      if (!c->capturing) GW_HIP(c, allow_lds(k_pair_rr<T, 2, A, B>, lds));                    \
      hipLaunchKernelGGL((k_pair_rr<T, 2, A, B>), dim3(gcs), blk, lds, c->stream, pu, ptc,    \
                         sc->ext[2], sc->gmax[1], sc->gmax[2], ncw, v0, nvt, c0, nct, n1,      \
                         em->ext[1], em->ext[2], em->gmax[1], em->gmax[2],                     \
                         vb, ty, tz, t2);                                                     \
    } else {                                                                                  \
      if (!c->capturing) GW_HIP(c, allow_lds(k_pair_rr<T, 1, A, B>, lds));                    \
      hipLaunchKernelGGL((k_pair_rr<T, 1, A, B>), dim3(gcs), blk, lds, c->stream, pu, ptc,    \
                         sc->ext[2], sc->gmax[1], sc->gmax[2], ncw, v0, nvt, c0, nct, n1,      \
                         em->ext[1], em->ext[2], em->gmax[1], em->gmax[2],                     \
                         vb, ty, tz, t2);                                                     \
    }                                                                                         \
  }
        GW_CS_SHAPES(X)
#undef X
      }
    }
#define X(A, B)                                                                              \
  if (!rf && n2 == A && n3 == B) {                                                           \
    rf = true;                                                                               \
    const size_t lds = rf_lds_elems<A, B>(em->ext[2]) * sizeof(cpx<T>);                      \
    if (nspinor == 2) {                                                                      \
      if (!c->capturing) GW_HIP(c, allow_lds(k_pair_plane_rf<T, 2, A, B>, lds));             \
      hipLaunchKernelGGL((k_pair_plane_rf<T, 2, A, B>), g, dim3(kThreads), lds, c->stream, pu, \
                         pc, v0, nvt, c0, n1, em->ext[1], em->ext[2], em->gmax[1],           \
                         em->gmax[2], ty, tz, t2, npairs);                                   \
    } else {                                                                                 \
      if (!c->capturing) GW_HIP(c, allow_lds(k_pair_plane_rf<T, 1, A, B>, lds));             \
      hipLaunchKernelGGL((k_pair_plane_rf<T, 1, A, B>), g, dim3(kThreads), lds, c->stream, pu, \
                         pc, v0, nvt, c0, n1, em->ext[1], em->ext[2], em->gmax[1],           \
                         em->gmax[2], ty, tz, t2, npairs);                                   \
    }                                                                                        \
  }
    GW_PLANE_SHAPES(X)
#undef X
    if (!rf)
      hipLaunchKernelGGL(kp, g, dim3(kThreads), lds_p, c->stream, pu, pc, v0, nvt, c0, n1, n2, n3,
                         em->ext[1], em->ext[2], em->gmax[1], em->gmax[2], py, pz, ty, tz, t2,
                         npairs);
    GW_CHECK_LAUNCH(c, "k_pair_plane");
  }
  {
    ProfScope ps(c, "pair_xpass");
    const T invN = (T)(1.0 / ((double)n1 * n2 * n3));
    bool done = false;
#define X(N)                                                                                   \
  if (!done && n1 == N) {                                                                      \
    done = true;                                                                               \
    const long long tot =                                                                      \
        (long long)((ncol + XpShape<T, N>::CPB - 1) / XpShape<T, N>::CPB) * npairs;            \
    const unsigned grid = (unsigned)(((tot + kXcd - 1) / kXcd) * kXcd);                        \
    hipLaunchKernelGGL((k_pair_x_rf<T, N>), dim3(grid), dim3(kThreads), 0, c->stream, t2,      \
                       ncol, em->ext[1], em->ext[2], em->gmax[0], em->d_cube,                  \
                       static_cast<const cpx<T>*>(twx), invN, v0, nvt, c0, nc_total, em->n,    \
                       npairs, static_cast<cpx<T>*>(mtxel));                                   \
  }
    GW_X_LENGTHS(X)
#undef X
    if (!done) {
      dim3 g((ncol + CH - 1) / CH, npairs);
      hipLaunchKernelGGL(kx, g, dim3(kThreads), lds_x, c->stream, t2, n1, ncol, CH, em->ext[0],
                         em->ext[1], em->ext[2], em->gmax[0], em->d_cube, px,
                         static_cast<const cpx<T>*>(twx), invN, v0, nvt, c0, nc_total, em->n,
                         static_cast<cpx<T>*>(mtxel));
    }
    GW_CHECK_LAUNCH(c, "k_pair_x");
  }
  return GW_OK;
}

template gw_status band_to_grid<double>(gw_ctx*, const int*, int, int, const void*,
                                        const SphereMap*, void*, void*, size_t);
template gw_status band_to_grid<float>(gw_ctx*, const int*, int, int, const void*,
                                       const SphereMap*, void*, void*, size_t);
template gw_status pair_to_eps<double>(gw_ctx*, const int*, int, const void*, const void*,
                                       const void*, const SphereMap*, int, int, int, int, int,
                                       const SphereMap*, void*, void*);
template gw_status pair_to_eps<float>(gw_ctx*, const int*, int, const void*, const void*,
                                      const void*, const SphereMap*, int, int, int, int, int,
                                      const SphereMap*, void*, void*);
template gw_status band_compact<double>(gw_ctx*, const int*, int, int, const void*,
                                        const SphereMap*, void*);
template gw_status band_compact<float>(gw_ctx*, const int*, int, int, const void*,
                                       const SphereMap*, void*);

}  // namespace gw
