// Register-resident DFTs of small compile-time lengths and the two-factor
// pencil transform built on them.
//
// y_k = sum_j a_j exp(+2 pi i jk/N) for N in {2,3,4,5,6,8,10,12,15,16,20},
// by a compile-time Cooley-Tukey split N = F*M (F the first of 4,2,3,5 that
// divides N) down to the radix-2/3/4/5 butterflies.  The internal twiddles
// exp(+2 pi i j/N) are evaluated at compile time from their Taylor series with
// the argument folded into [0, pi/4], so every constant is correctly rounded to
// double.
#pragma once

#include "common.h"

namespace gw {

// ------------------------------------------------------------------ compile-time trig
namespace ct_trig {
constexpr long double kPi = 3.141592653589793238462643383279502884L;
constexpr long double sin_series(long double x) {
  long double term = x, sum = x;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / ((2 * k) * (2 * k + 1));
    sum += term;
  }
  return sum;
}
constexpr long double cos_series(long double x) {
  long double term = 1.0L, sum = 1.0L;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / ((2 * k - 1) * (2 * k));
    sum += term;
  }
  return sum;
}
// cos and sin of 2 pi m / n, reduced by octant with exact integer arithmetic
constexpr void unit(long long m, long long n, long double* c, long double* s) {
  m %= n;
  if (m < 0) m += n;
  const long long q = (4 * m) / n, rem = 4 * m - q * n;
  long double cc = 0, ss = 0;
  if (2 * rem <= n) {
    const long double a = (kPi / 2) * (long double)rem / (long double)n;
    cc = cos_series(a);
    ss = sin_series(a);
  } else {
    const long double a = (kPi / 2) * (long double)(n - rem) / (long double)n;
    cc = sin_series(a);
    ss = cos_series(a);
  }
  switch (q) {
    case 0: *c = cc; *s = ss; break;
    case 1: *c = -ss; *s = cc; break;
    case 2: *c = -cc; *s = -ss; break;
    default: *c = ss; *s = -cc; break;
  }
}
constexpr double cosr(long long m, long long n) {
  long double c = 0, s = 0;
  unit(m, n, &c, &s);
  return (double)c;
}
constexpr double sinr(long long m, long long n) {
  long double c = 0, s = 0;
  unit(m, n, &c, &s);
  return (double)s;
}
}  // namespace ct_trig

// ------------------------------------------------------------------ base butterflies
template <typename T>
__host__ __device__ __forceinline__ void bfly2(cpx<T>* a) {
  cpx<T> t = a[0];
  a[0] = t + a[1];
  a[1] = t - a[1];
}
template <typename T>
__host__ __device__ __forceinline__ void bfly3(cpx<T>* a) {
  const T h = (T)0.86602540378443864676;  // sin(2 pi / 3)
  cpx<T> t1 = a[1] + a[2];
  cpx<T> t2 = a[0] - scal(t1, (T)0.5);
  cpx<T> t3 = scal(mul_i(a[1] - a[2]), h);
  a[0] = a[0] + t1;
  a[1] = t2 + t3;
  a[2] = t2 - t3;
}
template <typename T>
__host__ __device__ __forceinline__ void bfly4(cpx<T>* a) {
  cpx<T> t0 = a[0] + a[2], t1 = a[0] - a[2];
  cpx<T> t2 = a[1] + a[3], t3 = mul_i(a[1] - a[3]);
  a[0] = t0 + t2;
  a[2] = t0 - t2;
  a[1] = t1 + t3;
  a[3] = t1 - t3;
}
template <typename T>
__host__ __device__ __forceinline__ void bfly5(cpx<T>* a) {
  const T c1 = (T)0.30901699437494742410, s1 = (T)0.95105651629515357212;   // 2 pi / 5
  const T c2 = (T)-0.80901699437494742410, s2 = (T)0.58778525229247312917;  // 4 pi / 5
  cpx<T> t1 = a[1] + a[4], t2 = a[2] + a[3];
  cpx<T> t3 = a[1] - a[4], t4 = a[2] - a[3];
  cpx<T> b1 = a[0] + scal(t1, c1) + scal(t2, c2);
  cpx<T> b2 = a[0] + scal(t1, c2) + scal(t2, c1);
  cpx<T> d1 = mul_i(scal(t3, s1) + scal(t4, s2));
  cpx<T> d2 = mul_i(scal(t3, s2) - scal(t4, s1));
  a[0] = a[0] + t1 + t2;
  a[1] = b1 + d1;
  a[4] = b1 - d1;
  a[2] = b2 + d2;
  a[3] = b2 - d2;
}

constexpr int first_factor(int n) {
  return n % 4 == 0 ? 4 : n % 2 == 0 ? 2 : n % 3 == 0 ? 3 : n % 5 == 0 ? 5 : 0;
}

// ------------------------------------------------------------------ register DFT
template <typename T, int N>
__host__ __device__ __forceinline__ void reg_dft(cpx<T>* a) {
  if constexpr (N == 1) {
  } else if constexpr (N == 2) {
    bfly2<T>(a);
  } else if constexpr (N == 3) {
    bfly3<T>(a);
  } else if constexpr (N == 4) {
    bfly4<T>(a);
  } else if constexpr (N == 5) {
    bfly5<T>(a);
  } else {
    constexpr int F = first_factor(N);
    static_assert(F > 0, "length must factor into 2, 3, 5");
    constexpr int M = N / F;
    cpx<T> s[F][M];
#pragma unroll
    for (int n1 = 0; n1 < F; ++n1)
#pragma unroll
      for (int n2 = 0; n2 < M; ++n2) s[n1][n2] = a[n1 + F * n2];
#pragma unroll
    for (int n1 = 0; n1 < F; ++n1) reg_dft<T, M>(s[n1]);
#pragma unroll
    for (int n1 = 1; n1 < F; ++n1)
#pragma unroll
      for (int k2 = 1; k2 < M; ++k2) {
        const T c = (T)ct_trig::cosr((long long)n1 * k2, N);
        const T sn = (T)ct_trig::sinr((long long)n1 * k2, N);
        s[n1][k2] = cmul(s[n1][k2], mk(c, sn));
      }
#pragma unroll
    for (int k2 = 0; k2 < M; ++k2) {
      cpx<T> t[F];
#pragma unroll
      for (int n1 = 0; n1 < F; ++n1) t[n1] = s[n1][k2];
      reg_dft<T, F>(t);
#pragma unroll
      for (int k1 = 0; k1 < F; ++k1) a[k2 + M * k1] = t[k1];
    }
  }
}

// frequency of transform index k on an axis of length n, kept if |f| <= g
// (returns f + g, the index in the compact range), else -1
__device__ __forceinline__ int kept(int k, int n, int g) {
  const int f = (2 * k <= n) ? k : k - n;
  return (f >= -g && f <= g) ? f + g : -1;
}

// Workgroup barrier that orders LDS accesses only: global loads in flight are
// not waited for, so a register prefetch can stay outstanding across it.
__device__ __forceinline__ void lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

constexpr int pow2_at_least(int n) {
  int p = 1;
  while (p < n) p <<= 1;
  return p;
}

// threads per pencil for the two-factor transform of length N (N = N1 * N2)
constexpr int split_n1(int n) {
  return n == 160 ? 8 : n == 30 ? 5 : n == 60 ? 4 : n % 4 == 0 ? 4 : n % 2 == 0 ? 2 : 1;
}

}  // namespace gw
