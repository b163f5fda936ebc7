// Device-side tile bodies shared by the single-call and the batched (many-q)
// kernels: the chi0 band-pair contraction in FP64 and in split-BF16, and a
// plain complex-double GEMM tile.  Included by gemm.hip, lu.hip and plan.hip.
#pragma once

#include "common.h"

namespace gw {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int KT = 16;       // K step (pairs) of the FP64 tiles
constexpr int BK = 32;       // K step (pairs) of the split-BF16 tile = one 16x16x32 MFMA
constexpr int BKP = BK + 8;  // LDS pitch in bf16 (16-byte aligned rows)
constexpr int KFLUSH = 512;  // pairs accumulated in float before the double flush

// upper-triangle tile index -> (ti, tj), ti <= tj, row-major over the triangle
__device__ __forceinline__ void tri_tile(int idx, int nt, int* ti, int* tj) {
  int r = 0, start = 0;
  while (start + (nt - r) <= idx) { start += nt - r; ++r; }
  *ti = r;
  *tj = r + (idx - start);
}

// bf16 round-to-nearest-even from the IEEE-754 binary32 bit pattern (finite inputs).
__device__ __forceinline__ unsigned short bf16_rn_bits(float x) {
  unsigned int u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(unsigned short h) {
  return __uint_as_float(((unsigned int)h) << 16);
}

// Add a finished tile to C (Hermitian update): (i,j) gets the value, and for an
// off-diagonal tile (j,i) gets its conjugate.  Row/column skip_head is left out.
// A diagonal tile keeps its upper triangle only, mirrors it, and takes the
// diagonal as real, so that chi0 is Hermitian to the last bit.
__device__ __forceinline__ bool herm_keep(bool diag_tile, int i, int j, double* im, bool* offdiag) {
  if (!diag_tile) {
    *offdiag = true;
    return true;
  }
  if (i > j) return false;
  if (i == j) *im = 0.0;
  *offdiag = i < j;
  return true;
}

__device__ __forceinline__ void herm_add(cpx<double>* C, int neps, int i, int j, double re,
                                         double im, bool offdiag, int skip_head) {
  if (i >= neps || j >= neps) return;
  if (skip_head >= 0 && (i == skip_head || j == skip_head)) return;
  cpx<double>* d = C + (size_t)i * neps + j;
  *d = mk(d->x + re, d->y + im);
  if (offdiag) {
    cpx<double>* m = C + (size_t)j * neps + i;
    *m = mk(m->x + re, m->y - im);
  }
}

// Store a finished tile into a partial-sum matrix: (i,j) gets the value and, off
// the diagonal, (j,i) its conjugate; the skipped row/column get zeros so that
// every entry of the matrix is defined.
__device__ __forceinline__ void herm_store(cpx<double>* C, int neps, int i, int j, double re,
                                           double im, bool offdiag, int skip_head) {
  if (i >= neps || j >= neps) return;
  if (skip_head >= 0 && (i == skip_head || j == skip_head)) re = im = 0.0;
  C[(size_t)i * neps + j] = mk(re, im);
  if (offdiag) C[(size_t)j * neps + i] = mk(re, -im);
}

// ------------------------------------------------------------------ FP64 chi0 tile, direct LDS loads
// The 64x64 complex-double tile (2x2 wavefronts of 32x32) with its operand rows
// loaded straight into LDS by global_load_lds_dwordx4: a row of 64 columns of
// M (1 KiB) is one wavefront instruction, each lane's 16 bytes landing at
// lane * 16 of the row, so the slab needs no registers, no VALU and no LDS
// stores on its way in. Two slabs of 12 pairs alternate (49 KiB of LDS, so
// three workgroups fit a CU); the next one is in
// flight while the matrix cores work on the current one, and one barrier per
// slab both publishes it and retires the old one. The weight w[p] multiplies
// the B fragment as it is read; pairs past P read row P-1 and get weight 0,
// and columns past neps read column neps-1 and feed outputs that are not
// stored, so no operand needs a mask.
typedef __attribute__((address_space(3))) void lds_void;
__device__ __forceinline__ void chi0_f64_tile_dl(const cpx<double>* __restrict__ M, int P,
                                                 int neps, const double* __restrict__ w,
                                                 cpx<double>* __restrict__ C, int ti, int tj,
                                                 int skip_head, bool overwrite) {
  constexpr int TMv = 64, KD = 12;  // pairs per slab: 3 rows per wavefront and operand
  static_assert(KD % 4 == 0, "each wavefront loads KD/4 rows of each operand");
  // two slabs as separate LDS objects, so that the compiler can tell the
  // in-flight loads into one from the reads of the other
  __shared__ __align__(16) cpx<double> As0[KD][TMv], Bs0[KD][TMv];
  __shared__ __align__(16) cpx<double> As1[KD][TMv], Bs1[KD][TMv];
  __shared__ double Ws0[KD], Ws1[KD];
  const int i0 = ti * TMv, j0 = tj * TMv;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int l16 = lane & 15, lk = lane >> 4;
  const int ca = min(i0 + lane, neps - 1), cb = min(j0 + lane, neps - 1);
  d4 t1[2][2], t2[2][2], t3[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      t1[a][b] = (d4){0, 0, 0, 0};
      t2[a][b] = (d4){0, 0, 0, 0};
      t3[a][b] = (d4){0, 0, 0, 0};
    }
  // rows wave*KD/4 .. of both operands of the slab at p0
  auto issue = [&](cpx<double> (*As)[TMv], cpx<double> (*Bs)[TMv], int p0) {
#pragma unroll
    for (int r = 0; r < KD / 4; ++r) {
      const int kk = wave * (KD / 4) + r;
      const size_t row = (size_t)min(p0 + kk, P - 1) * neps;
      __builtin_amdgcn_global_load_lds((const void*)(M + row + ca), (lds_void*)&As[kk][0], 16, 0,
                                       0);
      __builtin_amdgcn_global_load_lds((const void*)(M + row + cb), (lds_void*)&Bs[kk][0], 16, 0,
                                       0);
    }
  };
  auto weight = [&](int p0) { return (tid < KD && p0 + tid < P) ? w[p0 + tid] : 0.0; };
  auto compute = [&](const cpx<double> (*As)[TMv], const cpx<double> (*Bs)[TMv],
                     const double* Ws) {
#pragma unroll
    for (int s = 0; s < KD / 4; ++s) {
      const int kk = s * 4 + lk;
      const double wk = Ws[kk];
      cpx<double> av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = As[kk][wr * 32 + a * 16 + l16];
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const cpx<double> v = Bs[kk][wc * 32 + b * 16 + l16];
        bv[b] = mk(wk * v.x, wk * v.y);
      }
      double dd[2], ss[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) dd[a] = av[a].x - av[a].y;
#pragma unroll
      for (int b = 0; b < 2; ++b) ss[b] = bv[b].x + bv[b].y;
      // t1 = sum ar br, t2 = sum ai bi, t3 = sum (ar - ai)(br + bi): Re conj(a) b
      // = t1 + t2 and Im = t3 - t1 + t2
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          t1[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a].x, bv[b].x, t1[a][b], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          t2[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a].y, bv[b].y, t2[a][b], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          t3[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(dd[a], ss[b], t3[a][b], 0, 0, 0);
    }
  };
  // one slab step: compute from (Ac, Bc, Wc) while the slab at pn streams into
  // (An, Bn, Wn); this wavefront's loads land before the barrier, which makes
  // every wavefront's visible and ends the reads of the current slab
  auto step = [&](const cpx<double> (*Ac)[TMv], const cpx<double> (*Bc)[TMv], const double* Wc,
                  cpx<double> (*An)[TMv], cpx<double> (*Bn)[TMv], double* Wn, int pn) {
    const bool more = pn < P;
    double wn = 0.0;
    if (more) {
      issue(An, Bn, pn);
      wn = weight(pn);
    }
    compute(Ac, Bc, Wc);
    if (more && tid < KD) Wn[tid] = wn;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  };
  issue(As0, Bs0, 0);
  const double w0 = weight(0);
  if (tid < KD) Ws0[tid] = w0;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  for (int p0 = 0; p0 < P; p0 += 2 * KD) {
    step(As0, Bs0, Ws0, As1, Bs1, Ws1, p0 + KD);
    if (p0 + KD < P) step(As1, Bs1, Ws1, As0, Bs0, Ws0, p0 + 2 * KD);
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {  // f64 16x16x4 D layout: row lk + 4r, column l16
        const int i = i0 + wr * 32 + a * 16 + lk + 4 * r, j = j0 + wc * 32 + b * 16 + l16;
        const double re = t1[a][b][r] + t2[a][b][r];
        double im = (t3[a][b][r] - t1[a][b][r]) + t2[a][b][r];
        bool od;
        if (!herm_keep(ti == tj, i, j, &im, &od)) continue;
        if (overwrite) herm_store(C, neps, i, j, re, im, od, skip_head);
        else herm_add(C, neps, i, j, re, im, od, skip_head);
      }
}

// ------------------------------------------------------------------ FP64 chi0 tile
// C[i][j] += sum_p conj(M[p][i]) w[p] M[p][j] for the (TM x TM) tile (ti, tj),
// TM = 32*WM, WM x WM waves of 32x32 (2x2 blocks of v_mfma_f64_16x16x4_f64).
// Planar re/im LDS tiles padded so each quarter-wave row group lands on its own
// half of the banks; the next K-tile is fetched into registers (clamped
// addresses, masked at the store) while the matrix cores work on this one.
template <int WM, typename Tin>
__device__ __forceinline__ void chi0_f64_tile(const cpx<Tin>* __restrict__ M, int P, int neps,
                                              const double* __restrict__ w,
                                              cpx<double>* __restrict__ C, int ti, int tj,
                                              int skip_head, bool overwrite = false) {
  if constexpr (WM == 2 && sizeof(Tin) == 8) {
    chi0_f64_tile_dl(reinterpret_cast<const cpx<double>*>(M), P, neps, w, C, ti, tj, skip_head,
                     overwrite);
    return;
  }
  constexpr int TMv = 32 * WM, NT = 64 * WM * WM, NE = (KT * TMv) / NT, PTv = TMv + 16;
  __shared__ double Ar[KT][PTv], Ai[KT][PTv], Br[KT][PTv], Bi[KT][PTv];
  const int i0 = ti * TMv, j0 = tj * TMv;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave / WM, wc = wave % WM;
  const int l16 = lane & 15, lk = lane >> 4;
  // t1 = sum ar br, t2 = sum ai bi, t3 = sum (ar - ai)(br + bi); then
  // Re conj(a) b = t1 + t2 and Im = t3 - t1 + t2 (three real products per
  // complex one instead of four)
  d4 t1[2][2], t2[2][2], t3[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      t1[a][b] = (d4){0, 0, 0, 0};
      t2[a][b] = (d4){0, 0, 0, 0};
      t3[a][b] = (d4){0, 0, 0, 0};
    }
  cpx<Tin> ra[NE], rb[NE];
  double rw[NE];
  auto gload = [&](int p0) {
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const int idx = tid + e * NT;
      const int kk = idx / TMv, ii = idx % TMv;
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
      const int idx = tid + e * NT;
      const int kk = idx / TMv, ii = idx % TMv;
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
      double dd[2], ss[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) dd[a] = ar[a] - ai[a];
#pragma unroll
      for (int b = 0; b < 2; ++b) ss[b] = br[b] + bi[b];
      // the three products are issued round-robin over the twelve accumulators
      // so that no MFMA waits on the one just issued
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          t1[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[a], br[b], t1[a][b], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          t2[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[a], bi[b], t2[a][b], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          t3[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(dd[a], ss[b], t3[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {  // f64 16x16x4 D layout: row lk + 4r, column l16
        const int i = i0 + wr * 32 + a * 16 + lk + 4 * r, j = j0 + wc * 32 + b * 16 + l16;
        const double re = t1[a][b][r] + t2[a][b][r];
        double im = (t3[a][b][r] - t1[a][b][r]) + t2[a][b][r];
        bool od;
        if (!herm_keep(ti == tj, i, j, &im, &od)) continue;
        if (overwrite) herm_store(C, neps, i, j, re, im, od, skip_head);
        else herm_add(C, neps, i, j, re, im, od, skip_head);
      }
}

// ------------------------------------------------------------------ split-BF16 chi0 tile
// Each float x = hi + lo, hi = bf16_rn(x), lo = bf16_rn(x - hi); every real
// product is hi*hi + hi*lo + lo*hi on v_mfma_f32_16x16x32_bf16 with float
// accumulation flushed into double registers every KFLUSH pairs. The operands
// are split once in advance (k_bf16_split): X[pb][q][G][32] holds, for pair
// block pb (32 pairs, zero-padded past P) and plane q = (re hi, re lo, im hi,
// im lo), the bf16 bits of column G. A slab is then a contiguous 4 KiB per
// plane and is staged with 16-byte loads and LDS stores, leaving the VALU free
// for the MFMA issue.
// WM = 2 form of the pre-split tile with the slabs loaded straight into LDS by
// global_load_lds_dwordx4 (one wavefront instruction = 16 rows x 64 bytes of
// one plane), into two slabs kept as separate LDS objects and alternated, one
// barrier per slab. Rows are stored unpadded; the four 16-byte chunks of row r
// are permuted by XOR with (r >> 1) & 3 on the way in and on the way out. With
// that permutation a fragment read (16 rows of 64 bytes, one chunk each) takes
// as many LDS cycles as a contiguous 1 KiB read, by the bank-conflict counter;
// ((r >> 1) ^ (r >> 3)) & 3, (r & 3), (r >> 2) & 3 and no permutation all take
// twice as many.
__device__ __forceinline__ void chi0_bf16s_tile_dl(const unsigned short* __restrict__ XA,
                                                   const unsigned short* __restrict__ XB, int pb0,
                                                   int npb, int neps, cpx<double>* __restrict__ C,
                                                   int ti, int tj, int skip_head, bool overwrite) {
  constexpr int TMv = 64;
  __shared__ __align__(16) unsigned short As0[4][TMv][BK], Bs0[4][TMv][BK];
  __shared__ __align__(16) unsigned short As1[4][TMv][BK], Bs1[4][TMv][BK];
  typedef unsigned short (*Slab)[TMv][BK];
  const int i0 = ti * TMv, j0 = tj * TMv;
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
  // this lane's row within a 16-row block and the logical chunk it carries
  const int lrow = lane >> 2, lchunk = (lane & 3) ^ ((lrow >> 1) & 3);
  const int ra = min(i0 + lrow, neps - 1), rb = min(j0 + lrow, neps - 1);
  // the wavefront's 8 of the slab's 32 row blocks (operand, plane, 16-row block)
  auto issue = [&](Slab A, Slab B, int pb) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = wave * 8 + u, opnd = idx >> 4, q = (idx >> 2) & 3, blk = idx & 3;
      const size_t plane = ((size_t)pb * 4 + q) * neps;
      const unsigned short* src =
          (opnd ? XB + (plane + min(rb + 16 * blk, neps - 1)) * BK
                : XA + (plane + min(ra + 16 * blk, neps - 1)) * BK) + lchunk * 8;
      unsigned short* dst = opnd ? &B[q][16 * blk][0] : &A[q][16 * blk][0];
      __builtin_amdgcn_global_load_lds((const void*)src, (lds_void*)dst, 16, 0, 0);
    }
  };
  // physical chunk of logical chunk lk in this lane's fragment rows
  const int pch = (lk ^ ((l16 >> 1) & 3)) * 8;
  int since_flush = 0;
  auto compute = [&](Slab A, Slab B, bool last) {
    bf8 a[2][4], b[2][4];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[x][q] = *reinterpret_cast<const bf8*>(&A[q][wr * 32 + x * 16 + l16][pch]);
        b[x][q] = *reinterpret_cast<const bf8*>(&B[q][wc * 32 + x * 16 + l16][pch]);
      }
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
#define GW_MF(ACC, A_, B_)                                                    \
  _Pragma("unroll") for (int x = 0; x < 2; ++x) _Pragma("unroll") for (int y = 0; y < 2; ++y) \
      ACC[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A_, B_, ACC[x][y], 0, 0, 0);
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
    if (since_flush >= KFLUSH || last) {
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
  };
  // compute from (Ac, Bc) while the slab pn streams into (An, Bn); this
  // wavefront's loads land before the barrier, which publishes every
  // wavefront's and ends the reads of the current slab
  const int pend = pb0 + npb;
  auto step = [&](Slab Ac, Slab Bc, Slab An, Slab Bn, int pn) {
    if (pn < pend) issue(An, Bn, pn);
    compute(Ac, Bc, pn >= pend);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  };
  if (npb <= 0) return;
  issue(As0, Bs0, pb0);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  for (int pb = pb0; pb < pend; pb += 2) {
    step(As0, Bs0, As1, Bs1, pb + 1);
    if (pb + 1 < pend) step(As1, Bs1, As0, Bs0, pb + 2);
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {  // f32 16x16x32 D layout: row 4*lk + r, column l16
        const int i = i0 + wr * 32 + x * 16 + lk * 4 + r, j = j0 + wc * 32 + y * 16 + l16;
        double im = di[x][y][r];
        bool od;
        if (!herm_keep(ti == tj, i, j, &im, &od)) continue;
        if (overwrite) herm_store(C, neps, i, j, dr[x][y][r], im, od, skip_head);
        else herm_add(C, neps, i, j, dr[x][y][r], im, od, skip_head);
      }
}

// ------------------------------------------------------------------ split-BF16 chi0 tile, 128 x 128
// The contraction's operand traffic per flop falls with the tile edge: a 64 x 64
// tile streams 32 KiB of staged operands per 32-pair slab for 3.1 MFLOP, which
// at the matrix cores' rate needs more operand feed than L2 and the CU's load
// path give. This tile is 128 x 128 on 8 wavefronts of 64 x 32 (4 x 2 blocks
// of v_mfma_f32_16x16x32_bf16): per slab 64 KiB in, 12.6 MFLOP, and each
// wavefront reads 24 fragments of 1 KiB from LDS for 96 MFMAs.
//   - Slabs go straight into LDS with global_load_lds_dwordx4 (16 rows x 64 B
//     of one plane per wavefront instruction, 8 per wavefront per slab), into
//     two slabs kept as separate LDS objects (128 KiB) and alternated, one
//     barrier per slab; the chunk XOR swizzle is the 64 x 64 tile's.
//   - The accumulation stays in float over the whole pair range of the
//     workgroup (the caller bounds it at 8192 pairs, 256 MFMA accumulations);
//     ranges are added in double.
constexpr int WT = 128;  // tile edge of chi0_bf16s_tile_w
__device__ __forceinline__ void chi0_bf16s_tile_w(const unsigned short* __restrict__ XA,
                                                  const unsigned short* __restrict__ XB, int pb0,
                                                  int npb, int neps, cpx<double>* __restrict__ C,
                                                  int ti, int tj, int skip_head, bool overwrite) {
  __shared__ __align__(16) unsigned short As0[4][WT][BK], Bs0[4][WT][BK];
  __shared__ __align__(16) unsigned short As1[4][WT][BK], Bs1[4][WT][BK];
  typedef unsigned short (*Slab)[WT][BK];
  const int i0 = ti * WT, j0 = tj * WT;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 2, wc = wave & 3;  // rows wr*64 .. +63, columns wc*32 .. +31
  const int l16 = lane & 15, lk = lane >> 4;
  // imaginary part = cp - cn: the conjugated operand's minus sign is taken
  // at the end instead of negating fragments in the loop
  f4 cr[4][2], cp[4][2], cn[4][2];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      cr[x][y] = (f4){0, 0, 0, 0};
      cp[x][y] = (f4){0, 0, 0, 0};
      cn[x][y] = (f4){0, 0, 0, 0};
    }
  const int lrow = lane >> 2, lchunk = (lane & 3) ^ ((lrow >> 1) & 3);
  // the wavefront's 8 of the slab's 64 row blocks (operand, plane, 16-row block)
  auto issue = [&](Slab A, Slab B, int pb) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = wave * 8 + u, opnd = idx >> 5, q = (idx >> 3) & 3, blk = idx & 7;
      const size_t plane = ((size_t)pb * 4 + q) * neps;
      const int r = 16 * blk + lrow;
      const unsigned short* src =
          (opnd ? XB + (plane + min(j0 + r, neps - 1)) * BK
                : XA + (plane + min(i0 + r, neps - 1)) * BK) + lchunk * 8;
      unsigned short* dst = opnd ? &B[q][16 * blk][0] : &A[q][16 * blk][0];
      __builtin_amdgcn_global_load_lds((const void*)src, (lds_void*)dst, 16, 0, 0);
    }
  };
  const int pch = (lk ^ ((l16 >> 1) & 3)) * 8;
  auto compute = [&](Slab A, Slab B) {
    bf8 b[2][4];
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        b[y][q] = *reinterpret_cast<const bf8*>(&B[q][wc * 32 + y * 16 + l16][pch]);
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      bf8 a[4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        a[q] = *reinterpret_cast<const bf8*>(&A[q][wr * 64 + x * 16 + l16][pch]);
      // the two column blocks interleaved, and the six real-part products
      // spread between the others, so that no accumulator is updated by
      // consecutive instructions
#define GW_MF(ACC, A_, Q)                                                                         \
  ACC[x][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A_, b[0][Q], ACC[x][0], 0, 0, 0);           \
  ACC[x][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A_, b[1][Q], ACC[x][1], 0, 0, 0);
      GW_MF(cr, a[0], 0)
      GW_MF(cp, a[0], 2)
      GW_MF(cr, a[0], 1)
      GW_MF(cn, a[2], 0)
      GW_MF(cr, a[1], 0)
      GW_MF(cp, a[0], 3)
      GW_MF(cr, a[2], 2)
      GW_MF(cn, a[2], 1)
      GW_MF(cr, a[2], 3)
      GW_MF(cp, a[1], 2)
      GW_MF(cr, a[3], 2)
      GW_MF(cn, a[3], 0)
#undef GW_MF
    }
  };
  const int pend = pb0 + npb;
  auto step = [&](Slab Ac, Slab Bc, Slab An, Slab Bn, int pn) {
    if (pn < pend) issue(An, Bn, pn);
    compute(Ac, Bc);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  };
  if (npb > 0) {
    issue(As0, Bs0, pb0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int pb = pb0; pb < pend; pb += 2) {
      step(As0, Bs0, As1, Bs1, pb + 1);
      if (pb + 1 < pend) step(As1, Bs1, As0, Bs0, pb + 2);
    }
  }
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {  // f32 16x16x32 D layout: row 4*lk + r, column l16
        const int i = i0 + wr * 64 + x * 16 + lk * 4 + r, j = j0 + wc * 32 + y * 16 + l16;
        double im = (double)cp[x][y][r] - (double)cn[x][y][r];
        bool od;
        if (!herm_keep(ti == tj, i, j, &im, &od)) continue;
        if (overwrite) herm_store(C, neps, i, j, (double)cr[x][y][r], im, od, skip_head);
        else herm_add(C, neps, i, j, (double)cr[x][y][r], im, od, skip_head);
      }
}

template <int WM>
__device__ __forceinline__ void chi0_bf16s_tile(const unsigned short* __restrict__ XA,
                                                const unsigned short* __restrict__ XB, int pb0,
                                                int npb, int neps, cpx<double>* __restrict__ C,
                                                int ti, int tj, int skip_head, bool overwrite) {
  if constexpr (WM == 2) {
    chi0_bf16s_tile_dl(XA, XB, pb0, npb, neps, C, ti, tj, skip_head, overwrite);
    return;
  }
  constexpr int TMv = 32 * WM, NT = 64 * WM * WM;
  constexpr int CH = 4 * TMv * (BK / 8);  // 16-byte chunks per operand slab
  constexpr int NE = CH / NT;
  static_assert(CH % NT == 0, "whole chunks per thread");
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  __shared__ __align__(16) unsigned short As[4][TMv][BKP];
  __shared__ __align__(16) unsigned short Bs[4][TMv][BKP];
  const int i0 = ti * TMv, j0 = tj * TMv;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave / WM, wc = wave % WM;
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
  u4 ra[NE], rb[NE];
  auto gload = [&](int pb) {
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const int c = tid + e * NT;
      const int q = c / (TMv * 4), row = (c / 4) % TMv, kc = c % 4;
      const size_t base = ((size_t)pb * 4 + q) * neps;
      ra[e] = *reinterpret_cast<const u4*>(XA + (base + min(i0 + row, neps - 1)) * BK + kc * 8);
      rb[e] = *reinterpret_cast<const u4*>(XB + (base + min(j0 + row, neps - 1)) * BK + kc * 8);
    }
  };
  gload(pb0);
  for (int pb = pb0; pb < pb0 + npb; ++pb) {
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const int c = tid + e * NT;
      const int q = c / (TMv * 4), row = (c / 4) % TMv, kc = c % 4;
      *reinterpret_cast<u4*>(&As[q][row][kc * 8]) = ra[e];
      *reinterpret_cast<u4*>(&Bs[q][row][kc * 8]) = rb[e];
    }
    __syncthreads();
    if (pb + 1 < pb0 + npb) gload(pb + 1);
    bf8 a[2][4], b[2][4];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[x][q] = *reinterpret_cast<const bf8*>(&As[q][wr * 32 + x * 16 + l16][lk * 8]);
        b[x][q] = *reinterpret_cast<const bf8*>(&Bs[q][wc * 32 + x * 16 + l16][lk * 8]);
      }
    // the fragments are in registers: the slab may be restaged after this point
    __syncthreads();
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
#define GW_MF(ACC, A, B)                                                      \
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
    if (since_flush >= KFLUSH || pb + 1 >= pb0 + npb) {
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
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {  // f32 16x16x32 D layout: row 4*lk + r, column l16
        const int i = i0 + wr * 32 + x * 16 + lk * 4 + r, j = j0 + wc * 32 + y * 16 + l16;
        double im = di[x][y][r];
        bool od;
        if (!herm_keep(ti == tj, i, j, &im, &od)) continue;
        if (overwrite) herm_store(C, neps, i, j, dr[x][y][r], im, od, skip_head);
        else herm_add(C, neps, i, j, dr[x][y][r], im, od, skip_head);
      }
}

// ------------------------------------------------------------------ 64x64 Gauss-Jordan inverse
// In-place inverse of the leading nbk x nbk block of a 64x64 matrix held by a
// workgroup of TG*TG threads: thread (ti, tj) = (tid / TG, tid % TG) holds
// entries (ti + TG a, tj + TG b) in d[a][b], the identity outside nbk (which
// leaves the leading inverse unchanged). Gauss-Jordan without pivoting; step t:
//   - the TG lanes that hold row t (one group inside a wavefront) take the
//     pivot p from the lane on the diagonal, form 1/p (hardware reciprocal and
//     two Newton steps), and publish row t times 1/p with 1/p at the pivot: that
//     is also the row's final value;
//   - the lanes that hold column t publish it with a zero in row t, and clear
//     their entries of it outside row t;
//   - after one barrier every thread subtracts col(i) row(j) from each entry.
// Only the owners of the pivot row and column branch, and 1/p is formed once
// per step. rowb and colb are two LDS buffers of 64 each, alternating by step
// parity. Returns true on the diagonal lane of a step whose pivot is not real
// and >= 1/2, which I minus a negative semidefinite matrix cannot give.
template <int TG>
__device__ __forceinline__ bool gj_invert_64(cpx<double> (&d)[64 / TG][64 / TG], int nbk,
                                             cpx<double> (*rowb)[64], cpx<double> (*colb)[64]) {
  constexpr int TE = 64 / TG;
  static_assert(TG * TE == 64 && 64 % TG == 0, "a row's owners must share a wavefront");
  const int tid = threadIdx.x, ti = tid / TG, tj = tid % TG;
  bool bad = false;
  for (int t = 0; t < nbk; ++t) {
    const int buf = t & 1, ta = t / TG, tr = t % TG;
    if (ti == tr) {
      cpx<double> own = d[0][0];
#pragma unroll
      for (int q = 1; q < TE; ++q)
        if (ta == q) own = d[q][q];
      const int src = (tid & 63 & ~(TG - 1)) + tr;  // the diagonal lane of this group
      const cpx<double> p = mk(__shfl(own.x, src), __shfl(own.y, src));
      if (tj == tr && !(p.x >= 0.5 && fabs(p.y) <= 0.25 * p.x && p.x < INFINITY)) bad = true;
      const double den = p.x * p.x + p.y * p.y;
      double r = __builtin_amdgcn_rcp(den);
      r = fma(r, fma(-den, r, 1.0), r);
      r = fma(r, fma(-den, r, 1.0), r);
      const cpx<double> pinv = den > 0.0 ? mk(p.x * r, -p.y * r) : mk(0.0, 0.0);
#pragma unroll
      for (int q = 0; q < TE; ++q)
        if (ta == q) {
#pragma unroll
          for (int b = 0; b < TE; ++b) {
            const int j = tj + TG * b;
            const cpx<double> v = j == t ? pinv : cmul(d[q][b], pinv);
            rowb[buf][j] = v;
            d[q][b] = v;
          }
        }
    }
    if (tj == tr) {
#pragma unroll
      for (int q = 0; q < TE; ++q)
        if (ta == q) {
#pragma unroll
          for (int a = 0; a < TE; ++a) {
            // row t's entry was replaced by 1/p above (same lane) and is not read
            if (ti + TG * a == t) {
              colb[buf][t] = mk(0.0, 0.0);
            } else {
              colb[buf][ti + TG * a] = d[a][q];
              d[a][q] = mk(0.0, 0.0);
            }
          }
        }
    }
    __syncthreads();
    cpx<double> rs[TE], cc[TE];
#pragma unroll
    for (int b = 0; b < TE; ++b) rs[b] = rowb[buf][tj + TG * b];
#pragma unroll
    for (int a = 0; a < TE; ++a) cc[a] = colb[buf][ti + TG * a];
#pragma unroll
    for (int a = 0; a < TE; ++a)
#pragma unroll
      for (int b = 0; b < TE; ++b) {
        const double xr = fma(-cc[a].x, rs[b].x, d[a][b].x);
        const double xi = fma(-cc[a].x, rs[b].y, d[a][b].y);
        d[a][b] = mk(fma(cc[a].y, rs[b].y, xr), fma(-cc[a].y, rs[b].x, xi));
      }
    // the other buffer pair was last read before this step's barrier
  }
  return bad;
}

// ------------------------------------------------------------------ Gauss-Jordan rank-update tile
// dst = A - Cb R on one 64x64 tile (i0, j0 per wavefront: 2x2 wavefronts of
// 32x32) for K = kdim <= 64, rows and columns below lim, dst entry (i, j) at
// (i - doff) * ldd + (j - doff). No LDS and no barrier: fragments come straight
// from Cb (N x ldcb) and R (kdim x N, row stride N), which stay in L2, with the
// next four K loaded while the current ones feed the matrix cores; 2x2
// v_mfma_f64_16x16x4_f64 blocks, three real products per complex one; A is read
// in the epilogue (dst may be A: each entry is read before it is written, by
// the same lane).
__device__ __forceinline__ void gj_update_tile(const cpx<double>* __restrict__ Cb, int ldcb,
                                               const cpx<double>* __restrict__ R,
                                               const cpx<double>* A, int N, int kdim,
                                               int i0, int j0, int lim, cpx<double>* dst,
                                               int ldd, int doff) {
  const int lane = threadIdx.x & 63;
  const int l16 = lane & 15, lk = lane >> 4;
  // fragment rows of Cb and columns of R; rows or columns past N are clamped
  // (their products land in outputs that are not stored)
  const int ia[2] = {min(i0 + l16, N - 1), min(i0 + 16 + l16, N - 1)};
  const int jb[2] = {min(j0 + l16, N - 1), min(j0 + 16 + l16, N - 1)};
  d4 t1[2][2], t2[2][2], t3[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      t1[a][b] = (d4){0, 0, 0, 0};
      t2[a][b] = (d4){0, 0, 0, 0};
      t3[a][b] = (d4){0, 0, 0, 0};
    }
  // K past kdim reads row/column kdim - 1 and is zeroed by selection (stale
  // panel entries may hold anything, so they are never multiplied)
  auto load = [&](int k0, cpx<double> (&fa)[2], cpx<double> (&fb)[2]) {
    const int k = k0 + lk, kc = min(k, kdim - 1);
    const bool ok = k < kdim;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const cpx<double> v = Cb[(size_t)ia[a] * ldcb + kc];
      fa[a] = ok ? v : mk(0.0, 0.0);
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const cpx<double> v = R[(size_t)kc * N + jb[b]];
      fb[b] = ok ? v : mk(0.0, 0.0);
    }
  };
  cpx<double> fa[2], fb[2];
  load(0, fa, fb);
  for (int k0 = 0; k0 < kdim; k0 += 4) {
    cpx<double> na[2], nb[2];
    if (k0 + 4 < kdim) load(k0 + 4, na, nb);
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
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      fa[a] = na[a];
      fb[a] = nb[a];
    }
  }
  // dst = A - product for rows and columns below lim: Re = t1 - t2,
  // Im = t3 - t1 - t2 (f64 16x16x4 D layout: row lk + 4r, column l16)
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + a * 16 + lk + 4 * r, j = j0 + b * 16 + l16;
        if (i < lim && j < lim) {
          const cpx<double> v = A[(size_t)i * N + j];
          dst[(size_t)(i - doff) * ldd + (j - doff)] =
              mk(v.x - (t1[a][b][r] - t2[a][b][r]),
                 v.y - ((t3[a][b][r] - t1[a][b][r]) - t2[a][b][r]));
        }
      }
}

// ------------------------------------------------------------------ complex-double GEMM tile
// C[i][j] = alpha * sum_k A[i][k] B[k][j] + beta * C[i][j] on the 64x64 tile at
// (i0, j0), 256 threads (beta is 0 or 1).
//   - Three real products per complex one: t1 = ar br, t2 = ai bi,
//     t3 = (ar + ai)(br + bi); Re = t1 - t2 and Im = t3 - t1 - t2.
//   - With beta 1 the accumulators start from C (t1 = Re C, t3 = Re C + Im C),
//     loaded before the first slab, so reading C overlaps the slab loads and
//     the epilogue is a plain store.
//   - alpha scales A as it is staged in LDS.
//   - K advances in slabs of KT through two LDS buffers; the next slab is
//     loaded into registers while the current one feeds the MFMAs, so there
//     is one barrier per slab.
constexpr int ZTM = 64, ZLP = ZTM + 1;
__device__ __forceinline__ void zgemm_tile(int m, int n, int kdim, double alpha, double beta,
                                           const cpx<double>* __restrict__ A, int lda,
                                           const cpx<double>* __restrict__ B, int ldb,
                                           cpx<double>* __restrict__ C, int ldc, int i0, int j0) {
  __shared__ cpx<double> As[2][KT][ZLP];
  __shared__ cpx<double> Bs[2][KT][ZLP];
  constexpr int PER = (KT * ZTM) / 256;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int l16 = lane & 15, lk = lane >> 4;
  d4 t1[2][2], t2[2][2], t3[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {  // f64 16x16x4 D layout: row lk + 4r, column l16
        const int i = i0 + wr * 32 + a * 16 + lk + 4 * r, j = j0 + wc * 32 + b * 16 + l16;
        cpx<double> v = mk(0.0, 0.0);
        if (beta != 0.0 && i < m && j < n) v = C[(size_t)i * ldc + j];
        t1[a][b][r] = v.x;
        t2[a][b][r] = 0.0;
        t3[a][b][r] = v.x + v.y;
      }
  cpx<double> ra[PER], rb[PER];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int idx = tid + e * 256;
      // A slab: ZTM rows x KT columns, k fastest for coalescing
      const int ai = idx / KT, ak = idx % KT;
      ra[e] = (i0 + ai < m && k0 + ak < kdim) ? A[(size_t)(i0 + ai) * lda + k0 + ak]
                                              : mk<double>(0, 0);
      const int bk = idx / ZTM, bj = idx % ZTM;
      rb[e] = (k0 + bk < kdim && j0 + bj < n) ? B[(size_t)(k0 + bk) * ldb + j0 + bj]
                                              : mk<double>(0, 0);
    }
  };
  fetch(0);
  int buf = 0;
  for (int k0 = 0; k0 < kdim; k0 += KT) {
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int idx = tid + e * 256;
      As[buf][idx % KT][idx / KT] = scal(ra[e], alpha);
      Bs[buf][idx / ZTM][idx % ZTM] = rb[e];
    }
    __syncthreads();
    if (k0 + KT < kdim) fetch(k0 + KT);
#pragma unroll
    for (int s = 0; s < KT / 4; ++s) {
      const int kk = s * 4 + lk;
      cpx<double> av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = As[buf][kk][wr * 32 + a * 16 + l16];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = Bs[buf][kk][wc * 32 + b * 16 + l16];
      double sa[2], sb[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) sa[a] = av[a].x + av[a].y;
#pragma unroll
      for (int b = 0; b < 2; ++b) sb[b] = bv[b].x + bv[b].y;
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          t1[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a].x, bv[b].x, t1[a][b], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          t2[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a].y, bv[b].y, t2[a][b], 0, 0, 0);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          t3[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(sa[a], sb[b], t3[a][b], 0, 0, 0);
    }
    // the other buffer was last read before this slab's barrier, so the next
    // slab can be stored into it without another barrier
    buf ^= 1;
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wr * 32 + a * 16 + lk + 4 * r;
        const int j = j0 + wc * 32 + b * 16 + l16;
        if (i < m && j < n)
          C[(size_t)i * ldc + j] = mk(t1[a][b][r] - t2[a][b][r],
                                      (t3[a][b][r] - t1[a][b][r]) - t2[a][b][r]);
      }
}

}  // namespace gw
