// Internal definitions shared by the libgwspinor translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <map>
#include <memory>
#include <set>
#include <string>
#include <vector>

#include "../../include/gw.h"

namespace gw {

// ---------------------------------------------------------------- complex
template <typename T> struct cpx { T x, y; };

template <typename T>
__host__ __device__ __forceinline__ cpx<T> mk(T a, T b) { cpx<T> r; r.x = a; r.y = b; return r; }
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename T>
__host__ __device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename T>
__host__ __device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
template <typename T>
__host__ __device__ __forceinline__ cpx<T> cmulc(cpx<T> a, cpx<T> b) {
  return mk(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
template <typename T>
__host__ __device__ __forceinline__ cpx<T> scal(cpx<T> a, T s) { return mk(a.x * s, a.y * s); }
// multiply by +i
template <typename T>
__host__ __device__ __forceinline__ cpx<T> mul_i(cpx<T> a) { return mk(-a.y, a.x); }

// Workgroups are dispatched to the 8 XCDs round-robin by linear id, and each XCD
// has its own L2.  Renumber so that XCD k receives the k-th contiguous slice of
// the logical order (a grid of kXcd * ceil(total / kXcd) blocks); returns -1
// for padding blocks.
constexpr int kXcd = 8;
__device__ __forceinline__ long long xcd_linear(long long b, long long total) {
  const long long per = (total + kXcd - 1) / kXcd;
  const long long l = (b % kXcd) * per + b / kXcd;
  return l < total ? l : -1;
}

// ---------------------------------------------------------------- FFT plan
// Length n = product of radices (each 2, 3, 4 or 5), executed as Stockham passes.
struct FftPlan {
  int n;
  int npass;
  int radix[12];
};
FftPlan make_fft_plan(int n);  // n must factor into 2, 3, 5

// ---------------------------------------------------------------- geometry
// A G-sphere placed in a box: compact cube [2gx+1][2gy+1][2gz+1] -> sphere index or -1.
struct SphereMap {
  int gmax[3];
  int ext[3];            // 2*gmax+1
  int* d_cube = nullptr; // device int32[ext0*ext1*ext2]
  int n = 0;             // sphere size
  // the (x, y) columns of the compact cube that hold a sphere point: d_disk
  // [ext1*ext0] maps jy*ext0 + jx to the column's index (or -1), followed by
  // [ndisk] entries giving each column's jy*ext0 + jx (device, one allocation)
  int ndisk = 0;
  int* d_disk = nullptr;
};

struct ProfRec {
  std::string name;
  hipEvent_t a, b;
};

struct ProfAcc {
  int launches = 0;
  double ms = 0.0;
};

struct PinRec {
  size_t a, b;     // byte range of the staging ring read by one copy
  hipEvent_t ev;   // recorded after that copy
};

}  // namespace gw

struct gw_ctx {
  int device = 0;
  int cus = 256;                                  // compute units of the device
  hipStream_t stream = nullptr;
  std::string err;
  // growable workspace (bump sub-allocation per call)
  char* ws = nullptr;
  size_t ws_cap = 0;
  size_t ws_used = 0;
  // cached device tables
  std::map<std::string, gw::SphereMap> spheres;
  std::map<std::pair<int, int>, void*> twiddles;  // (n, is_double) -> device table
  std::map<long long, void*> tile_orders;         // (tiles, block shape) -> chi0 tile order (int2)
  int* d_flag = nullptr;                          // device status flags
  bool capturing = false;                         // inside a graph capture: no attribute calls
  // networks and plans created on this context (freed with it)
  std::set<gw_mlp*> mlps;
  std::set<gw_plan*> plans;
  // profiling
  bool profiling = false;
  std::string prof_only;  // non-empty: only scopes of this name record events
  std::vector<gw::ProfRec> prof_pending;
  std::vector<hipEvent_t> ev_pool;
  std::map<std::string, gw::ProfAcc> prof;
  std::vector<std::string> prof_names;
  // pinned host staging ring for small host arrays (frequencies, G lists)
  // copied to the device by calls that return before the device finishes:
  // each copy records an event, and a region is rewritten only after the
  // copies that read it have completed
  char* pin = nullptr;
  size_t pin_cap = 0;
  size_t pin_off = 0;
  std::vector<gw::PinRec> pin_recs;
};

namespace gw {

gw_status fail(gw_ctx* c, gw_status s, const char* fmt, ...);
void mlp_free(gw_mlp* n);    // closure.hip: release without touching the context
void plan_free(gw_plan* p);  // plan.hip
gw_status hip_fail(gw_ctx* c, hipError_t e, const char* what);

// Workspace: reset at the start of a call, then carve aligned pieces.
gw_status ws_begin(gw_ctx* c, size_t total_bytes);
void* ws_take(gw_ctx* c, size_t bytes);
inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }
// Copy `bytes` of host memory to device memory `dst` on the context stream
// through the pinned staging ring; the host buffer may be reused as soon as this
// returns, and the call does not wait for the device.
gw_status stage_h2d(gw_ctx* c, void* dst, const void* src, size_t bytes);

// Device tables.
gw_status sphere_map(gw_ctx* c, const int32_t* g, int n, const int box[3], SphereMap** out);
gw_status twiddle_table(gw_ctx* c, int n, bool dbl, const void** out);

// Profiling scope around a launch.
struct ProfScope {
  gw_ctx* c;
  const char* name;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(gw_ctx* cc, const char* nm);
  ~ProfScope();
};

#define GW_CHECK_LAUNCH(ctx, what)                                   \
  do {                                                               \
    hipError_t _e = hipGetLastError();                               \
    if (_e != hipSuccess) return ::gw::hip_fail((ctx), _e, (what));  \
  } while (0)

#define GW_HIP(ctx, call)                                            \
  do {                                                               \
    hipError_t _e = (call);                                          \
    if (_e != hipSuccess) return ::gw::hip_fail((ctx), _e, #call);   \
  } while (0)

// ---- launchers implemented in the kernel translation units ----
// FFT stage (fft.hip)
template <typename T>
gw_status band_to_grid(gw_ctx* c, const int box[3], int nbs, int ng, const void* coef,
                       const SphereMap* sm, void* u_out, void* scratch, size_t scratch_bytes);
// Pairs (v, c) for v in [v0, v0+nvt), c in [c0, c0+nct) into M. The conduction
// bands come either as full real-space fields uc, or (box shapes for which
// pair_compact_shape holds) as compact x-transformed slabs tc on sphere sc,
// from which the pair kernels build each plane themselves.
template <typename T>
gw_status pair_to_eps(gw_ctx* c, const int box[3], int nspinor, const void* uv, const void* uc,
                      const void* tc, const SphereMap* sc, int v0, int nvt, int c0, int nct,
                      int nc_total, const SphereMap* em, void* mtxel, void* scratch);
template <typename T>
gw_status band_compact(gw_ctx* c, const int box[3], int nbs, int ng, const void* coef,
                       const SphereMap* sm, void* out);
bool pair_compact_shape(const int box[3]);
// Boxes whose xy-planes have a built pair kernel (fft_xy.hip): conduction bands
// as compact z-transformed slabs [c][s][z][jy][jx] on sphere sc, valence bands
// as full fields in [v][s][z][y][x] order, pair intermediate
// T[pair][z][jy][jx] on the eps sphere's (x, y) extent.
bool pair_xy_shape(const int box[3]);
size_t band_zc_bytes(const int box[3], const SphereMap* sm, int nbs, size_t elem);
size_t pair_xy_scratch_bytes(const int box[3], const SphereMap* em, int npairs, size_t elem);
template <typename T>
gw_status band_zc(gw_ctx* c, const int box[3], int nbs, int ng, const void* coef,
                  const SphereMap* sm, void* out);
template <typename T>
gw_status grid_to_zyx(gw_ctx* c, const int box[3], int nbs, const void* u, void* w);
template <typename T>
gw_status pair_to_eps_xy(gw_ctx* c, const int box[3], int nspinor, const void* uvz,
                         const void* tcz, const SphereMap* sc, int v0, int nvt, int c0, int nct,
                         int nc_total, const SphereMap* em, void* mtxel, void* scratch);
size_t band_compact_bytes(const int box[3], const SphereMap* sm, int nbs, size_t elem);
size_t band_scratch_bytes(const int box[3], const SphereMap* sm, int nbs, size_t elem);
size_t pair_scratch_bytes(const int box[3], const SphereMap* em, int npairs, size_t elem);

// Head overlap (head.hip)
gw_status head_dipole(gw_ctx* c, gw_dtype dt, int nspinor, int nv, int nc, int ng,
                      const void* cv, const void* cc, const int* d_g, const double sq[3],
                      double q0k, const double* ev, const double* ec, double* mhead);
gw_status head_overlap(gw_ctx* c, gw_dtype dt, int nspinor, int nv, int ngv, const void* cv,
                       int nc, int ngc, const void* cc, const int* d_match, int nmatch,
                       double* mhead);
gw_status chi0_wings(gw_ctx* c, int P, int neps, const void* mtxel, gw_dtype dt,
                     const double* mhead, int head, int nfreq, const double* wts, double* chi0);

// chi0 contraction (gemm.hip)
gw_status chi0_weights(gw_ctx* c, int nv, int nc, const double* ev, const double* ec, int nfreq,
                       const double* d_omega, double pref, double* wts);
// The pair sum of the contraction is cut into `split` ranges when that fills
// the last round of workgroups better; ranges 1.. write their tiles to `part`
// (split-1 matrices per frequency), which are then added to chi0 in order.
// real-axis weights (Re and Im of the bracket as 2*nfreq real sets) and the
// combination chi0[f] += h[f] + i h[nfreq + f] of the two Hermitian results
gw_status chi0_weights_real(gw_ctx* c, int nv, int nc, const double* ev, const double* ec,
                            int nfreq, const double* d_omega, double eta, double pref,
                            double* wts);
gw_status chi0_combine_real(gw_ctx* c, int neps, int nfreq, const double* h, double* chi0);
int chi0_split(gw_ctx* c, int P, int neps, int nfreq, gw_prec prec, gw_dtype dt);
// no_alloc: use no device table that would be allocated on first use
gw_status chi0_fp64(gw_ctx* c, int P, int neps, const void* mtxel, gw_dtype dt, int nfreq,
                    const double* wts, int skip_head, double* chi0, int split, double* part,
                    bool no_alloc = false);
// The split-BF16 contraction first splits its operands into `xsplit`
// (bf16_split_bytes(P, neps, nfreq) bytes of device workspace).
size_t bf16_split_bytes(int P, int neps, int nfreq);
gw_status split_bf16(gw_ctx* c, int P, int neps, const void* mtxel, int nfreq, const double* wts,
                     void* xsplit);
gw_status chi0_splitbf16(gw_ctx* c, int P, int neps, const void* mtxel, int nfreq,
                         const double* wts, int skip_head, double* chi0, int split, double* part,
                         void* xsplit);
// generic batched C[i][j] = alpha * sum_k A[i][k] B[k][j] + beta * C[i][j] (complex
// double, row-major, beta 0 or 1); offsets, leading dimensions, batch strides and
// extents in complex elements
gw_status zgemm_nn(gw_ctx* c, int m, int n, int k, double alpha, const double* A, size_t offA,
                   int lda, long long sA, const double* B, size_t offB, int ldb, long long sB,
                   double* C, size_t offC, int ldc, long long sC, int batch, size_t extA,
                   size_t extB, size_t extC, double beta = 1.0);

// eps and its inverse (lu.hip): Gauss-Jordan on eps~ with the pivoted fallback,
// or LU with partial pivoting for any matrix
gw_status epsinv_run(gw_ctx* c, int neps, int nfreq, const double* chi0, const double* vcoul,
                     double* epsinv);
gw_status epsinv_pivoted_one(gw_ctx* c, int N, int nfreq, const double* chi0,
                             const double* vcoul, double* epsinv);
// consumers of eps^-1 (lu.hip): W = eps^-1 v, and the static screened exchange
gw_status screened_w(gw_ctx* c, int N, int nfreq, const double* epsinv, const double* vcoul,
                     double* w);
gw_status sigma_sx_static(gw_ctx* c, int nocc, int nband, int N, const void* mtxel, gw_dtype dt,
                          const double* epsinv, const double* vcoul, double prefactor,
                          double* sigma);

}  // namespace gw
