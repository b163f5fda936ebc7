// Batched many-q plan: every q-point of a grid through the whole path in one
// captured HIP graph.
//
//   per q     : valence band transforms, pair transforms -> M_q, FP64 head
//               overlap for the q0 point, Adler-Wiser weights
//   all q     : one persistent contraction kernel over every (q, tile, omega)
//               work item, items assigned to workgroups on the host by
//               longest-processing-time order (static, so the graph needs no
//               atomics and no counter resets); tile edge and grid size picked
//               by timed trial launches
//   all q     : Gauss-Jordan inversion of eps~ = I - S chi0 S for every (q, omega)
//               in the same launches (each matrix stops at its own size)
// Conduction bands at k shared by every q (same pointer and G set) are brought
// to the grid once.  After the graph, any matrix whose pivots show it is not of
// the positive-definite form is redone by LU with partial pivoting.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <fstream>
#include <functional>
#include <numeric>
#include <queue>
#include <sstream>
#include <tuple>

#include "tiles.h"

namespace gw {


struct ChiQ {
  const void* M;
  const unsigned short* X;  // split-BF16 operands (split_bf16 layout), or null
  const double* w;
  double* chi;
  int P, neps, skip, pad;
};

struct GjM {
  cpx<double>* A;          // eps~ in place, then eps^-1 (the caller's epsinv slice)
  const cpx<double>* chi;  // chi0 slice
  const double* v;         // v(q+G)
  cpx<double>* R;          // [PB][N]
  cpx<double>* Cb;         // [N][PB]
  cpx<double>* D;          // [PB][PB]
  int N, pad;
};

constexpr int PB = 64;  // Gauss-Jordan block width of the batched inversion

// ------------------------------------------------------------------ batched contraction
template <int WM, int BF16, typename Tin>
__global__ void __launch_bounds__(64 * WM * WM, WM == 2 ? 2 : 1) k_chi0_items(const ChiQ* __restrict__ qs,
                                                             const int4* __restrict__ items,
                                                             const int* __restrict__ bins) {
  for (int it = bins[blockIdx.x]; it < bins[blockIdx.x + 1]; ++it) {
    const int4 m = items[it];  // (q, ti, tj, f)
    const ChiQ q = qs[m.x];
    const double* w = q.w + (size_t)m.w * q.P;
    cpx<double>* C = reinterpret_cast<cpx<double>*>(q.chi) + (size_t)m.w * q.neps * q.neps;
    if constexpr (BF16) {
      const int Pb = (q.P + BK - 1) / BK;
      const size_t osz = (size_t)Pb * 4 * q.neps * BK;
      chi0_bf16s_tile<WM>(q.X, q.X + (size_t)(1 + m.w) * osz, 0, Pb, q.neps, C, m.y, m.z, q.skip,
                          false);
    } else
      chi0_f64_tile<WM, Tin>(static_cast<const cpx<Tin>*>(q.M), q.P, q.neps, w, C, m.y, m.z,
                             q.skip);
  }
}

__global__ void k_zero_c128(cpx<double>* p, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = mk(0.0, 0.0);
}

__global__ void k_zero_i32(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// ------------------------------------------------------------------ batched Gauss-Jordan
// flags[m] = 1: some v <= 0 or a pivot that is not real and >= 1/2 (eps~ >= I).
__global__ void k_gjb_build(const GjM* __restrict__ ms, int* __restrict__ flags) {
  const GjM m = ms[blockIdx.y];
  const size_t nn = (size_t)m.N * m.N;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nn) return;
  const int i = (int)(idx / m.N), j = (int)(idx % m.N);
  const double vi = m.v[i], vj = m.v[j];
  if (!(vi > 0.0) || !(vi < INFINITY)) flags[blockIdx.y] = 1;
  const double s = sqrt(vi) * sqrt(vj);
  const cpx<double> x = m.chi[idx];
  m.A[idx] = mk((i == j ? 1.0 : 0.0) - s * x.x, -s * x.y);
}

// Inverse of the diagonal block, register resident (gj_invert_64), as in the
// single-matrix inversion; a ragged block is padded with the identity.
__global__ void __launch_bounds__(1024) k_gjb_diag(const GjM* __restrict__ ms, int k,
                                                   int* __restrict__ flags) {
  static_assert(PB == 64, "gj_invert_64 holds a 64x64 block");
  const GjM m = ms[blockIdx.x];
  if (k >= m.N) return;
  const int N = m.N, nbk = min(PB, N - k);
  __shared__ cpx<double> rowb[2][PB], colb[2][PB];
  const int tid = threadIdx.x, ti = tid / 32, tj = tid % 32;
  cpx<double> d[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int i = ti + 32 * a, j = tj + 32 * b;
      d[a][b] = (i < nbk && j < nbk) ? m.A[(size_t)(k + i) * N + k + j]
                                     : mk(i == j ? 1.0 : 0.0, 0.0);
    }
  if (gj_invert_64<32>(d, nbk, rowb, colb)) flags[blockIdx.x] = 1;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int i = ti + 32 * a, j = tj + 32 * b;
      if (i < nbk && j < nbk) m.D[i * PB + j] = d[a][b];
    }
}

// R = Dinv A[K, :] (rows nbk.. of R are never read)
__global__ void __launch_bounds__(256, 2) k_gjb_rpanel(const GjM* __restrict__ ms, int k) {
  const GjM m = ms[blockIdx.z];
  if (k >= m.N) return;
  const int N = m.N, nbk = min(PB, N - k);
  const int j0 = blockIdx.x * ZTM;
  if (j0 >= N) return;
  zgemm_tile(nbk, N, nbk, 1.0, 0.0, m.D, PB, m.A + (size_t)k * N, N, m.R, N, 0, j0);
}

// Cb = A[:, K]; R[:, K] = I + Dinv, so that A - Cb R leaves -Cb Dinv in the
// column block (its Gauss-Jordan value)
__global__ void k_gjb_prep(const GjM* __restrict__ ms, int k) {
  const GjM m = ms[blockIdx.y];
  if (k >= m.N) return;
  const int N = m.N, nbk = min(PB, N - k);
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < N * nbk) {
    const int i = e / nbk, t = e % nbk;
    m.Cb[(size_t)i * PB + t] = m.A[(size_t)i * N + k + t];
  }
  if (e < nbk * nbk) {
    const int t = e / nbk, j = e % nbk;
    const cpx<double> dv = m.D[t * PB + j];
    m.R[(size_t)t * N + k + j] = mk(dv.x + (t == j ? 1.0 : 0.0), dv.y);
  }
}

// A -= Cb R over the whole matrix (the LDS-free rank-update tile)
__global__ void __launch_bounds__(256, 3) k_gjb_update(const GjM* __restrict__ ms, int k) {
  static_assert(PB == 64, "one 64x64 tile per workgroup");
  const GjM m = ms[blockIdx.z];
  if (k >= m.N) return;
  const int N = m.N, nbk = min(PB, N - k);
  const int i0 = blockIdx.y * PB, j0 = blockIdx.x * PB;
  if (i0 >= N || j0 >= N) return;
  const int wave = threadIdx.x >> 6;
  gj_update_tile(m.Cb, PB, m.R, m.A, N, nbk, i0 + (wave >> 1) * 32, j0 + (wave & 1) * 32, N,
                 m.A, N, 0);
}

// row block K <- R outside the K columns and Dinv inside
__global__ void k_gjb_fix(const GjM* __restrict__ ms, int k) {
  const GjM m = ms[blockIdx.y];
  if (k >= m.N) return;
  const int N = m.N, nbk = min(PB, N - k);
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nbk * N) return;
  const int t = e / N, j = e % N;
  m.A[(size_t)(k + t) * N + j] =
      (j >= k && j < k + nbk) ? m.D[t * PB + (j - k)] : m.R[(size_t)t * N + j];
}

__global__ void k_gjb_unscale(const GjM* __restrict__ ms) {
  const GjM m = ms[blockIdx.y];
  const size_t nn = (size_t)m.N * m.N;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nn) return;
  const int i = (int)(idx / m.N), j = (int)(idx % m.N);
  m.A[idx] = scal(m.A[idx], sqrt(m.v[i]) / sqrt(m.v[j]));
}

}  // namespace gw

// ------------------------------------------------------------------ plan object
struct gw_plan_q {
  gw_q_desc d;
  gw::SphereMap *sv = nullptr, *sc = nullptr, *se = nullptr;
  int P = 0;
  void* M = nullptr;
  double* mhead = nullptr;
  int* dmatch = nullptr;
  int nmatch = 0;
  double* wts = nullptr;
  void* X = nullptr;  // split-BF16 operands of the contraction
  std::vector<int> match;
};

struct gw_plan {
  gw_ctx* ctx = nullptr;
  int box[3];
  int nspinor;
  gw_dtype dtype;
  gw_prec prec;
  int nfreq;
  std::vector<double> omega;
  double pref;
  std::vector<gw_plan_q> q;
  bool shared_c = false;
  int nc_shared = 0;
  bool compact = false;  // conduction kept as compact x-transformed slabs
  // device memory (one allocation)
  char* base = nullptr;
  size_t bytes = 0;
  void *uc = nullptr, *uv = nullptr, *bscr = nullptr, *pscr = nullptr;
  size_t bscr_bytes = 0;
  int pair_chunk = 1;
  double* d_omega = nullptr;
  gw::ChiQ* d_chiq = nullptr;
  int4* d_items = nullptr;
  int* d_bins = nullptr;
  int nitems = 0;
  int nbins = 0;
  gw::GjM* d_gj = nullptr;
  int* d_flags = nullptr;
  int nmat = 0;
  int nmax = 0;
  int wm = 2;
  std::vector<gw::GjM> h_gj;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool compiled = false;
  std::string desc;
};

namespace gw {

void plan_free(gw_plan* p) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->cap) (void)hipStreamDestroy(p->cap);
  if (p->base) (void)hipFree(p->base);
  delete p;
}

static gw_status plan_fail(gw_plan* p, gw_status s, const std::string& m) {
  return fail(p->ctx, s, "%s", m.c_str());
}

// LPT assignment of contraction items to `nb` workgroups; cost ~ P * TM^2.
static void lpt_bins(const std::vector<int4>& items, const std::vector<double>& cost, int nb,
                     std::vector<int4>* out_items, std::vector<int>* out_bins) {
  std::vector<int> order(items.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  typedef std::pair<double, int> L;
  std::priority_queue<L, std::vector<L>, std::greater<L>> heap;
  for (int b = 0; b < nb; ++b) heap.push(L(0.0, b));
  std::vector<std::vector<int>> bins(nb);
  for (int i : order) {
    L l = heap.top();
    heap.pop();
    bins[l.second].push_back(i);
    heap.push(L(l.first + cost[i], l.second));
  }
  out_items->clear();
  out_bins->assign(1, 0);
  for (int b = 0; b < nb; ++b) {
    for (int i : bins[b]) out_items->push_back(items[i]);
    out_bins->push_back((int)out_items->size());
  }
}

static gw_status build_schedule(gw_plan* p, int wm, int nbins) {
  gw_ctx* c = p->ctx;
  const int tmv = 32 * wm;
  std::vector<int4> items;
  std::vector<double> cost;
  for (int iq = 0; iq < (int)p->q.size(); ++iq) {
    const auto& q = p->q[iq];
    const int nt = (q.d.neps + tmv - 1) / tmv;
    for (int f = 0; f < p->nfreq; ++f)
      for (int ti = 0; ti < nt; ++ti)
        for (int tj = ti; tj < nt; ++tj) {
          items.push_back(make_int4(iq, ti, tj, f));
          cost.push_back((double)q.P * tmv * tmv);
        }
  }
  std::vector<int4> it;
  std::vector<int> bins;
  lpt_bins(items, cost, nbins, &it, &bins);
  if ((int)it.size() > p->nitems || nbins > p->nbins)
    return fail(c, GW_EINVAL, "schedule larger than its reservation");
  GW_HIP(c, hipMemcpy(p->d_items, it.data(), it.size() * sizeof(int4), hipMemcpyHostToDevice));
  GW_HIP(c, hipMemcpy(p->d_bins, bins.data(), bins.size() * sizeof(int), hipMemcpyHostToDevice));
  return GW_OK;
}

static gw_status launch_chi0(gw_plan* p, int wm, int nbins) {
  gw_ctx* c = p->ctx;
  ProfScope ps(c, "plan_chi0");
  const dim3 g(nbins), b(64 * wm * wm);
  const bool bf = p->prec == GW_PREC_SPLITBF16;
  const bool dbl = p->dtype == GW_C128;
  if (wm == 2) {
    if (bf) hipLaunchKernelGGL((k_chi0_items<2, 1, float>), g, b, 0, c->stream, p->d_chiq, p->d_items, p->d_bins);
    else if (dbl) hipLaunchKernelGGL((k_chi0_items<2, 0, double>), g, b, 0, c->stream, p->d_chiq, p->d_items, p->d_bins);
    else hipLaunchKernelGGL((k_chi0_items<2, 0, float>), g, b, 0, c->stream, p->d_chiq, p->d_items, p->d_bins);
  } else {
    if (bf) hipLaunchKernelGGL((k_chi0_items<1, 1, float>), g, b, 0, c->stream, p->d_chiq, p->d_items, p->d_bins);
    else if (dbl) hipLaunchKernelGGL((k_chi0_items<1, 0, double>), g, b, 0, c->stream, p->d_chiq, p->d_items, p->d_bins);
    else hipLaunchKernelGGL((k_chi0_items<1, 0, float>), g, b, 0, c->stream, p->d_chiq, p->d_items, p->d_bins);
  }
  GW_CHECK_LAUNCH(c, "k_chi0_items");
  return GW_OK;
}

static gw_status zero_chi(gw_plan* p) {
  gw_ctx* c = p->ctx;
  ProfScope ps(c, "plan_zero");
  for (auto& q : p->q) {
    const size_t n = (size_t)p->nfreq * q.d.neps * q.d.neps;
    hipLaunchKernelGGL(k_zero_c128, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream,
                       reinterpret_cast<cpx<double>*>(q.d.chi0), n);
    GW_CHECK_LAUNCH(c, "k_zero_c128");
  }
  return GW_OK;
}

// mtxel + weights for every q (the part before the contraction)
static gw_status enqueue_front(gw_plan* p) {
  gw_ctx* c = p->ctx;
  gw_status st;
  const bool dbl = p->dtype == GW_C128;
  const int ns = p->nspinor;
  auto conduction = [&](int nbs, int ng, const void* cc, const SphereMap* sc) {
    if (p->compact)
      return dbl ? band_compact<double>(c, p->box, nbs, ng, cc, sc, p->uc)
                 : band_compact<float>(c, p->box, nbs, ng, cc, sc, p->uc);
    return dbl ? band_to_grid<double>(c, p->box, nbs, ng, cc, sc, p->uc, p->bscr, p->bscr_bytes)
               : band_to_grid<float>(c, p->box, nbs, ng, cc, sc, p->uc, p->bscr, p->bscr_bytes);
  };
  if (p->shared_c) {
    const auto& q0 = p->q[0];
    if ((st = conduction(p->nc_shared * ns, q0.d.ngc, q0.d.cc, q0.sc)) != GW_OK) return st;
  }
  const void* ucf = p->compact ? nullptr : p->uc;
  const void* tcs = p->compact ? p->uc : nullptr;
  for (auto& q : p->q) {
    const int nv = q.d.nv, nc = q.d.nc;
    if (!p->shared_c) {
      if ((st = conduction(nc * ns, q.d.ngc, q.d.cc, q.sc)) != GW_OK) return st;
    }
    st = dbl ? band_to_grid<double>(c, p->box, nv * ns, q.d.ngv, q.d.cv, q.sv, p->uv, p->bscr,
                                    p->bscr_bytes)
             : band_to_grid<float>(c, p->box, nv * ns, q.d.ngv, q.d.cv, q.sv, p->uv, p->bscr,
                                   p->bscr_bytes);
    if (st != GW_OK) return st;
    const int vt = std::min(nv, p->pair_chunk);
    const int ct = std::max(1, std::min(nc, p->pair_chunk / vt));
    for (int v0 = 0; v0 < nv; v0 += vt)
      for (int c0 = 0; c0 < nc; c0 += ct) {
        const int nvt = std::min(vt, nv - v0), nct = std::min(ct, nc - c0);
        st = dbl ? pair_to_eps<double>(c, p->box, ns, p->uv, ucf, tcs, q.sc, v0, nvt, c0, nct, nc,
                                       q.se, q.M, p->pscr)
                 : pair_to_eps<float>(c, p->box, ns, p->uv, ucf, tcs, q.sc, v0, nvt, c0, nct, nc,
                                      q.se, q.M, p->pscr);
        if (st != GW_OK) return st;
      }
    if (q.mhead) {
      st = head_overlap(c, p->dtype, ns, nv, q.d.ngv, q.d.cv, nc, q.d.ngc, q.d.cc, q.dmatch,
                        q.nmatch, q.mhead);
      if (st != GW_OK) return st;
    }
    st = chi0_weights(c, nv, nc, q.d.ev, q.d.ec, p->nfreq, p->d_omega, p->pref, q.wts);
    if (st != GW_OK) return st;
    if (q.X) {
      st = split_bf16(c, q.P, q.d.neps, q.M, p->nfreq, q.wts, q.X);
      if (st != GW_OK) return st;
    }
  }
  return GW_OK;
}

static gw_status enqueue_back(gw_plan* p) {
  gw_ctx* c = p->ctx;
  gw_status st;
  for (auto& q : p->q)
    if (q.mhead) {
      st = chi0_wings(c, q.P, q.d.neps, q.M, p->dtype, q.mhead, q.d.head_index, p->nfreq, q.wts,
                      q.d.chi0);
      if (st != GW_OK) return st;
    }
  // batched Gauss-Jordan over every (q, omega)
  {
    ProfScope ps(c, "plan_gj_build");
    hipLaunchKernelGGL(k_zero_i32, dim3((p->nmat + 255) / 256), dim3(256), 0, c->stream, p->d_flags,
                       p->nmat);
    GW_CHECK_LAUNCH(c, "k_zero_i32");
    const size_t nn = (size_t)p->nmax * p->nmax;
    hipLaunchKernelGGL(k_gjb_build, dim3((unsigned)((nn + 255) / 256), p->nmat), dim3(256), 0,
                       c->stream, p->d_gj, p->d_flags);
    GW_CHECK_LAUNCH(c, "k_gjb_build");
  }
  const int tiles = (p->nmax + ZTM - 1) / ZTM;
  for (int k = 0; k < p->nmax; k += PB) {
    {
      ProfScope ps(c, "plan_gj_small");
      hipLaunchKernelGGL(k_gjb_diag, dim3(p->nmat), dim3(1024), 0, c->stream, p->d_gj, k,
                         p->d_flags);
      GW_CHECK_LAUNCH(c, "k_gjb_diag");
      hipLaunchKernelGGL(k_gjb_rpanel, dim3(tiles, 1, p->nmat), dim3(256), 0, c->stream,
                         p->d_gj, k);
      GW_CHECK_LAUNCH(c, "k_gjb_rpanel");
      hipLaunchKernelGGL(k_gjb_prep, dim3((PB * p->nmax + 255) / 256, p->nmat), dim3(256), 0,
                         c->stream, p->d_gj, k);
      GW_CHECK_LAUNCH(c, "k_gjb_prep");
    }
    {
      ProfScope ps(c, "plan_gj_update");
      hipLaunchKernelGGL(k_gjb_update, dim3(tiles, tiles, p->nmat), dim3(256), 0, c->stream,
                         p->d_gj, k);
      GW_CHECK_LAUNCH(c, "k_gjb_update");
    }
    {
      ProfScope ps(c, "plan_gj_small");
      hipLaunchKernelGGL(k_gjb_fix, dim3((PB * p->nmax + 255) / 256, p->nmat), dim3(256), 0,
                         c->stream, p->d_gj, k);
      GW_CHECK_LAUNCH(c, "k_gjb_fix");
    }
  }
  {
    ProfScope ps(c, "plan_gj_build");
    const size_t nn = (size_t)p->nmax * p->nmax;
    hipLaunchKernelGGL(k_gjb_unscale, dim3((unsigned)((nn + 255) / 256), p->nmat), dim3(256), 0,
                       c->stream, p->d_gj);
    GW_CHECK_LAUNCH(c, "k_gjb_unscale");
  }
  (void)st;
  return GW_OK;
}

static gw_status enqueue_all(gw_plan* p, int nbins) {
  gw_status st;
  if ((st = enqueue_front(p)) != GW_OK) return st;
  if ((st = zero_chi(p)) != GW_OK) return st;
  if ((st = launch_chi0(p, p->wm, nbins)) != GW_OK) return st;
  return enqueue_back(p);
}

static std::string tune_key(const gw_plan* p) {
  std::ostringstream k;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, p->ctx->device) == hipSuccess) k << prop.gcnArchName;
  k << "|" << (int)p->dtype << "|" << (int)p->prec << "|" << p->nfreq << "|" << p->q.size();
  long long ps = 0, es = 0;
  for (auto& q : p->q) { ps += q.P; es += q.d.neps; }
  // shape class: pair and eps sizes rounded to 3 significant digits
  auto round3 = [](long long x) {
    long long m = 1;
    while (x >= 1000 * m) m *= 10;
    return (x / m) * m;
  };
  k << "|" << round3(ps) << "|" << round3(es);
  return k.str();
}

static bool cache_lookup(const std::string& key, int* wm, int* mult) {
  const char* path = std::getenv("GW_AUTOTUNE_CACHE");
  if (!path) return false;
  std::ifstream in(path);
  std::string line;
  while (std::getline(in, line)) {
    // one JSON object per line: {"key": "...", "wm": 2, "mult": 2}
    const auto kp = line.find("\"key\": \"");
    if (kp == std::string::npos) continue;
    const auto ke = line.find('"', kp + 8);
    if (line.substr(kp + 8, ke - kp - 8) != key) continue;
    const auto wp = line.find("\"wm\": "), mp = line.find("\"mult\": ");
    if (wp == std::string::npos || mp == std::string::npos) continue;
    *wm = std::atoi(line.c_str() + wp + 6);
    *mult = std::atoi(line.c_str() + mp + 8);
    return (*wm == 1 || *wm == 2) && *mult > 0 && *mult <= 16;
  }
  return false;
}

static void cache_store(const std::string& key, int wm, int mult) {
  const char* path = std::getenv("GW_AUTOTUNE_CACHE");
  if (!path) return;
  std::ofstream out(path, std::ios::app);
  out << "{\"key\": \"" << key << "\", \"wm\": " << wm << ", \"mult\": " << mult << "}\n";
}

}  // namespace gw

using namespace gw;

extern "C" {

gw_status gw_plan_create(gw_ctx* c, gw_plan** out, const int box[3], int nspinor, gw_dtype dtype,
                         gw_prec prec, int nfreq, const double* omega, double prefactor, int nq,
                         const gw_q_desc* qd) {
  if (!c || !out) return GW_EINVAL;
  *out = nullptr;
  c->err.clear();
  if (!box || !omega || !qd || nq <= 0 || nfreq <= 0)
    return fail(c, GW_EINVAL, "plan needs a box, frequencies and at least one q");
  if (nspinor != 1 && nspinor != 2) return fail(c, GW_EINVAL, "nspinor must be 1 or 2");
  if (dtype != GW_C128 && dtype != GW_C64) return fail(c, GW_EINVAL, "unknown dtype");
  if (prec != GW_PREC_FP64 && prec != GW_PREC_SPLITBF16) return fail(c, GW_EINVAL, "unknown precision");
  if (prec == GW_PREC_SPLITBF16 && dtype != GW_C64)
    return fail(c, GW_EINVAL, "split-BF16 contraction needs GW_C64 matrix elements");
  for (int f = 0; f < nfreq; ++f)
    if (!(omega[f] >= 0.0) || !std::isfinite(omega[f]))
      return fail(c, GW_EINVAL, "omega[%d] must be finite and >= 0", f);
  for (int a = 0; a < 3; ++a) {
    if (make_fft_plan(box[a]).npass < 0 || box[a] <= 0 || box[a] > 4096)
      return fail(c, GW_EINVAL, "box[%d] must be a product of 2, 3 and 5", a);
  }
  for (int i = 0; i < nq; ++i) {
    const gw_q_desc& d = qd[i];
    if (d.nv <= 0 || d.nc <= 0 || d.neps <= 0 || d.ngv <= 0 || d.ngc <= 0)
      return fail(c, GW_EINVAL, "q %d: empty band set or sphere", i);
    if (!d.gv || !d.gc || !d.geps || !d.cv || !d.cc || !d.ev || !d.ec || !d.vcoul || !d.chi0 ||
        !d.epsinv)
      return fail(c, GW_EINVAL, "q %d: NULL pointer", i);
    if (d.head_index >= d.neps) return fail(c, GW_EINVAL, "q %d: head_index >= neps", i);
    if (d.head_index >= 0 && (d.geps[3 * d.head_index] != 0 || d.geps[3 * d.head_index + 1] != 0 ||
                              d.geps[3 * d.head_index + 2] != 0))
      return fail(c, GW_EINVAL, "q %d: geps[head_index] is not G = 0", i);
    if ((long long)d.nv * d.nc > 65535LL * 1024) return fail(c, GW_EINVAL, "q %d: too many pairs", i);
  }
  gw_plan* p = new gw_plan();
  p->ctx = c;
  for (int a = 0; a < 3; ++a) p->box[a] = box[a];
  p->nspinor = nspinor;
  p->dtype = dtype;
  p->prec = prec;
  p->nfreq = nfreq;
  p->omega.assign(omega, omega + nfreq);
  p->pref = prefactor;
  p->q.resize(nq);
  for (int i = 0; i < nq; ++i) {
    p->q[i].d = qd[i];
    p->q[i].P = qd[i].nv * qd[i].nc;
    // the G lists are host memory read during the call: build the maps now
    gw_status st;
    if ((st = sphere_map(c, qd[i].gv, qd[i].ngv, box, &p->q[i].sv)) != GW_OK ||
        (st = sphere_map(c, qd[i].gc, qd[i].ngc, box, &p->q[i].sc)) != GW_OK ||
        (st = sphere_map(c, qd[i].geps, qd[i].neps, box, &p->q[i].se)) != GW_OK) {
      delete p;
      return st;
    }
    for (int a = 0; a < 3; ++a)
      if (box[a] <= p->q[i].sv->gmax[a] + p->q[i].sc->gmax[a] + p->q[i].se->gmax[a]) {
        delete p;
        return fail(c, GW_EALIAS, "q %d: box[%d] too small, the pair product aliases", i, a);
      }
    if (qd[i].head_index >= 0) {
      std::map<std::tuple<int, int, int>, int> lut;
      for (int g = 0; g < qd[i].ngc; ++g)
        lut[std::make_tuple(qd[i].gc[3 * g], qd[i].gc[3 * g + 1], qd[i].gc[3 * g + 2])] = g;
      for (int g = 0; g < qd[i].ngv; ++g) {
        auto it = lut.find(std::make_tuple(qd[i].gv[3 * g], qd[i].gv[3 * g + 1], qd[i].gv[3 * g + 2]));
        if (it != lut.end()) { p->q[i].match.push_back(g); p->q[i].match.push_back(it->second); }
      }
    }
  }
  // shared conduction: same pointer and same G set for every q
  p->shared_c = true;
  for (int i = 1; i < nq; ++i)
    if (qd[i].cc != qd[0].cc || p->q[i].sc != p->q[0].sc) p->shared_c = false;
  for (int i = 0; i < nq; ++i) p->nc_shared = std::max(p->nc_shared, qd[i].nc);
  c->plans.insert(p);
  *out = p;
  return GW_OK;
}

gw_status gw_plan_compile(gw_plan* p) {
  if (!p) return GW_EINVAL;
  gw_ctx* c = p->ctx;
  c->err.clear();
  if (p->compiled) return GW_OK;
  (void)hipSetDevice(c->device);
  const size_t elem = p->dtype == GW_C128 ? 16 : 8;
  const size_t nbox = (size_t)p->box[0] * p->box[1] * p->box[2];
  const int ns = p->nspinor;
  int nv_max = 0, nc_max = 0;
  size_t band_per = 0, pair_per = 0;
  for (auto& q : p->q) {
    nv_max = std::max(nv_max, q.d.nv);
    nc_max = std::max(nc_max, q.d.nc);
    band_per = std::max({band_per, band_scratch_bytes(p->box, q.sv, 1, elem),
                         band_scratch_bytes(p->box, q.sc, 1, elem)});
    pair_per = std::max(pair_per, pair_scratch_bytes(p->box, q.se, 1, elem));
  }
  const int nbs_max = std::max(nv_max, p->shared_c ? p->nc_shared : nc_max) * ns;
  const int band_chunk = (int)std::max<size_t>(1, std::min<size_t>(nbs_max, (512ull << 20) / band_per));
  p->bscr_bytes = band_per * band_chunk;
  p->pair_chunk = (int)std::max<size_t>(1, std::min<size_t>(65535, (1ull << 30) / pair_per));
  const size_t pscr_bytes = pair_per * p->pair_chunk;
  // matrices
  p->nmat = (int)p->q.size() * p->nfreq;
  p->nmax = 0;
  for (auto& q : p->q) p->nmax = std::max(p->nmax, q.d.neps);
  // schedule reservation: the larger of the two tile edges
  long long items = 0;
  for (auto& q : p->q) {
    const long long nt = (q.d.neps + 31) / 32;
    items += p->nfreq * nt * (nt + 1) / 2;
  }
  hipDeviceProp_t prop;
  GW_HIP(c, hipGetDeviceProperties(&prop, c->device));
  const int ncu = prop.multiProcessorCount;
  p->nbins = 16 * ncu;
  p->nitems = (int)items;
  // one allocation
  std::vector<std::pair<void**, size_t>> parts;
  p->compact = pair_compact_shape(p->box);
  size_t uc_bytes = (size_t)(p->shared_c ? p->nc_shared : nc_max) * ns * nbox * elem;
  if (p->compact) {
    uc_bytes = 0;
    for (auto& q : p->q)
      uc_bytes = std::max(uc_bytes, band_compact_bytes(p->box, q.sc,
                                                       (p->shared_c ? p->nc_shared : q.d.nc) * ns,
                                                       elem));
  }
  const size_t uv_bytes = (size_t)nv_max * ns * nbox * elem;
  parts.push_back({&p->uc, uc_bytes});
  parts.push_back({&p->uv, uv_bytes});
  parts.push_back({&p->bscr, p->bscr_bytes});
  parts.push_back({&p->pscr, pscr_bytes});
  parts.push_back({reinterpret_cast<void**>(&p->d_omega), p->nfreq * sizeof(double)});
  parts.push_back({reinterpret_cast<void**>(&p->d_chiq), p->q.size() * sizeof(ChiQ)});
  parts.push_back({reinterpret_cast<void**>(&p->d_items), (size_t)p->nitems * sizeof(int4)});
  parts.push_back({reinterpret_cast<void**>(&p->d_bins), ((size_t)p->nbins + 1) * sizeof(int)});
  parts.push_back({reinterpret_cast<void**>(&p->d_gj), (size_t)p->nmat * sizeof(GjM)});
  parts.push_back({reinterpret_cast<void**>(&p->d_flags), (size_t)p->nmat * sizeof(int)});
  std::vector<void*> gjR(p->nmat), gjC(p->nmat), gjD(p->nmat);
  for (auto& q : p->q) {
    parts.push_back({&q.M, (size_t)q.P * q.d.neps * elem});
    parts.push_back({reinterpret_cast<void**>(&q.wts), (size_t)p->nfreq * q.P * sizeof(double)});
    if (p->prec == GW_PREC_SPLITBF16)
      parts.push_back({&q.X, bf16_split_bytes(q.P, q.d.neps, p->nfreq)});
    if (q.d.head_index >= 0) {
      parts.push_back({reinterpret_cast<void**>(&q.mhead), (size_t)q.P * 16});
      parts.push_back({reinterpret_cast<void**>(&q.dmatch), std::max<size_t>(16, q.match.size() * 4)});
    }
  }
  for (int iq = 0; iq < (int)p->q.size(); ++iq)
    for (int f = 0; f < p->nfreq; ++f) {
      const int m = iq * p->nfreq + f;
      const size_t N = p->q[iq].d.neps;
      parts.push_back({&gjR[m], PB * N * 16});
      parts.push_back({&gjC[m], N * PB * 16});
      parts.push_back({&gjD[m], PB * PB * 16});
    }
  size_t total = 0;
  for (auto& pt : parts) total += align_up(pt.second);
  void* base = nullptr;
  hipError_t e = hipMalloc(&base, total);
  if (e != hipSuccess) return fail(c, GW_ENOMEM, "plan workspace of %zu bytes: %s", total, hipGetErrorString(e));
  p->base = static_cast<char*>(base);
  p->bytes = total;
  size_t off = 0;
  for (auto& pt : parts) {
    *pt.first = p->base + off;
    off += align_up(pt.second);
  }
  // small tables
  GW_HIP(c, hipMemcpy(p->d_omega, p->omega.data(), p->nfreq * sizeof(double), hipMemcpyHostToDevice));
  std::vector<ChiQ> hq(p->q.size());
  for (size_t i = 0; i < p->q.size(); ++i) {
    auto& q = p->q[i];
    q.nmatch = (int)q.match.size() / 2;
    if (q.dmatch && q.nmatch)
      GW_HIP(c, hipMemcpy(q.dmatch, q.match.data(), q.match.size() * 4, hipMemcpyHostToDevice));
    if (q.d.head_index >= 0 && q.nmatch == 0)
      return fail(c, GW_EINVAL, "q %zu: no common G between the valence and conduction spheres", i);
    hq[i].M = q.M;
    hq[i].X = static_cast<const unsigned short*>(q.X);
    hq[i].w = q.wts;
    hq[i].chi = q.d.chi0;
    hq[i].P = q.P;
    hq[i].neps = q.d.neps;
    hq[i].skip = q.mhead ? q.d.head_index : -1;
    hq[i].pad = 0;
  }
  GW_HIP(c, hipMemcpy(p->d_chiq, hq.data(), hq.size() * sizeof(ChiQ), hipMemcpyHostToDevice));
  p->h_gj.resize(p->nmat);
  for (int iq = 0; iq < (int)p->q.size(); ++iq)
    for (int f = 0; f < p->nfreq; ++f) {
      const int m = iq * p->nfreq + f;
      const auto& d = p->q[iq].d;
      const size_t nn = (size_t)d.neps * d.neps;
      GjM g;
      g.A = reinterpret_cast<cpx<double>*>(d.epsinv) + f * nn;
      g.chi = reinterpret_cast<const cpx<double>*>(d.chi0) + f * nn;
      g.v = d.vcoul;
      g.R = static_cast<cpx<double>*>(gjR[m]);
      g.Cb = static_cast<cpx<double>*>(gjC[m]);
      g.D = static_cast<cpx<double>*>(gjD[m]);
      g.N = d.neps;
      g.pad = 0;
      p->h_gj[m] = g;
    }
  GW_HIP(c, hipMemcpy(p->d_gj, p->h_gj.data(), p->h_gj.size() * sizeof(GjM), hipMemcpyHostToDevice));

  // eager pass: builds every cached table, runs each kernel once
  const bool prof = c->profiling;
  c->profiling = false;
  gw_status st = enqueue_front(p);
  if (st != GW_OK) { c->profiling = prof; return st; }

  // autotune the contraction: tile edge x persistent grid size
  std::ostringstream ds;
  const std::string key = tune_key(p);
  int best_wm = 2, best_mult = 2;
  if (cache_lookup(key, &best_wm, &best_mult)) {
    ds << "autotune: cache hit (" << key << ")";
  } else {
    hipEvent_t e0, e1;
    GW_HIP(c, hipEventCreate(&e0));
    GW_HIP(c, hipEventCreate(&e1));
    float best = 1e30f;
    ds << "autotune [" << key << "]:";
    for (int wm : {2, 1}) {
      for (int mult : {1, 2, 4, 8}) {
        const int occ = wm == 2 ? 2 : 8;  // resident workgroups per CU for the tile edge
        const int nb = std::min(p->nbins, mult * occ * ncu / 2);
        if ((st = build_schedule(p, wm, nb)) != GW_OK) { c->profiling = prof; return st; }
        if ((st = zero_chi(p)) != GW_OK) { c->profiling = prof; return st; }
        GW_HIP(c, hipEventRecord(e0, c->stream));
        if ((st = launch_chi0(p, wm, nb)) != GW_OK) { c->profiling = prof; return st; }
        GW_HIP(c, hipEventRecord(e1, c->stream));
        GW_HIP(c, hipEventSynchronize(e1));
        float ms = 0.f;
        GW_HIP(c, hipEventElapsedTime(&ms, e0, e1));
        ds << " tm" << 32 * wm << "/g" << nb << "=" << ms << "ms";
        if (ms < best) { best = ms; best_wm = wm; best_mult = mult; }
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    cache_store(key, best_wm, best_mult);
  }
  p->wm = best_wm;
  const int occ = best_wm == 2 ? 2 : 8;
  const int nb = std::min(p->nbins, best_mult * occ * ncu / 2);
  if ((st = build_schedule(p, best_wm, nb)) != GW_OK) { c->profiling = prof; return st; }
  ds << " -> tile " << 32 * best_wm << ", " << nb << " workgroups";
  p->desc = ds.str();
  p->nbins = nb;

  // capture every stage on a private stream
  GW_HIP(c, hipStreamSynchronize(c->stream));
  GW_HIP(c, hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking));
  hipStream_t user = c->stream;
  c->stream = p->cap;
  e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) { c->stream = user; c->profiling = prof; return hip_fail(c, e, "hipStreamBeginCapture"); }
  c->capturing = true;
  st = enqueue_all(p, nb);
  c->capturing = false;
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(p->cap, &g);
  c->stream = user;
  c->profiling = prof;
  if (st != GW_OK) { if (g) (void)hipGraphDestroy(g); return st; }
  if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
  p->graph = g;
  e = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) return hip_fail(c, e, "hipGraphInstantiate");
  p->compiled = true;
  return GW_OK;
}

gw_status gw_plan_launch(gw_plan* p) {
  if (!p) return GW_EINVAL;
  gw_ctx* c = p->ctx;
  c->err.clear();
  if (!p->compiled) return fail(c, GW_EINVAL, "gw_plan_compile has not run");
  (void)hipSetDevice(c->device);
  {
    ProfScope ps(c, "plan_graph");
    GW_HIP(c, hipGraphLaunch(p->exec, c->stream));
  }
  std::vector<int> flags(p->nmat);
  GW_HIP(c, hipMemcpyAsync(flags.data(), p->d_flags, p->nmat * sizeof(int), hipMemcpyDeviceToHost,
                           c->stream));
  GW_HIP(c, hipStreamSynchronize(c->stream));
  gw_status worst = GW_OK;
  for (int m = 0; m < p->nmat; ++m) {
    if (!flags[m]) continue;
    // not of the positive-definite form: LU with partial pivoting for this matrix
    const int iq = m / p->nfreq, f = m % p->nfreq;
    const auto& d = p->q[iq].d;
    const size_t nn = (size_t)d.neps * d.neps;
    gw_status st = epsinv_pivoted_one(c, d.neps, 1, d.chi0 + 2 * f * nn, d.vcoul,
                                      d.epsinv + 2 * f * nn);
    if (st != GW_OK) worst = st;
  }
  return worst;
}

gw_status gw_plan_destroy(gw_plan* p) {
  if (!p) return GW_EINVAL;
  (void)hipSetDevice(p->ctx->device);
  (void)hipStreamSynchronize(p->ctx->stream);
  p->ctx->plans.erase(p);
  gw::plan_free(p);
  return GW_OK;
}

const char* gw_plan_describe(const gw_plan* p) { return p ? p->desc.c_str() : ""; }

}  // extern "C"
