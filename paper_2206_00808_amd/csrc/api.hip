// C ABI of libgwspinor: argument validation, device tables, workspace,
// per-kernel event timing, and the entry points declared in include/gw.h.
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <set>
#include <tuple>

#include "common.h"

namespace gw {

gw_status fail(gw_ctx* c, gw_status s, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return s;
}

gw_status hip_fail(gw_ctx* c, hipError_t e, const char* what) {
  const gw_status s = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? GW_ENOMEM
                                                                                  : GW_EDEVICE;
  return fail(c, s, "%s: %s", what, hipGetErrorString(e));
}

gw_status ws_begin(gw_ctx* c, size_t total) {
  total = align_up(total + 256);
  if (total > c->ws_cap) {
    if (c->ws) {
      hipError_t e = hipStreamSynchronize(c->stream);
      if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
      (void)hipFree(c->ws);
      c->ws = nullptr;
      c->ws_cap = 0;
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, total);
    if (e != hipSuccess) return fail(c, GW_ENOMEM, "workspace of %zu bytes: %s", total,
                                     hipGetErrorString(e));
    c->ws = static_cast<char*>(p);
    c->ws_cap = total;
  }
  c->ws_used = 0;
  return GW_OK;
}

void* ws_take(gw_ctx* c, size_t bytes) {
  void* p = c->ws + c->ws_used;
  c->ws_used += align_up(bytes);
  return p;
}

static void pin_release(gw_ctx* c) {
  for (auto& r : c->pin_recs) (void)hipEventDestroy(r.ev);
  c->pin_recs.clear();
  if (c->pin) (void)hipHostFree(c->pin);
  c->pin = nullptr;
  c->pin_cap = 0;
  c->pin_off = 0;
}

gw_status stage_h2d(gw_ctx* c, void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return GW_OK;
  const size_t need = align_up(bytes);
  if (need > c->pin_cap) {
    // grow: every earlier copy must have read its range before the free
    for (auto& r : c->pin_recs) {
      const hipError_t e = hipEventSynchronize(r.ev);
      if (e != hipSuccess) return hip_fail(c, e, "hipEventSynchronize");
    }
    pin_release(c);
    const size_t cap = std::max<size_t>(64u << 10, 2 * need);
    void* p = nullptr;
    const hipError_t e = hipHostMalloc(&p, cap, hipHostMallocDefault);
    if (e != hipSuccess) return fail(c, GW_ENOMEM, "pinned staging of %zu bytes: %s", cap,
                                     hipGetErrorString(e));
    c->pin = static_cast<char*>(p);
    c->pin_cap = cap;
    c->pin_off = 0;
  }
  if (c->pin_off + need > c->pin_cap) c->pin_off = 0;
  const size_t a = c->pin_off, b = a + need;
  // wait for (almost always long finished) copies that still read [a, b)
  for (size_t i = 0; i < c->pin_recs.size();) {
    PinRec& r = c->pin_recs[i];
    if (r.a < b && a < r.b) {
      const hipError_t e = hipEventSynchronize(r.ev);
      if (e != hipSuccess) return hip_fail(c, e, "hipEventSynchronize");
      (void)hipEventDestroy(r.ev);
      c->pin_recs.erase(c->pin_recs.begin() + i);
    } else {
      ++i;
    }
  }
  std::memcpy(c->pin + a, src, bytes);
  GW_HIP(c, hipMemcpyAsync(dst, c->pin + a, bytes, hipMemcpyHostToDevice, c->stream));
  hipEvent_t ev;
  GW_HIP(c, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  const hipError_t e = hipEventRecord(ev, c->stream);
  if (e != hipSuccess) { (void)hipEventDestroy(ev); return hip_fail(c, e, "hipEventRecord"); }
  c->pin_recs.push_back(PinRec{a, b, ev});
  c->pin_off = b;
  return GW_OK;
}

static uint64_t fnv1a(const void* data, size_t n, uint64_t h = 1469598103934665603ull) {
  const unsigned char* p = static_cast<const unsigned char*>(data);
  for (size_t i = 0; i < n; ++i) { h ^= p[i]; h *= 1099511628211ull; }
  return h;
}

gw_status sphere_map(gw_ctx* c, const int32_t* g, int n, const int box[3], SphereMap** out) {
  char key[96];
  const uint64_t h = fnv1a(g, (size_t)n * 3 * sizeof(int32_t));
  snprintf(key, sizeof key, "%d:%d:%d:%d:%016llx", box[0], box[1], box[2], n,
           (unsigned long long)h);
  auto it = c->spheres.find(key);
  if (it != c->spheres.end()) { *out = &it->second; return GW_OK; }
  SphereMap sm;
  sm.n = n;
  for (int a = 0; a < 3; ++a) sm.gmax[a] = 0;
  for (int i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) sm.gmax[a] = std::max(sm.gmax[a], std::abs(g[3 * i + a]));
  for (int a = 0; a < 3; ++a) {
    sm.ext[a] = 2 * sm.gmax[a] + 1;
    if (sm.ext[a] > box[a])
      return fail(c, GW_EINVAL, "G vectors span %d points along axis %d but the box has %d",
                  sm.ext[a], a, box[a]);
  }
  const size_t ncube = (size_t)sm.ext[0] * sm.ext[1] * sm.ext[2];
  std::vector<int> cube(ncube, -1);
  for (int i = 0; i < n; ++i) {
    const size_t idx = ((size_t)(g[3 * i] + sm.gmax[0]) * sm.ext[1] + (g[3 * i + 1] + sm.gmax[1])) *
                           sm.ext[2] + (g[3 * i + 2] + sm.gmax[2]);
    if (cube[idx] >= 0) return fail(c, GW_EINVAL, "duplicate G vector at index %d", i);
    cube[idx] = i;
  }
  GW_HIP(c, hipMalloc(&sm.d_cube, ncube * sizeof(int)));
  GW_HIP(c, hipMemcpy(sm.d_cube, cube.data(), ncube * sizeof(int), hipMemcpyHostToDevice));
  // columns (jx, jy) with at least one sphere point, y-major
  const int nxy = sm.ext[0] * sm.ext[1];
  std::vector<int> disk(nxy, -1), cols;
  for (int jy = 0; jy < sm.ext[1]; ++jy)
    for (int jx = 0; jx < sm.ext[0]; ++jx) {
      bool any = false;
      for (int jz = 0; jz < sm.ext[2] && !any; ++jz)
        any = cube[((size_t)jx * sm.ext[1] + jy) * sm.ext[2] + jz] >= 0;
      if (any) {
        disk[jy * sm.ext[0] + jx] = (int)cols.size();
        cols.push_back(jy * sm.ext[0] + jx);
      }
    }
  sm.ndisk = (int)cols.size();
  disk.insert(disk.end(), cols.begin(), cols.end());
  GW_HIP(c, hipMalloc(&sm.d_disk, disk.size() * sizeof(int)));
  GW_HIP(c, hipMemcpy(sm.d_disk, disk.data(), disk.size() * sizeof(int), hipMemcpyHostToDevice));
  auto res = c->spheres.emplace(key, sm);
  *out = &res.first->second;
  return GW_OK;
}

ProfScope::ProfScope(gw_ctx* cc, const char* nm) : c(cc), name(nm) {
  if (!c->profiling) return;
  if (!c->prof_only.empty() && c->prof_only != name) return;
  auto get = [&]() {
    hipEvent_t e;
    if (!c->ev_pool.empty()) { e = c->ev_pool.back(); c->ev_pool.pop_back(); }
    else (void)hipEventCreate(&e);
    return e;
  };
  a = get();
  b = get();
  (void)hipEventRecord(a, c->stream);
}

ProfScope::~ProfScope() {
  if (!a) return;
  (void)hipEventRecord(b, c->stream);
  c->prof_pending.push_back(ProfRec{name, a, b});
}

static void prof_collect(gw_ctx* c) {
  if (c->prof_pending.empty()) return;
  (void)hipStreamSynchronize(c->stream);
  for (auto& r : c->prof_pending) {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, r.a, r.b);
    auto it = c->prof.find(r.name);
    if (it == c->prof.end()) {
      c->prof_names.push_back(r.name);
      it = c->prof.emplace(r.name, ProfAcc{}).first;
    }
    it->second.launches += 1;
    it->second.ms += ms;
    c->ev_pool.push_back(r.a);
    c->ev_pool.push_back(r.b);
  }
  c->prof_pending.clear();
}

static bool factorable(int n) {
  if (n <= 0) return false;
  for (int p : {2, 3, 5})
    while (n % p == 0) n /= p;
  return n == 1;
}

static bool g_ok(const int32_t* g, int n) { return n == 0 || g != nullptr; }

// FP64 G = 0 overlaps of the small-q head (head.hip), from the G vectors the
// two spheres share
static gw_status mtxel_head(gw_ctx* c, gw_dtype dtype, int nspinor, int nv, int ngv,
                            const int32_t* gv, const void* cv, int nc, int ngc,
                            const int32_t* gc, const void* cc, double* mhead) {
  std::vector<int> match;
  std::map<std::tuple<int, int, int>, int> lut;
  for (int i = 0; i < ngc; ++i) lut[std::make_tuple(gc[3 * i], gc[3 * i + 1], gc[3 * i + 2])] = i;
  for (int i = 0; i < ngv; ++i) {
    auto it = lut.find(std::make_tuple(gv[3 * i], gv[3 * i + 1], gv[3 * i + 2]));
    if (it != lut.end()) { match.push_back(i); match.push_back(it->second); }
  }
  const int nm = (int)match.size() / 2;
  if (nm == 0) {
    GW_HIP(c, hipMemsetAsync(mhead, 0, (size_t)nv * nc * 16, c->stream));
    return GW_OK;
  }
  gw_status st = ws_begin(c, align_up(match.size() * sizeof(int)));
  if (st != GW_OK) return st;
  int* dmatch = static_cast<int*>(ws_take(c, match.size() * sizeof(int)));
  if ((st = stage_h2d(c, dmatch, match.data(), match.size() * sizeof(int))) != GW_OK) return st;
  return head_overlap(c, dtype, nspinor, nv, ngv, cv, nc, ngc, cc, dmatch, nm, mhead);
}

// Matrix elements on boxes with a built xy-plane pair kernel (fft_xy.hip):
// valence bands as full fields in [v][s][z][y][x] order, conduction bands as
// compact z-transformed slabs, pairs in chunks of at most 4 GiB of intermediate.
static gw_status mtxel_xy(gw_ctx* c, const int box[3], int nspinor, int nv, int ngv,
                          const void* cv, int nc, int ngc, const void* cc, gw_dtype dtype,
                          const SphereMap* sv, const SphereMap* sc, const SphereMap* se,
                          void* mtxel, int head_index, double* mhead, const int32_t* gv,
                          const int32_t* gc) {
  const size_t elem = dtype == GW_C128 ? 16 : 8;
  const size_t nbox = (size_t)box[0] * box[1] * box[2];
  const size_t uv_bytes = (size_t)nv * nspinor * nbox * elem;
  const size_t uc_bytes = band_zc_bytes(box, sc, nc * nspinor, elem);
  const size_t band_per = band_scratch_bytes(box, sv, 1, elem);
  const int band_chunk = (int)std::max<size_t>(1, std::min<size_t>((size_t)nv * nspinor,
                                                                   (512ull << 20) / band_per));
  const size_t band_bytes = band_per * band_chunk;
  const size_t pair_per = pair_xy_scratch_bytes(box, se, 1, elem);
  int max_pairs = (int)std::max<size_t>(1, (4ull << 30) / pair_per);
  if (max_pairs > 65535) max_pairs = 65535;
  const int vt = std::min(nv, max_pairs);
  const int ct = std::max(1, std::min(nc, max_pairs / vt));
  // the valence fields in (x, y, z) order pass through the pair scratch
  const size_t pair_bytes = std::max(pair_per * (size_t)vt * ct, uv_bytes);
  gw_status st = ws_begin(c, align_up(uv_bytes) + align_up(uc_bytes) + align_up(band_bytes) +
                                 align_up(pair_bytes));
  if (st != GW_OK) return st;
  void* uv = ws_take(c, uv_bytes);
  void* uc = ws_take(c, uc_bytes);
  void* bscr = ws_take(c, band_bytes);
  void* pscr = ws_take(c, pair_bytes);
  const bool dbl = dtype == GW_C128;
  st = dbl ? band_to_grid<double>(c, box, nv * nspinor, ngv, cv, sv, pscr, bscr, band_bytes)
           : band_to_grid<float>(c, box, nv * nspinor, ngv, cv, sv, pscr, bscr, band_bytes);
  if (st != GW_OK) return st;
  st = dbl ? grid_to_zyx<double>(c, box, nv * nspinor, pscr, uv)
           : grid_to_zyx<float>(c, box, nv * nspinor, pscr, uv);
  if (st != GW_OK) return st;
  st = dbl ? band_zc<double>(c, box, nc * nspinor, ngc, cc, sc, uc)
           : band_zc<float>(c, box, nc * nspinor, ngc, cc, sc, uc);
  if (st != GW_OK) return st;
  for (int v0 = 0; v0 < nv; v0 += vt) {
    const int nvt = std::min(vt, nv - v0);
    for (int c0 = 0; c0 < nc; c0 += ct) {
      const int nct = std::min(ct, nc - c0);
      st = dbl ? pair_to_eps_xy<double>(c, box, nspinor, uv, uc, sc, v0, nvt, c0, nct, nc, se,
                                        mtxel, pscr)
               : pair_to_eps_xy<float>(c, box, nspinor, uv, uc, sc, v0, nvt, c0, nct, nc, se,
                                       mtxel, pscr);
      if (st != GW_OK) return st;
    }
  }
  if (mhead)
    return mtxel_head(c, dtype, nspinor, nv, ngv, gv, cv, nc, ngc, gc, cc, mhead);
  return GW_OK;
}

}  // namespace gw

using namespace gw;

extern "C" {

const char* gw_status_string(gw_status s) {
  switch (s) {
    case GW_OK: return "GW_OK";
    case GW_EINVAL: return "GW_EINVAL";
    case GW_ENOMEM: return "GW_ENOMEM";
    case GW_EDEVICE: return "GW_EDEVICE";
    case GW_EALIAS: return "GW_EALIAS";
    case GW_ESINGULAR: return "GW_ESINGULAR";
    case GW_ENOTTRAINED: return "GW_ENOTTRAINED";
    case GW_EUNSUPPORTED: return "GW_EUNSUPPORTED";
    case GW_EFALLBACK: return "GW_EFALLBACK";
  }
  return "GW_UNKNOWN";
}

gw_status gw_ctx_create(gw_ctx** out, int device, void* stream) {
  if (!out) return GW_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return GW_EDEVICE;
  if (device < 0 || device >= ndev) return GW_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return GW_EDEVICE;
  gw_ctx* c = new gw_ctx();
  c->device = device;
  c->stream = static_cast<hipStream_t>(stream);
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
      cus > 0)
    c->cus = cus;
  if (hipMalloc(&c->d_flag, 64) != hipSuccess) { delete c; return GW_ENOMEM; }
  if (hipMemset(c->d_flag, 0, 64) != hipSuccess) { (void)hipFree(c->d_flag); delete c; return GW_EDEVICE; }
  *out = c;
  return GW_OK;
}

gw_status gw_ctx_destroy(gw_ctx* c) {
  if (!c) return GW_EINVAL;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  // children still alive are released with their context
  for (gw_mlp* n : std::vector<gw_mlp*>(c->mlps.begin(), c->mlps.end())) mlp_free(n);
  for (gw_plan* p : std::vector<gw_plan*>(c->plans.begin(), c->plans.end())) plan_free(p);
  for (auto& r : c->prof_pending) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
  for (auto e : c->ev_pool) (void)hipEventDestroy(e);
  for (auto& kv : c->spheres) {
    (void)hipFree(kv.second.d_cube);
    (void)hipFree(kv.second.d_disk);
  }
  for (auto& kv : c->twiddles) (void)hipFree(kv.second);
  for (auto& kv : c->tile_orders) (void)hipFree(kv.second);
  if (c->ws) (void)hipFree(c->ws);
  if (c->d_flag) (void)hipFree(c->d_flag);
  pin_release(c);
  delete c;
  return GW_OK;
}

gw_status gw_ctx_set_stream(gw_ctx* c, void* stream) {
  if (!c) return GW_EINVAL;
  c->stream = static_cast<hipStream_t>(stream);
  return GW_OK;
}

const char* gw_last_error(const gw_ctx* c) { return c ? c->err.c_str() : "null context"; }

gw_status gw_ctx_profile(gw_ctx* c, int enable) {
  if (!c) return GW_EINVAL;
  c->profiling = enable != 0;
  return GW_OK;
}

gw_status gw_ctx_profile_only(gw_ctx* c, const char* name) {
  if (!c) return GW_EINVAL;
  c->prof_only = name ? name : "";
  return GW_OK;
}

gw_status gw_ctx_profile_reset(gw_ctx* c) {
  if (!c) return GW_EINVAL;
  prof_collect(c);
  c->prof.clear();
  c->prof_names.clear();
  return GW_OK;
}

int gw_ctx_profile_count(gw_ctx* c) {
  if (!c) return 0;
  prof_collect(c);
  return (int)c->prof_names.size();
}

gw_status gw_ctx_profile_entry(gw_ctx* c, int i, const char** name, int* launches,
                               double* total_ms) {
  if (!c) return GW_EINVAL;
  prof_collect(c);
  if (i < 0 || i >= (int)c->prof_names.size()) return fail(c, GW_EINVAL, "profile index %d", i);
  const auto& nm = c->prof_names[i];
  const auto& acc = c->prof[nm];
  if (name) *name = nm.c_str();
  if (launches) *launches = acc.launches;
  if (total_ms) *total_ms = acc.ms;
  return GW_OK;
}

gw_status gw_mtxel_spinor(gw_ctx* c, const int box[3], int nspinor, int nv, int ngv,
                          const int32_t* gv, const void* cv, int nc, int ngc, const int32_t* gc,
                          const void* cc, int neps, const int32_t* geps, gw_dtype dtype,
                          void* mtxel, int head_index, double* mhead) {
  if (!c) return GW_EINVAL;
  c->err.clear();
  if (!box) return fail(c, GW_EINVAL, "box is NULL");
  for (int a = 0; a < 3; ++a)
    if (!factorable(box[a]))
      return fail(c, GW_EINVAL, "box[%d] = %d must be a positive product of 2, 3 and 5", a, box[a]);
  if (box[0] > 4096 || box[1] > 4096 || box[2] > 4096)
    return fail(c, GW_EINVAL, "box dimension above 4096");
  if (nspinor != 1 && nspinor != 2) return fail(c, GW_EINVAL, "nspinor must be 1 or 2");
  if (nv < 0 || nc < 0 || neps < 0 || ngv < 0 || ngc < 0)
    return fail(c, GW_EINVAL, "negative size");
  if (dtype != GW_C128 && dtype != GW_C64) return fail(c, GW_EINVAL, "unknown dtype");
  if (nv == 0 || nc == 0 || neps == 0) return GW_OK;
  if (ngv == 0 || ngc == 0) return fail(c, GW_EINVAL, "empty wavefunction sphere");
  if (!g_ok(gv, ngv) || !g_ok(gc, ngc) || !g_ok(geps, neps) || !cv || !cc || !mtxel)
    return fail(c, GW_EINVAL, "NULL array argument");
  if (head_index >= neps) return fail(c, GW_EINVAL, "head_index %d >= neps %d", head_index, neps);
  if (head_index >= 0 &&
      (geps[3 * head_index] != 0 || geps[3 * head_index + 1] != 0 || geps[3 * head_index + 2] != 0))
    return fail(c, GW_EINVAL, "geps[head_index] is not G = 0");
  if ((long long)nv * nc > (1LL << 31) / 2) return fail(c, GW_EINVAL, "too many pairs");
  (void)hipSetDevice(c->device);

  SphereMap *sv, *sc, *se;
  gw_status st;
  if ((st = sphere_map(c, gv, ngv, box, &sv)) != GW_OK) return st;
  if ((st = sphere_map(c, gc, ngc, box, &sc)) != GW_OK) return st;
  if ((st = sphere_map(c, geps, neps, box, &se)) != GW_OK) return st;
  for (int a = 0; a < 3; ++a)
    if (box[a] <= sv->gmax[a] + sc->gmax[a] + se->gmax[a])
      return fail(c, GW_EALIAS,
                  "box[%d] = %d <= %d + %d + %d: the pair product would alias onto an eps G", a,
                  box[a], sv->gmax[a], sc->gmax[a], se->gmax[a]);

  const size_t elem = dtype == GW_C128 ? 16 : 8;
  const size_t nbox = (size_t)box[0] * box[1] * box[2];
  const size_t uv_bytes = (size_t)nv * nspinor * nbox * elem;
  if (!pair_compact_shape(box) && pair_xy_shape(box))
    return mtxel_xy(c, box, nspinor, nv, ngv, cv, nc, ngc, cc, dtype, sv, sc, se, mtxel,
                    head_index, mhead, gv, gc);
  // conduction bands: compact x-transformed slabs when the pair kernels build
  // their planes themselves, full real-space fields otherwise
  const bool compact = pair_compact_shape(box);
  const size_t uc_bytes = compact ? band_compact_bytes(box, sc, nc * nspinor, elem)
                                  : (size_t)nc * nspinor * nbox * elem;
  // band scratch: a chunk of band-spins of the compact x-pass output
  const size_t band_per = band_scratch_bytes(box, sv, 1, elem) > band_scratch_bytes(box, sc, 1, elem)
                              ? band_scratch_bytes(box, sv, 1, elem)
                              : band_scratch_bytes(box, sc, 1, elem);
  const int nbs_max = std::max(nv, nc) * nspinor;
  const int band_chunk = (int)std::max<size_t>(1, std::min<size_t>(nbs_max, (512ull << 20) / band_per));
  const size_t band_bytes = band_per * band_chunk;
  // pair scratch: all valence bands times a tile of conduction bands
  const size_t pair_per = pair_scratch_bytes(box, se, 1, elem);
  size_t pair_budget = 1ull << 30;
  int max_pairs = (int)std::max<size_t>(1, pair_budget / pair_per);
  if (max_pairs > 65535) max_pairs = 65535;
  int vt = std::min(nv, max_pairs);
  int ct = std::max(1, std::min(nc, max_pairs / vt));
  const size_t pair_bytes = pair_per * (size_t)vt * ct;
  // head match list
  std::vector<int> match;
  if (mhead) {
    std::map<std::tuple<int, int, int>, int> lut;
    for (int i = 0; i < ngc; ++i) lut[std::make_tuple(gc[3 * i], gc[3 * i + 1], gc[3 * i + 2])] = i;
    for (int i = 0; i < ngv; ++i) {
      auto it = lut.find(std::make_tuple(gv[3 * i], gv[3 * i + 1], gv[3 * i + 2]));
      if (it != lut.end()) { match.push_back(i); match.push_back(it->second); }
    }
  }
  const size_t match_bytes = match.size() * sizeof(int) + 16;
  st = ws_begin(c, align_up(uv_bytes) + align_up(uc_bytes) + align_up(band_bytes) +
                       align_up(pair_bytes) + align_up(match_bytes));
  if (st != GW_OK) return st;
  void* uv = ws_take(c, uv_bytes);
  void* uc = ws_take(c, uc_bytes);
  void* bscr = ws_take(c, band_bytes);
  void* pscr = ws_take(c, pair_bytes);
  int* dmatch = static_cast<int*>(ws_take(c, match_bytes));

  if (dtype == GW_C128) {
    if ((st = band_to_grid<double>(c, box, nv * nspinor, ngv, cv, sv, uv, bscr, band_bytes)) != GW_OK) return st;
    st = compact ? band_compact<double>(c, box, nc * nspinor, ngc, cc, sc, uc)
                 : band_to_grid<double>(c, box, nc * nspinor, ngc, cc, sc, uc, bscr, band_bytes);
    if (st != GW_OK) return st;
  } else {
    if ((st = band_to_grid<float>(c, box, nv * nspinor, ngv, cv, sv, uv, bscr, band_bytes)) != GW_OK) return st;
    st = compact ? band_compact<float>(c, box, nc * nspinor, ngc, cc, sc, uc)
                 : band_to_grid<float>(c, box, nc * nspinor, ngc, cc, sc, uc, bscr, band_bytes);
    if (st != GW_OK) return st;
  }
  for (int v0 = 0; v0 < nv; v0 += vt) {
    const int nvt = std::min(vt, nv - v0);
    for (int c0 = 0; c0 < nc; c0 += ct) {
      const int nct = std::min(ct, nc - c0);
      const void* ucf = compact ? nullptr : uc;
      const void* tcs = compact ? uc : nullptr;
      if (dtype == GW_C128)
        st = pair_to_eps<double>(c, box, nspinor, uv, ucf, tcs, sc, v0, nvt, c0, nct, nc, se,
                                 mtxel, pscr);
      else
        st = pair_to_eps<float>(c, box, nspinor, uv, ucf, tcs, sc, v0, nvt, c0, nct, nc, se,
                                mtxel, pscr);
      if (st != GW_OK) return st;
    }
  }
  if (mhead) {
    const int nm = (int)match.size() / 2;
    if (nm > 0) {
      if ((st = stage_h2d(c, dmatch, match.data(), match.size() * sizeof(int))) != GW_OK)
        return st;
      if ((st = head_overlap(c, dtype, nspinor, nv, ngv, cv, nc, ngc, cc, dmatch, nm, mhead)) != GW_OK)
        return st;
    } else {
      GW_HIP(c, hipMemsetAsync(mhead, 0, (size_t)nv * nc * 16, c->stream));
    }
  }
  return GW_OK;
}

gw_status gw_chi0_accumulate(gw_ctx* c, int nv, int nc, int neps, const void* mtxel,
                             gw_dtype dtype, const double* ev, const double* ec, int nfreq,
                             const double* omega, double prefactor, gw_prec prec,
                             const double* mhead, int head_index, double* chi0) {
  if (!c) return GW_EINVAL;
  c->err.clear();
  if (nv < 0 || nc < 0 || neps < 0 || nfreq < 0) return fail(c, GW_EINVAL, "negative size");
  if (dtype != GW_C128 && dtype != GW_C64) return fail(c, GW_EINVAL, "unknown dtype");
  if (prec != GW_PREC_FP64 && prec != GW_PREC_SPLITBF16) return fail(c, GW_EINVAL, "unknown precision");
  if (prec == GW_PREC_SPLITBF16 && dtype != GW_C64)
    return fail(c, GW_EINVAL, "split-BF16 contraction needs GW_C64 matrix elements");
  if (nv == 0 || nc == 0 || neps == 0 || nfreq == 0) return GW_OK;
  if (!mtxel || !ev || !ec || !omega || !chi0) return fail(c, GW_EINVAL, "NULL array argument");
  if (!std::isfinite(prefactor)) return fail(c, GW_EINVAL, "non-finite prefactor");
  for (int f = 0; f < nfreq; ++f)
    if (!(omega[f] >= 0.0) || !std::isfinite(omega[f]))
      return fail(c, GW_EINVAL, "omega[%d] must be finite and >= 0", f);
  if (head_index >= neps) return fail(c, GW_EINVAL, "head_index >= neps");
  if ((long long)neps * neps > (1LL << 40)) return fail(c, GW_EINVAL, "neps too large");
  if ((long long)nv * nc > (1LL << 31) / 2) return fail(c, GW_EINVAL, "too many pairs");
  (void)hipSetDevice(c->device);
  const int P = nv * nc;
  const bool use_head = mhead != nullptr && head_index >= 0;
  const int split = chi0_split(c, P, neps, nfreq, prec, dtype);
  const size_t part_bytes = (size_t)(split - 1) * nfreq * neps * neps * 16;
  const size_t xs_bytes = prec == GW_PREC_SPLITBF16 ? bf16_split_bytes(P, neps, nfreq) : 0;
  gw_status st = ws_begin(c, align_up((size_t)nfreq * 8) + align_up((size_t)nfreq * P * 8) +
                                 align_up(part_bytes) + align_up(xs_bytes));
  if (st != GW_OK) return st;
  double* d_om = static_cast<double*>(ws_take(c, (size_t)nfreq * 8));
  double* wts = static_cast<double*>(ws_take(c, (size_t)nfreq * P * 8));
  double* part = part_bytes ? static_cast<double*>(ws_take(c, part_bytes)) : nullptr;
  void* xsplit = xs_bytes ? ws_take(c, xs_bytes) : nullptr;
  if ((st = stage_h2d(c, d_om, omega, (size_t)nfreq * 8)) != GW_OK) return st;
  if ((st = chi0_weights(c, nv, nc, ev, ec, nfreq, d_om, prefactor, wts)) != GW_OK) return st;
  const int skip = use_head ? head_index : -1;
  if (prec == GW_PREC_FP64)
    st = chi0_fp64(c, P, neps, mtxel, dtype, nfreq, wts, skip, chi0, split, part);
  else
    st = chi0_splitbf16(c, P, neps, mtxel, nfreq, wts, skip, chi0, split, part, xsplit);
  if (st != GW_OK) return st;
  if (use_head) {
    if ((st = chi0_wings(c, P, neps, mtxel, dtype, mhead, head_index, nfreq, wts, chi0)) != GW_OK)
      return st;
  }
  return GW_OK;
}

gw_status gw_head_dipole(gw_ctx* c, int nspinor, int nv, int nc, int ng, const int* g,
                         const void* cv, const void* cc, gw_dtype dtype, const double* cell,
                         const double* kpt, const double* qcart, const double* ev,
                         const double* ec, double* mhead) {
  if (!c) return GW_EINVAL;
  c->err.clear();
  if (nspinor != 1 && nspinor != 2) return fail(c, GW_EINVAL, "nspinor must be 1 or 2");
  if (nv < 0 || nc < 0 || ng < 0) return fail(c, GW_EINVAL, "negative size");
  if (dtype != GW_C128 && dtype != GW_C64) return fail(c, GW_EINVAL, "unknown dtype");
  if (nv == 0 || nc == 0) return GW_OK;
  if (!cell || !kpt || !qcart || !ev || !ec || !mhead || (ng > 0 && (!g || !cv || !cc)))
    return fail(c, GW_EINVAL, "NULL array argument");
  if ((long long)nv * nc > (1LL << 31) - 1) return fail(c, GW_EINVAL, "nv*nc too large");
  double sq[3], q0k = 0.0;
  for (int i = 0; i < 3; ++i) {
    if (!(cell[i] > 0.0) || !std::isfinite(cell[i]) || !std::isfinite(kpt[i]) ||
        !std::isfinite(qcart[i]))
      return fail(c, GW_EINVAL, "cell must be positive and k, q finite");
    sq[i] = 2.0 * M_PI * qcart[i] / cell[i];
    q0k += kpt[i] * sq[i];
  }
  (void)hipSetDevice(c->device);
  gw_status st = ws_begin(c, align_up((size_t)std::max(ng, 1) * 3 * sizeof(int)));
  if (st != GW_OK) return st;
  int* d_g = static_cast<int*>(ws_take(c, (size_t)std::max(ng, 1) * 3 * sizeof(int)));
  if ((st = stage_h2d(c, d_g, g, (size_t)ng * 3 * sizeof(int))) != GW_OK) return st;
  return head_dipole(c, dtype, nspinor, nv, nc, ng, cv, cc, d_g, sq, q0k, ev, ec, mhead);
}

gw_status gw_chi0_accumulate_real(gw_ctx* c, int nv, int nc, int neps, const void* mtxel,
                                  gw_dtype dtype, const double* ev, const double* ec, int nfreq,
                                  const double* omega, double eta, double prefactor, gw_prec prec,
                                  double* chi0) {
  if (!c) return GW_EINVAL;
  c->err.clear();
  if (nv < 0 || nc < 0 || neps < 0 || nfreq < 0) return fail(c, GW_EINVAL, "negative size");
  if (dtype != GW_C128 && dtype != GW_C64) return fail(c, GW_EINVAL, "unknown dtype");
  if (prec != GW_PREC_FP64 && prec != GW_PREC_SPLITBF16) return fail(c, GW_EINVAL, "unknown precision");
  if (prec == GW_PREC_SPLITBF16 && dtype != GW_C64)
    return fail(c, GW_EINVAL, "split-BF16 contraction needs GW_C64 matrix elements");
  if (!(eta > 0.0) || !std::isfinite(eta)) return fail(c, GW_EINVAL, "eta must be finite and > 0");
  if (nv == 0 || nc == 0 || neps == 0 || nfreq == 0) return GW_OK;
  if (!mtxel || !ev || !ec || !omega || !chi0) return fail(c, GW_EINVAL, "NULL array argument");
  if (!std::isfinite(prefactor)) return fail(c, GW_EINVAL, "non-finite prefactor");
  for (int f = 0; f < nfreq; ++f)
    if (!std::isfinite(omega[f])) return fail(c, GW_EINVAL, "omega[%d] must be finite", f);
  if ((long long)neps * neps > (1LL << 40)) return fail(c, GW_EINVAL, "neps too large");
  if (nfreq > 32767) return fail(c, GW_EINVAL, "nfreq above 32767");
  if ((long long)nv * nc > (1LL << 31) / 2) return fail(c, GW_EINVAL, "too many pairs");
  (void)hipSetDevice(c->device);
  const int P = nv * nc, nw = 2 * nfreq;
  const size_t nn = (size_t)neps * neps;
  const int split = chi0_split(c, P, neps, nw, prec, dtype);
  const size_t part_bytes = (size_t)(split - 1) * nw * nn * 16;
  const size_t xs_bytes = prec == GW_PREC_SPLITBF16 ? bf16_split_bytes(P, neps, nw) : 0;
  gw_status st = ws_begin(c, align_up((size_t)nfreq * 8) + align_up((size_t)nw * P * 8) +
                                 align_up((size_t)nw * nn * 16) + align_up(part_bytes) +
                                 align_up(xs_bytes));
  if (st != GW_OK) return st;
  double* d_om = static_cast<double*>(ws_take(c, (size_t)nfreq * 8));
  double* wts = static_cast<double*>(ws_take(c, (size_t)nw * P * 8));
  double* h = static_cast<double*>(ws_take(c, (size_t)nw * nn * 16));
  double* part = part_bytes ? static_cast<double*>(ws_take(c, part_bytes)) : nullptr;
  void* xsplit = xs_bytes ? ws_take(c, xs_bytes) : nullptr;
  if ((st = stage_h2d(c, d_om, omega, (size_t)nfreq * 8)) != GW_OK) return st;
  GW_HIP(c, hipMemsetAsync(h, 0, (size_t)nw * nn * 16, c->stream));
  if ((st = chi0_weights_real(c, nv, nc, ev, ec, nfreq, d_om, eta, prefactor, wts)) != GW_OK)
    return st;
  // the two real weight sets give two Hermitian contractions A and B, and
  // chi0 += A + i B
  if (prec == GW_PREC_FP64)
    st = chi0_fp64(c, P, neps, mtxel, dtype, nw, wts, -1, h, split, part);
  else
    st = chi0_splitbf16(c, P, neps, mtxel, nw, wts, -1, h, split, part, xsplit);
  if (st != GW_OK) return st;
  return chi0_combine_real(c, neps, nfreq, h, chi0);
}

gw_status gw_epsinv_lu(gw_ctx* c, int neps, int nfreq, const double* chi0, const double* vcoul,
                       double* epsinv) {
  if (!c) return GW_EINVAL;
  c->err.clear();
  if (neps < 0 || nfreq < 0) return fail(c, GW_EINVAL, "negative size");
  if (neps == 0 || nfreq == 0) return GW_OK;
  if (!chi0 || !vcoul || !epsinv) return fail(c, GW_EINVAL, "NULL array argument");
  if (chi0 == epsinv) return fail(c, GW_EINVAL, "epsinv may not alias chi0");
  if (neps > 16384) return fail(c, GW_EINVAL, "neps above 16384");
  if (nfreq > 65535) return fail(c, GW_EINVAL, "nfreq above 65535");
  (void)hipSetDevice(c->device);
  return epsinv_pivoted_one(c, neps, nfreq, chi0, vcoul, epsinv);
}

gw_status gw_screened_w(gw_ctx* c, int neps, int nfreq, const double* epsinv,
                        const double* vcoul, double* w) {
  if (!c) return GW_EINVAL;
  c->err.clear();
  if (neps < 0 || nfreq < 0) return fail(c, GW_EINVAL, "negative size");
  if (neps == 0 || nfreq == 0) return GW_OK;
  if (!epsinv || !vcoul || !w) return fail(c, GW_EINVAL, "NULL array argument");
  if (nfreq > 65535) return fail(c, GW_EINVAL, "nfreq above 65535");
  if ((long long)neps * neps > (1LL << 40)) return fail(c, GW_EINVAL, "neps too large");
  (void)hipSetDevice(c->device);
  return screened_w(c, neps, nfreq, epsinv, vcoul, w);
}

gw_status gw_sigma_sx(gw_ctx* c, int nocc, int nband, int neps, const void* mtxel,
                      gw_dtype dtype, const double* epsinv, const double* vcoul,
                      double prefactor, double* sigma) {
  if (!c) return GW_EINVAL;
  c->err.clear();
  if (nocc < 0 || nband < 0 || neps < 0) return fail(c, GW_EINVAL, "negative size");
  if (dtype != GW_C128 && dtype != GW_C64) return fail(c, GW_EINVAL, "unknown dtype");
  if (nocc == 0 || nband == 0 || neps == 0) return GW_OK;
  if (!mtxel || !epsinv || !vcoul || !sigma) return fail(c, GW_EINVAL, "NULL array argument");
  if (!std::isfinite(prefactor)) return fail(c, GW_EINVAL, "non-finite prefactor");
  if ((long long)nocc * nband > 65535 || neps > 16384)
    return fail(c, GW_EINVAL, "nocc*nband above 65535 or neps above 16384");
  if (static_cast<const void*>(sigma) == mtxel || sigma == epsinv)
    return fail(c, GW_EINVAL, "sigma aliases an input");
  (void)hipSetDevice(c->device);
  return sigma_sx_static(c, nocc, nband, neps, mtxel, dtype, epsinv, vcoul, prefactor, sigma);
}

gw_status gw_epsinv(gw_ctx* c, int neps, int nfreq, const double* chi0, const double* vcoul,
                    double* epsinv) {
  if (!c) return GW_EINVAL;
  c->err.clear();
  if (neps < 0 || nfreq < 0) return fail(c, GW_EINVAL, "negative size");
  if (neps == 0 || nfreq == 0) return GW_OK;
  if (!chi0 || !vcoul || !epsinv) return fail(c, GW_EINVAL, "NULL array argument");
  if (chi0 == epsinv) return fail(c, GW_EINVAL, "epsinv may not alias chi0");
  if (neps > 16384) return fail(c, GW_EINVAL, "neps above 16384");
  if (nfreq > 65535) return fail(c, GW_EINVAL, "nfreq above 65535");
  (void)hipSetDevice(c->device);
  return epsinv_run(c, neps, nfreq, chi0, vcoul, epsinv);
}

}  // extern "C"
