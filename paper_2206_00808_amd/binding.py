"""ctypes binding of libgwspinor (include/gw.h): argument marshalling only.

Every function here has the name of the C entry point it wraps and passes
torch device tensors by pointer; all computation happens in the library's HIP
kernels.  The library must be built (``paper_2206_00808_amd.build.build()``);
importing this module without it raises ImportError.
"""
from __future__ import annotations

import ctypes as ct
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libgwspinor.so")

GW_OK, GW_EINVAL, GW_ENOMEM, GW_EDEVICE = 0, -1, -2, -3
GW_EALIAS, GW_ESINGULAR, GW_ENOTTRAINED, GW_EUNSUPPORTED, GW_EFALLBACK = -4, -5, -6, -7, 1
GW_C128, GW_C64 = 0, 1
GW_PREC_FP64, GW_PREC_SPLITBF16 = 0, 1
GW_CLOSURE_INFER, GW_CLOSURE_TRAIN_STEP, GW_CLOSURE_FULL_FALLBACK = 0, 1, 2

EXPORTED = [
    "gw_ctx_create", "gw_ctx_destroy", "gw_ctx_set_stream", "gw_last_error", "gw_status_string",
    "gw_ctx_profile", "gw_ctx_profile_only", "gw_ctx_profile_reset", "gw_ctx_profile_count",
    "gw_ctx_profile_entry",
    "gw_mtxel_spinor", "gw_chi0_accumulate", "gw_chi0_accumulate_noalloc", "gw_epsinv",
    "gw_chi0_accumulate_real",
    "gw_epsinv_lu", "gw_head_dipole", "gw_screened_w", "gw_sigma_sx",
    "gw_unfold_spinor", "gw_gpp_modes", "gw_sigma_gpp", "gw_chi0_symmetrize",
    "gw_bse_kernel", "gw_little_group", "gw_kgrid_orbits", "gw_epsinv_lowrank",
    "gw_lowrank_basis", "gw_mtxel_project", "gw_epsinv_from_basis", "gw_peak_probe",
    "gw_mlp_create", "gw_mlp_destroy", "gw_mlp_save", "gw_mlp_load", "gw_mlp_set_tolerance",
    "gw_chi0_closure",
    "gw_plan_create", "gw_plan_compile", "gw_plan_launch", "gw_plan_destroy", "gw_plan_describe",
]

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run paper_2206_00808_amd.build.build() "
                      "(or __graft_entry__.build()) first")

# torch's HIP runtime is loaded before this library, so that a process that
# creates a context before touching torch still sees its devices through torch
try:
    import torch  # noqa: F401
except ImportError:  # the library itself does not need torch
    pass

_lib = ct.CDLL(LIB_PATH)

_vp, _i, _d, _u64 = ct.c_void_p, ct.c_int, ct.c_double, ct.c_uint64
_ip = ct.POINTER(ct.c_int)


class QDesc(ct.Structure):
    _fields_ = [
        ("nv", _i), ("ngv", _i), ("gv", _vp), ("cv", _vp),
        ("nc", _i), ("ngc", _i), ("gc", _vp), ("cc", _vp),
        ("neps", _i), ("geps", _vp),
        ("ev", _vp), ("ec", _vp), ("vcoul", _vp),
        ("head_index", _i), ("chi0", _vp), ("epsinv", _vp),
    ]


_SIG = {
    "gw_ctx_create": (_i, [ct.POINTER(_vp), _i, _vp]),
    "gw_ctx_destroy": (_i, [_vp]),
    "gw_ctx_set_stream": (_i, [_vp, _vp]),
    "gw_last_error": (ct.c_char_p, [_vp]),
    "gw_status_string": (ct.c_char_p, [_i]),
    "gw_ctx_profile": (_i, [_vp, _i]),
    "gw_ctx_profile_only": (_i, [_vp, ct.c_char_p]),
    "gw_ctx_profile_reset": (_i, [_vp]),
    "gw_ctx_profile_count": (_i, [_vp]),
    "gw_ctx_profile_entry": (_i, [_vp, _i, ct.POINTER(ct.c_char_p), _ip, ct.POINTER(_d)]),
    "gw_mtxel_spinor": (_i, [_vp, _ip, _i, _i, _i, _vp, _vp, _i, _i, _vp, _vp, _i, _vp, _i,
                             _vp, _i, _vp]),
    "gw_chi0_accumulate": (_i, [_vp, _i, _i, _i, _vp, _i, _vp, _vp, _i, _vp, _d, _i, _vp, _i,
                                _vp]),
    "gw_chi0_accumulate_noalloc": (_i, [_vp, _i, _i, _i, _vp, _i, _vp, _vp, _i, _vp, _d, _vp,
                                        _i, _vp]),
    "gw_epsinv": (_i, [_vp, _i, _i, _vp, _vp, _vp]),
    "gw_chi0_accumulate_real": (_i, [_vp, _i, _i, _i, _vp, _i, _vp, _vp, _i, _vp, _d, _d, _i,
                                     _vp]),
    "gw_epsinv_lu": (_i, [_vp, _i, _i, _vp, _vp, _vp]),
    "gw_peak_probe": (_i, [_vp, _i, _vp]),
    "gw_lowrank_basis": (_i, [_vp, _i, _vp, _vp, _i, _vp, _vp]),
    "gw_mtxel_project": (_i, [_vp, _i, _i, _vp, _i, _vp, _i, _vp, _vp]),
    "gw_epsinv_from_basis": (_i, [_vp, _i, _i, _i, _vp, _vp, _vp, _vp]),
    "gw_epsinv_lowrank": (_i, [_vp, _i, _i, _vp, _vp, _i, _vp, _vp]),
    "gw_little_group": (_i, [_i, _vp, _vp, _vp, _vp]),
    "gw_kgrid_orbits": (_i, [_i, _i, _i, _i, _vp, _vp, _vp, _vp, _vp, _vp]),
    "gw_bse_kernel": (_i, [_vp, _i, _i, _i, _vp, _vp, _vp, _i, _vp, _vp, _vp, _vp]),
    "gw_chi0_symmetrize": (_i, [_vp, _i, _i, _vp, _vp, _i, _vp, _vp, _vp, _vp]),
    "gw_gpp_modes": (_i, [_vp, _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "gw_sigma_gpp": (_i, [_vp, _i, _i, _i, _i, _vp, _i, _vp, _vp, _vp, _vp, _i, _vp, _d, _vp,
                          _vp]),
    "gw_unfold_spinor": (_i, [_vp, _i, _i, _i, _vp, _vp, _i, _i, _vp, _vp, _vp, _vp, _vp,
                              _vp]),
    "gw_screened_w": (_i, [_vp, _i, _i, _vp, _vp, _vp]),
    "gw_sigma_sx": (_i, [_vp, _i, _i, _i, _vp, _i, _vp, _vp, _d, _vp]),
    "gw_head_dipole": (_i, [_vp, _i, _i, _i, _i, _vp, _vp, _vp, _i, _vp, _vp, _vp, _vp, _vp,
                            _vp]),
    "gw_mlp_create": (_i, [_vp, ct.POINTER(_vp), _i, _i, _i, _i, _u64]),
    "gw_mlp_destroy": (_i, [_vp]),
    "gw_mlp_save": (_i, [_vp, _vp, ct.POINTER(ct.c_size_t)]),
    "gw_mlp_load": (_i, [_vp, _vp, ct.c_size_t]),
    "gw_mlp_set_tolerance": (_i, [_vp, _d]),
    "gw_chi0_closure": (_i, [_vp, _vp, _i, _i, _vp, _vp, _d, _d, _vp, ct.c_float,
                             ct.POINTER(ct.c_float), _vp]),
    "gw_plan_create": (_i, [_vp, ct.POINTER(_vp), _ip, _i, _i, _i, _i, _vp, _d, _i,
                            ct.POINTER(QDesc)]),
    "gw_plan_compile": (_i, [_vp]),
    "gw_plan_launch": (_i, [_vp]),
    "gw_plan_destroy": (_i, [_vp]),
    "gw_plan_describe": (ct.c_char_p, [_vp]),
}
for _name, (_res, _args) in _SIG.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class GwError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{status_string(status)}: {message}")
        self.status = status


def status_string(s):
    return _lib.gw_status_string(int(s)).decode()


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _host_i32(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.int32))
    return a


def _check(ctx, status, ok=(GW_OK,)):
    if status not in ok:
        raise GwError(status, _lib.gw_last_error(ctx.handle).decode() if ctx else "")
    return status


class Context:
    """Owns a gw_ctx on one HIP device; calls run on torch's current stream."""

    def __init__(self, device=0):
        h = _vp()
        s = _lib.gw_ctx_create(ct.byref(h), int(device), None)
        if s != GW_OK:
            raise GwError(s, "gw_ctx_create failed (no usable HIP device?)")
        self.handle = h
        self.device = device
        self._children = weakref.WeakSet()

    def close(self):
        if getattr(self, "handle", None):
            # the library frees networks and plans with their context
            for ch in list(self._children):
                ch.handle = None
            _lib.gw_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sync_stream(self):
        import torch
        st = torch.cuda.current_stream(self.device).cuda_stream
        _lib.gw_ctx_set_stream(self.handle, ct.c_void_p(st))

    # profiling -------------------------------------------------------------
    def profile(self, enable=True):
        _check(self, _lib.gw_ctx_profile(self.handle, 1 if enable else 0))

    def profile_only(self, name=None):
        """Record events around kernels of this name only (None: all)."""
        _check(self, _lib.gw_ctx_profile_only(self.handle, None if name is None else name.encode()))

    def profile_reset(self):
        _check(self, _lib.gw_ctx_profile_reset(self.handle))

    def profile_table(self):
        out = {}
        n = _lib.gw_ctx_profile_count(self.handle)
        for i in range(n):
            name = ct.c_char_p()
            launches = ct.c_int()
            ms = ct.c_double()
            _check(self, _lib.gw_ctx_profile_entry(self.handle, i, ct.byref(name),
                                                   ct.byref(launches), ct.byref(ms)))
            out[name.value.decode()] = (launches.value, ms.value)
        return out


def _dtype_code(t):
    import torch
    if t.dtype == torch.complex128:
        return GW_C128
    if t.dtype == torch.complex64:
        return GW_C64
    raise TypeError(f"complex128 or complex64 expected, got {t.dtype}")


def gw_mtxel_spinor(ctx, box, nspinor, gv, cv, gc, cc, geps, mtxel, head_index=-1, mhead=None):
    """M[v][c][G] on the eps sphere (see include/gw.h).  gv/gc/geps: host int arrays [n][3];
    cv [nv][nspinor][ngv], cc [nc][nspinor][ngc], mtxel [nv][nc][neps]: device tensors."""
    ctx.sync_stream()
    box_a = (ct.c_int * 3)(*[int(x) for x in box])
    gv, gc, geps = _host_i32(gv), _host_i32(gc), _host_i32(geps)
    nv, nc, neps = cv.shape[0], cc.shape[0], geps.shape[0]
    for t in (cv, cc, mtxel):
        if not t.is_contiguous():
            raise ValueError("tensors must be contiguous")
    dt = _dtype_code(cv)
    if _dtype_code(cc) != dt or _dtype_code(mtxel) != dt:
        raise TypeError("cv, cc and mtxel must share one complex dtype")
    if tuple(mtxel.shape) != (nv, nc, neps):
        raise ValueError(f"mtxel shape {tuple(mtxel.shape)} != {(nv, nc, neps)}")
    if cv.shape[1] != nspinor or cc.shape[1] != nspinor:
        raise ValueError("spinor dimension mismatch")
    if cv.shape[2] != gv.shape[0] or cc.shape[2] != gc.shape[0]:
        raise ValueError("sphere size mismatch")
    s = _lib.gw_mtxel_spinor(ctx.handle, ct.cast(box_a, _ip), int(nspinor), nv, gv.shape[0],
                             gv.ctypes.data, _ptr(cv), nc, gc.shape[0], gc.ctypes.data, _ptr(cc),
                             neps, geps.ctypes.data, dt, _ptr(mtxel), int(head_index),
                             _ptr(mhead))
    return _check(ctx, s)


def gw_chi0_accumulate(ctx, nv, nc, neps, mtxel, ev, ec, omega, prefactor, prec, chi0,
                       mhead=None, head_index=-1):
    """chi0[f] += prefactor * sum_p w_p(omega_f) conj(M_p) M_p^T (see include/gw.h)."""
    ctx.sync_stream()
    om = np.ascontiguousarray(np.asarray(omega, dtype=np.float64))
    dt = _dtype_code(mtxel)
    s = _lib.gw_chi0_accumulate(ctx.handle, int(nv), int(nc), int(neps), _ptr(mtxel), dt,
                                _ptr(ev), _ptr(ec), len(om), om.ctypes.data, float(prefactor),
                                int(prec), _ptr(mhead), int(head_index), _ptr(chi0))
    return _check(ctx, s)


def gw_chi0_accumulate_noalloc(ctx, nv, nc, neps, mtxel, ev, ec, omega, prefactor, chi0,
                               mhead=None, head_index=-1):
    """gw_chi0_accumulate in FP64 without any allocation (see include/gw.h)."""
    ctx.sync_stream()
    om = np.ascontiguousarray(np.asarray(omega, dtype=np.float64))
    dt = _dtype_code(mtxel)
    s = _lib.gw_chi0_accumulate_noalloc(ctx.handle, int(nv), int(nc), int(neps), _ptr(mtxel), dt,
                                        _ptr(ev), _ptr(ec), len(om), om.ctypes.data,
                                        float(prefactor), _ptr(mhead), int(head_index),
                                        _ptr(chi0))
    return _check(ctx, s)


def gw_epsinv(ctx, neps, nfreq, chi0, vcoul, epsinv):
    """epsinv[f] = (I - diag(vcoul) chi0[f])^-1 (see include/gw.h)."""
    ctx.sync_stream()
    s = _lib.gw_epsinv(ctx.handle, int(neps), int(nfreq), _ptr(chi0), _ptr(vcoul), _ptr(epsinv))
    return _check(ctx, s)


def gw_chi0_accumulate_real(ctx, nv, nc, neps, mtxel, ev, ec, omega, eta, prefactor, prec,
                            chi0):
    """chi0[f] += prefactor * sum_p b_p(omega_f) conj(M_p) M_p^T on the real axis
    with broadening eta (see include/gw.h)."""
    ctx.sync_stream()
    om = np.ascontiguousarray(np.asarray(omega, dtype=np.float64))
    dt = _dtype_code(mtxel)
    s = _lib.gw_chi0_accumulate_real(ctx.handle, int(nv), int(nc), int(neps), _ptr(mtxel), dt,
                                     _ptr(ev), _ptr(ec), len(om), om.ctypes.data, float(eta),
                                     float(prefactor), int(prec), _ptr(chi0))
    return _check(ctx, s)


def gw_epsinv_lu(ctx, neps, nfreq, chi0, vcoul, epsinv):
    """epsinv[f] = (I - diag(vcoul) chi0[f])^-1 by pivoted LU (see include/gw.h)."""
    ctx.sync_stream()
    s = _lib.gw_epsinv_lu(ctx.handle, int(neps), int(nfreq), _ptr(chi0), _ptr(vcoul),
                          _ptr(epsinv))
    return _check(ctx, s)


def gw_head_dipole(ctx, nspinor, g, cv, cc, cell, kpt, qcart, ev, ec, mhead):
    """mhead[v*nc + c] = q.P_vc / (E_v - E_c) from momentum matrix elements (see
    include/gw.h); g is a host int array [ng][3], cv/cc device tensors."""
    ctx.sync_stream()
    gh = np.ascontiguousarray(np.asarray(g, dtype=np.int32))
    cl = np.ascontiguousarray(np.asarray(cell, dtype=np.float64))
    kp = np.ascontiguousarray(np.asarray(kpt, dtype=np.float64))
    qc = np.ascontiguousarray(np.asarray(qcart, dtype=np.float64))
    nv, nc, ng = int(cv.shape[0]), int(cc.shape[0]), int(gh.shape[0])
    s = _lib.gw_head_dipole(ctx.handle, int(nspinor), nv, nc, ng, gh.ctypes.data, _ptr(cv),
                            _ptr(cc), _dtype_code(cv), cl.ctypes.data, kp.ctypes.data,
                            qc.ctypes.data, _ptr(ev), _ptr(ec), _ptr(mhead))
    return _check(ctx, s)


def gw_screened_w(ctx, neps, nfreq, epsinv, vcoul, w):
    """w[f] = epsinv[f] diag(vcoul) (see include/gw.h)."""
    ctx.sync_stream()
    s = _lib.gw_screened_w(ctx.handle, int(neps), int(nfreq), _ptr(epsinv), _ptr(vcoul), _ptr(w))
    return _check(ctx, s)


def gw_sigma_sx(ctx, nocc, nband, neps, mtxel, epsinv, vcoul, prefactor, sigma):
    """sigma[n] -= prefactor sum_occ M^H epsinv diag(v) M (static SX; see include/gw.h)."""
    ctx.sync_stream()
    s = _lib.gw_sigma_sx(ctx.handle, int(nocc), int(nband), int(neps), _ptr(mtxel),
                         _dtype_code(mtxel), _ptr(epsinv), _ptr(vcoul), float(prefactor),
                         _ptr(sigma))
    return _check(ctx, s)


def gw_unfold_spinor(ctx, nspinor, gin, cin, gout, rot, tau, cell, cout, g0=None):
    """cout = U cin(S^-1 (gout - g0)) e^{-i (gout - g0).tau} (see include/gw.h)."""
    gin = _host_i32(gin).reshape(-1, 3)
    gout = _host_i32(gout).reshape(-1, 3)
    rot = _host_i32(rot).reshape(9)
    tau = np.ascontiguousarray(np.asarray(tau, dtype=np.float64).reshape(3))
    cell = np.ascontiguousarray(np.asarray(cell, dtype=np.float64).reshape(3))
    g0a = None if g0 is None else _host_i32(g0).reshape(3)
    nb = cin.shape[0] if hasattr(cin, "shape") else 0
    ctx.sync_stream()
    s = _lib.gw_unfold_spinor(ctx.handle, int(nspinor), int(nb), gin.shape[0], gin.ctypes.data,
                              _ptr(cin), _dtype_code(cin), gout.shape[0], gout.ctypes.data,
                              rot.ctypes.data, tau.ctypes.data,
                              None if g0a is None else g0a.ctypes.data, cell.ctypes.data,
                              _ptr(cout))
    return _check(ctx, s)


def gw_gpp_modes(ctx, geps, cell, qred, rho, epsinv, amp, wtilde):
    """Plasmon-pole amp = Omega^2/wt and wtilde from the static eps^-1 (see include/gw.h).
    rho: device complex128 tensor [n1][n2][n3] (the box is its shape)."""
    geps = _host_i32(geps).reshape(-1, 3)
    cell = np.ascontiguousarray(np.asarray(cell, dtype=np.float64).reshape(3))
    q = np.ascontiguousarray(np.asarray(qred, dtype=np.float64).reshape(3))
    box = _host_i32(list(rho.shape))
    ctx.sync_stream()
    s = _lib.gw_gpp_modes(ctx.handle, geps.shape[0], geps.ctypes.data, cell.ctypes.data,
                          q.ctypes.data, box.ctypes.data, _ptr(rho), _ptr(epsinv), _ptr(amp),
                          _ptr(wtilde))
    return _check(ctx, s)


def gw_sigma_gpp(ctx, nn, nocc, nband, neps, mtxel, en, vcoul, amp, wtilde, energies, prefactor,
                 sigma_sx, sigma_coh):
    """Plasmon-pole SX and COH added to sigma_sx, sigma_coh [nband][ne] (see include/gw.h)."""
    ne = energies.shape[-1]
    ctx.sync_stream()
    s = _lib.gw_sigma_gpp(ctx.handle, int(nn), int(nocc), int(nband), int(neps), _ptr(mtxel),
                          _dtype_code(mtxel), _ptr(en), _ptr(vcoul), _ptr(amp), _ptr(wtilde),
                          int(ne), _ptr(energies), float(prefactor), _ptr(sigma_sx),
                          _ptr(sigma_coh))
    return _check(ctx, s)


def gw_chi0_symmetrize(ctx, geps, qred, ops, chi_in, chi_out):
    """chi_out = little-group average of chi_in (see include/gw.h); ops = [(rot, tau), ...]."""
    geps = _host_i32(geps).reshape(-1, 3)
    q = np.ascontiguousarray(np.asarray(qred, dtype=np.float64).reshape(3))
    rots = _host_i32([np.asarray(r).reshape(9) for r, _ in ops]).reshape(-1)
    taus = np.ascontiguousarray(np.asarray([np.asarray(t, dtype=np.float64).reshape(3)
                                            for _, t in ops]).reshape(-1))
    nfreq = chi_in.shape[0] if chi_in.dim() == 3 else 1
    ctx.sync_stream()
    s = _lib.gw_chi0_symmetrize(ctx.handle, geps.shape[0], nfreq, geps.ctypes.data, q.ctypes.data,
                                len(ops), rots.ctypes.data, taus.ctypes.data, _ptr(chi_in),
                                _ptr(chi_out))
    return _check(ctx, s)


def gw_bse_kernel(ctx, mvc, mcc, mvv, vx, w, kx, kd):
    """BSE exchange and direct kernels for one k-point (see include/gw.h)."""
    nv, nc, neps = mvc.shape
    dt = _dtype_code(mvc)
    if _dtype_code(mcc) != dt or _dtype_code(mvv) != dt:
        raise TypeError("mvc, mcc and mvv must share one complex dtype")
    if tuple(mcc.shape) != (nc, nc, neps) or tuple(mvv.shape) != (nv, nv, neps):
        raise ValueError("mcc must be [nc][nc][neps] and mvv [nv][nv][neps]")
    ctx.sync_stream()
    s = _lib.gw_bse_kernel(ctx.handle, nv, nc, neps, _ptr(mvc), _ptr(mcc), _ptr(mvv), dt, _ptr(vx),
                           _ptr(w), _ptr(kx), _ptr(kd))
    return _check(ctx, s)


def _host_rots(ops):
    return _host_i32([np.asarray(op[0] if isinstance(op, tuple) else op).reshape(9)
                      for op in ops]).reshape(-1)


def gw_little_group(ops, qred):
    """(in_group bool[nops], gshift int[nops][3]) for S q = q + G_S (see include/gw.h).
    Host only: needs no device and no context."""
    rots = _host_rots(ops)
    q = np.ascontiguousarray(np.asarray(qred, dtype=np.float64).reshape(3))
    ing = np.zeros(len(ops), dtype=np.int32)
    gs = np.zeros((len(ops), 3), dtype=np.int32)
    s = _lib.gw_little_group(len(ops), rots.ctypes.data, q.ctypes.data, ing.ctypes.data,
                             gs.ctypes.data)
    if s != GW_OK:
        raise GwError(s, "gw_little_group: bad operation")
    return ing.astype(bool), gs


def gw_kgrid_orbits(n, ops):
    """(rep, op, g0, weight, nirr) for the unshifted grid n under ops (see include/gw.h).
    Host only: needs no device and no context."""
    rots = _host_rots(ops)
    npts = int(n[0]) * int(n[1]) * int(n[2])
    rep = np.zeros(npts, dtype=np.int32)
    op = np.zeros(npts, dtype=np.int32)
    g0 = np.zeros((npts, 3), dtype=np.int32)
    w = np.zeros(npts, dtype=np.int32)
    nirr = ct.c_int()
    s = _lib.gw_kgrid_orbits(int(n[0]), int(n[1]), int(n[2]), len(ops), rots.ctypes.data,
                             rep.ctypes.data, op.ctypes.data, g0.ctypes.data, w.ctypes.data,
                             ct.byref(nirr))
    if s != GW_OK:
        raise GwError(s, "gw_kgrid_orbits: bad grid or operation")
    return rep, op, g0, w, nirr.value


def gw_epsinv_lowrank(ctx, neps, nfreq, chi0, vcoul, nb, epsinv, eigenvalues=None):
    """eps^-1 in a basis of nb static eigenvectors (see include/gw.h)."""
    ctx.sync_stream()
    s = _lib.gw_epsinv_lowrank(ctx.handle, int(neps), int(nfreq), _ptr(chi0), _ptr(vcoul), int(nb),
                               _ptr(epsinv), _ptr(eigenvalues))
    return _check(ctx, s)


def gw_lowrank_basis(ctx, neps, chi0_static, vcoul, nb, basis, eigenvalues=None):
    """U [neps][nb]: the leading eigenvectors of epst(0) (see include/gw.h)."""
    ctx.sync_stream()
    s = _lib.gw_lowrank_basis(ctx.handle, int(neps), _ptr(chi0_static), _ptr(vcoul), int(nb),
                              _ptr(basis), _ptr(eigenvalues))
    return _check(ctx, s)


def gw_mtxel_project(ctx, mtxel, vcoul, basis, out):
    """out [npairs][nb] = M diag(sqrt v) U (see include/gw.h)."""
    neps = mtxel.shape[-1]
    npairs = mtxel.numel() // neps
    ctx.sync_stream()
    s = _lib.gw_mtxel_project(ctx.handle, npairs, neps, _ptr(mtxel), _dtype_code(mtxel),
                              _ptr(vcoul), basis.shape[1], _ptr(basis), _ptr(out))
    return _check(ctx, s)


def gw_epsinv_from_basis(ctx, chi_b, vcoul, basis, epsinv):
    """eps^-1 from the projected chi_B [nfreq][nb][nb] (see include/gw.h)."""
    neps, nb = basis.shape
    ctx.sync_stream()
    s = _lib.gw_epsinv_from_basis(ctx.handle, int(neps), int(nb), chi_b.shape[0], _ptr(chi_b),
                                  _ptr(vcoul), _ptr(basis), _ptr(epsinv))
    return _check(ctx, s)


def gw_peak_probe(ctx, kind):
    """Measured FP64 MFMA TFLOP/s (0), FP64 vector TFLOP/s (1) or copy GB/s (2)."""
    r = ct.c_double()
    ctx.sync_stream()
    s = _lib.gw_peak_probe(ctx.handle, int(kind), ct.byref(r))
    _check(ctx, s)
    return r.value


def raw():
    """The loaded ctypes library (for tests of the exported symbol table)."""
    return _lib


class Plan:
    """gw_plan_* wrapper: one captured graph over many q-points.

    `qs` is a list of dicts holding, per q: host int arrays gv, gc, geps; device
    tensors cv, cc, ev, ec, vcoul, chi0 (out), epsinv (out); and head_index.
    The tensors must stay alive (and at the same addresses) for the plan's life.
    """

    def __init__(self, ctx, box, nspinor, dtype, prec, omega, prefactor, qs):
        ctx.sync_stream()
        self.ctx = ctx
        self._keep = qs
        om = np.ascontiguousarray(np.asarray(omega, dtype=np.float64))
        self._om = om
        arr = (QDesc * len(qs))()
        self._host = []
        for i, q in enumerate(qs):
            gv, gc, geps = _host_i32(q["gv"]), _host_i32(q["gc"]), _host_i32(q["geps"])
            self._host.append((gv, gc, geps))
            d = arr[i]
            d.nv, d.ngv, d.gv, d.cv = q["cv"].shape[0], gv.shape[0], gv.ctypes.data, _ptr(q["cv"])
            d.nc, d.ngc, d.gc, d.cc = q["nc"], gc.shape[0], gc.ctypes.data, _ptr(q["cc"])
            d.neps, d.geps = geps.shape[0], geps.ctypes.data
            d.ev, d.ec, d.vcoul = _ptr(q["ev"]), _ptr(q["ec"]), _ptr(q["vcoul"])
            d.head_index = int(q.get("head_index", -1))
            d.chi0, d.epsinv = _ptr(q["chi0"]), _ptr(q["epsinv"])
        h = _vp()
        box_a = (ct.c_int * 3)(*[int(x) for x in box])
        s = _lib.gw_plan_create(ctx.handle, ct.byref(h), ct.cast(box_a, _ip), int(nspinor),
                                int(dtype), int(prec), len(om), om.ctypes.data, float(prefactor),
                                len(qs), arr)
        _check(ctx, s)
        self.handle = h
        ctx._children.add(self)

    def compile(self):
        self.ctx.sync_stream()
        return _check(self.ctx, _lib.gw_plan_compile(self.handle))

    def launch(self):
        self.ctx.sync_stream()
        return _check(self.ctx, _lib.gw_plan_launch(self.handle))

    def describe(self):
        return _lib.gw_plan_describe(self.handle).decode()

    def close(self):
        if getattr(self, "handle", None) and getattr(self.ctx, "handle", None):
            _lib.gw_plan_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gw_plan_create(ctx, box, nspinor, dtype, prec, omega, prefactor, qs):
    return Plan(ctx, box, nspinor, dtype, prec, omega, prefactor, qs)


def gw_plan_compile(plan):
    return plan.compile()


def gw_plan_launch(plan):
    return plan.launch()


class Mlp:
    """gw_mlp_* wrapper (the closure network)."""

    def __init__(self, ctx, nin=7, width=256, depth=3, nout=2, seed=0):
        self.ctx = ctx
        h = _vp()
        _check(ctx, _lib.gw_mlp_create(ctx.handle, ct.byref(h), int(nin), int(width), int(depth),
                                       int(nout), ct.c_uint64(seed)))
        self.handle = h
        self.shape = (nin, width, depth, nout)
        ctx._children.add(self)

    def save(self):
        n = ct.c_size_t(0)
        _check(self.ctx, _lib.gw_mlp_save(self.handle, None, ct.byref(n)))
        buf = ct.create_string_buffer(n.value)
        _check(self.ctx, _lib.gw_mlp_save(self.handle, buf, ct.byref(n)))
        return bytes(buf.raw[:n.value])

    def load(self, blob):
        buf = ct.create_string_buffer(blob, len(blob))
        _check(self.ctx, _lib.gw_mlp_load(self.handle, buf, len(blob)))

    def set_tolerance(self, tol):
        """Largest rel_F against the full sum at which a judged prediction is kept."""
        _check(self.ctx, _lib.gw_mlp_set_tolerance(self.handle, float(tol)))

    def close(self):
        if getattr(self, "handle", None) and getattr(self.ctx, "handle", None):
            _lib.gw_mlp_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gw_chi0_closure(ctx, net, mode, neps, qg, chi0_trunc, gap, emax, chi0_full=None, lr=0.0,
                    chi0_out=None):
    """Returns (status, loss): status GW_OK or GW_EFALLBACK; loss for TRAIN_STEP."""
    ctx.sync_stream()
    loss = ct.c_float(float("nan"))
    s = _lib.gw_chi0_closure(ctx.handle, net.handle if net is not None else None, int(mode),
                             int(neps), _ptr(qg), _ptr(chi0_trunc), float(gap), float(emax),
                             _ptr(chi0_full), ct.c_float(lr), ct.byref(loss), _ptr(chi0_out))
    _check(ctx, s, ok=(GW_OK, GW_EFALLBACK))
    return s, loss.value


# serialised network layout (gw_mlp_save): header then float arrays
MLP_HEADER_BYTES = 48


def mlp_blob_unpack(blob):
    hdr = np.frombuffer(blob, dtype=np.uint32, count=2)
    dims = np.frombuffer(blob, dtype=np.int32, count=6, offset=8)
    step, count = np.frombuffer(blob, dtype=np.int64, count=2, offset=32)
    arr = np.frombuffer(blob, dtype=np.float32, offset=MLP_HEADER_BYTES).reshape(3, count)
    return dict(magic=int(hdr[0]), nin=int(dims[0]), width=int(dims[1]), depth=int(dims[2]),
                nout=int(dims[3]), kpad=int(dims[4]), opad=int(dims[5]), step=int(step),
                params=arr[0].copy(), m=arr[1].copy(), v=arr[2].copy())


def mlp_blob_pack(meta, params, m=None, v=None):
    count = params.size
    m = np.zeros(count, np.float32) if m is None else m
    v = np.zeros(count, np.float32) if v is None else v
    head = np.array([meta["magic"], 1], dtype=np.uint32).tobytes()
    head += np.array([meta["nin"], meta["width"], meta["depth"], meta["nout"], meta["kpad"],
                      meta["opad"]], dtype=np.int32).tobytes()
    head += np.array([meta["step"], count], dtype=np.int64).tobytes()
    return head + np.concatenate([params, m, v]).astype(np.float32).tobytes()


def mlp_layers(meta):
    """(din, dout) of each padded linear layer, in the order stored."""
    dims = [meta["kpad"]] + [meta["width"]] * meta["depth"] + [meta["opad"]]
    return list(zip(dims[:-1], dims[1:]))
