"""Seeded synthetic spinor systems with the shapes of the paper's workloads.

The paper's Epsilon stage consumes fully relativistic Kohn-Sham spinors
phi_nk = sum_alpha phi_nk,alpha |alpha> expanded in plane waves on a kinetic
energy sphere (Sec. II, the non-collinear spinor definition; Sec. III, the
wavefunction-sphere storage), band energies, and the dielectric G-sphere set by
epsilon_cut (Table "tab:parameters").  No DFT data ships here, so every input is
drawn from a seeded generator:

* G-spheres: integer triples g with |k+G|^2 < E_cut, G = 2*pi*g/a on an
  orthorhombic cell, energies in Rydberg (so the cutoff is on |k+G|^2 in
  bohr^-2), sorted by ascending |k+G|^2 with ties broken lexicographically.
* Spinors: complex N(0,1) coefficients on the stacked (up block, down block)
  2*N_G vector, orthonormalised by a Householder QR; band n is column n.
* Energies: E_v ~ U[-6, 0] eV, E_c ~ U[1, 20] eV, each sorted, in Hartree.
* The small-q head construction: valence at k+q0 is the valence at k plus
  |q0| times a random spinor, re-orthonormalised, so that the G=0 matrix
  element is O(|q0|) as it is for a physical q -> 0 limit.

Draw order per system (numpy default_rng(seed)):
  joint case (q0 head): X_joint (real, imag) -> R (real, imag) -> E_v -> E_c
  separate case:        X_c (real, imag) -> X_v (real, imag) -> E_v -> E_c
"""
from __future__ import annotations

import dataclasses
import hashlib
import json
import math
from dataclasses import dataclass, field

import numpy as np

EV_PER_HA = 27.211386245988


@dataclass(frozen=True)
class SystemConfig:
    name: str
    seed: int
    cell: tuple            # orthorhombic lattice constants a1, a2, a3 (bohr)
    box: tuple             # FFT box n1, n2, n3
    ecut_wfn: float        # Ry: wavefunction sphere |k+G|^2 < ecut_wfn
    ecut_eps: float        # Ry: dielectric sphere |q+G|^2 < ecut_eps
    nv: int
    nc: int
    q: tuple               # reduced coordinates of the momentum transfer
    omega_ev: tuple = (0.0,)   # imaginary-axis frequencies (eV); 0 is static
    nspinor: int = 2
    q0_head: bool = False  # q is a small q0 near Gamma (FP64 head/wings)


def _c2_omegas():
    return (0.0,) + tuple(0.5 * 80.0 ** (j / 7.0) for j in range(8))


CONFIGS = {
    # Plain FP64 single-q static chi0 on a 16^3 box.
    "C1": SystemConfig("C1", 1, (7.5, 7.75, 9.5), (16, 16, 16), 12.324, 3.367,
                       8, 32, (0.1, 0.0, 0.0)),
    # Si-like size (800 empty states, Table tab:parameters), static + 8 iw.
    "C2": SystemConfig("C2", 2, (10.0, 10.4, 10.8), (48, 48, 48), 22.419, 13.980,
                       16, 800, (0.1, 0.0, 0.0), _c2_omegas()),
    # Layered (Bi2Se3-like) size for the mixed-precision path.
    "C3": SystemConfig("C3", 3, (15.0, 15.4, 40.0), (60, 60, 160), 14.922, 8.742,
                       56, 2000, (0.1, 0.0, 0.0)),
    # Small cases used by the tests (not benchmark workloads).
    "T1": SystemConfig("T1", 11, (7.5, 7.75, 9.5), (16, 16, 16), 12.324, 3.367,
                       4, 12, (0.1, 0.0, 0.0), (0.0, 1.0, 10.0)),
    "T1Q0": SystemConfig("T1Q0", 12, (7.5, 7.75, 9.5), (16, 16, 16), 12.324, 3.367,
                         6, 20, (1e-3, 0.0, 0.0), (0.0, 2.0), q0_head=True),
    "T2": SystemConfig("T2", 13, (10.0, 10.4, 10.8), (20, 24, 30), 9.0, 4.5,
                       6, 40, (0.25, -0.25, 0.5), (0.0, 3.0)),
    # Box lengths outside the compile-time FFT lengths and plane shapes: the
    # runtime-length transform kernels.
    "T3": SystemConfig("T3", 14, (10.0, 10.4, 10.8), (18, 20, 25), 8.0, 3.5,
                       5, 30, (0.25, 0.0, -0.25), (0.0, 2.0)),
    # An elongated box whose transforms run x and y on xy-planes and z last
    # (the layout of the layered-cell workload, at a size the oracle handles).
    "T4": SystemConfig("T4", 15, (7.5, 7.75, 18.0), (16, 16, 40), 9.0, 3.0,
                       5, 21, (0.1, 0.0, 0.05), (0.0, 1.5)),
}


def config_by_name(name: str) -> SystemConfig:
    return CONFIGS[name]


def config_digest(cfg: SystemConfig) -> str:
    """First 12 hex digits of the SHA-256 of the workload's parameters (sorted
    JSON): the key of a stored reference computed for that workload."""
    text = json.dumps(dataclasses.asdict(cfg), sort_keys=True)
    return hashlib.sha256(text.encode()).hexdigest()[:12]


def _cart(cell, kred, g):
    a = np.asarray(cell, dtype=np.float64)
    return (np.asarray(g, dtype=np.float64) + np.asarray(kred, dtype=np.float64)) * (2.0 * np.pi / a)


def _g_candidates(cell, ecut, kred):
    a = np.asarray(cell, dtype=np.float64)
    lim = np.floor(np.sqrt(ecut) * a / (2.0 * np.pi) + np.abs(np.asarray(kred)) + 2).astype(int)
    axes = [np.arange(-l, l + 1) for l in lim]
    g = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, 3)
    e = (_cart(cell, kred, g) ** 2).sum(axis=1)
    return g, e


def g_sphere(cell, kred, ecut):
    """Integer G with |k+G|^2 < ecut, sorted by |k+G|^2 then lexicographically."""
    g, e = _g_candidates(cell, ecut, kred)
    keep = e < ecut
    g, e = g[keep], e[keep]
    order = np.lexsort((g[:, 2], g[:, 1], g[:, 0], e))
    return np.ascontiguousarray(g[order].astype(np.int32))


def cutoff_for_count(cell, kred, target):
    """A cutoff halfway between two distinct shells whose sphere holds about `target` G."""
    ecut = 1.0
    while True:
        g, e = _g_candidates(cell, ecut, kred)
        if (e < ecut).sum() > target + 64:
            break
        ecut *= 1.5
    e = np.sort(e[e < ecut])
    n = int(target)
    # walk to the nearest count that ends on a shell boundary
    best = None
    for m in range(max(1, n - 64), min(len(e) - 1, n + 64) + 1):
        if e[m] - e[m - 1] > 1e-9 * max(1.0, e[m]):
            if best is None or abs(m - n) < abs(best - n):
                best = m
    return 0.5 * (e[best - 1] + e[best])


def _random_spinors(rng, ng, nb, nspinor):
    shape = (nspinor * ng, nb)
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    qm, _ = np.linalg.qr(x)
    return np.ascontiguousarray(qm.T.reshape(nb, nspinor, ng))


def _energies(rng, nv, nc):
    ev = np.sort(rng.uniform(-6.0, 0.0, nv)) / EV_PER_HA
    ec = np.sort(rng.uniform(1.0, 20.0, nc)) / EV_PER_HA
    return ev, ec


def vcoul(cell, q, geps):
    """Bare Coulomb potential v(q+G) = 4 pi / (Omega |q+G|^2) in Hartree."""
    omega_cell = float(np.prod(np.asarray(cell, dtype=np.float64)))
    qg2 = (_cart(cell, q, geps) ** 2).sum(axis=1)
    return 4.0 * np.pi / (omega_cell * qg2)


def charge_density(seed, cell, box, nelec, decay=2.5):
    """Fourier components rho(G) of a synthetic valence density on the FFT box,
    stored at g mod n: rho(0) = nelec / Omega (electrons per bohr^3), rho(-G) =
    conj(rho(G)) (a real density), and |rho(G)| ~ 0.4 rho(0) exp(-|G|^2 / (2 decay^2))
    with random phases.  Stands in for the DFT density the plasmon-pole model reads."""
    rng = np.random.default_rng(seed)
    n = np.asarray(box, dtype=np.int64)
    axes = [np.fft.fftfreq(int(m), 1.0 / int(m)).astype(np.int64) for m in n]
    g = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1)
    gc = 2.0 * np.pi * g / np.asarray(cell, dtype=np.float64)
    rho0 = nelec / float(np.prod(cell))
    amp = 0.4 * rho0 * np.exp(-(gc ** 2).sum(-1) / (2.0 * decay ** 2))
    z = (rng.standard_normal(amp.shape) + 1j * rng.standard_normal(amp.shape)) / np.sqrt(2.0)
    r = amp * z
    # Hermitise: rho(-G) = conj(rho(G)); -g mod n is the reversed index on every axis
    neg = r[tuple(np.ix_(*[(-np.arange(int(m))) % int(m) for m in n]))]
    r = 0.5 * (r + np.conj(neg))
    r[0, 0, 0] = rho0
    return np.ascontiguousarray(r.astype(np.complex128))


def _map_coeffs(c_src, g_src, g_dst):
    """Re-express coefficients given on g_src on the sphere g_dst (zero where absent)."""
    lut = {tuple(g): i for i, g in enumerate(g_src.tolist())}
    idx = np.array([lut.get(tuple(g), -1) for g in g_dst.tolist()])
    out = np.zeros(c_src.shape[:-1] + (len(g_dst),), dtype=c_src.dtype)
    ok = idx >= 0
    out[..., ok] = c_src[..., idx[ok]]
    return out


def build_system(cfg: SystemConfig, nc_override=None, ecut_eps_override=None,
                 gc=None, cc=None):
    """Draw one system. Returns a dict of numpy arrays (complex128 / int32 / float64)."""
    rng = np.random.default_rng(cfg.seed)
    nc = cfg.nc if nc_override is None else nc_override
    ecut_eps = cfg.ecut_eps if ecut_eps_override is None else ecut_eps_override
    k0 = (0.0, 0.0, 0.0)
    gk = g_sphere(cfg.cell, k0, cfg.ecut_wfn) if gc is None else gc
    gkq = g_sphere(cfg.cell, cfg.q, cfg.ecut_wfn)
    geps = g_sphere(cfg.cell, cfg.q, ecut_eps)
    ns = cfg.nspinor
    if cfg.q0_head:
        joint = _random_spinors(rng, len(gk), cfg.nv + nc, ns)
        cv_k = joint[:cfg.nv]
        cc_k = joint[cfg.nv:]
        shape = (ns * len(gkq), cfg.nv)
        r = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
        qnorm = float(np.linalg.norm(_cart(cfg.cell, cfg.q, np.zeros((1, 3)))))
        base = _map_coeffs(cv_k, gk, gkq).reshape(cfg.nv, ns * len(gkq)).T
        qm, _ = np.linalg.qr(base + qnorm * r)
        cv = np.ascontiguousarray(qm.T.reshape(cfg.nv, ns, len(gkq)))
    else:
        cc_k = _random_spinors(rng, len(gk), nc, ns) if cc is None else None
        cv = _random_spinors(rng, len(gkq), cfg.nv, ns)
    if cc is not None:
        cc_k = cc
    ev, ec = _energies(rng, cfg.nv, nc)
    omega = np.asarray(cfg.omega_ev, dtype=np.float64) / EV_PER_HA
    head = -1
    if cfg.q0_head:
        zero = np.where((geps == 0).all(axis=1))[0]
        head = int(zero[0]) if len(zero) else -1
    return dict(
        name=cfg.name, box=np.asarray(cfg.box, dtype=np.int32),
        cell=np.asarray(cfg.cell, dtype=np.float64), q=np.asarray(cfg.q, dtype=np.float64),
        nspinor=ns, gv=gkq, gc=gk, geps=geps,
        cv=cv, cc=np.ascontiguousarray(cc_k), ev=ev, ec=ec, omega=omega,
        vcoul=vcoul(cfg.cell, cfg.q, geps), qg=_cart(cfg.cell, cfg.q, geps),
        head_index=head,
    )


# --------------------------------------------------------------------------
# Many-q batch: a Gamma-centred 4x4x4 q-grid, Gamma replaced by a small q0.
# Conduction bands at k=0 are shared by every q; valence bands live at k+q.
# --------------------------------------------------------------------------
BATCH_DEFAULT = dict(seed=4000, cell=(10.0, 10.4, 10.8), box=(48, 48, 48), ecut_wfn=22.419,
                     nv=16, nc_range=(400, 1600), neps_range=(600, 2400), grid=4, q0=1e-3)


def batch_systems(nq=64, seed=4000, cell=(10.0, 10.4, 10.8), box=(48, 48, 48),
                  ecut_wfn=22.419, nv=16, nc_range=(400, 1600), neps_range=(600, 2400),
                  grid=4, q0=1e-3, omega_ev=(0.0,)):
    """Per-q systems for the batched launch; conduction at k=0 is drawn once."""
    rng = np.random.default_rng(seed)
    qs = []
    for i in range(grid):
        for j in range(grid):
            for l in range(grid):
                qs.append((i / grid, j / grid, l / grid))
    qs = qs[:nq]
    nc_q = rng.integers(nc_range[0], nc_range[1] + 1, size=len(qs))
    neps_q = rng.integers(neps_range[0], neps_range[1] + 1, size=len(qs))
    ncmax = int(nc_q.max())
    gk = g_sphere(cell, (0.0, 0.0, 0.0), ecut_wfn)
    # shared conduction (and the valence at k used for the q0 construction)
    joint = _random_spinors(rng, len(gk), nv + ncmax, 2)
    cv_k, cc_k = joint[:nv], np.ascontiguousarray(joint[nv:])
    ec_all = np.sort(rng.uniform(1.0, 20.0, ncmax)) / EV_PER_HA
    ev_k = np.sort(rng.uniform(-6.0, 0.0, nv)) / EV_PER_HA
    out = []
    for iq, qred in enumerate(qs):
        is_gamma = all(abs(x) < 1e-12 for x in qred)
        qv = (q0, 0.0, 0.0) if is_gamma else qred
        sub = np.random.default_rng(seed + 1 + iq)
        gkq = g_sphere(cell, qv, ecut_wfn)
        if is_gamma:
            shape = (2 * len(gkq), nv)
            r = sub.standard_normal(shape) + 1j * sub.standard_normal(shape)
            qnorm = float(np.linalg.norm(_cart(cell, qv, np.zeros((1, 3)))))
            base = _map_coeffs(cv_k, gk, gkq).reshape(nv, 2 * len(gkq)).T
            qm, _ = np.linalg.qr(base + qnorm * r)
            cv = np.ascontiguousarray(qm.T.reshape(nv, 2, len(gkq)))
            ev = ev_k.copy()
        else:
            cv = _random_spinors(sub, len(gkq), nv, 2)
            ev = np.sort(sub.uniform(-6.0, 0.0, nv)) / EV_PER_HA
        ecut_eps = cutoff_for_count(cell, qv, int(neps_q[iq]))
        geps = g_sphere(cell, qv, ecut_eps)
        head = -1
        if is_gamma:
            head = int(np.where((geps == 0).all(axis=1))[0][0])
        nc = int(nc_q[iq])
        out.append(dict(
            name=f"B{iq}", box=np.asarray(box, dtype=np.int32), cell=np.asarray(cell),
            q=np.asarray(qv, dtype=np.float64), nspinor=2, gv=gkq, gc=gk, geps=geps,
            cv=cv, cc=cc_k, nc=nc, ev=ev, ec=ec_all[:nc],
            omega=np.asarray(omega_ev, dtype=np.float64) / EV_PER_HA,
            vcoul=vcoul(cell, qv, geps), qg=_cart(cell, qv, geps), head_index=head))
    return out


# --------------------------------------------------------------------------
# Closure data: many small systems, each with a truncated and a full band sum.
# --------------------------------------------------------------------------
def closure_systems(indices, seed0=5000, cell=(10.0, 10.4, 10.8), box=(32, 32, 32),
                    ecut_wfn=15.017, nv=16, nc_full=2000, neps_range=(300, 800), jitter=0.05,
                    grid=4):
    """Systems i in `indices` (i < 256 train, 256 <= i < 288 held out)."""
    qs = []
    for i in range(grid):
        for j in range(grid):
            for l in range(grid):
                if (i, j, l) != (0, 0, 0):
                    qs.append((i / grid, j / grid, l / grid))
    out = []
    for i in indices:
        rng = np.random.default_rng(seed0 + i)
        scale = 1.0 + jitter * rng.uniform(-1.0, 1.0, 3)
        cl = tuple(float(x) for x in np.asarray(cell) * scale)
        qv = qs[i % len(qs)]
        target = int(rng.integers(neps_range[0], neps_range[1] + 1))
        ecut_eps = cutoff_for_count(cl, qv, target)
        # a shrunken cell holds fewer plane waves: raise the cutoff until both
        # spheres carry enough spinor components for N_v + N_c orthonormal bands
        ec_i = ecut_wfn
        while min(len(g_sphere(cl, (0.0, 0.0, 0.0), ec_i)), len(g_sphere(cl, qv, ec_i))) * 2 < \
                nv + nc_full + 16:
            ec_i *= 1.05
        cfg = SystemConfig(f"S{i}", seed0 + 100000 + i, cl, box, ec_i, ecut_eps, nv, nc_full, qv)
        out.append(build_system(cfg))
    return out
