"""Pins of the symmetry-unfolding oracle against what the mathematics fixes.

The physics pin is a plane-wave Hamiltonian with a local potential and
spin-orbit coupling, H = T + V(r) + lambda sigma . (grad W x p), whose V and W
are symmetrised over a space group with a 4_2 screw axis, inversion and a
two-fold axis: an unfolded eigenvector must be an eigenvector of H at the
rotated k with the same energy, and chi0 summed over a full k grid from
unfolded states must equal the sum over states diagonalised at every k.
"""
import itertools

import numpy as np
import pytest

import oracle
from oracle.symmetry import PAULI
from synth.generate import g_sphere

CELL = (5.0, 5.0, 6.2)
ECUT = 9.0


# ----------------------------------------------------------------- group and model
def _compose(a, b):
    """{S1|t1}{S2|t2} = {S1 S2 | S1 t2 + t1}, fractional translation mod 1."""
    s = a[0] @ b[0]
    t = np.mod(a[0] @ b[1] + a[1], 1.0)
    return s, np.where(np.isclose(t, 1.0), 0.0, t)


def _key(op):
    return tuple(op[0].ravel().tolist()) + tuple(np.round(op[1], 9).tolist())


def space_group():
    c4 = np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1]])
    c2x = np.array([[1, 0, 0], [0, -1, 0], [0, 0, -1]])
    gens = [(c4, np.array([0.0, 0.0, 0.5])), (-np.eye(3, dtype=int), np.zeros(3)),
            (c2x, np.zeros(3))]
    ops = {_key((np.eye(3, dtype=int), np.zeros(3))): (np.eye(3, dtype=int), np.zeros(3))}
    frontier = list(ops.values())
    while frontier:
        new = []
        for a in frontier:
            for g in gens:
                b = _compose(g, a)
                if _key(b) not in ops:
                    ops[_key(b)] = b
                    new.append(b)
        frontier = new
    return list(ops.values())


def _cart(g, k=(0, 0, 0)):
    return 2 * np.pi * (np.asarray(g, dtype=np.float64) + np.asarray(k)) / np.asarray(CELL)


def symmetrised_field(rng, ops, gcut, scale):
    """Fourier components of a real field invariant under every {S|tau}:
    f(G) = mean over ops of f0(S^-1 G) e^{-i G.tau}."""
    g = g_sphere(CELL, (0, 0, 0), gcut).astype(np.int64)
    f0 = {}
    for gi in g.tolist():
        t = tuple(gi)
        if t in f0:
            continue
        z = complex(rng.standard_normal(), rng.standard_normal()) * scale
        f0[t] = z
        f0[tuple(-x for x in gi)] = np.conj(z)
    f0[(0, 0, 0)] = complex(f0[(0, 0, 0)].real, 0.0)
    f = {}
    for gi in g.tolist():
        acc = 0.0
        for s, tau in ops:
            src = tuple((np.asarray(gi) @ s).tolist())  # S_lat^T g
            acc += f0.get(src, 0.0) * np.exp(-2j * np.pi * np.dot(gi, tau))
        f[tuple(gi)] = acc / len(ops)
    return f


class Model:
    def __init__(self, seed=5, lam=0.08):
        rng = np.random.default_rng(seed)
        self.ops = space_group()
        self.v = symmetrised_field(rng, self.ops, 7.0, 0.35)
        self.w = symmetrised_field(rng, self.ops, 7.0, 0.25)
        self.lam = lam

    def hamiltonian(self, k, g):
        g = np.asarray(g, dtype=np.int64)
        ng = len(g)
        kg = _cart(g, k)
        h = np.zeros((2, ng, 2, ng), dtype=np.complex128)
        dg = g[:, None, :] - g[None, :, :]
        vv = np.array([[self.v.get(tuple(d), 0.0) for d in row] for row in dg.tolist()])
        ww = np.array([[self.w.get(tuple(d), 0.0) for d in row] for row in dg.tolist()])
        cr = np.cross(kg[:, None, :], kg[None, :, :])
        for s in range(2):
            h[s, :, s, :] += vv
            h[s, np.arange(ng), s, np.arange(ng)] += 0.5 * (kg ** 2).sum(1)
        for j in range(3):
            blk = 1j * self.lam * ww * cr[:, :, j]
            for s, t in itertools.product(range(2), range(2)):
                h[s, :, t, :] += blk * PAULI[j][s, t]
        h = h.reshape(2 * ng, 2 * ng)
        assert np.abs(h - h.conj().T).max() < 1e-12
        return h

    def states(self, k, nb):
        g = g_sphere(CELL, k, ECUT)
        e, v = np.linalg.eigh(self.hamiltonian(k, g))
        c = np.ascontiguousarray(v[:, :nb].T.reshape(nb, 2, len(g)))
        return e, c, g


def _kprime(s_lat, k):
    return np.linalg.inv(np.asarray(s_lat, dtype=np.float64)).T @ np.asarray(k)


@pytest.fixture(scope="module")
def model():
    return Model()


# ----------------------------------------------------------------- rotations
def _rand_rot(rng):
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    x, y, z, w = q
    return np.array([
        [w * w + x * x - y * y - z * z, 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), w * w - x * x + y * y - z * z, 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), w * w - x * x - y * y + z * z]])


def _axis_angle(n, th):
    n = np.asarray(n, dtype=np.float64) / np.linalg.norm(n)
    k = np.array([[0, -n[2], n[1]], [n[2], 0, -n[0]], [-n[1], n[0], 0]])
    return np.eye(3) + np.sin(th) * k + (1 - np.cos(th)) * k @ k


def test_group_closes_and_ops_are_orthogonal(model):
    assert len(model.ops) == 16
    for s, _ in model.ops:
        r = oracle.rotation_lat_to_cart(s, CELL)
        assert np.abs(r.T @ r - np.eye(3)).max() < 1e-14
        # the reciprocal-basis form (B^T)^-1 S_lat B^T with B = 2 pi A^-T
        b = 2 * np.pi * np.linalg.inv(np.diag(CELL)).T
        assert np.abs(np.linalg.inv(b.T) @ s @ b.T - r).max() < 1e-13


@pytest.mark.parametrize("angle", [0.0, 1e-9, 0.7, np.pi / 2, np.pi - 1e-9, np.pi])
def test_quaternion_recovers_axis_and_angle(angle):
    rng = np.random.default_rng(3)
    for _ in range(8):
        n = rng.standard_normal(3)
        r = _axis_angle(n, angle)
        q = oracle.quaternion_from_rotation(r)
        assert abs(np.linalg.norm(q) - 1) < 1e-14
        # R rebuilt from q (the Rodrigues form with sin, 1 - cos written in q)
        th = 2 * np.arctan2(np.linalg.norm(q[:3]), q[3])
        nn = q[:3] / max(np.linalg.norm(q[:3]), 1e-300)
        assert np.abs(_axis_angle(nn, th) - r).max() < 1e-12 if angle > 0 else True
        want = np.concatenate([n / np.linalg.norm(n) * np.sin(angle / 2), [np.cos(angle / 2)]])
        assert min(np.abs(q - want).max(), np.abs(q + want).max()) < 1e-8


def test_su2_is_unitary_and_turns_the_spin_vector():
    rng = np.random.default_rng(11)
    mats = [_rand_rot(rng) for _ in range(20)] + [_axis_angle((1, 1, 0), np.pi),
                                                   _axis_angle((0, 0, 1), np.pi), np.eye(3)]
    for r in mats:
        u = oracle.su2_from_rotation(r)
        assert np.abs(u.conj().T @ u - np.eye(2)).max() < 1e-14
        assert abs(np.linalg.det(u) - 1) < 1e-14
        for i in range(3):
            rot = sum(r[i, j] * PAULI[j] for j in range(3))
            assert np.abs(u.conj().T @ PAULI[i] @ u - rot).max() < 1e-14
        # an improper operation takes the rotation part
        assert np.abs(oracle.su2_from_rotation(-r) - u).max() == 0.0


def test_printed_spin_matrix_is_not_su2():
    """The reading: the matrix with (-n_y + i n_x) sin(theta/2) in its lower-left
    corner has determinant cos^2 + (n_z^2 - n_x^2 - n_y^2) sin^2, not 1."""
    n, th = np.array([0.6, 0.8, 0.0]), 1.1
    c, s = np.cos(th / 2), np.sin(th / 2)
    printed = np.array([[c - 1j * n[2] * s, (-n[1] - 1j * n[0]) * s],
                        [(-n[1] + 1j * n[0]) * s, c + 1j * n[2] * s]])
    assert abs(np.linalg.det(printed) - 1) > 0.5


# ----------------------------------------------------------------- unfolding
K0 = (0.13, 0.27, 0.19)


@pytest.mark.parametrize("iop", range(16))
def test_unfolded_state_is_an_eigenstate_at_sk(model, iop):
    s, tau = model.ops[iop]
    e, c, g = model.states(K0, 6)
    k1 = _kprime(s, K0)
    for g0 in ((0, 0, 0), tuple(np.rint(k1).astype(int) + np.array([1, 0, -1]))):
        kk = k1 - np.asarray(g0)
        gout = g_sphere(CELL, kk, ECUT)
        assert len(gout) == len(g)
        c1 = oracle.unfold_spinor(c, g, gout, s, tau, CELL, g0=g0)
        h = model.hamiltonian(kk, gout)
        for b in range(6):
            x = c1[b].reshape(-1)
            assert abs(np.linalg.norm(x) - 1) < 1e-13
            assert np.linalg.norm(h @ x - e[b] * x) < 1e-10


def test_unfolding_pin_catches_planted_mistakes(model, monkeypatch):
    """Mistakes planted in the oracle on the CPU break the eigenstate pin: the
    conjugate transpose of U, a dropped fractional-translation phase, S in place
    of S^-1 (the operation applied the wrong way round)."""
    import oracle.symmetry as sym
    e, c, g = model.states(K0, 2)

    def resid(s, tau, s_unfold=None):
        k1 = _kprime(s, K0)
        gout = g_sphere(CELL, k1, ECUT)
        try:
            c1 = sym.unfold_spinor(c, g, gout, s if s_unfold is None else s_unfold, tau, CELL)
        except ValueError:
            return np.inf
        x = c1[0].reshape(-1)
        return np.linalg.norm(model.hamiltonian(k1, gout) @ x - e[0] * x)

    screw = [op for op in model.ops
             if np.array_equal(op[0], [[0, -1, 0], [1, 0, 0], [0, 0, 1]])][0]
    assert resid(*screw) < 1e-10
    assert resid(screw[0], np.zeros(3)) > 1e-3
    real = sym.su2_from_rotation
    monkeypatch.setattr(sym, "su2_from_rotation", lambda r: real(r).conj().T)
    assert resid(*screw) > 1e-3
    monkeypatch.setattr(sym, "su2_from_rotation", real)
    assert resid(screw[0], screw[1], s_unfold=screw[0].T) > 1e-3


def test_chi0_over_the_full_grid_from_unfolded_states(model):
    """chi0(q) summed over a 3x3x3 grid: states unfolded from the irreducible
    points of the little group of q against states diagonalised at every k."""
    nv, nc = 4, 4
    q = np.array([0.0, 0.0, 1.0 / 3.0])
    geps = g_sphere(CELL, q, 3.0)
    omega = np.array([0.0, 0.4])
    grid = [np.array([i / 3, j / 3, l / 3]) for i in range(3) for j in range(3) for l in range(3)]
    little = [op for op in model.ops
              if np.allclose(np.mod(_kprime(op[0], q) - q + 1e-12, 1.0), 0.0, atol=1e-9)]
    assert 1 < len(little) < len(model.ops)

    def chi_at(ev, cv, gv, ec, cc, gc):
        m = oracle.mtxel_convolution(cv, gv, cc, gc, geps)
        return oracle.chi0(m, ev, ec, omega)

    direct = 0
    for k in grid:
        e1, c1, g1 = model.states(k, nv + nc)
        e2, c2, g2 = model.states(k + q, nv)
        for e in (e1, e2):
            assert e[nv] - e[nv - 1] > 1e-6 and e[nv + nc] - e[nv + nc - 1] > 1e-6
        direct = direct + chi_at(e2[:nv], c2[:nv], g2, e1[nv:nv + nc], c1[nv:], g1)

    unfolded = 0
    covered = set()
    for k in grid:
        key = tuple(np.round(np.mod(k, 1.0), 9))
        if key in covered:
            continue
        ec_, cc_, gc_ = model.states(k, nv + nc)
        ev_, cv_, gv_ = model.states(k + q, nv)
        for s, tau in little:
            sk = _kprime(s, k)
            kf = np.mod(sk + 1e-12, 1.0)
            kf = np.where(kf > 1 - 1e-9, 0.0, kf)
            kkey = tuple(np.round(kf, 9))
            if kkey in covered:
                continue
            covered.add(kkey)
            g0 = np.rint(sk - kf).astype(int)
            gq = np.rint(_kprime(s, q) - q).astype(int)
            gc1 = g_sphere(CELL, kf, ECUT)
            gv1 = g_sphere(CELL, kf + q, ECUT)
            cc1 = oracle.unfold_spinor(cc_[nv:], gc_, gc1, s, tau, CELL, g0=g0)
            cv1 = oracle.unfold_spinor(cv_, gv_, gv1, s, tau, CELL, g0=g0 + gq)
            unfolded = unfolded + chi_at(ev_[:nv], cv1, gv1, ec_[nv:nv + nc], cc1, gc1)
    assert len(covered) == len(grid)
    assert oracle.rel_f(unfolded, direct) < 1e-10
    # the +- branch of the quaternion flips U for every band: M*M does not see it
    s, tau = little[1]
    e, c, g = model.states(grid[5], nv)
    gout = g_sphere(CELL, _kprime(s, grid[5]), ECUT)
    a = oracle.unfold_spinor(c, g, gout, s, tau, CELL)
    import oracle.symmetry as sym
    real = sym.su2_from_rotation
    try:
        sym.su2_from_rotation = lambda r: -real(r)
        b = oracle.unfold_spinor(c, g, gout, s, tau, CELL)
    finally:
        sym.su2_from_rotation = real
    assert np.abs(a + b).max() < 1e-15


def test_chi0_from_the_irreducible_wedge_symmetrised(model):
    """chi0(q) over the 3x3x3 grid from the irreducible points of the little group
    of q only (states diagonalised there, weighted by orbit size) and averaged over
    the little group equals chi0 from states diagonalised at every k.  Dropping the
    translation phase breaks it, and the result is invariant under each operation."""
    nv, nc = 4, 4
    q = np.array([0.0, 0.0, 1.0 / 3.0])
    geps = g_sphere(CELL, q, 3.0)
    omega = np.array([0.0, 0.4])
    grid = [np.array([i / 3, j / 3, l / 3]) for i in range(3) for j in range(3) for l in range(3)]
    little = [op for op in model.ops if oracle.little_group_shift(op[0], q) is not None]

    def chi_at(k):
        e1, c1, g1 = model.states(k, nv + nc)
        e2, c2, g2 = model.states(k + q, nv)
        m = oracle.mtxel_convolution(c2[:nv], g2, c1[nv:], g1, geps)
        return oracle.chi0(m, e2[:nv], e1[nv:nv + nc], omega)

    def key(k):
        kf = np.mod(k + 1e-12, 1.0)
        return tuple(np.round(np.where(kf > 1 - 1e-9, 0.0, kf), 9))

    direct = sum(chi_at(k) for k in grid)
    seen, irr = set(), 0
    for k in grid:
        if key(k) in seen:
            continue
        orbit = {key(_kprime(s, k)) for s, _ in little}
        seen |= orbit
        irr = irr + len(orbit) * chi_at(k)
    assert len(seen) == len(grid)
    # the same sum over the representatives and weights kgrid_orbits returns
    rep, _, _, w = oracle.kgrid_orbits((3, 3, 3), little)
    irr2 = sum(int(w[i]) * chi_at(np.array([i // 9, (i // 3) % 3, i % 3]) / 3.0)
               for i in np.nonzero(w)[0])
    assert oracle.rel_f(oracle.chi0_symmetrize(irr2, geps, little, q), direct) < 1e-10
    sym = oracle.chi0_symmetrize(irr, geps, little, q)
    assert oracle.rel_f(sym, direct) < 1e-10
    assert oracle.rel_f(oracle.chi0_symmetrize(sym, geps, little[1:2], q), sym) < 1e-13
    no_phase = [(s, np.zeros(3)) for s, _ in little]
    assert oracle.rel_f(oracle.chi0_symmetrize(irr, geps, no_phase, q), direct) > 1e-3


def test_kgrid_orbits_partition_the_grid(model):
    q = np.array([0.0, 0.0, 1.0 / 3.0])
    little = [op for op in model.ops if oracle.little_group_shift(op[0], q) is not None]
    for n, ops in (((3, 3, 3), little), ((4, 4, 2), model.ops), ((4, 4, 3), little[:4])):
        rep, op, g0, w = oracle.kgrid_orbits(n, ops)
        npts = int(np.prod(n))
        assert w.sum() == npts and np.all(w[rep[w > 0]] > 0)
        idx = np.stack(np.meshgrid(*[np.arange(m) for m in n], indexing="ij"), -1).reshape(-1, 3)
        k = idx / np.asarray(n)
        for i in range(npts):
            s = ops[op[i]][0]
            assert np.allclose(_kprime(s, k[rep[i]]), k[i] + g0[i], atol=1e-12)
            assert w[rep[i]] == np.sum(rep == rep[i])
    # the 16-element group folds the 4x4x2 grid; the trivial group leaves it
    assert (oracle.kgrid_orbits((4, 4, 2), model.ops)[3] > 0).sum() < 32
    assert (oracle.kgrid_orbits((2, 2, 2), model.ops[:1])[3] > 0).sum() == 8
