"""GPU parity of the spinor unfolding (gw_unfold_spinor) and of the little-group
average of chi0 (gw_chi0_symmetrize) against the oracle, and chi0 over a full k
grid on the GPU, from unfolded states or from the irreducible points alone,
against the oracle's sum over states diagonalised at every k."""
import numpy as np
import pytest

import oracle
from synth.generate import _random_spinors, g_sphere
from test_symmetry_pins import CELL, ECUT, Model, _kprime

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    import paper_2206_00808_amd as P
    return P


@pytest.fixture(scope="module")
def ctx(P):
    return P.Context(0)


@pytest.fixture(scope="module")
def model():
    return Model()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _same_up_to_branch(x, ref):
    """The two quaternion branches give U and -U; both are valid.  Returns the
    relative error after taking the branch that fits, and that branch."""
    s = 1.0 if np.vdot(ref.ravel(), x.ravel()).real >= 0 else -1.0
    return float(np.abs(s * x - ref).max() / np.abs(ref).max()), s


@pytest.mark.parametrize("dtype", [np.complex128, np.complex64])
@pytest.mark.parametrize("nspinor", [2, 1])
def test_unfold_matches_oracle_for_every_operation(P, ctx, model, dtype, nspinor):
    rng = np.random.default_rng(7 + nspinor)
    k = np.array([0.13, 0.27, 0.19])
    gin = g_sphere(CELL, k, 30.0)
    nb = 21
    c = _random_spinors(rng, len(gin), nb, nspinor).astype(dtype)
    dc = _dev(c)
    for s, tau in model.ops:
        k1 = _kprime(s, k)
        for g0 in ((0, 0, 0), (1, -2, 1)):
            gout = g_sphere(CELL, k1 - np.asarray(g0), 30.0)[::-1].copy()  # any order
            out = torch.empty((nb, nspinor, len(gout)), dtype=dc.dtype, device="cuda:0")
            P.gw_unfold_spinor(ctx, nspinor, gin, dc, gout, s, tau, CELL, out, g0=g0)
            torch.cuda.synchronize()
            want = oracle.unfold_spinor(c.astype(np.complex128), gin, gout, s, tau, CELL, g0=g0)
            err, br = _same_up_to_branch(out.cpu().numpy().astype(np.complex128), want)
            assert br == 1.0
            assert err < (1e-15 if dtype == np.complex128 else 1e-7)


def test_unfold_rejects_bad_arguments(P, ctx, model):
    rng = np.random.default_rng(1)
    gin = g_sphere(CELL, (0, 0, 0), 20.0)
    c = _dev(_random_spinors(rng, len(gin), 3, 2))
    out = torch.empty_like(c)
    s, tau = model.ops[1]
    with pytest.raises(P.GwError):  # an output vector outside the rotated sphere
        P.gw_unfold_spinor(ctx, 2, gin, c, gin + np.array([5, 0, 0]), s, tau, CELL, out)
    with pytest.raises(P.GwError):  # a shear is no rotation of this lattice
        P.gw_unfold_spinor(ctx, 2, gin, c, gin, [[1, 1, 0], [0, 1, 0], [0, 0, 1]], tau, CELL,
                           out)
    with pytest.raises(P.GwError):  # C4 about z in a cell with a1 != a2
        P.gw_unfold_spinor(ctx, 2, gin, c, gin, [[0, -1, 0], [1, 0, 0], [0, 0, 1]], tau,
                           (5.0, 5.5, 6.2), out)
    with pytest.raises(P.GwError):
        P.gw_unfold_spinor(ctx, 2, np.concatenate([gin, gin[:1]]), c, gin, s, tau, CELL, out)
    with pytest.raises(P.GwError):
        P.gw_unfold_spinor(ctx, 2, gin, c, gin, s, tau, CELL, c)


def test_chi0_over_the_full_grid_from_gpu_unfolded_states(P, ctx, model):
    """Per irreducible point of the little group of q: states diagonalised on the
    CPU (the inputs), unfolded to every k of its orbit on the GPU, matrix elements
    and chi0 accumulated there; against the oracle's chi0 summed over states
    diagonalised at every k of the 3x3x3 grid."""
    nv, nc = 4, 4
    q = np.array([0.0, 0.0, 1.0 / 3.0])
    geps = g_sphere(CELL, q, 3.0)
    omega = [0.0, 0.4]
    grid = [np.array([i / 3, j / 3, l / 3]) for i in range(3) for j in range(3) for l in range(3)]
    little = [op for op in model.ops
              if np.allclose(np.mod(_kprime(op[0], q) - q + 1e-12, 1.0), 0.0, atol=1e-9)]
    direct = 0
    for k in grid:
        e1, c1, g1 = model.states(k, nv + nc)
        e2, c2, g2 = model.states(k + q, nv)
        m = oracle.mtxel_convolution(c2[:nv], g2, c1[nv:], g1, geps)
        direct = direct + oracle.chi0(m, e2[:nv], e1[nv:nv + nc], np.asarray(omega))

    box = (16, 16, 16)
    chi = torch.zeros((len(omega), len(geps), len(geps)), dtype=torch.complex128, device="cuda:0")
    covered = set()
    for k in grid:
        if tuple(np.round(np.mod(k, 1.0), 9)) in covered:
            continue
        ec_, cc_, gc_ = model.states(k, nv + nc)
        ev_, cv_, gv_ = model.states(k + q, nv)
        dcc, dcv = _dev(cc_[nv:]), _dev(cv_)
        dev_, dec_ = _dev(ev_[:nv]), _dev(ec_[nv:nv + nc])
        for s, tau in little:
            sk = _kprime(s, k)
            kf = np.mod(sk + 1e-12, 1.0)
            kf = np.where(kf > 1 - 1e-9, 0.0, kf)
            if tuple(np.round(kf, 9)) in covered:
                continue
            covered.add(tuple(np.round(kf, 9)))
            g0 = np.rint(sk - kf).astype(int)
            gq = np.rint(_kprime(s, q) - q).astype(int)
            gc1 = g_sphere(CELL, kf, ECUT)
            gv1 = g_sphere(CELL, kf + q, ECUT)
            uc = torch.empty((nc, 2, len(gc1)), dtype=torch.complex128, device="cuda:0")
            uv = torch.empty((nv, 2, len(gv1)), dtype=torch.complex128, device="cuda:0")
            P.gw_unfold_spinor(ctx, 2, gc_, dcc, gc1, s, tau, CELL, uc, g0=g0)
            P.gw_unfold_spinor(ctx, 2, gv_, dcv, gv1, s, tau, CELL, uv, g0=g0 + gq)
            m = torch.empty((nv, nc, len(geps)), dtype=torch.complex128, device="cuda:0")
            P.gw_mtxel_spinor(ctx, box, 2, gv1, uv, gc1, uc, geps, m)
            P.gw_chi0_accumulate(ctx, nv, nc, len(geps), m, dev_, dec_, omega, 1.0,
                                 P.GW_PREC_FP64, chi)
    torch.cuda.synchronize()
    assert len(covered) == len(grid)
    assert oracle.rel_f(chi.cpu().numpy(), direct) < 1e-10


def _little(model, q):
    return [op for op in model.ops if oracle.little_group_shift(op[0], q) is not None]


def test_chi0_symmetrize_matches_oracle(P, ctx, model):
    rng = np.random.default_rng(4)
    q = np.array([0.0, 0.0, 1.0 / 3.0])
    geps = g_sphere(CELL, q, 8.0)
    n = len(geps)
    x = rng.standard_normal((3, n, n)) + 1j * rng.standard_normal((3, n, n))
    little = _little(model, q)
    out = torch.empty((3, n, n), dtype=torch.complex128, device="cuda:0")
    P.gw_chi0_symmetrize(ctx, geps, q, little, _dev(x), out)
    torch.cuda.synchronize()
    want = oracle.chi0_symmetrize(x, geps, little, q)
    assert np.abs(out.cpu().numpy() - want).max() < 1e-14 * np.abs(want).max()


def test_empty_calls_are_no_ops(P, ctx, model):
    gin = g_sphere(CELL, (0, 0, 0), 20.0)
    c = torch.zeros((0, 2, len(gin)), dtype=torch.complex128, device="cuda:0")
    out = torch.zeros((0, 2, len(gin)), dtype=torch.complex128, device="cuda:0")
    s, tau = model.ops[1]
    P.gw_unfold_spinor(ctx, 2, gin, c, gin, s, tau, CELL, out)  # no bands
    q = np.array([0.0, 0.0, 1.0 / 3.0])
    geps = g_sphere(CELL, q, 3.0)
    x = torch.zeros((0, len(geps), len(geps)), dtype=torch.complex128, device="cuda:0")
    P.gw_chi0_symmetrize(ctx, geps, q, _little(model, q), x, torch.empty_like(x))  # no frequencies
    torch.cuda.synchronize()


def test_chi0_symmetrize_rejects_bad_arguments(P, ctx, model):
    q = np.array([0.0, 0.0, 1.0 / 3.0])
    geps = g_sphere(CELL, q, 3.0)
    n = len(geps)
    x = _dev(np.zeros((1, n, n), np.complex128))
    y = torch.empty_like(x)
    outside = [op for op in model.ops if oracle.little_group_shift(op[0], q) is None]
    with pytest.raises(P.GwError):
        P.gw_chi0_symmetrize(ctx, geps, q, outside[:1], x, y)
    with pytest.raises(P.GwError):
        P.gw_chi0_symmetrize(ctx, geps, q, _little(model, q), x, x)
    with pytest.raises(P.GwError):  # a sphere that is not closed under C4
        P.gw_chi0_symmetrize(ctx, geps[:-3], q, _little(model, q), _dev(np.zeros((1, n - 3, n - 3),
                             np.complex128)), torch.empty((1, n - 3, n - 3), dtype=torch.complex128,
                                                          device="cuda:0"))


def test_chi0_from_irreducible_points_on_the_gpu(P, ctx, model):
    """Only the irreducible points of q's little group, found by the library's host
    bookkeeping: states diagonalised there (CPU inputs), matrix elements and chi0
    on the GPU weighted by orbit size, then gw_chi0_symmetrize; against the
    oracle's chi0 over states at every k of the grid."""
    nv, nc = 4, 4
    q = np.array([0.0, 0.0, 1.0 / 3.0])
    geps = g_sphere(CELL, q, 3.0)
    omega = [0.0, 0.4]
    grid = [np.array([i / 3, j / 3, l / 3]) for i in range(3) for j in range(3) for l in range(3)]
    direct = 0
    for k in grid:
        e1, c1, g1 = model.states(k, nv + nc)
        e2, c2, g2 = model.states(k + q, nv)
        m = oracle.mtxel_convolution(c2[:nv], g2, c1[nv:], g1, geps)
        direct = direct + oracle.chi0(m, e2[:nv], e1[nv:nv + nc], np.asarray(omega))

    chi = torch.zeros((2, len(geps), len(geps)), dtype=torch.complex128, device="cuda:0")
    # the library's own bookkeeping: the little group of q and the grid's orbits
    ing, _ = P.gw_little_group(model.ops, q)
    little = [op for op, keep in zip(model.ops, ing) if keep]
    rep, _, _, weight, nirr = P.gw_kgrid_orbits((3, 3, 3), little)
    for i in np.nonzero(weight)[0]:
        k = np.array([i // 9, (i // 3) % 3, i % 3]) / 3.0
        ec_, cc_, gc_ = model.states(k, nv + nc)
        ev_, cv_, gv_ = model.states(k + q, nv)
        m = torch.empty((nv, nc, len(geps)), dtype=torch.complex128, device="cuda:0")
        P.gw_mtxel_spinor(ctx, (16, 16, 16), 2, gv_, _dev(cv_), gc_, _dev(cc_[nv:]), geps, m)
        P.gw_chi0_accumulate(ctx, nv, nc, len(geps), m, _dev(ev_[:nv]), _dev(ec_[nv:nv + nc]),
                             omega, float(weight[i]), P.GW_PREC_FP64, chi)
    seen = set(rep.tolist())
    out = torch.empty_like(chi)
    P.gw_chi0_symmetrize(ctx, geps, q, little, chi, out)
    torch.cuda.synchronize()
    assert len(seen) == nirr < len(grid) and weight.sum() == len(grid)
    assert oracle.rel_f(out.cpu().numpy(), direct) < 1e-10
