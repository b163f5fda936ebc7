"""Pins of the BSE kernel oracle: real-space double sums, the spin trace for
collinear spinors, Hermiticity."""
import numpy as np

import oracle
from synth.generate import _random_spinors, g_sphere

CELL = (5.0, 5.3, 5.7)
BOX = (12, 12, 12)


def _sets(seed=1, nv=3, nc=4, ns=2):
    rng = np.random.default_rng(seed)
    g = g_sphere(CELL, (0, 0, 0), 5.0)
    geps = g_sphere(CELL, (0, 0, 0), 2.5)
    c = _random_spinors(rng, len(g), nv + nc, ns)
    return rng, g, geps, c[:nv], c[nv:]


def _mt(a, ga, b, gb, geps):
    return oracle.mtxel_convolution(a, ga, b, gb, geps)


def _density(a, b, g):
    """rho_ab(r_j) = sum_sigma conj(u_a^sigma(r_j)) u_b^sigma(r_j) on the grid."""
    ua = oracle.wavefunction_on_box(a, g, BOX)
    ub = oracle.wavefunction_on_box(b, g, BOX)
    return np.einsum("asr,bsr->abr", np.conj(ua.reshape(ua.shape[0], ua.shape[1], -1)),
                     ub.reshape(ub.shape[0], ub.shape[1], -1))


def test_kernels_equal_real_space_double_sums():
    rng, g, geps, cv, cc = _sets()
    assert oracle.alias_free(g, g, geps, BOX)
    nv, nc, n = len(cv), len(cc), len(geps)
    vx = rng.uniform(0.1, 3.0, n)
    a = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    w = a @ a.conj().T / n + np.diag(vx)
    kx, kd = oracle.bse_kernel(_mt(cv, g, cc, g, geps), _mt(cc, g, cc, g, geps),
                               _mt(cv, g, cv, g, geps), vx, w)
    # grid positions and the kernels' Fourier series
    idx = np.stack(np.meshgrid(*[np.arange(m) for m in BOX], indexing="ij"), -1).reshape(-1, 3)
    ph = np.exp(2j * np.pi * (idx / np.asarray(BOX)) @ geps.T)  # e^{+iG.r_j}   [Nr][N]
    nr = len(idx)
    vr = ph.conj() @ (vx[:, None] * ph.T)          # V(r1, r2) = sum_G v e^{-iG r1} e^{+iG r2}
    wr = ph.conj() @ w @ ph.T                      # W(r1, r2) = sum e^{-iG r1} W_GG' e^{+iG' r2}
    rvc = _density(cv, cc, g).reshape(nv * nc, nr)
    rcc = _density(cc, cc, g)
    rvv = _density(cv, cv, g)
    kx_r = np.conj(rvc) @ vr @ rvc.T / nr ** 2
    kd_r = -np.einsum("cdr,rs,vus->vcud", np.conj(rcc), wr, rvv).reshape(nv * nc, nv * nc) / nr ** 2
    assert np.abs(kx - kx_r).max() < 1e-13 * np.abs(kx).max()
    assert np.abs(kd - kd_r).max() < 1e-13 * np.abs(kd).max()
    # exchange Hermitian positive semidefinite; the TDA Hamiltonian Hermitian
    assert np.abs(kx - kx.conj().T).max() < 1e-14 * np.abs(kx).max()
    assert np.linalg.eigvalsh(kx).min() > -1e-13 * np.abs(kx).max()
    # with W Hermitian and real in real space (W_{-G,-G'} = conj W_GG', the static
    # screened interaction of a time-reversal symmetric system) the TDA
    # Hamiltonian D + K^X + K^D is Hermitian; a W without the second property
    # breaks it
    lut = {tuple(v): i for i, v in enumerate(geps.tolist())}
    minus = np.array([lut[tuple(-x for x in v)] for v in geps.tolist()])
    wt = 0.5 * (w + np.conj(w[np.ix_(minus, minus)]))
    kd_t = oracle.bse_kernel(_mt(cv, g, cc, g, geps), _mt(cc, g, cc, g, geps),
                             _mt(cv, g, cv, g, geps), vx, wt)[1]
    d = np.diag(rng.uniform(1, 2, nv * nc))
    h = d + kx + kd_t
    assert np.abs(h - h.conj().T).max() < 1e-13 * np.abs(h).max()
    h_bad = d + kx + kd
    assert np.abs(h_bad - h_bad.conj().T).max() > 1e-3 * np.abs(h_bad).max()


def test_collinear_spinors_give_the_spinless_kernels():
    """Orbitals phi as (phi, 0) and (0, phi): same-spin transition blocks carry the
    spinless kernels (exchange also across the two spins), spin-flip transitions
    have no exchange, and the direct term does not couple different spins."""
    rng, g, geps, pv, pc = _sets(seed=4, ns=1)
    n = len(geps)
    vx = rng.uniform(0.1, 3.0, n)
    a = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    w = a @ a.conj().T / n
    ks = oracle.bse_kernel(_mt(pv, g, pc, g, geps), _mt(pc, g, pc, g, geps),
                           _mt(pv, g, pv, g, geps), vx, w)

    def spin(c, s):
        out = np.zeros((c.shape[0], 2, c.shape[2]), dtype=np.complex128)
        out[:, s] = c[:, 0]
        return out

    cv = np.concatenate([spin(pv, 0), spin(pv, 1)])
    cc = np.concatenate([spin(pc, 0), spin(pc, 1)])
    kx, kd = oracle.bse_kernel(_mt(cv, g, cc, g, geps), _mt(cc, g, cc, g, geps),
                               _mt(cv, g, cv, g, geps), vx, w)
    nv, nc = len(pv), len(pc)
    kx4 = kx.reshape(2, nv, 2, nc, 2, nv, 2, nc)
    kd4 = kd.reshape(2, nv, 2, nc, 2, nv, 2, nc)
    sx, sd = ks[0].reshape(nv, nc, nv, nc), ks[1].reshape(nv, nc, nv, nc)
    for s in range(2):
        for t in range(2):
            assert np.abs(kx4[s, :, s, :, t, :, t, :] - sx).max() < 1e-13
            assert np.abs(kx4[s, :, 1 - s, :, t, :, 1 - t, :]).max() == 0.0
        assert np.abs(kd4[s, :, s, :, s, :, s, :] - sd).max() < 1e-13
        assert np.abs(kd4[s, :, s, :, 1 - s, :, 1 - s, :]).max() == 0.0
