"""Pins of the plasmon-pole oracle (gpp_modes, epsinv_gpp, sigma_gpp) against what
the model and the mathematics fix: the static eps^-1 it reproduces, the plasma
frequency of the uniform electron gas, the f-sum rule of a single pole, the
Hermitian pole weight of W, and the SX/COH limits at E = E_n''."""
import numpy as np
import pytest
from scipy import integrate

import oracle
import synth
from synth.generate import g_sphere

CELL = (7.5, 7.75, 9.5)
BOX = (16, 16, 16)
Q = (0.05, -0.02, 0.03)


def _system(seed=3, nv=4, nb=10, ecut=4.0):
    rng = np.random.default_rng(seed)
    geps = g_sphere(CELL, Q, ecut)
    n = len(geps)
    v = synth.vcoul(CELL, Q, geps)
    # a static chi0 <= 0 from random pair elements -> eps^-1 through the oracle
    m = (rng.standard_normal((40, n)) + 1j * rng.standard_normal((40, n))) * 0.05
    chi = -(np.conj(m).T @ m)
    einv = oracle.epsilon_inverse(chi[None], v)[0]
    rho = synth.charge_density(seed, CELL, BOX, nelec=8.0)
    mt = (rng.standard_normal((nb, 5, n)) + 1j * rng.standard_normal((nb, 5, n))) / 4
    en = np.sort(rng.uniform(-0.5, 0.8, nb))
    return geps, v, einv, rho, mt, en, nv


def test_modes_reproduce_the_static_epsinv():
    geps, v, einv, rho, *_ = _system()
    o2, wt, keep = oracle.gpp_modes(einv, geps, CELL, Q, rho)
    assert keep.mean() > 0.3
    static = oracle.epsinv_gpp(o2, wt, 0.0)
    assert np.abs(static[keep] - einv[keep]).max() < 1e-12
    n = len(geps)
    assert np.abs(static[~keep] - np.eye(n)[~keep]).max() == 0.0
    assert np.all(wt[keep].real > 0)


def test_uniform_gas_pole_is_the_plasma_frequency():
    """Uniform density (rho(G) = 0 for G != 0), perfect screening of the head as
    q -> 0: the head's pole sits at omega_p = sqrt(4 pi n) = sqrt(3 / r_s^3)."""
    rs = 2.0
    n_el = 3.0 / (4.0 * np.pi * rs ** 3)
    rho = np.zeros(BOX, dtype=np.complex128)
    rho[0, 0, 0] = n_el
    for qx in (1e-2, 1e-3):
        q = (qx, 0.0, 0.0)
        geps = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]])
        qg2 = ((2 * np.pi * (geps + np.array(q)) / np.array(CELL)) ** 2).sum(1)
        ktf2 = 4.0 * (3.0 * n_el / np.pi) ** (1.0 / 3.0)  # Thomas-Fermi k^2
        einv = np.diag(1.0 / (1.0 + ktf2 / qg2)).astype(np.complex128)
        o2, wt, keep = oracle.gpp_modes(einv, geps, CELL, q, rho)
        assert keep[0, 0] and not keep[0, 1] and np.abs(o2[0, 1:]).max() == 0.0
        wp = np.sqrt(3.0 / rs ** 3)
        assert abs(wt[0, 0].real - wp) / wp < 2 * qg2[0] / ktf2
    assert abs(np.sqrt(3.0 / 8.0) * 27.211386 - 16.66) < 0.01  # r_s = 2: 16.7 eV


def test_single_pole_satisfies_the_f_sum_rule():
    """int_0^inf w Im eps^-1(w) dw = -(pi/2) Omega^2 for the broadened pole."""
    o2, wt, eta = 0.7, 0.9, 1e-3

    def im(w):
        return (o2 / (w * w - (wt - 1j * eta) ** 2)).imag * w

    val = integrate.quad(im, 0, wt, limit=400, points=[wt])[0] + \
        integrate.quad(im, wt, 60.0, limit=400)[0] + integrate.quad(im, 60.0, np.inf)[0]
    assert abs(val + np.pi / 2 * o2) / (np.pi / 2 * o2) < 5e-3


def test_pole_weight_of_w_is_hermitian():
    """Omega^2_GG' v(q+G') is Hermitian for a real density; the index of the
    |q+G|^2 denominator fixes it (the other choice fails)."""
    geps, v, einv, rho, *_ = _system()
    n = len(geps)
    # delta - eps^-1 = 0.3 everywhere: a mode is dropped only where Re Omega^2 <= 0,
    # a set that is symmetric when the pole weight of W is Hermitian
    o2, wt, keep = oracle.gpp_modes(np.eye(n) - 0.3, geps, CELL, Q, rho)
    assert keep.mean() > 0.3
    w = o2 * v[None, :]
    assert np.abs(w - w.conj().T).max() < 1e-12 * np.abs(w).max()
    qg = 2 * np.pi * (geps + np.array(Q)) / np.array(CELL)
    qg2 = (qg ** 2).sum(1)
    wrong = o2 * (qg2[:, None] / qg2[None, :]) * v[None, :]
    assert np.abs(wrong - wrong.conj().T).max() > 1e-3 * np.abs(wrong).max()


def test_sx_and_coh_at_e_equal_e_occupied():
    """With every E_n'' equal to E: SX is the static SX with the GPP's static eps^-1,
    and COH is 1/2 m^H (eps^-1_GPP(0) - 1) v m summed over every n''."""
    geps, v, einv, rho, mt, en, nv = _system()
    o2, wt, keep = oracle.gpp_modes(einv, geps, CELL, Q, rho)
    nn, nband, n = mt.shape
    e0 = 0.3
    en0 = np.full(nn, e0)
    energies = np.full((nband, 1), e0)
    sx, coh = oracle.sigma_gpp(mt, en0, nv, v, o2, wt, energies, prefactor=0.7)
    stat = oracle.epsinv_gpp(o2, wt, 0.0)
    want_sx = oracle.sigma_sx_static(mt[:nv], stat, v, 0.7)
    assert np.abs(sx[:, 0] - want_sx).max() < 1e-12 * np.abs(want_sx).max()
    d = (stat - np.eye(n)) * v[None, :]
    want_coh = 0.5 * 0.7 * np.einsum("ang,gh,anh->n", np.conj(mt), d, mt)
    assert np.abs(coh[:, 0] - want_coh).max() < 1e-12 * np.abs(want_coh).max()
    # COH lowers the energy: 1 - eps^-1 weighted by v is positive semidefinite here
    assert np.all(want_coh.real < 0)


@pytest.mark.parametrize("delta", [-0.8, -0.2, 0.3])
def test_coh_term_is_the_positive_frequency_integral(delta):
    """One element: prefactor-free COH from the w' > 0 integral of the broadened
    pole's spectral weight -(1/pi) Im eps^-1(w') against 1/(delta - w') tends to
    Omega^2 / (2 wtilde (delta - wtilde)) as eta -> 0."""
    o2, wt = 0.6, 0.95
    m = np.array([1.0 + 0.0j])
    v = np.array([1.0])
    got = oracle.sigma_gpp(m[None, None, :], [0.0], 0, v, np.array([[o2]]),
                           np.array([[wt + 0j]]), [[delta]])[1][0, 0]
    errs = []
    for eta in (4e-3, 2e-3):
        def integrand(w, part):
            a = -(o2 / (w * w - (wt - 1j * eta) ** 2)).imag / np.pi
            z = a / (delta - w + 1j * eta)
            return z.real if part == 0 else z.imag
        brk = sorted({wt, max(delta, 1e-6)})
        val = sum(integrate.quad(integrand, lo, hi, args=(0,), limit=800)[0]
                  for lo, hi in zip([0.0] + brk, brk + [50.0]))
        errs.append(abs(val - got.real) / abs(got.real))
    assert errs[1] < errs[0] and errs[1] < 2e-2


def test_sx_pole_term_matches_partial_fractions():
    """Omega^2/(d^2 - wt^2) = Omega^2/(2 wt) [1/(d - wt) - 1/(d + wt)] for complex
    wtilde: the identity the GPU kernel evaluates."""
    rng = np.random.default_rng(0)
    o2 = rng.standard_normal(50) + 1j * rng.standard_normal(50)
    wt = np.sqrt(rng.uniform(0.2, 3, 50) + 1j * rng.uniform(-1, 1, 50))
    d = rng.uniform(-2, 2, 50)
    lhs = o2 / (d * d - wt * wt)
    rhs = o2 / (2 * wt) * (1 / (d - wt) - 1 / (d + wt))
    assert np.abs(lhs - rhs).max() < 1e-12 * np.abs(lhs).max()
