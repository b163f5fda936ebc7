"""Pins of the CPU oracle against closed forms, brute force and library routines.

Each check is chosen so that a plausible slip in the oracle (a dropped spin
term, a wrong transform sign or normalisation, a transposed operand, a missing
conjugate, a wrong energy denominator) fails at least one of them.
"""
import numpy as np
import pytest
import scipy.linalg
import scipy.linalg.blas

import oracle
import synth
from synth.generate import SystemConfig, _random_spinors, g_sphere, vcoul


def tiny_system(seed=7, q=(0.25, 0.0, -0.25), nv=3, nc=5, ns=2, box=(8, 9, 10),
                cell=(5.0, 5.3, 5.7), ecut=8.0, ecut_eps=3.0):
    rng = np.random.default_rng(seed)
    gk = g_sphere(cell, (0, 0, 0), ecut)
    gkq = g_sphere(cell, q, ecut)
    geps = g_sphere(cell, q, ecut_eps)
    cc = _random_spinors(rng, len(gk), nc, ns)
    cv = _random_spinors(rng, len(gkq), nv, ns)
    ev = np.sort(rng.uniform(-6, 0, nv)) / synth.EV_PER_HA
    ec = np.sort(rng.uniform(1, 20, nc)) / synth.EV_PER_HA
    return dict(cv=cv, gv=gkq, cc=cc, gc=gk, geps=geps, box=box, ev=ev, ec=ec,
                vcoul=vcoul(cell, q, geps), cell=cell, q=q)


@pytest.fixture(scope="module")
def tiny():
    s = tiny_system()
    assert oracle.alias_free(s["gv"], s["gc"], s["geps"], s["box"])
    return s


def test_wavefunction_matches_explicit_synthesis(tiny):
    s = tiny
    u = oracle.wavefunction_on_box(s["cv"], s["gv"], s["box"])
    box = np.array(s["box"])
    rng = np.random.default_rng(1)
    for _ in range(20):
        j = rng.integers(0, box)
        b, sp = rng.integers(0, s["cv"].shape[0]), rng.integers(0, 2)
        val = np.sum(s["cv"][b, sp] * np.exp(2j * np.pi * (s["gv"] @ (j / box))))
        assert abs(u[b, sp, j[0], j[1], j[2]] - val) < 1e-13


def test_wavefunction_parseval(tiny):
    # orthonormal spinors: (1/N) sum_r sum_sigma |u|^2 = 1 and cross terms vanish
    u = oracle.wavefunction_on_box(tiny["cv"], tiny["gv"], tiny["box"])
    n = np.prod(tiny["box"])
    flat = u.reshape(u.shape[0], -1)
    gram = np.conj(flat) @ flat.T / n
    assert np.allclose(gram, np.eye(u.shape[0]), atol=1e-13)


def test_mtxel_three_routes_agree(tiny):
    s = tiny
    m_fft = oracle.mtxel_fft(s["cv"], s["gv"], s["cc"], s["gc"], s["geps"], s["box"])
    m_conv = oracle.mtxel_convolution(s["cv"], s["gv"], s["cc"], s["gc"], s["geps"])
    m_bf = oracle.mtxel_bruteforce(s["cv"], s["gv"], s["cc"], s["gc"], s["geps"], s["box"])
    assert oracle.rel_f(m_fft, m_conv) < 1e-13
    assert oracle.rel_f(m_bf, m_conv) < 1e-12


def test_aliasing_box_breaks_fft_route():
    # a box at the alias limit must disagree with the grid-free definition
    s = tiny_system(box=(5, 5, 5))
    assert not oracle.alias_free(s["gv"], s["gc"], s["geps"], s["box"])
    m_fft = oracle.mtxel_fft(s["cv"], s["gv"], s["cc"], s["gc"], s["geps"], s["box"])
    m_conv = oracle.mtxel_convolution(s["cv"], s["gv"], s["cc"], s["gc"], s["geps"])
    assert oracle.rel_f(m_fft, m_conv) > 1e-3


@pytest.mark.parametrize("sa,sb", [(0, 0), (1, 1), (0, 1), (1, 0)])
def test_single_plane_wave_pair_gives_delta(tiny, sa, sb):
    s = tiny
    gv, gc, geps = s["gv"], s["gc"], s["geps"]
    ia, ib = 5, 3
    cv = np.zeros((1, 2, len(gv)), complex)
    cc = np.zeros((1, 2, len(gc)), complex)
    cv[0, sa, ia] = 1.0
    cc[0, sb, ib] = 1.0
    want = np.zeros(len(geps), complex)
    if sa == sb:
        d = gv[ia] - gc[ib]
        hit = np.where((geps == d).all(axis=1))[0]
        want[hit] = 1.0
    for m in (oracle.mtxel_fft(cv, gv, cc, gc, geps, s["box"])[0, 0],
              oracle.mtxel_convolution(cv, gv, cc, gc, geps)[0, 0],
              oracle.mtxel_bruteforce(cv, gv, cc, gc, geps, s["box"])[0, 0]):
        assert np.abs(m - want).max() < 1e-13


def test_head_vanishes_for_orthonormal_states_at_q0():
    # q = 0: valence and conduction from one orthonormal set -> M_vc(G=0) = 0
    rng = np.random.default_rng(3)
    cell = (5.0, 5.3, 5.7)
    gk = g_sphere(cell, (0, 0, 0), 8.0)
    geps = g_sphere(cell, (0, 0, 0), 3.0)
    joint = _random_spinors(rng, len(gk), 9, 2)
    cv, cc = joint[:3], joint[3:]
    m = oracle.mtxel_fft(cv, gk, cc, gk, geps, (8, 9, 10))
    i0 = np.where((geps == 0).all(axis=1))[0][0]
    assert np.abs(m[:, :, i0]).max() < 1e-14
    # and the diagonal overlap of a state with itself is 1
    h = oracle.head_overlap(joint, gk, joint, gk)
    assert np.allclose(h, np.eye(9), atol=1e-14)


def test_zero_down_component_is_spinless(tiny):
    s = tiny
    cv, cc = s["cv"].copy(), s["cc"].copy()
    cv[:, 1] = 0.0
    cc[:, 1] = 0.0
    m2 = oracle.mtxel_fft(cv, s["gv"], cc, s["gc"], s["geps"], s["box"])
    m1 = oracle.mtxel_fft(cv[:, :1], s["gv"], cc[:, :1], s["gc"], s["geps"], s["box"])
    assert np.abs(m2 - m1).max() < 1e-15


def test_doubled_collinear_set_doubles_chi0(tiny):
    # Sec. II: the spinor P has the spinless form with spin traced and both
    # band counts doubled.  Spinor set {(phi,0),(0,phi)} => chi0 = 2 chi0_spinless.
    s = tiny
    phi_v, phi_c = s["cv"][:, :1], s["cc"][:, :1]
    m1 = oracle.mtxel_fft(phi_v, s["gv"], phi_c, s["gc"], s["geps"], s["box"])
    x1 = oracle.chi0(m1, s["ev"], s["ec"], [0.0, 1.5])

    def doubled(phi):
        nb, _, ng = phi.shape
        out = np.zeros((2 * nb, 2, ng), complex)
        out[:nb, 0] = phi[:, 0]
        out[nb:, 1] = phi[:, 0]
        return out

    m2 = oracle.mtxel_fft(doubled(phi_v), s["gv"], doubled(phi_c), s["gc"], s["geps"], s["box"])
    x2 = oracle.chi0(m2, np.tile(s["ev"], 2), np.tile(s["ec"], 2), [0.0, 1.5])
    assert oracle.rel_f(x2, 2 * x1) < 1e-14


def test_completeness_sum_rule():
    # sum over a complete basis at k of M*_vn(G) M_vn(G') equals
    # sum_sigma sum_{a in S_k} c_v(a+G) conj(c_v(a+G')), from the M definition
    rng = np.random.default_rng(11)
    cell, q = (5.0, 5.3, 5.7), (0.25, 0.0, 0.0)
    gk = g_sphere(cell, (0, 0, 0), 6.0)
    gkq = g_sphere(cell, q, 6.0)
    geps = g_sphere(cell, q, 2.5)
    full = _random_spinors(rng, len(gk), 2 * len(gk), 2)   # unitary basis at k
    cv = _random_spinors(rng, len(gkq), 2, 2)
    m = oracle.mtxel_fft(cv, gkq, full, gk, geps, (12, 12, 12))
    lhs = np.einsum("vng,vnh->vgh", np.conj(m), m)
    lutv = {tuple(g): i for i, g in enumerate(gkq.tolist())}
    rhs = np.zeros_like(lhs)
    for v in range(cv.shape[0]):
        for ig, G in enumerate(geps.tolist()):
            for jg, H in enumerate(geps.tolist()):
                acc = 0j
                for a in gk.tolist():
                    i1 = lutv.get((a[0] + G[0], a[1] + G[1], a[2] + G[2]))
                    i2 = lutv.get((a[0] + H[0], a[1] + H[1], a[2] + H[2]))
                    if i1 is not None and i2 is not None:
                        acc += np.sum(cv[v, :, i1] * np.conj(cv[v, :, i2]))
                rhs[v, ig, jg] = acc
    assert np.abs(lhs - rhs).max() < 1e-13


def test_weight_closed_form():
    ev = np.array([-0.2, -0.05])
    ec = np.array([0.1, 0.3, 0.7])
    om = np.array([0.0, 0.4])
    w = oracle.chi0_weight(ev, ec, om)
    d = (ev[:, None] - ec[None, :]).ravel()
    for f, o in enumerate(om):
        assert np.allclose(w[f], 2 * d / (d * d + o * o), rtol=1e-15, atol=0)
    assert np.all(w < 0)


def test_real_axis_weight_forms():
    ev = np.array([-0.2, -0.05])
    ec = np.array([0.1, 0.3, 0.7])
    d = (ev[:, None] - ec[None, :]).ravel()
    # at w = i*omega and eta = 0 the bracket is the imaginary-axis factor
    om = np.array([0.0, 0.4, 3.0])
    w = oracle.chi0_weight_real(ev, ec, 1j * om, 0.0)
    assert np.allclose(w, oracle.chi0_weight(ev, ec, om), rtol=1e-15, atol=0)
    # on the real axis the two terms sum to 2a / (a^2 - w^2), a = delta + i eta
    eta = 0.01
    wr = np.array([0.0, 0.15, 0.5, 2.0])
    w = oracle.chi0_weight_real(ev, ec, wr, eta)
    a = d + 1j * eta
    for f, o in enumerate(wr):
        assert np.allclose(w[f], 2 * a / (a * a - o * o), rtol=1e-13, atol=0)
    assert np.all(w.imag < 0)  # absorptive: both poles sit below the real axis


def test_chi0_real_splits_into_hermitian_parts(tiny):
    """Re and Im of the bracket are real weights, so P(w) = A + iB with A, B
    Hermitian contractions; each is rebuilt with scipy ZHERK from the positive and
    negative parts of its weight."""
    s = tiny
    m = oracle.mtxel_convolution(s["cv"], s["gv"], s["cc"], s["gc"], s["geps"])
    flat = m.reshape(-1, m.shape[-1])
    wr = [0.0, 0.12, 0.4]
    eta = 0.02
    x = oracle.chi0_real(m, s["ev"], s["ec"], wr, eta, prefactor=0.5)
    w = oracle.chi0_weight_real(s["ev"], s["ec"], wr, eta)

    def herk(weights):
        out = np.zeros((flat.shape[1], flat.shape[1]), dtype=np.complex128)
        for sign in (1.0, -1.0):
            part = np.clip(sign * weights, 0.0, None)
            a = np.sqrt(part)[:, None] * flat
            up = scipy.linalg.blas.zherk(0.5 * sign, a, trans=2)
            out += np.triu(up) + np.triu(up, 1).conj().T
        return out

    for f in range(len(wr)):
        ref = herk(w[f].real) + 1j * herk(w[f].imag)
        assert oracle.rel_f(x[f], ref) < 1e-14
        # absorptive diagonal for eta > 0
        assert np.all(np.diag(x[f]).imag < 0)
    # even in w
    xm = oracle.chi0_real(m, s["ev"], s["ec"], [-v for v in wr], eta, prefactor=0.5)
    assert oracle.rel_f(xm, x) < 1e-15
    # static limit: at w = 0 the difference from the imaginary-axis chi0 at
    # omega = 0 is first order in eta (an imaginary part -2 eta / delta^2 per pair)
    ref0 = oracle.chi0(m, s["ev"], s["ec"], [0.0])[0]
    errs = [oracle.rel_f(oracle.chi0_real(m, s["ev"], s["ec"], [0.0], e)[0], ref0)
            for e in (1e-6, 1e-9)]
    assert errs[1] < 1e-7 and 500 < errs[0] / errs[1] < 2000


def test_chi0_matches_zherk_and_is_hermitian_nsd(tiny):
    s = tiny
    m = oracle.mtxel_convolution(s["cv"], s["gv"], s["cc"], s["gc"], s["geps"])
    om = [0.0, 0.2, 1.0, 5.0]
    x = oracle.chi0(m, s["ev"], s["ec"], om, prefactor=0.5)
    flat = m.reshape(-1, m.shape[-1])
    d = (s["ev"][:, None] - s["ec"][None, :]).ravel()
    for f, o in enumerate(om):
        a = np.sqrt(-2 * d / (d * d + o * o))[:, None] * flat
        up = scipy.linalg.blas.zherk(-0.5, a, trans=2)       # -0.5 * a^H a, upper
        ref = np.triu(up) + np.triu(up, 1).conj().T
        assert oracle.rel_f(x[f], ref) < 1e-14
        assert np.abs(x[f] - x[f].conj().T).max() < 1e-15 * np.abs(x[f]).max()
        assert np.linalg.eigvalsh(x[f]).max() < 1e-14 * np.abs(x[f]).max()
    # Loewner monotone in omega: chi0(i w2) - chi0(i w1) is PSD for w2 > w1
    for f in range(len(om) - 1):
        assert np.linalg.eigvalsh(x[f + 1] - x[f]).min() > -1e-14 * np.abs(x[f]).max()


def test_chi0_large_omega_asymptote(tiny):
    s = tiny
    m = oracle.mtxel_convolution(s["cv"], s["gv"], s["cc"], s["gc"], s["geps"])
    big = 1e4
    x = oracle.chi0(m, s["ev"], s["ec"], [big])[0] * big * big
    flat = m.reshape(-1, m.shape[-1])
    d = (s["ev"][:, None] - s["ec"][None, :]).ravel()
    lim = (np.conj(flat).T * (2 * d)[None, :]) @ flat
    assert oracle.rel_f(x, lim) < 1e-6


def test_chi0_chunked_accumulation(tiny):
    s = tiny
    m = oracle.mtxel_convolution(s["cv"], s["gv"], s["cc"], s["gc"], s["geps"])
    om = [0.0, 0.7]
    full = oracle.chi0(m, s["ev"], s["ec"], om)
    part = oracle.chi0(m[:, :2], s["ev"], s["ec"][:2], om) + oracle.chi0(m[:, 2:], s["ev"], s["ec"][2:], om)
    assert oracle.rel_f(part, full) < 1e-15


def test_epsinv_sherman_morrison_single_pair(tiny):
    s = tiny
    m = oracle.mtxel_convolution(s["cv"][:1], s["gv"], s["cc"][:1], s["gc"], s["geps"])
    om = [0.0, 0.3]
    x = oracle.chi0(m, s["ev"][:1], s["ec"][:1], om)
    einv = oracle.epsilon_inverse(x, s["vcoul"])
    mv = m[0, 0]
    d = s["ev"][0] - s["ec"][0]
    for f, o in enumerate(om):
        w = 2 * d / (d * d + o * o)
        u = w * s["vcoul"] * np.conj(mv)
        ref = np.eye(len(mv)) + np.outer(u, mv) / (1 - mv @ u)
        assert oracle.rel_f(einv[f], ref) < 1e-13


def test_eps_spectrum_bounds_and_lu_solve():
    s = synth.build_system(synth.CONFIGS["C1"])
    m = oracle.mtxel_convolution(s["cv"], s["gv"], s["cc"], s["gc"], s["geps"])
    x = oracle.chi0(m, s["ev"], s["ec"], [0.0, 1.0])
    einv = oracle.epsilon_inverse(x, s["vcoul"])
    vh = np.sqrt(s["vcoul"])
    for f in range(2):
        eps = oracle.epsilon(x[f], s["vcoul"])
        # eps is similar to I - V^1/2 chi0 V^1/2 (Hermitian, >= 1)
        ev_eps = np.linalg.eigvals(eps)
        assert np.abs(ev_eps.imag).max() < 1e-10
        assert ev_eps.real.min() > 1 - 1e-12
        sym = np.eye(len(vh)) - vh[:, None] * x[f] * vh[None, :]
        lam = np.linalg.eigvalsh(sym)
        assert lam.min() > 1 - 1e-12
        inv_ev = np.linalg.eigvals(einv[f])
        assert inv_ev.real.min() > 0 and inv_ev.real.max() < 1 + 1e-12
        lu = scipy.linalg.lu_factor(eps)
        ref = scipy.linalg.lu_solve(lu, np.eye(len(vh)))
        assert oracle.rel_f(einv[f], ref) < 1e-13


def _spinor_model(cell, g, kred, vpot):
    """Eigenpairs of H(k) = |k+G|^2/2 + V(G - G') (2x2 in spin) on the list g:
    a local, spin-dependent potential, so the velocity is exactly p + k."""
    ng = len(g)
    kg = (g + np.asarray(kred)) * (2 * np.pi / np.asarray(cell))
    h = np.zeros((2 * ng, 2 * ng), dtype=np.complex128)
    for a in range(ng):
        for b in range(ng):
            h[2 * a:2 * a + 2, 2 * b:2 * b + 2] = vpot(tuple(g[a] - g[b]))
    h += np.diag(np.repeat(0.5 * np.sum(kg * kg, axis=1), 2))
    e, u = np.linalg.eigh(h)
    # coefficients c[n][sigma][G]
    return e, np.transpose(u.reshape(ng, 2, 2 * ng), (2, 1, 0))


def test_head_dipole_is_the_kp_limit_of_the_overlap():
    """In a plane-wave model with a local spin-dependent potential (no time
    reversal, so no degeneracies), the G = 0 matrix element <u_v,k+q|u_c,k> from
    wavefunctions diagonalised at k+q matches q.P_vc/(E_v - E_c) from k alone, with
    an error second order in q."""
    cell = (5.0, 5.3, 5.7)
    g = g_sphere(cell, (0, 0, 0), 6.0)
    rng = np.random.default_rng(11)
    table = {}

    def vpot(dg):
        if dg == (0, 0, 0):
            return np.array([[0.3, 0.1 - 0.05j], [0.1 + 0.05j, -0.2]])
        key = min(dg, tuple(-x for x in dg))
        if key not in table:
            table[key] = 0.15 * (rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2)))
        m = table[key]
        return m if dg == key else m.conj().T

    nv, nc = 2, 3
    e0, c0 = _spinor_model(cell, g, (0, 0, 0), vpot)
    assert np.min(np.diff(e0[:nv + nc])) > 1e-3
    qdir = np.array([0.6, -0.3, 0.74])
    qdir /= np.linalg.norm(qdir)
    errs = []
    for qn in (2e-3, 1e-3):
        qcart = qn * qdir
        qred = qcart * np.asarray(cell) / (2 * np.pi)
        eq, cq = _spinor_model(cell, g, qred, vpot)
        # fix the arbitrary phase of each band at k+q to its k counterpart
        for n in range(nv):
            ov = np.vdot(c0[n].ravel(), cq[n].ravel())
            cq[n] *= np.conj(ov) / abs(ov)
        over = oracle.head_overlap(cq[:nv], g, c0[nv:nv + nc], g)
        dip = oracle.head_dipole(c0[:nv], c0[nv:nv + nc], g, cell, (0, 0, 0), qcart, e0[:nv],
                                 e0[nv:nv + nc])
        errs.append(np.abs(over - dip).max() / np.abs(dip).max())
    assert errs[0] < 5e-3
    # M itself is first order in q and the difference second order, so the
    # relative difference halves with q
    assert 1.8 < errs[0] / errs[1] < 2.2


def test_head_dipole_hermiticity_and_plane_waves():
    cell = (5.0, 5.3, 5.7)
    g = g_sphere(cell, (0, 0, 0), 8.0)
    rng = np.random.default_rng(3)
    nv, nc = 2, 3
    cv = _random_spinors(rng, len(g), nv, 2)
    cc = _random_spinors(rng, len(g), nc, 2)
    ev = np.array([-0.3, -0.1])
    ec = np.array([0.2, 0.4, 0.9])
    k = (0.1, -0.2, 0.05)
    q = np.array([1e-3, -2e-3, 0.5e-3])
    d_vc = oracle.head_dipole(cv, cc, g, cell, k, q, ev, ec) * (ev[:, None] - ec[None, :])
    d_cv = oracle.head_dipole(cc, cv, g, cell, k, q, ec, ev) * (ec[:, None] - ev[None, :])
    assert np.allclose(d_vc, np.conj(d_cv).T, rtol=1e-14, atol=1e-16)
    # single plane waves: P = delta_{G1 G2} delta_{ab} (k + G1)
    i1, i2 = 5, 9
    a = np.zeros((1, 2, len(g)), dtype=np.complex128)
    b = np.zeros((2, 2, len(g)), dtype=np.complex128)
    a[0, 1, i1] = 1.0
    b[0, 1, i1] = 1.0
    b[1, 1, i2] = 1.0
    m = oracle.head_dipole(a, b, g, cell, k, q, [0.0], [1.0, 1.0])
    kg1 = (np.asarray(g[i1], dtype=np.float64) + np.asarray(k)) * 2 * np.pi / np.asarray(cell)
    assert np.isclose(m[0, 0], -(kg1 @ q), rtol=1e-14, atol=0)
    assert m[0, 1] == 0


def test_static_screened_exchange_bounds(tiny):
    """Sigma^SX with the static eps^-1: at eps^-1 = I it is the bare exchange
    -sum |M(G)|^2 v(G); with chi0 <= 0 the screened W = eps^-1 v is Hermitian
    positive semidefinite and no larger than v, so Sigma^SX is real and lies
    between the bare exchange and 0, band by band."""
    s = tiny
    m = oracle.mtxel_convolution(s["cv"], s["gv"], s["cc"], s["gc"], s["geps"])  # [3][5][neps]
    v = s["vcoul"]
    neps = m.shape[-1]
    bare = oracle.sigma_sx_static(m, np.eye(neps), v, prefactor=0.5)
    assert np.allclose(bare, -0.5 * np.einsum("ang,g->n", np.abs(m) ** 2, v), rtol=1e-14, atol=0)
    x = oracle.chi0(m, s["ev"], s["ec"], [0.0])[0]
    einv = oracle.epsilon_inverse(x[None], v)[0]
    w = oracle.screened_w(einv[None], v)[0]
    assert np.abs(w - w.conj().T).max() < 1e-13 * np.abs(w).max()
    sx = oracle.sigma_sx_static(m, einv, v, prefactor=0.5)
    assert np.abs(sx.imag).max() < 1e-12 * np.abs(sx).max()
    assert np.all(sx.real < 0) and np.all(sx.real > bare.real)


def test_generator_is_deterministic():
    a = synth.build_system(synth.CONFIGS["C1"])
    b = synth.build_system(synth.CONFIGS["C1"])
    for k in ("cv", "cc", "gv", "gc", "geps", "ev", "ec", "vcoul"):
        assert np.array_equal(a[k], b[k])
    assert a["geps"].shape[0] == 59
    assert a["gc"].shape[0] == 395 and a["gv"].shape[0] == 399
    # orthonormal stacked spinors
    flat = a["cc"].reshape(a["cc"].shape[0], -1)
    assert np.allclose(np.conj(flat) @ flat.T, np.eye(flat.shape[0]), atol=1e-13)


def test_q0_head_construction_scales_with_q():
    s = synth.build_system(synth.CONFIGS["T1Q0"])
    h = oracle.head_overlap(s["cv"], s["gv"], s["cc"], s["gc"])
    qn = np.linalg.norm(s["qg"][s["head_index"]])
    assert s["head_index"] >= 0
    assert np.abs(h).max() < 20 * qn and np.abs(h).max() > 1e-3 * qn
    m = oracle.mtxel_convolution(s["cv"], s["gv"], s["cc"], s["gc"], s["geps"])
    assert np.allclose(m[:, :, s["head_index"]], h, atol=1e-15)


# ----------------------------------------------------------------- low-rank eps^-1
def _lr_system(seed, n=40, nf=3, rank=None):
    rng = np.random.default_rng(seed)
    v = rng.uniform(0.2, 3.0, n)
    r = n if rank is None else rank
    m = (rng.standard_normal((r, n)) + 1j * rng.standard_normal((r, n))) * 0.3
    chi = np.stack([-(np.conj(m).T @ m) / (1.0 + f) for f in range(nf)])
    return chi, v


def test_lowrank_full_basis_is_the_exact_inverse():
    chi, v = _lr_system(1)
    lr, _ = oracle.epsinv_lowrank(chi, v, chi.shape[-1])
    ex = oracle.epsilon_inverse(chi, v)
    assert np.abs(lr - ex).max() < 1e-12 * np.abs(ex).max()


def test_lowrank_rank_one_chi_is_exact_with_one_vector():
    """chi0(w) = -a(w) x x^H: epst - I has rank one, so one eigenvector carries all
    of it and the Sherman-Morrison inverse follows exactly."""
    rng = np.random.default_rng(2)
    n = 30
    v = rng.uniform(0.2, 3.0, n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    chi = np.stack([-a * np.outer(np.conj(x), x) for a in (0.7, 0.3, 0.05)])
    lr, _ = oracle.epsinv_lowrank(chi, v, 1)
    ex = oracle.epsilon_inverse(chi, v)
    assert np.abs(lr - ex).max() < 1e-12 * np.abs(ex).max()


def test_lowrank_static_error_is_the_discarded_spectrum():
    """At w = 0: epst^-1 - approx = sum over discarded eigenpairs of (1/lambda - 1) u u^H,
    whose 2-norm is max |1/lambda - 1| over the discarded eigenvalues."""
    chi, v = _lr_system(3)
    n, nb = chi.shape[-1], 12
    lr, lam = oracle.epsinv_lowrank(chi, v, nb)
    ex = oracle.epsilon_inverse(chi, v)
    sv = np.sqrt(v)
    d = (lr[0] - ex[0]) * sv[None, :] / sv[:, None]  # back to the symmetric form
    want = np.max(np.abs(1.0 / lam[:n - nb] - 1.0))
    assert abs(np.linalg.norm(d, 2) - want) < 1e-10 * want
    assert np.all(lam >= 1.0 - 1e-12)


def test_projected_chi0_route_equals_the_projected_inverse():
    """Building chi0 in the basis (M projected first) gives the same reduced-basis
    eps^-1 as projecting the full chi0; when every M_p lies in an nb-dimensional
    space the reduced basis is exact."""
    rng = np.random.default_rng(8)
    nv, nc, n, nb = 3, 7, 36, 9
    m = (rng.standard_normal((nv, nc, n)) + 1j * rng.standard_normal((nv, nc, n))) / 3
    ev = np.sort(rng.uniform(-0.5, -0.05, nv))
    ec = np.sort(rng.uniform(0.05, 0.9, nc))
    om = np.array([0.0, 0.3, 1.1])
    v = rng.uniform(0.2, 3.0, n)
    chi = oracle.chi0(m, ev, ec, om)
    lr, _ = oracle.epsinv_lowrank(chi, v, nb)
    sv = np.sqrt(v)
    u = np.linalg.eigh(np.eye(n) - sv[:, None] * chi[0] * sv[None, :])[1][:, n - nb:]
    pr = oracle.epsinv_projected(m, ev, ec, om, v, u)
    assert np.abs(pr - lr).max() < 1e-12 * np.abs(lr).max()
    # M_p = coefficients x a fixed nb-row basis / sqrt(v): chi0(w) has an nb-dim range
    basis = (rng.standard_normal((nb, n)) + 1j * rng.standard_normal((nb, n))) / sv[None, :]
    m2 = (rng.standard_normal((nv, nc, nb)) + 1j * rng.standard_normal((nv, nc, nb))) @ basis / 4
    chi2 = oracle.chi0(m2, ev, ec, om)
    u2 = np.linalg.eigh(np.eye(n) - sv[:, None] * chi2[0] * sv[None, :])[1][:, n - nb:]
    ex = oracle.epsilon_inverse(chi2, v)
    pr2 = oracle.epsinv_projected(m2, ev, ec, om, v, u2)
    assert np.abs(pr2 - ex).max() < 1e-10 * np.abs(ex).max()


def test_threaded_fft_route_equals_the_plain_one():
    """The threaded scipy FFT (the CPU baseline's setting) computes the same M."""
    s = synth.build_system(synth.CONFIGS["T4"])
    a = oracle.mtxel_fft(s["cv"][:2], s["gv"], s["cc"][:3], s["gc"], s["geps"], s["box"])
    b = oracle.mtxel_fft(s["cv"][:2], s["gv"], s["cc"][:3], s["gc"], s["geps"], s["box"],
                         workers=2)
    assert np.abs(a - b).max() <= 1e-14 * np.abs(a).max()
    ref = oracle.mtxel_convolution(s["cv"][:2], s["gv"], s["cc"][:3], s["gc"], s["geps"])
    assert np.abs(b - ref).max() <= 1e-13 * np.abs(ref).max()
