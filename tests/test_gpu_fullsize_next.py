"""The rows beyond the Epsilon path at the full C2 sizes, in the launch shapes the
benchmark times, against the oracle on all outputs (unfolding, little-group
average, W) or on sampled bands and states (static SX, plasmon-pole Sigma)."""
import numpy as np
import pytest

import oracle
import synth
from synth.generate import g_sphere

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    import paper_2206_00808_amd as P
    return P


@pytest.fixture(scope="module")
def ctx(P):
    return P.Context(0)


@pytest.fixture(scope="module")
def c2():
    return synth.build_system(synth.CONFIGS["C2"])


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def test_unfold_full_size(P, ctx, c2):
    rot = np.diag([-1, -1, 1])
    tau = (0.0, 0.0, 0.5)
    cc = c2["cc"]
    out = torch.empty(cc.shape, dtype=torch.complex128, device="cuda:0")
    P.gw_unfold_spinor(ctx, 2, c2["gc"], _dev(cc), c2["gc"], rot, tau, c2["cell"], out)
    torch.cuda.synchronize()
    want = oracle.unfold_spinor(cc, c2["gc"], c2["gc"], rot, tau, c2["cell"])
    assert np.abs(out.cpu().numpy() - want).max() < 1e-15


def _random_epsinv(rng, n, v):
    m = (rng.standard_normal((60, n)) + 1j * rng.standard_normal((60, n))) * 0.03
    return oracle.epsilon_inverse((-(np.conj(m).T @ m))[None], v)[0]


def test_symmetrize_and_w_full_size(P, ctx, c2):
    rng = np.random.default_rng(12)
    n = len(c2["geps"])
    x = rng.standard_normal((9, n, n)) + 1j * rng.standard_normal((9, n, n))
    ops = [(np.diag(d), (0.0, 0.0, 0.0)) for d in ((1, 1, 1), (1, -1, -1), (1, -1, 1), (1, 1, -1))]
    dx = _dev(x)
    out = torch.empty_like(dx)
    P.gw_chi0_symmetrize(ctx, c2["geps"], c2["q"], ops, dx, out)
    w = torch.empty_like(dx)
    P.gw_screened_w(ctx, n, 9, dx, _dev(c2["vcoul"]), w)
    torch.cuda.synchronize()
    want = oracle.chi0_symmetrize(x, c2["geps"], ops, c2["q"])
    assert np.abs(out.cpu().numpy() - want).max() < 1e-14 * np.abs(want).max()
    assert np.array_equal(w.cpu().numpy(), oracle.screened_w(x, c2["vcoul"]))


def test_sigma_sx_full_size_sampled_bands(P, ctx, c2):
    rng = np.random.default_rng(13)
    nv, nc, n = 16, 800, len(c2["geps"])
    m = (rng.standard_normal((nv, nc, n)) + 1j * rng.standard_normal((nv, nc, n))) / np.sqrt(n)
    e = _random_epsinv(rng, n, c2["vcoul"])
    sig = torch.zeros(nc, dtype=torch.complex128, device="cuda:0")
    P.gw_sigma_sx(ctx, nv, nc, n, _dev(m), _dev(e), _dev(c2["vcoul"]), 0.5, sig)
    torch.cuda.synchronize()
    sel = [0, 1, 399, 799]
    want = oracle.sigma_sx_static(m[:, sel], e, c2["vcoul"], 0.5)
    got = sig.cpu().numpy()[sel]
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()


def test_sigma_gpp_full_size_sampled_states(P, ctx, c2):
    """N_eps = 1000 (63 x 16 tiles), 24 states n'' (16 occupied), 2 bands, 3 energies."""
    rng = np.random.default_rng(14)
    n = len(c2["geps"])
    nn, nocc, nband = 24, 16, 2
    e = _random_epsinv(rng, n, c2["vcoul"])
    rho = synth.charge_density(15, c2["cell"], c2["box"], nelec=16.0)
    amp = torch.empty((n, n), dtype=torch.complex128, device="cuda:0")
    wt = torch.empty_like(amp)
    P.gw_gpp_modes(ctx, c2["geps"], c2["cell"], c2["q"], _dev(rho), _dev(e), amp, wt)
    m = (rng.standard_normal((nn, nband, n)) + 1j * rng.standard_normal((nn, nband, n))) / n
    en = np.sort(rng.uniform(-0.3, 0.8, nn))
    energies = rng.uniform(-0.2, 0.5, (nband, 3))
    sx = torch.zeros((nband, 3), dtype=torch.complex128, device="cuda:0")
    coh = torch.zeros_like(sx)
    P.gw_sigma_gpp(ctx, nn, nocc, nband, n, _dev(m), _dev(en), _dev(c2["vcoul"]), amp, wt,
                   _dev(energies), 1.0, sx, coh)
    torch.cuda.synchronize()
    o2, wto, keep = oracle.gpp_modes(e, c2["geps"], c2["cell"], c2["q"], rho)
    a = amp.cpu().numpy()
    assert np.array_equal(a != 0, keep)
    want_a = np.where(keep, o2 / wto, 0.0)
    assert np.abs(a - want_a).max() < 1e-12 * np.abs(want_a).max()
    wsx, wcoh = oracle.sigma_gpp(m, en, nocc, c2["vcoul"], o2, wto, energies)
    for got, want in ((sx, wsx), (coh, wcoh)):
        assert np.abs(got.cpu().numpy() - want).max() < 1e-10 * np.abs(want).max()


def test_lowrank_full_size(P, ctx, c2):
    """N_eps = 1000 (block Jacobi), 100 eigenvectors, 3 frequencies:
    V^1/2 chi0(w) V^1/2 = -Q diag(l_i / (1 + a_i w)) Q^H with a random unitary Q, 100
    modes l in [1, 5] and 900 in [0, 0.1] (a clear gap, so the basis is unique),
    the same input on both sides."""
    rng = np.random.default_rng(16)
    n, nb = len(c2["geps"]), 100
    q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    lam0 = np.concatenate([rng.uniform(1.0, 5.0, nb), rng.uniform(0.0, 0.1, n - nb)])
    a = rng.uniform(0.2, 2.0, n)
    v = c2["vcoul"]
    sv = np.sqrt(v)
    chi = np.stack([-(q * (lam0 / (1.0 + a * w))[None, :]) @ q.conj().T / sv[:, None] / sv[None, :]
                    for w in (0.0, 0.5, 3.0)])
    out = torch.empty(chi.shape, dtype=torch.complex128, device="cuda:0")
    lam = torch.empty(n, dtype=torch.float64, device="cuda:0")
    P.gw_epsinv_lowrank(ctx, n, 3, _dev(chi), _dev(v), nb, out, lam)
    torch.cuda.synchronize()
    want, wlam = oracle.epsinv_lowrank(chi, v, nb)
    gap = (wlam[n - nb] - wlam[n - nb - 1]) / wlam[-1]
    assert gap > 0.1
    # block Jacobi: about 500 dense 32 x 32 unitary updates per entry; a backward
    # error of order N eps ||A|| (1.3e-10 here) bounds the eigenvalue error
    assert np.abs(lam.cpu().numpy() - wlam).max() < n * np.finfo(float).eps * wlam.max() * 100
    got = out.cpu().numpy()
    for f in range(3):
        assert oracle.rel_f(got[f], want[f]) < 1e-9
