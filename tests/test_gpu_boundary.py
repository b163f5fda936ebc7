"""GPU checks of the C ABI's conventions: calls return before the device
finishes (host arrays are staged through the context's pinned ring, so the
caller may reuse them at once), and eps^-1 of a non-Hermitian chi0 whose
Gauss-Jordan pivots look Hermitian positive definite still goes through the
residual check."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    import paper_2206_00808_amd as P
    return P


@pytest.fixture(scope="module")
def ctx(P):
    return P.Context(0)


def test_mtxel_and_chi0_return_before_the_device_finishes(P, ctx):
    from paper_2206_00808_amd import pipeline
    s = synth.build_system(synth.CONFIGS["C2"])
    d = pipeline.upload(s, dtype="c128")
    out = pipeline.alloc_outputs(d)
    stages = ("mtxel", "chi0")
    pipeline.run_path(ctx, d, out, stages=stages)   # tables built, workspace grown
    torch.cuda.synchronize()
    first = out["chi0"].clone()
    m_first = out["mtxel"].clone()
    # C2 is several milliseconds of device work; the host calls take far less
    pipeline.run_path(ctx, d, out, stages=stages)
    pending = not torch.cuda.current_stream().query()
    torch.cuda.synchronize()
    assert pending, "the calls waited for the device"
    assert torch.equal(out["mtxel"], m_first)
    assert torch.equal(out["chi0"], first)


def test_staged_frequencies_may_be_overwritten_after_the_call(P, ctx):
    """Many chi0 calls, each with its own host frequency array that is
    overwritten as soon as the call returns: every result must use the
    frequencies the call was given."""
    s = synth.build_system(synth.CONFIGS["T1"])
    m = oracle.mtxel_convolution(s["cv"], s["gv"], s["cc"], s["gc"], s["geps"])
    nv, nc, neps = m.shape
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    dm, dev_v, dec = dev(m), dev(s["ev"]), dev(s["ec"])
    ncall = 300      # 300 staged copies of 256 bytes wrap the 64 KiB ring
    chi = torch.zeros((ncall, 2, neps, neps), dtype=torch.complex128, device="cuda:0")
    omegas = []
    buf = np.zeros(2)
    for k in range(ncall):
        buf[:] = (0.05 * k, 0.05 * k + 1.0)
        omegas.append(buf.copy())
        P.gw_chi0_accumulate(ctx, nv, nc, neps, dm, dev_v, dec, buf, 1.0, P.GW_PREC_FP64, chi[k])
        buf[:] = -1.0   # a reused host buffer: the library must have staged it
    torch.cuda.synchronize()
    got = chi.cpu().numpy()
    for k in (0, 1, 77, 150, ncall - 1):
        want = oracle.chi0(m, s["ev"], s["ec"], omegas[k])
        assert oracle.rel_f(got[k], want) < 1e-12


def _hermitian_nsd(rng, n, rank, scale):
    a = rng.standard_normal((n, rank)) + 1j * rng.standard_normal((n, rank))
    return -(a @ a.conj().T) * (scale / rank)


def test_non_hermitian_chi_with_passing_pivots_is_verified(P, ctx):
    rng = np.random.default_rng(8)
    n = 150
    v = rng.uniform(0.5, 2.0, n)
    h = _hermitian_nsd(rng, n, 40, 0.5)
    b = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    k = 1e-3 * (b + b.conj().T)                  # Hermitian
    chis = {"hermitian": h, "non_hermitian": h + 1j * k}   # chi^H != chi
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    for name, chi in chis.items():
        c = dev(chi[None])
        out = torch.empty_like(c)
        ctx.profile_reset()
        ctx.profile(True)
        P.gw_epsinv(ctx, n, 1, c, dev(v), out)
        tab = ctx.profile_table()
        ctx.profile(False)
        ctx.profile_reset()
        want = oracle.epsilon_inverse(chi[None], v)
        assert oracle.rel_f(out.cpu().numpy(), want) < 1e-10, name
        # the Hermitian matrix needs no residual check; the other one gets it
        assert ("eps_verify" in tab) == (name == "non_hermitian"), (name, sorted(tab))


def test_nan_coefficient_is_reported_by_epsinv(P, ctx):
    """Error injection: one NaN coefficient in a conduction band spreads through
    the matrix elements and chi0 (the calls do not read device data back), and
    gw_epsinv, which reads its flags, reports it as GW_EINVAL."""
    from paper_2206_00808_amd import pipeline
    s = synth.build_system(synth.CONFIGS["T1"])
    bad = dict(s, cc=s["cc"].copy())
    bad["cc"][3, 1, 7] = np.nan
    d = pipeline.upload(bad)
    out = pipeline.alloc_outputs(d)
    pipeline.run_path(ctx, d, out, stages=("mtxel", "chi0"))
    torch.cuda.synchronize()
    m = out["mtxel"].cpu().numpy()
    assert np.isnan(m[:, 3]).any() and np.isfinite(np.delete(m, 3, axis=1)).all()
    with pytest.raises(P.GwError) as ei:
        P.gw_epsinv(ctx, d["neps"], len(d["omega"]), out["chi0"], d["vcoul"], out["epsinv"])
    assert ei.value.status == P.GW_EINVAL
    # the context stays usable: the clean system goes through
    good = pipeline.upload(s)
    o2 = pipeline.alloc_outputs(good)
    pipeline.run_path(ctx, good, o2)
    torch.cuda.synchronize()
    mref = oracle.mtxel_convolution(s["cv"], s["gv"], s["cc"], s["gc"], s["geps"])
    x = oracle.chi0(mref, s["ev"], s["ec"], s["omega"])
    e = oracle.epsilon_inverse(x, s["vcoul"])
    assert oracle.rel_f(o2["epsinv"].cpu().numpy(), e) < 1e-10
