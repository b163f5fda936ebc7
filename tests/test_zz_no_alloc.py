"""gw_chi0_accumulate_noalloc (no allocation: its scratch is a fixed device
array of the library) against gw_chi0_accumulate on the same inputs, twice in a
row, the second call smaller than the first, through the C ABI."""
import ctypes as ct

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


def _noalloc(P, ctx, nv, nc, neps, m, ev, ec, omega, pref, chi, mhead=None, head=-1):
    lib = P.binding.raw()
    f = lib.gw_chi0_accumulate_noalloc
    vp, i, d = ct.c_void_p, ct.c_int, ct.c_double
    f.restype = i
    f.argtypes = [vp, i, i, i, vp, i, vp, vp, i, vp, d, vp, i, vp]
    om = np.ascontiguousarray(np.asarray(omega, dtype=np.float64))
    ctx.sync_stream()
    dt = P.GW_C128 if m.dtype == torch.complex128 else P.GW_C64
    ptr = lambda t: None if t is None else t.data_ptr()  # noqa: E731
    return f(ctx.handle, nv, nc, neps, ptr(m), dt, ptr(ev), ptr(ec), len(om), om.ctypes.data, pref,
             ptr(mhead), head, ptr(chi))


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_noalloc_matches_the_allocating_call_twice(P, dtype):
    ctx = P.Context(0)
    rng = np.random.default_rng(21)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")  # noqa: E731
    for nv, nc, neps, nf in ((12, 400, 333, 5), (5, 37, 70, 2)):   # second call smaller
        m = (rng.standard_normal((nv, nc, neps)) + 1j * rng.standard_normal((nv, nc, neps))) / 9
        ev = np.sort(rng.uniform(-0.3, 0.0, nv))
        ec = np.sort(rng.uniform(0.05, 0.7, nc))
        omega = np.linspace(0.0, 1.5, nf)
        dm = dev(m).to(dtype)
        a = torch.zeros((nf, neps, neps), dtype=torch.complex128, device="cuda:0")
        b = torch.zeros_like(a)
        P.gw_chi0_accumulate(ctx, nv, nc, neps, dm, dev(ev), dev(ec), omega, 0.7,
                             P.GW_PREC_FP64, a)
        st = _noalloc(P, ctx, nv, nc, neps, dm, dev(ev), dev(ec), omega, 0.7, b)
        assert st == P.GW_OK, P.binding.raw().gw_last_error(ctx.handle)
        torch.cuda.synchronize()
        an, bn = a.cpu().numpy(), b.cpu().numpy()
        for f in range(nf):
            assert oracle.rel_f(bn[f], an[f]) < 1e-12
        # and against the oracle itself
        x = oracle.chi0(dm.cpu().numpy().astype(np.complex128), ev, ec, omega, prefactor=0.7)
        for f in range(nf):
            assert oracle.rel_f(bn[f], x[f]) < 1e-10
    ctx.close()


def test_noalloc_head_and_wings(P):
    ctx = P.Context(0)
    s = synth.build_system(synth.CONFIGS["T1Q0"])
    from paper_2206_00808_amd import pipeline
    d = pipeline.upload(s)
    out = pipeline.alloc_outputs(d, with_head=True)
    pipeline.run_path(ctx, d, out, stages=("mtxel", "chi0"))
    b = torch.zeros_like(out["chi0"])
    st = _noalloc(P, ctx, d["nv"], d["nc"], d["neps"], out["mtxel"], d["ev"], d["ec"], d["omega"],
                  1.0, b, out["mhead"], d["head_index"])
    assert st == P.GW_OK
    torch.cuda.synchronize()
    assert oracle.rel_f(b.cpu().numpy(), out["chi0"].cpu().numpy()) < 1e-12
    ctx.close()


def test_noalloc_rejects_sizes_beyond_its_scratch(P):
    ctx = P.Context(0)
    nv, nc, neps = 64, 70000, 4      # 64 * 70000 doubles > 32 MiB
    m = torch.zeros((1,), dtype=torch.complex128, device="cuda:0")
    ev = torch.zeros(nv, dtype=torch.float64, device="cuda:0")
    ec = torch.zeros(nc, dtype=torch.float64, device="cuda:0")
    chi = torch.zeros((1, neps, neps), dtype=torch.complex128, device="cuda:0")
    st = _noalloc(P, ctx, nv, nc, neps, m, ev, ec, [0.0], 1.0, chi)
    assert st == P.GW_EINVAL
    st = _noalloc(P, ctx, 2, 3, neps, m, ev, ec, np.zeros(65), 1.0, chi)   # 65 frequencies
    assert st == P.GW_EINVAL
    torch.cuda.synchronize()
    assert torch.count_nonzero(chi) == 0
    ctx.close()
