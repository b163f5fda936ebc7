"""Full-size parity at the workloads' own sizes, through the C ABI.

- Si-like system (48^3 box, N_v 16, N_c 800, N_eps 1000, 9 frequencies), FP64:
  every matrix element, chi0 at every frequency and eps^-1 against the oracle
  chain (plane-wave convolution -> chi0 -> LAPACK inverse), each with rel_F and
  a max-element bound.
- Layered-cell system (60 x 60 x 160 box, N_v 56, N_c 2000, N_eps 4000):
  FP64 matrix elements of sampled pairs against the convolution form; chi0 on
  index blocks that straddle the contraction's 64-wide tile boundaries against
  the oracle's chi0 of the same matrix elements; eps^-1 against LAPACK's
  inverse of the same chi0; the mixed path's chi0 and eps^-1 against the FP64
  path, within 1e-4.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    import paper_2206_00808_amd as P
    return P


@pytest.fixture(scope="module")
def ctx(P):
    return P.Context(0)


def _run(ctx, P, s, dtype, prec):
    from paper_2206_00808_amd import pipeline
    d = pipeline.upload(s, dtype=dtype)
    o = pipeline.alloc_outputs(d)
    pipeline.run_path(ctx, d, o, prec=prec)
    torch.cuda.synchronize()
    return d, o


def _errs(x, ref):
    rel = oracle.rel_f(x, ref)
    mx = float(np.abs(x - ref).max() / np.abs(ref).max())
    return rel, mx


def test_si_like_fp64_every_element(P, ctx):
    s = synth.build_system(synth.CONFIGS["C2"])
    d, o = _run(ctx, P, s, "c128", P.GW_PREC_FP64)
    m = oracle.mtxel_convolution(s["cv"], s["gv"], s["cc"], s["gc"], s["geps"])
    rel, mx = _errs(o["mtxel"].cpu().numpy(), m)
    print(f"C2 M: rel_F {rel:.2e} max {mx:.2e}")
    assert rel < 1e-12 and mx < 1e-12
    x = oracle.chi0(m, s["ev"], s["ec"], s["omega"])
    e = oracle.epsilon_inverse(x, s["vcoul"])
    gx, ge = o["chi0"].cpu().numpy(), o["epsinv"].cpu().numpy()
    for f in range(len(s["omega"])):
        rc, mc = _errs(gx[f], x[f])
        ri, mi = _errs(ge[f], e[f])
        print(f"C2 omega {f}: chi0 rel_F {rc:.2e} max {mc:.2e}; eps^-1 rel_F {ri:.2e} max {mi:.2e}")
        assert rc < 1e-10 and mc < 1e-10
        assert ri < 1e-10 and mi < 1e-10


@pytest.fixture(scope="module")
def layered(P, ctx):
    s = synth.build_system(synth.CONFIGS["C3"])
    d, o = _run(ctx, P, s, "c128", P.GW_PREC_FP64)
    out = {"sys": s, "chi0": o["chi0"].cpu().numpy(), "epsinv": o["epsinv"].cpu().numpy()}
    rng = np.random.default_rng(3)
    nv, nc = d["nv"], d["nc"]
    picks = [(0, 0), (nv - 1, nc - 1)] + [(int(rng.integers(nv)), int(rng.integers(nc)))
                                          for _ in range(6)]
    out["m_pairs"] = [(v, c, o["mtxel"][v, c].cpu().numpy()) for v, c in picks]
    # every pair's elements at G indices on both sides of 64-wide tile edges, and
    # at the sphere's extreme g_x, g_y and g_z (the outermost kept columns of the
    # xy-plane pass and the last kept z frequencies)
    ge = np.asarray(s["geps"])
    ext = [int(np.argmax(ge[:, a])) for a in range(3)] + [int(np.argmin(ge[:, a])) for a in range(3)]
    sel = np.unique(np.array([0, 1, 62, 63, 64, 65, 127, 128, 2047, 2048, 3967, 3968, 3999] + ext))
    out["sel"] = sel
    out["m_sel"] = o["mtxel"][:, :, sel].cpu().numpy()
    del o, d
    torch.cuda.empty_cache()
    return out


def test_layered_fp64_sampled_pairs(layered):
    s = layered["sys"]
    for v, c, got in layered["m_pairs"]:
        ref = oracle.mtxel_convolution(s["cv"][v:v + 1], s["gv"], s["cc"][c:c + 1], s["gc"],
                                       s["geps"])[0, 0]
        rel, mx = _errs(got, ref)
        assert rel < 1e-12 and mx < 1e-12, (v, c, rel, mx)


def test_layered_fp64_chi0_across_tile_edges(layered):
    s = layered["sys"]
    sel = layered["sel"]
    m = oracle.mtxel_convolution(s["cv"], s["gv"], s["cc"], s["gc"], s["geps"][sel])
    rel, mx = _errs(layered["m_sel"], m)
    assert rel < 1e-12 and mx < 1e-12
    x = oracle.chi0(m, s["ev"], s["ec"], s["omega"])
    got = layered["chi0"][:, sel][:, :, sel]
    rel, mx = _errs(got, x)
    print(f"C3 chi0 block: rel_F {rel:.2e} max {mx:.2e}")
    assert rel < 1e-10 and mx < 1e-10


def test_layered_fp64_epsinv_against_lapack(layered):
    s = layered["sys"]
    want = oracle.epsilon_inverse(layered["chi0"], s["vcoul"])
    rel, mx = _errs(layered["epsinv"], want)
    print(f"C3 eps^-1 vs LAPACK on the same chi0: rel_F {rel:.2e} max {mx:.2e}")
    assert rel < 1e-10 and mx < 1e-10


def test_layered_mixed_against_fp64(P, ctx, layered):
    s = layered["sys"]
    d, o = _run(ctx, P, s, "c64", P.GW_PREC_SPLITBF16)
    rc, mc = _errs(o["chi0"].cpu().numpy(), layered["chi0"])
    ri, mi = _errs(o["epsinv"].cpu().numpy(), layered["epsinv"])
    print(f"C3 mixed vs FP64: chi0 rel_F {rc:.2e} max {mc:.2e}; eps^-1 rel_F {ri:.2e} max {mi:.2e}")
    assert rc < 1e-4 and mc < 1e-4
    assert ri < 1e-4 and mi < 1e-4
