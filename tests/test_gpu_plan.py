"""GPU parity of the batched many-q plan (one captured graph over every q)."""
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


def small_batch(omega_ev=(0.0, 2.0)):
    return synth.batch_systems(nq=5, seed=77, cell=(7.5, 7.75, 9.5), box=(16, 16, 16),
                               ecut_wfn=12.324, nv=4, nc_range=(8, 24), neps_range=(30, 80),
                               grid=2, omega_ev=omega_ev)


def oracle_q(s):
    nc = s["nc"]
    m = oracle.mtxel_convolution(s["cv"], s["gv"], s["cc"][:nc], s["gc"], s["geps"])
    x = oracle.chi0(m, s["ev"], s["ec"][:nc], s["omega"])
    return m, x, oracle.epsilon_inverse(x, s["vcoul"])


def run_plan(P, ctx, systems, dtype, prec):
    from paper_2206_00808_amd import pipeline
    from paper_2206_00808_amd.binding import Plan
    qs = pipeline.upload_batch(systems, dtype=dtype)
    dt = P.GW_C128 if dtype == "c128" else P.GW_C64
    plan = Plan(ctx, systems[0]["box"], 2, dt, prec, systems[0]["omega"], 1.0, qs)
    plan.compile()
    plan.launch()
    torch.cuda.synchronize()
    return plan, qs


def test_small_batch_fp64_matches_oracle(P, ctx):
    systems = small_batch()
    assert systems[0]["head_index"] >= 0
    plan, qs = run_plan(P, ctx, systems, "c128", P.GW_PREC_FP64)
    assert "tile" in plan.describe()
    for s, q in zip(systems, qs):
        _, x, e = oracle_q(s)
        for f in range(len(s["omega"])):
            assert oracle.rel_f(q["chi0"][f].cpu().numpy(), x[f]) < 1e-10
            assert oracle.rel_f(q["epsinv"][f].cpu().numpy(), e[f]) < 1e-10
    plan.close()


def test_small_batch_mixed_matches_oracle(P, ctx):
    systems = small_batch()
    plan, qs = run_plan(P, ctx, systems, "c64", P.GW_PREC_SPLITBF16)
    for s, q in zip(systems, qs):
        _, x, e = oracle_q(s)
        for f in range(len(s["omega"])):
            assert oracle.rel_f(q["chi0"][f].cpu().numpy(), x[f]) < 1e-4
            assert oracle.rel_f(q["epsinv"][f].cpu().numpy(), e[f]) < 1e-4
        if s["head_index"] >= 0:
            h = s["head_index"]
            for f in range(len(s["omega"])):
                got = q["chi0"][f][h, h].item()
                assert abs(got - x[f][h, h]) / abs(x[f][h, h]) < 1e-5
    plan.close()


def test_plan_equals_single_calls_and_replays_identically(P, ctx):
    from paper_2206_00808_amd import pipeline
    systems = small_batch()
    plan, qs = run_plan(P, ctx, systems, "c128", P.GW_PREC_FP64)
    first = [(q["chi0"].clone(), q["epsinv"].clone()) for q in qs]
    # eager work between replays
    for s, q in zip(systems, qs):
        d = pipeline.upload(dict(s, cc=s["cc"][:s["nc"]], ec=s["ec"][:s["nc"]]), dtype="c128")
        out = pipeline.alloc_outputs(d, with_head=True)
        pipeline.run_path(ctx, d, out)
        torch.cuda.synchronize()
        assert oracle.rel_f(q["chi0"].cpu().numpy(), out["chi0"].cpu().numpy()) < 1e-12
        assert oracle.rel_f(q["epsinv"].cpu().numpy(), out["epsinv"].cpu().numpy()) < 1e-12
    for _ in range(3):
        plan.launch()
        torch.cuda.synchronize()
        for q, (c0, e0) in zip(qs, first):
            assert torch.equal(q["chi0"], c0)
            assert torch.equal(q["epsinv"], e0)
    plan.close()


@pytest.mark.slow
def test_c4_full_batch_mixed(P, ctx):
    """The 64-q batch (mixed precision, one graph) against three references:
    the single-call path on every q (the same precision through gw_mtxel_spinor,
    gw_chi0_accumulate and gw_epsinv, whose parity with the oracle is tested
    elsewhere); the oracle on a 12 x 12 (G, G') block, the head included, for
    four q; and, for the same q, eps^-1 against LAPACK's FP64 inverse of the eps
    built from the plan's own chi0, element by element."""
    from paper_2206_00808_amd import pipeline
    systems = synth.batch_systems()
    assert len(systems) == 64
    plan, qs = run_plan(P, ctx, systems, "c64", P.GW_PREC_SPLITBF16)
    worst_chi, worst_inv = 0.0, 0.0
    for s, q in zip(systems, qs):
        d = pipeline.upload(dict(s, cc=s["cc"][:s["nc"]], ec=s["ec"][:s["nc"]]), dtype="c64")
        out = pipeline.alloc_outputs(d, with_head=True)
        pipeline.run_path(ctx, d, out, prec=P.GW_PREC_SPLITBF16)
        torch.cuda.synchronize()
        worst_chi = max(worst_chi, oracle.rel_f(q["chi0"].cpu().numpy(), out["chi0"].cpu().numpy()))
        worst_inv = max(worst_inv,
                        oracle.rel_f(q["epsinv"].cpu().numpy(), out["epsinv"].cpu().numpy()))
        del d, out
    print(f"C4 plan vs single calls (rel_F, worst q): chi0 {worst_chi:.2e}, eps^-1 {worst_inv:.2e}")
    # two split-BF16 contractions with different tiles and float chunks
    assert worst_chi < 1e-5 and worst_inv < 1e-5, (worst_chi, worst_inv)
    rng = np.random.default_rng(3)
    for iq in [0] + list(rng.choice(np.arange(1, 64), size=3, replace=False)):
        s, q = systems[iq], qs[iq]
        nc = s["nc"]
        neps = s["geps"].shape[0]
        sel = np.sort(rng.choice(neps, size=12, replace=False))
        if s["head_index"] >= 0 and s["head_index"] not in sel:
            sel[0] = s["head_index"]
            sel = np.sort(sel)
        msel = oracle.mtxel_convolution(s["cv"], s["gv"], s["cc"][:nc], s["gc"], s["geps"][sel])
        xref = oracle.chi0(msel, s["ev"], s["ec"][:nc], s["omega"])
        got = q["chi0"].cpu().numpy()[:, sel][:, :, sel]
        assert oracle.rel_f(got[0], xref[0]) < 1e-4
        assert np.abs(got[0] - xref[0]).max() < 1e-4 * np.abs(xref[0]).max()
        x = q["chi0"][0].cpu().numpy()
        einv = q["epsinv"][0].cpu().numpy()
        want = np.linalg.inv(np.eye(neps) - s["vcoul"][:, None] * x)
        assert np.abs(einv - want).max() < 1e-10 * np.abs(want).max()
    plan.close()
