"""GPU path against the stored oracle references under tests/golden/: the HIP
path through the C ABI on the seeded workload, compared with the values the
CPU FP64 oracle wrote there (no oracle call on the device's host): M_vc(q+G)
(Sec. II, Eq. (matrix_el)) at 1e-12, chi0 and eps^-1 (Sec. II) at 1e-10 in
FP64, and chi0 and eps^-1 at 1e-4 on the mixed path (complex64 transforms,
split-BF16 contraction, FP64 inverse), each relative to the largest stored
magnitude of its kind."""
import os
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_golden  # noqa: E402


@pytest.fixture(scope="module")
def P():
    import paper_2206_00808_amd as P
    return P


@pytest.fixture(scope="module")
def ctx(P):
    return P.Context(0)


def _run(P, ctx, name, dtype, prec):
    from paper_2206_00808_amd import pipeline
    s = synth.build_system(synth.CONFIGS[name])
    d = pipeline.upload(s, dtype=dtype)
    out = pipeline.alloc_outputs(d)
    pipeline.run_path(ctx, d, out, prec=prec)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}


def _worst(got, stored):
    """max |got - stored| over the stored entries, relative to the largest stored |value|."""
    top = max(abs(z) for z in stored.values())
    return max(abs(got[k] - z) for k, z in stored.items()) / top


@pytest.mark.parametrize("name", sorted(make_golden.WORKLOADS))
def test_fp64_path_matches_the_stored_reference(P, ctx, name):
    ref = make_golden.read(make_golden.path_for(name))
    out = _run(P, ctx, name, "c128", P.GW_PREC_FP64)
    assert _worst(out["mtxel"], ref["M"]) < 1e-12
    for kind, key in (("chi0", "chi0"), ("epsinv", "epsinv")):
        assert _worst(out[key], ref[kind]) < 1e-10, kind
        for f in range(out[key].shape[0]):
            assert np.isclose(np.linalg.norm(out[key][f]), ref["norm"][(kind, f)], rtol=1e-10)


@pytest.mark.parametrize("name", sorted(make_golden.WORKLOADS))
def test_mixed_path_matches_the_stored_reference(P, ctx, name):
    ref = make_golden.read(make_golden.path_for(name))
    out = _run(P, ctx, name, "c64", P.GW_PREC_SPLITBF16)
    assert _worst(out["mtxel"], ref["M"]) < 4e-6
    for kind in ("chi0", "epsinv"):
        assert _worst(out[kind], ref[kind]) < 1e-4, kind
