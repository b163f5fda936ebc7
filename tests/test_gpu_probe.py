"""The device peak probes (gw_peak_probe) return plausible rates."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_peak_probes_are_plausible():
    import paper_2206_00808_amd as P
    ctx = P.Context(0)
    mfma, fma, copy = (P.gw_peak_probe(ctx, k) for k in (0, 1, 2))
    # nominal 78.6 TFLOP/s FP64 (matrix and vector) and 8 TB/s HBM
    assert 20.0 < mfma < 100.0
    assert 10.0 < fma < 100.0
    assert 1000.0 < copy < 9000.0
    with pytest.raises(P.GwError):
        P.gw_peak_probe(ctx, 3)
