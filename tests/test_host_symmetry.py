"""The library's host bookkeeping for the symmetry row (gw_little_group,
gw_kgrid_orbits) against the oracle.  No device is needed: these entry points do
no GPU work and take no context."""
import numpy as np
import pytest

import oracle
from test_symmetry_pins import space_group


@pytest.fixture(scope="module")
def P():
    import paper_2206_00808_amd as P
    return P


@pytest.mark.parametrize("q", [(0.0, 0.0, 1 / 3), (0.25, 0.0, 0.0), (0.1, 0.2, 0.3),
                               (0.5, 0.5, 0.5), (0.0, 0.0, 0.0)])
def test_little_group_matches_oracle(P, q):
    ops = space_group()
    ing, gs = P.gw_little_group(ops, q)
    for j, (s, _) in enumerate(ops):
        want = oracle.little_group_shift(s, q)
        assert ing[j] == (want is not None)
        if want is not None:
            assert np.array_equal(gs[j], want)


@pytest.mark.parametrize("n,q", [((3, 3, 3), (0, 0, 1 / 3)), ((4, 4, 2), (0, 0, 0)),
                                 ((6, 6, 4), (0, 0, 0.25)), ((4, 4, 4), (0.25, 0.25, 0))])
def test_kgrid_orbits_match_oracle(P, n, q):
    ops = [op for op in space_group() if oracle.little_group_shift(op[0], q) is not None]
    rep, op, g0, w, nirr = P.gw_kgrid_orbits(n, ops)
    wrep, wop, wg0, ww = oracle.kgrid_orbits(n, ops)
    assert np.array_equal(rep, wrep) and np.array_equal(op, wop)
    assert np.array_equal(g0, wg0) and np.array_equal(w, ww)
    assert nirr == int((ww > 0).sum()) and w.sum() == np.prod(n)


def test_host_bookkeeping_rejects_bad_input(P):
    ops = space_group()
    with pytest.raises(P.GwError):  # C4 about z does not map a 4 x 3 x 2 grid onto itself
        P.gw_kgrid_orbits((4, 3, 2), ops)
    with pytest.raises(P.GwError):
        P.gw_little_group([np.array([[1, 1, 0], [0, 1, 1], [1, 0, 1]])], (0, 0, 0))
    with pytest.raises(P.GwError):
        P.gw_kgrid_orbits((0, 2, 2), ops)
