"""The stored oracle references under tests/golden/ (written by
tests/golden/make_golden.py from oracle/ and synth/ only) still describe the
current workloads and the current oracle: each file is found under the digest
of its workload's parameters, and the oracle reproduces every stored value.
A change to the oracle's arithmetic or to the input generator that moves a
value shows up here, and the files are then rewritten by the script."""
import os
import sys

import numpy as np
import pytest

import synth

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_golden  # noqa: E402


@pytest.mark.parametrize("name", sorted(make_golden.WORKLOADS))
def test_reference_file_is_keyed_by_the_workload(name):
    path = make_golden.path_for(name)
    assert os.path.exists(path), f"no stored reference for {name}: run tests/golden/make_golden.py"
    with open(path) as fh:
        head = fh.read(1024)
    assert f"digest {synth.config_digest(synth.CONFIGS[name])}" in head


@pytest.mark.parametrize("name", sorted(make_golden.WORKLOADS))
def test_oracle_reproduces_the_stored_values(name):
    ref = make_golden.read(make_golden.path_for(name))
    s, m, x, e = make_golden.reference(name)
    assert ref["shape"] == (m.shape[0], m.shape[1], len(s["geps"]), len(s["omega"]))
    mm = np.abs(m).max()
    for (v, c, g), z in ref["M"].items():
        assert abs(m[v, c, g] - z) <= 1e-13 * mm
    for kind, a in (("chi0", x), ("epsinv", e)):
        amax = np.abs(a).max()
        for (f, i, j), z in ref[kind].items():
            assert abs(a[f, i, j] - z) <= 1e-13 * amax, (kind, f, i, j)
        for f in range(a.shape[0]):
            assert np.isclose(np.linalg.norm(a[f]), ref["norm"][(kind, f)], rtol=1e-13, atol=0)


def test_reference_covers_diagonal_head_row_and_samples():
    ref = make_golden.read(make_golden.path_for("C1"))
    nv, nc, n, nf = ref["shape"]
    keys = set(ref["chi0"])
    assert all((0, i, i) in keys for i in range(n))
    assert all((0, 0, j) in keys for j in range(n))
    assert len(keys) == n + (n - 1) + make_golden.N_OFF
    assert len(ref["M"]) == make_golden.N_M
