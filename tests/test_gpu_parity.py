"""GPU parity: the HIP path through the C ABI against the CPU FP64 oracle.

Small systems are compared element by element; the full-size workloads are
checked on outputs the oracle can compute one by one (sampled pairs, sampled
(G, G') blocks) and on properties that hold at any size.
"""
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


def _sys(name):
    return synth.build_system(synth.CONFIGS[name])


def _run(P, ctx, s, dtype="c128", prec=None, with_head=False, nc=None):
    from paper_2206_00808_amd import pipeline
    prec = P.GW_PREC_FP64 if prec is None else prec
    d = pipeline.upload(s, dtype=dtype, nc=nc)
    out = pipeline.alloc_outputs(d, with_head=with_head)
    pipeline.run_path(ctx, d, out, prec=prec)
    torch.cuda.synchronize()
    return d, {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}


def _max_rel(x, ref):
    return float(np.abs(x - ref).max() / np.abs(ref).max())


# ----------------------------------------------------------------- matrix elements
@pytest.mark.parametrize("name", ["C1", "T1", "T2", "T3", "T4"])
def test_mtxel_fp64_matches_definition(P, ctx, name):
    s = _sys(name)
    _, out = _run(P, ctx, s)
    ref = oracle.mtxel_convolution(s["cv"], s["gv"], s["cc"], s["gc"], s["geps"])
    assert _max_rel(out["mtxel"], ref) < 1e-12


@pytest.mark.parametrize("name", ["C1", "T2", "T3", "T4"])
def test_mtxel_fp32_matches_definition(P, ctx, name):
    s = _sys(name)
    _, out = _run(P, ctx, s, dtype="c64", prec=P.GW_PREC_SPLITBF16)
    ref = oracle.mtxel_convolution(s["cv"], s["gv"], s["cc"], s["gc"], s["geps"])
    assert _max_rel(out["mtxel"], ref) < 2e-6


@pytest.mark.parametrize("name", ["T2", "T4"])
def test_single_plane_wave_pairs_give_deltas(P, ctx, name):
    s = _sys(name)
    gv, gc, geps = s["gv"], s["gc"], s["geps"]
    cv = np.zeros((2, 2, len(gv)), complex)
    cc = np.zeros((3, 2, len(gc)), complex)
    cv[0, 0, 4] = 1.0
    cv[1, 1, 9] = 1.0
    cc[0, 0, 2] = 1.0
    cc[1, 1, 2] = 1.0
    cc[2, 0, 7] = 1.0
    t = dict(s, cv=cv, cc=cc, ev=s["ev"][:2], ec=s["ec"][:3])
    _, out = _run(P, ctx, t)
    want = np.zeros((2, 3, len(geps)), complex)
    for v, (sv, iv) in enumerate([(0, 4), (1, 9)]):
        for c, (sc, ic) in enumerate([(0, 2), (1, 2), (0, 7)]):
            if sv == sc:
                hit = np.where((geps == gv[iv] - gc[ic]).all(axis=1))[0]
                want[v, c, hit] = 1.0
    assert np.abs(out["mtxel"] - want).max() < 1e-14


@pytest.mark.parametrize("name", ["T1", "T4"])
def test_zero_down_equals_spinless(P, ctx, name):
    s = _sys(name)
    z = dict(s, cv=s["cv"].copy(), cc=s["cc"].copy())
    z["cv"][:, 1] = 0
    z["cc"][:, 1] = 0
    one = dict(s, cv=np.ascontiguousarray(s["cv"][:, :1]), cc=np.ascontiguousarray(s["cc"][:, :1]))
    _, o2 = _run(P, ctx, z)
    _, o1 = _run(P, ctx, one)
    assert np.abs(o2["mtxel"] - o1["mtxel"]).max() < 1e-15
    assert np.abs(o2["chi0"] - o1["chi0"]).max() <= 1e-14 * np.abs(o1["chi0"]).max()


def test_orthonormal_head_vanishes_at_q0(P, ctx):
    s = _sys("T1Q0")
    # replace the q0 valence by states of the same orthonormal set as the conduction
    rng = np.random.default_rng(5)
    from synth.generate import _random_spinors, g_sphere
    cell = tuple(s["cell"])
    gk = s["gc"]
    geps = g_sphere(cell, (0, 0, 0), 3.367)
    joint = _random_spinors(rng, len(gk), 10, 2)
    t = dict(s, cv=joint[:3], gv=gk, cc=joint[3:], geps=geps, ev=s["ev"][:3], ec=s["ec"][:7],
             vcoul=np.ones(len(geps)), head_index=-1)
    _, out = _run(P, ctx, t)
    i0 = np.where((geps == 0).all(axis=1))[0][0]
    assert np.abs(out["mtxel"][:, :, i0]).max() < 1e-14


# ----------------------------------------------------------------- chi0 and eps^-1, FP64
@pytest.mark.parametrize("name", ["C1", "T1", "T2", "T3", "T4"])
def test_chi0_and_epsinv_fp64(P, ctx, name):
    s = _sys(name)
    _, out = _run(P, ctx, s)
    m = oracle.mtxel_convolution(s["cv"], s["gv"], s["cc"], s["gc"], s["geps"])
    x = oracle.chi0(m, s["ev"], s["ec"], s["omega"])
    e = oracle.epsilon_inverse(x, s["vcoul"])
    for f in range(len(s["omega"])):
        assert oracle.rel_f(out["chi0"][f], x[f]) < 1e-10
        assert oracle.rel_f(out["epsinv"][f], e[f]) < 1e-10
        assert _max_rel(out["chi0"][f], x[f]) < 1e-10
        assert _max_rel(out["epsinv"][f], e[f]) < 1e-10
    # Hermitian by construction (mirrored tiles)
    c = out["chi0"]
    assert np.abs(c - np.conj(np.transpose(c, (0, 2, 1)))).max() <= 1e-15 * np.abs(c).max()


def test_chi0_accumulates_in_chunks(P, ctx):
    from paper_2206_00808_amd import pipeline
    s = _sys("T1")
    d = pipeline.upload(s)
    out = pipeline.alloc_outputs(d)
    pipeline.run_path(ctx, d, out, stages=("mtxel", "chi0"))
    full = out["chi0"].clone()
    m = out["mtxel"]
    acc = torch.zeros_like(full)
    half = d["nc"] // 2
    for lo, hi in ((0, half), (half, d["nc"])):
        part = m[:, lo:hi].contiguous()
        P.gw_chi0_accumulate(ctx, d["nv"], hi - lo, d["neps"], part, d["ev"], d["ec"][lo:hi].contiguous(),
                             d["omega"], 1.0, P.GW_PREC_FP64, acc)
    torch.cuda.synchronize()
    assert oracle.rel_f(acc.cpu().numpy(), full.cpu().numpy()) < 1e-14


def _split_case(seed, dtype):
    """Random matrix elements large enough that the library cuts the pair sum
    into ranges on a full device (12 frequencies x 55 upper tiles, 3200 pairs)."""
    rng = np.random.default_rng(seed)
    nv, nc, neps, nf = 16, 200, 600, 12
    m = (rng.standard_normal((nv, nc, neps)) + 1j * rng.standard_normal((nv, nc, neps))) / np.sqrt(2)
    m = m.astype(dtype)
    ev = rng.uniform(-0.44, 0.0, nv)
    ec = rng.uniform(0.07, 1.5, nc)
    omega = np.concatenate([[0.0], np.geomspace(0.02, 3.0, nf - 1)])
    mh = (rng.standard_normal(nv * nc) + 1j * rng.standard_normal(nv * nc)) / np.sqrt(2)
    return m, ev, ec, omega, mh


@pytest.mark.parametrize("prec", ["fp64", "splitbf16"])
def test_chi0_pair_ranges_and_wings_match_oracle(P, ctx, prec):
    """Pair-sum ranges, their ordered reduction and the head/wings on top: the
    wings are the contraction with column h of M replaced by the head overlaps."""
    dt = np.complex128 if prec == "fp64" else np.complex64
    m, ev, ec, omega, mh = _split_case(4242, dt)
    nv, nc, neps = m.shape
    h = 7
    mx = m.astype(np.complex128).copy()
    mx[:, :, h] = mh.reshape(nv, nc)
    x = oracle.chi0(mx, ev, ec, omega)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    chi = torch.zeros((len(omega), neps, neps), dtype=torch.complex128, device="cuda:0")
    code = P.GW_PREC_FP64 if prec == "fp64" else P.GW_PREC_SPLITBF16
    P.gw_chi0_accumulate(ctx, nv, nc, neps, dev(m), dev(ev), dev(ec), omega, 1.0, code, chi,
                         mhead=dev(mh), head_index=h)
    torch.cuda.synchronize()
    got = chi.cpu().numpy()
    tol = 1e-12 if prec == "fp64" else 1e-4
    for f in range(len(omega)):
        assert oracle.rel_f(got[f], x[f]) < tol, (prec, f)
        # head row and column come from the FP64 wing sums in both precisions
        assert np.abs(got[f][h] - x[f][h]).max() <= 1e-12 * np.abs(x[f][h]).max(), (prec, f)


@pytest.mark.parametrize("prec", ["fp64", "splitbf16"])
@pytest.mark.parametrize("shape", [(1, 3, 5), (3, 37, 70), (5, 41, 129), (2, 17, 64)])
def test_chi0_ragged_sizes_match_oracle(P, ctx, prec, shape):
    """Pair counts that are not a multiple of the 16/32-pair slabs and sphere sizes
    that are not a multiple of the 64-wide tile (including a sphere smaller than
    one tile and fewer pairs than one slab): the clamped rows and the zero weights
    past the last pair must leave exactly the oracle's sum."""
    nv, nc, neps = shape
    rng = np.random.default_rng(100 + nv * 1000 + nc + neps)
    dt = np.complex128 if prec == "fp64" else np.complex64
    m = ((rng.standard_normal((nv, nc, neps)) + 1j * rng.standard_normal((nv, nc, neps)))
         / np.sqrt(2)).astype(dt)
    ev = rng.uniform(-0.44, 0.0, nv)
    ec = rng.uniform(0.07, 1.5, nc)
    omega = np.array([0.0, 0.3])
    x = oracle.chi0(m.astype(np.complex128), ev, ec, omega)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    chi = torch.zeros((len(omega), neps, neps), dtype=torch.complex128, device="cuda:0")
    code = P.GW_PREC_FP64 if prec == "fp64" else P.GW_PREC_SPLITBF16
    P.gw_chi0_accumulate(ctx, nv, nc, neps, dev(m), dev(ev), dev(ec), omega, 1.0, code, chi)
    torch.cuda.synchronize()
    got = chi.cpu().numpy()
    tol = 1e-12 if prec == "fp64" else 1e-4
    for f in range(len(omega)):
        assert oracle.rel_f(got[f], x[f]) < tol, (prec, shape, f)


# ----------------------------------------------------------------- q -> 0 head from momenta
@pytest.mark.parametrize("dtype", [np.complex128, np.complex64])
def test_head_dipole_matches_oracle(P, ctx, dtype):
    from synth.generate import _random_spinors, g_sphere
    rng = np.random.default_rng(17)
    cell = (5.0, 5.3, 5.7)
    g = g_sphere(cell, (0, 0, 0), 9.0)
    nv, nc = 5, 11
    cv = _random_spinors(rng, len(g), nv, 2).astype(dtype)
    cc = _random_spinors(rng, len(g), nc, 2).astype(dtype)
    ev = np.sort(rng.uniform(-0.4, -0.01, nv))
    ec = np.sort(rng.uniform(0.02, 0.9, nc))
    k = (0.25, 0.0, -0.25)
    q = np.array([1.0e-3, -0.4e-3, 0.7e-3])
    want = oracle.head_dipole(cv.astype(np.complex128), cc.astype(np.complex128), g, cell, k, q,
                              ev, ec).ravel()
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    mh = torch.empty(nv * nc, dtype=torch.complex128, device="cuda:0")
    P.gw_head_dipole(ctx, 2, g, dev(cv), dev(cc), cell, k, q, dev(ev), dev(ec), mh)
    torch.cuda.synchronize()
    assert oracle.rel_f(mh.cpu().numpy(), want) < 1e-12


def test_head_dipole_feeds_the_chi0_head_and_wings(P, ctx):
    """The dipole head as gw_chi0_accumulate's mhead: the head row and column of chi0
    are the contraction with column h of M replaced by it."""
    from synth.generate import _random_spinors, g_sphere
    rng = np.random.default_rng(23)
    cell = (5.0, 5.3, 5.7)
    g = g_sphere(cell, (0, 0, 0), 9.0)
    nv, nc, neps, h = 4, 9, 90, 0
    cv = _random_spinors(rng, len(g), nv, 2)
    cc = _random_spinors(rng, len(g), nc, 2)
    ev = np.sort(rng.uniform(-0.4, -0.01, nv))
    ec = np.sort(rng.uniform(0.02, 0.9, nc))
    q = np.array([0.0, 2e-3, 0.0])
    m = (rng.standard_normal((nv, nc, neps)) + 1j * rng.standard_normal((nv, nc, neps))) / 3
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    mh = torch.empty(nv * nc, dtype=torch.complex128, device="cuda:0")
    P.gw_head_dipole(ctx, 2, g, dev(cv), dev(cc), cell, (0, 0, 0), q, dev(ev), dev(ec), mh)
    omega = [0.0, 0.5]
    chi = torch.zeros((2, neps, neps), dtype=torch.complex128, device="cuda:0")
    P.gw_chi0_accumulate(ctx, nv, nc, neps, dev(m), dev(ev), dev(ec), omega, 1.0,
                         P.GW_PREC_FP64, chi, mhead=mh, head_index=h)
    torch.cuda.synchronize()
    mx = m.copy()
    mx[:, :, h] = oracle.head_dipole(cv, cc, g, cell, (0, 0, 0), q, ev, ec)
    x = oracle.chi0(mx, ev, ec, omega)
    got = chi.cpu().numpy()
    for f in range(2):
        assert oracle.rel_f(got[f], x[f]) < 1e-12
        assert np.abs(got[f][h] - x[f][h]).max() <= 1e-12 * np.abs(x[f][h]).max()


# ----------------------------------------------------------------- real frequency axis
@pytest.mark.parametrize("prec", ["fp64", "splitbf16"])
@pytest.mark.parametrize("shape", [(3, 37, 70), (16, 50, 200)])
def test_chi0_real_axis_matches_oracle(P, ctx, prec, shape):
    """Real-frequency chi0 with broadening (the Sec. II bracket with complex
    weights) against the oracle: non-Hermitian result, frequencies of both signs
    and one on a pole region, accumulated on top of an existing chi0."""
    nv, nc, neps = shape
    rng = np.random.default_rng(300 + nv + nc + neps)
    dt = np.complex128 if prec == "fp64" else np.complex64
    m = ((rng.standard_normal((nv, nc, neps)) + 1j * rng.standard_normal((nv, nc, neps)))
         / np.sqrt(2)).astype(dt)
    ev = rng.uniform(-0.44, 0.0, nv)
    ec = rng.uniform(0.07, 1.5, nc)
    omega = np.array([0.0, 0.35, -0.35, 0.9])
    eta = 0.02
    base = (rng.standard_normal((len(omega), neps, neps))
            + 1j * rng.standard_normal((len(omega), neps, neps)))
    want = base + oracle.chi0_real(m.astype(np.complex128), ev, ec, omega, eta, prefactor=0.5)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    chi = dev(base)
    code = P.GW_PREC_FP64 if prec == "fp64" else P.GW_PREC_SPLITBF16
    P.gw_chi0_accumulate_real(ctx, nv, nc, neps, dev(m), dev(ev), dev(ec), omega, eta, 0.5, code,
                              chi)
    torch.cuda.synchronize()
    got = chi.cpu().numpy()
    tol = 1e-12 if prec == "fp64" else 1e-4
    for f in range(len(omega)):
        assert oracle.rel_f(got[f] - base[f], want[f] - base[f]) < tol, (prec, shape, f)
    # the update is not Hermitian; its anti-Hermitian part is i times the
    # contraction with Im b, which is negative on the diagonal (absorption)
    upd = got[1] - base[1]
    assert np.abs(upd - upd.conj().T).max() > 1e-3 * np.abs(upd).max()
    assert np.all(np.diag(upd).imag < 0)


def test_chi0_real_axis_from_pipeline_and_lu_inverse(P, ctx):
    """The whole real-axis path on a synthetic system: matrix elements from the
    library, chi0 on the real axis, eps^-1 by the pivoted LU entry point, against
    the oracle's chi0_real and numpy's inverse of the non-Hermitian eps."""
    s = _sys("T1")
    from paper_2206_00808_amd import pipeline
    d = pipeline.upload(s)
    out = pipeline.alloc_outputs(d)
    pipeline.run_path(ctx, d, out, stages=("mtxel",))
    m = out["mtxel"]
    omega = np.array([0.0, 0.2, 0.5])
    eta = 0.01
    neps = d["neps"]
    chi = torch.zeros((len(omega), neps, neps), dtype=torch.complex128, device="cuda:0")
    P.gw_chi0_accumulate_real(ctx, d["nv"], d["nc"], neps, m, d["ev"], d["ec"], omega, eta, 1.0,
                              P.GW_PREC_FP64, chi)
    einv = torch.empty_like(chi)
    P.gw_epsinv_lu(ctx, neps, len(omega), chi, d["vcoul"], einv)
    # the default entry point: eps~ is not >= I on the real axis, so the
    # Gauss-Jordan result goes through the residual check; for this well-conditioned
    # eps it is kept, and the LU path does not run
    einv2 = torch.empty_like(chi)
    ctx.profile(True)
    ctx.profile_reset()
    P.gw_epsinv(ctx, neps, len(omega), chi, d["vcoul"], einv2)
    torch.cuda.synchronize()
    names = set(ctx.profile_table())
    ctx.profile(False)
    assert "eps_verify" in names and "lu_panel" not in names, names
    mh = m.cpu().numpy().reshape(d["nv"], d["nc"], neps)
    x = oracle.chi0_real(mh, d["ev"].cpu().numpy(), d["ec"].cpu().numpy(), omega, eta)
    e = oracle.epsilon_inverse(x, d["vcoul"].cpu().numpy())
    for f in range(len(omega)):
        assert oracle.rel_f(chi[f].cpu().numpy(), x[f]) < 1e-12
        assert oracle.rel_f(einv[f].cpu().numpy(), e[f]) < 1e-10
        assert oracle.rel_f(einv2[f].cpu().numpy(), e[f]) < 1e-10


def test_chi0_real_axis_rejects_bad_arguments(P, ctx):
    m = torch.zeros((2, 3, 4), dtype=torch.complex128, device="cuda")
    ev = torch.zeros(2, dtype=torch.float64, device="cuda")
    ec = torch.ones(3, dtype=torch.float64, device="cuda")
    chi = torch.zeros((1, 4, 4), dtype=torch.complex128, device="cuda")
    for eta in (0.0, -1.0, float("nan")):
        with pytest.raises(P.GwError) as ei:
            P.gw_chi0_accumulate_real(ctx, 2, 3, 4, m, ev, ec, [0.1], eta, 1.0, P.GW_PREC_FP64, chi)
        assert ei.value.status == P.GW_EINVAL
    with pytest.raises(P.GwError) as ei:
        P.gw_chi0_accumulate_real(ctx, 2, 3, 4, m, ev, ec, [float("inf")], 0.1, 1.0,
                                  P.GW_PREC_FP64, chi)
    assert ei.value.status == P.GW_EINVAL
    torch.cuda.synchronize()
    assert torch.count_nonzero(chi) == 0


# ----------------------------------------------------------------- mixed precision
@pytest.mark.parametrize("name", ["C1", "T1", "T2", "T3", "T4"])
def test_mixed_path_within_1e4(P, ctx, name):
    s = _sys(name)
    _, out = _run(P, ctx, s, dtype="c64", prec=P.GW_PREC_SPLITBF16)
    m = oracle.mtxel_convolution(s["cv"], s["gv"], s["cc"], s["gc"], s["geps"])
    x = oracle.chi0(m, s["ev"], s["ec"], s["omega"])
    e = oracle.epsilon_inverse(x, s["vcoul"])
    for f in range(len(s["omega"])):
        assert oracle.rel_f(out["chi0"][f], x[f]) < 1e-4
        assert oracle.rel_f(out["epsinv"][f], e[f]) < 1e-4
        assert _max_rel(out["chi0"][f], x[f]) < 1e-4
        assert _max_rel(out["epsinv"][f], e[f]) < 1e-4


def test_mixed_head_wings_in_fp64(P, ctx):
    s = _sys("T1Q0")
    h = s["head_index"]
    m = oracle.mtxel_convolution(s["cv"], s["gv"], s["cc"], s["gc"], s["geps"])
    x = oracle.chi0(m, s["ev"], s["ec"], s["omega"])
    e = oracle.epsilon_inverse(x, s["vcoul"])
    _, out = _run(P, ctx, s, dtype="c64", prec=P.GW_PREC_SPLITBF16, with_head=True)
    mh = oracle.head_overlap(s["cv"], s["gv"], s["cc"], s["gc"]).reshape(-1)
    # float coefficients summed in double: |dM| <= 2^-23 ||c_v|| ||c_c|| = 2^-23 (unit spinors)
    assert np.abs(out["mhead"] - mh).max() < 2.0 ** -23
    for f in range(len(s["omega"])):
        assert abs(out["chi0"][f][h, h] - x[f][h, h]) / abs(x[f][h, h]) < 1e-5
        assert oracle.rel_f(out["epsinv"][f], e[f]) < 1e-4
    # FP64 path with the FP64 head: identical math, tight bound
    _, o64 = _run(P, ctx, s, with_head=True)
    for f in range(len(s["omega"])):
        assert oracle.rel_f(o64["chi0"][f], x[f]) < 1e-10
        assert oracle.rel_f(o64["epsinv"][f], e[f]) < 1e-10


# ----------------------------------------------------------------- error paths
def test_alias_box_rejected(P, ctx):
    s = _sys("C1")
    from paper_2206_00808_amd import pipeline
    d = pipeline.upload(s)
    out = pipeline.alloc_outputs(d)
    before = out["mtxel"].clone()
    with pytest.raises(P.GwError) as ei:
        P.gw_mtxel_spinor(ctx, (12, 12, 12), 2, d["gv"], d["cv"], d["gc"], d["cc"], d["geps"],
                          out["mtxel"])
    assert ei.value.status == P.GW_EALIAS
    torch.cuda.synchronize()
    assert torch.equal(before, out["mtxel"])
    with pytest.raises(P.GwError) as ei:
        P.gw_mtxel_spinor(ctx, (16, 16, 7), 2, d["gv"], d["cv"], d["gc"], d["cc"], d["geps"],
                          out["mtxel"])
    assert ei.value.status == P.GW_EINVAL


@pytest.mark.parametrize("n,kind", [(n, "definite") for n in (1, 63, 64, 65, 129, 200, 2048, 2113)]
                         + [(n, "indefinite") for n in (65, 129)])
def test_epsinv_block_counts_match_oracle(P, ctx, n, kind):
    """eps^-1 at sizes around the 64-wide Gauss-Jordan blocks (one block, a ragged
    last block, the look-ahead block skipped by the rank update), three
    frequencies at once; from N = 2048 (whole blocks, and a last block of one
    column) the rank update stages its panels in LDS. 'definite' is chi0 <= 0 (the Gauss-Jordan path); in
    'indefinite' one frequency has chi0 with eigenvalues above 1/v, so eps~ is not
    positive definite and the call must take the pivoted LU path."""
    rng = np.random.default_rng(7 * n + (kind == "indefinite"))
    nf = 3
    v = rng.uniform(0.5, 3.0, n)
    chi = np.empty((nf, n, n), dtype=np.complex128)
    for f in range(nf):
        x = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2 * n)
        chi[f] = -(x @ x.conj().T) * (0.3 + f)
    if kind == "indefinite":
        # a Hermitian chi0 with eigenvalues of both signs and size well above 1/v
        y = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2 * n)
        chi[1] = (y + y.conj().T) * 2.0 + 1.5 * np.eye(n)
    want = oracle.epsilon_inverse(chi, v)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    out = torch.empty((nf, n, n), dtype=torch.complex128, device="cuda:0")
    P.gw_epsinv(ctx, n, nf, dev(chi), dev(v), out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for f in range(nf):
        assert oracle.rel_f(got[f], want[f]) < 1e-10, (n, kind, f)


def test_singular_eps_reported(P, ctx):
    n = 70
    chi = torch.eye(n, dtype=torch.complex128, device="cuda").reshape(1, n, n).contiguous()
    v = torch.ones(n, dtype=torch.float64, device="cuda")
    out = torch.empty_like(chi)
    with pytest.raises(P.GwError) as ei:
        P.gw_epsinv(ctx, n, 1, chi, v, out)
    assert ei.value.status == P.GW_ESINGULAR
    # the flag is cleared for the next call
    chi2 = torch.zeros_like(chi)
    P.gw_epsinv(ctx, n, 1, chi2, v, out)
    torch.cuda.synchronize()
    assert torch.allclose(out[0], torch.eye(n, dtype=torch.complex128, device="cuda"))


def test_empty_inputs_are_noops(P, ctx):
    chi = torch.zeros((1, 5, 5), dtype=torch.complex128, device="cuda")
    m = torch.zeros((0, 3, 5), dtype=torch.complex128, device="cuda")
    ev = torch.zeros(0, dtype=torch.float64, device="cuda")
    ec = torch.zeros(3, dtype=torch.float64, device="cuda")
    P.gw_chi0_accumulate(ctx, 0, 3, 5, m, ev, ec, [0.0], 1.0, P.GW_PREC_FP64, chi)
    torch.cuda.synchronize()
    assert torch.count_nonzero(chi) == 0


# ----------------------------------------------------------------- full-size workloads
def _sampled_checks(P, ctx, name, dtype, prec, tol_m, tol_chi, tol_inv, seed=0):
    s = _sys(name)
    d, out = None, None
    from paper_2206_00808_amd import pipeline
    d = pipeline.upload(s, dtype=dtype)
    o = pipeline.alloc_outputs(d)
    pipeline.run_path(ctx, d, o, prec=prec)
    torch.cuda.synchronize()
    rng = np.random.default_rng(seed)
    nv, nc, neps = d["nv"], d["nc"], d["neps"]
    # sampled pairs, all G
    for _ in range(6):
        v, c = int(rng.integers(nv)), int(rng.integers(nc))
        ref = oracle.mtxel_convolution(s["cv"][v:v + 1], s["gv"], s["cc"][c:c + 1], s["gc"],
                                       s["geps"])[0, 0]
        got = o["mtxel"][v, c].cpu().numpy()
        assert np.abs(got - ref).max() / np.abs(ref).max() < tol_m
    # sampled (G, G') block over every pair
    sel = np.sort(rng.choice(neps, size=6, replace=False))
    sel[0] = 0
    msel = oracle.mtxel_convolution(s["cv"], s["gv"], s["cc"], s["gc"], s["geps"][sel])
    xref = oracle.chi0(msel, s["ev"], s["ec"], s["omega"])
    got = o["chi0"].cpu().numpy()[:, sel][:, :, sel]
    for f in range(len(s["omega"])):
        assert oracle.rel_f(got[f], xref[f]) < tol_chi
    # eps^-1 against the property eps(chi0) eps^-1 = I
    x = o["chi0"].cpu().numpy()
    einv = o["epsinv"].cpu().numpy()
    for f in range(len(s["omega"])):
        eps = np.eye(neps) - s["vcoul"][:, None] * x[f]
        r = eps @ einv[f] - np.eye(neps)
        assert np.linalg.norm(r) / np.sqrt(neps) < tol_inv


@pytest.mark.slow
def test_c3_full_size_mixed(P, ctx):
    _sampled_checks(P, ctx, "C3", "c64", P.GW_PREC_SPLITBF16, 2e-6, 1e-4, 1e-6)


# ----------------------------------------------------------------- consumers of eps^-1
def _rand_c(rng, shape, dtype=np.complex128):
    return ((rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / 3).astype(dtype)


@pytest.mark.parametrize("inplace", [False, True])
def test_screened_w_matches_oracle(P, ctx, inplace):
    rng = np.random.default_rng(41)
    nfreq, neps = 3, 137
    e = _rand_c(rng, (nfreq, neps, neps))
    v = rng.uniform(0.01, 20.0, neps)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    de = dev(e)
    w = de if inplace else torch.empty_like(de)
    P.gw_screened_w(ctx, neps, nfreq, de, dev(v), w)
    torch.cuda.synchronize()
    # one product per element, correctly rounded on both sides
    assert np.array_equal(w.cpu().numpy(), oracle.screened_w(e, v))


@pytest.mark.parametrize("dtype,nocc,nband,neps", [
    (np.complex128, 5, 13, 200), (np.complex128, 1, 1, 1), (np.complex128, 3, 70, 64),
    (np.complex64, 4, 9, 129)])
def test_sigma_sx_matches_oracle(P, ctx, dtype, nocc, nband, neps):
    rng = np.random.default_rng(nocc * 1000 + neps)
    m = _rand_c(rng, (nocc, nband, neps), dtype)
    a = _rand_c(rng, (neps, neps))
    e = np.eye(neps) + 0.2 * (a + a.conj().T) / np.sqrt(neps)
    v = rng.uniform(0.01, 20.0, neps)
    s0 = _rand_c(rng, nband)
    pref = 0.37
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")
    sig = dev(s0)
    P.gw_sigma_sx(ctx, nocc, nband, neps, dev(m), dev(e), dev(v), pref, sig)
    torch.cuda.synchronize()
    want = s0 + oracle.sigma_sx_static(m.astype(np.complex128), e, v, pref)
    # widened inputs, FP64 arithmetic on both sides: only the summation order differs
    assert oracle.rel_f(sig.cpu().numpy(), want) < 1e-12


def test_sigma_sx_from_the_gpu_chain_matches_the_oracle_chain(P, ctx):
    """M -> chi0 -> eps^-1 on the GPU, then the static SX with the valence bands as
    the occupied n'' and the conduction bands as n, against the same chain in the oracle."""
    s = _sys("C1")
    d, out = _run(P, ctx, s)
    m = oracle.mtxel_convolution(s["cv"], s["gv"], s["cc"], s["gc"], s["geps"])
    x = oracle.chi0(m, s["ev"], s["ec"], s["omega"])
    e = oracle.epsilon_inverse(x, s["vcoul"])
    assert s["omega"][0] == 0.0
    want = oracle.sigma_sx_static(m, e[0], s["vcoul"], 0.5)
    nv, nc, neps = m.shape
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    sig = torch.zeros(nc, dtype=torch.complex128, device="cuda:0")
    P.gw_sigma_sx(ctx, nv, nc, neps, dev(out["mtxel"]), dev(out["epsinv"][0]), d["vcoul"], 0.5,
                  sig)
    torch.cuda.synchronize()
    assert oracle.rel_f(sig.cpu().numpy(), want) < 1e-10


def test_sigma_sx_rejects_bad_arguments(P, ctx):
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    m = dev(np.zeros((2, 3, 4), np.complex128))
    e = dev(np.eye(4, dtype=np.complex128))
    v = dev(np.ones(4))
    sig = dev(np.zeros(3, np.complex128))
    with pytest.raises(P.GwError):
        P.gw_sigma_sx(ctx, 2, 3, 4, m, e, v, float("nan"), sig)
    with pytest.raises(P.GwError):
        P.gw_sigma_sx(ctx, 2, 3, 4, m, e, v, 1.0, m)
    with pytest.raises(P.GwError):
        P.gw_sigma_sx(ctx, 2, 3, 4, m, e, v, 1.0, None)
    # empty sizes are a no-op
    P.gw_sigma_sx(ctx, 0, 3, 4, m, e, v, 1.0, sig)
    torch.cuda.synchronize()
    assert np.abs(sig.cpu().numpy()).max() == 0.0
