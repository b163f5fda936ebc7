#!/usr/bin/env python3
"""Throughput of the spinor chi0 / eps^-1 hot path on one MI355X.

One step = one pass of the whole path over one q-point, inputs resident in HBM:
  band transforms -> pair products + pruned transforms (M) -> chi0 contraction
  -> eps build + inverse.
The default workload is the layered-cell (Bi2Se3-like) system: FFT box
60 x 60 x 160, ~9,000 G per spinor component, N_v = 56, N_c = 2,000, eps sphere
4,000 G, static chi0.  The FP64 path gives the headline value; the mixed path
(float transforms, split-BF16 contraction, FP64 eps^-1) runs the same step and
reports its chi0 and eps^-1 errors against the FP64 path.  --config C2 runs the
Si-like system (48^3 box, 9 frequencies), C4 the 64-q batch, C5 the learned
closure.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("chi0 TFLOP/s + (v,c) pairs/s, mixed vs FP64 path at stated "
          "ε⁻¹ rel error")
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
BF16_PEAK_TFLOPS = 2500.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="C3")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--extras", action="store_true",
                    help="also time the consumers of eps^-1 and the next rows on this workload "
                         "(real axis, dipole head, W and SX, unfolding, plasmon pole, symmetrisation, "
                         "BSE kernels, reduced basis)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--closure-train", type=int, default=256)
    ap.add_argument("--closure-held", type=int, default=32)
    ap.add_argument("--closure-epochs", type=int, default=20)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (for HBM counter scaling)")
    return ap.parse_args()


# vector-ALU peaks of the chip (256 CUs at 2.4 GHz): FP64 78.6 TFLOP/s, FP32
# 157.3 TFLOP/s (the FP32 figure counts the packed instructions this build does
# not emit, so it is an upper bound the FP32 kernels cannot reach)
VECTOR_PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}
# plane shapes (n1, n2) that take the xy-plane pair kernels (x and y transforms
# per z, z last); other boxes transform z and y per x, x last
XY_PLANES = {(60, 60), (16, 16)}


def fft_stage_bytes(d, elem):
    """Algorithmic HBM bytes of the FFT stage (band + pair transforms) per q in
    the full-field accounting: every band field written and read back, and both
    spinor planes of the conduction band per pair."""
    nbox = int(np.prod(d["box"]))
    nv, nc, neps = d["nv"], d["nc"], d["neps"]
    ngv, ngc = d["gv"].shape[0], d["gc"].shape[0]
    ns = d["nspinor"]
    band = elem * (ns * (nv * ngv + nc * ngc) + ns * (nv + nc) * nbox)
    pair = nv * nc * elem * (ns * nbox + neps)
    return band, pair


def pair_work(d):
    """Flop-equivalents of the pair transforms per step, by stage: the
    spin-summed product (6 flops per complex product conj(a) b, 2 per complex
    add) on every grid point, then 5 n log2 n per pruned transform of length n
    that the kernels run (each pass only on the columns the previous pass
    kept)."""
    n1, n2, n3 = (int(x) for x in d["box"])
    nbox = n1 * n2 * n3
    ns = d["nspinor"]
    P = d["nv"] * d["nc"]
    g = np.abs(np.asarray(d["geps"])).max(0)
    e = 2 * g + 1
    f = lambda n: 5.0 * n * np.log2(n)  # noqa: E731
    prod = (8 * ns - 2) * nbox
    if (n1, n2) in XY_PLANES:    # x on every row, y on kept x, z last on the (x, y)
        plane = prod + f(n1) * n2 * n3 + f(n2) * e[0] * n3   # columns holding sphere points
        cols = {(int(a), int(b)) for a, b in np.asarray(d["geps"])[:, :2]}
        last = f(n3) * len(cols)
    else:                        # z on every row, y on kept z, x last on kept (y, z)
        plane = prod + f(n3) * n1 * n2 + f(n2) * e[2] * n1
        last = f(n1) * e[1] * e[2]
    return {"pair_plane": P * plane, "pair_xpass": P * last}


def measured_traffic(kernel, config, path="fp64"):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter record
    (FETCH_SIZE and WRITE_SIZE per dispatch, each scaled by the ratio a plain copy
    of known size reads back), or None when no record exists for this workload or
    the kernel's source changed after the counters were taken."""
    import hashlib
    fn = os.path.join(ROOT, "profiles", f"traffic_{config.lower()}_{path}.json")
    if not os.path.exists(fn):
        return None
    rec = json.load(open(fn)).get(kernel)
    if rec is None:
        return None
    for src, digest in rec["sources"].items():
        sp = os.path.join(ROOT, src)
        if not os.path.exists(sp) or hashlib.sha256(open(sp, "rb").read()).hexdigest() != digest:
            return None
    kib = rec["fetch_kib_per_dispatch"] * rec["fetch_scale"] + \
        rec["write_kib_per_dispatch"] * rec["write_scale"]
    return kib * 1024.0


def chi0_flops(d):
    """Algorithmic flops of the contraction: 4 N_eps^2 P n_omega (8 real flops
    per complex multiply-add over the Hermitian half)."""
    return 4.0 * d["neps"] ** 2 * d["nv"] * d["nc"] * len(d["omega"])


# executed flops per algorithmic flop: FP64 forms each complex product from
# three real products (6 flops for 8); split-BF16 takes three BF16 products per
# real product over the same upper-triangle tiles
CHI0_EXECUTED = {"chi0_fp64": 0.75, "chi0_bf16x3": 3.0}


def time_path(ctx, P, pipeline, d, out, prec, steps, warmup, pick):
    """Warm up, then one breakdown pass of at most 3 steps with events around
    every kernel (per-stage times; `pick` chooses the roofline kernel from it),
    then `steps` timed passes with events around that kernel only (events
    between short dependent kernels would lengthen the gaps between them).
    Returns (ms per step, wall s, roofline kernel, its (launches, ms) per step
    over the timed steps, per-stage (launches, ms) per step)."""
    import torch
    for _ in range(warmup):
        pipeline.run_path(ctx, d, out, prec=prec)
    torch.cuda.synchronize()
    ctx.profile_only(None)
    ctx.profile_reset()
    ctx.profile(True)
    nst = max(1, min(steps, 3))
    for _ in range(nst):
        pipeline.run_path(ctx, d, out, prec=prec)
    torch.cuda.synchronize()
    stage = {k: (n / nst, t / nst) for k, (n, t) in ctx.profile_table().items()}
    roof = pick(stage)
    ctx.profile_reset()
    ctx.profile_only(roof)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    t0 = time.perf_counter()
    for _ in range(steps):
        pipeline.run_path(ctx, d, out, prec=prec)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / steps
    n, t = ctx.profile_table().get(roof, (0, float("nan")))
    ctx.profile_only(None)
    ctx.profile_reset()
    ctx.profile(False)
    return ms, wall, roof, (n / steps, t / steps), stage


def roofline_of(kernel, launches, ms, d, config, path):
    """Roofline entry of one kernel from its per-step time: the contractions
    against their matrix-core peak by executed flops, the pair-plane kernel
    against the vector-ALU peak by its flop-equivalents, anything else by its
    measured HBM traffic when a counter record exists."""
    sec = ms * 1e-3
    per = max(launches, 1.0)
    traffic = measured_traffic(kernel, config, path)
    r = {"kernel": kernel, "launches_per_step": launches, "avg_launch_ms": ms / per,
         "traffic": traffic}
    if kernel in CHI0_EXECUTED:
        alg = chi0_flops(d)
        ex = alg * CHI0_EXECUTED[kernel]
        peak = FP64_PEAK_TFLOPS if kernel == "chi0_fp64" else BF16_PEAK_TFLOPS
        r.update(bound="mfma", achieved=ex / sec / 1e12, peak=peak, unit="TFLOP/s",
                 algorithmic_TFLOP_per_s=alg / sec / 1e12,
                 note="achieved = executed MFMA flops (%.2f x the algorithmic 4 N^2 P n_w) "
                      "over the kernel's event time" % CHI0_EXECUTED[kernel])
    elif kernel in ("pair_plane", "pair_xpass"):
        w = pair_work(d)[kernel]
        dt = "f64" if d["dtype"] == "c128" else "f32"
        r.update(bound="alu", achieved=w / sec / 1e12, peak=VECTOR_PEAK_TFLOPS[dt],
                 unit="TFLOP/s",
                 note="achieved = flop-equivalents of the product and pruned transforms "
                      f"(5 n log2 n each) over the kernel's event time; {dt} vector peak")
    else:
        r.update(bound="hbm", achieved=None if traffic is None else traffic / (sec / per) / 1e9,
                 peak=HBM_PEAK_GBS, unit="GB/s")
    r["frac"] = None if r.get("achieved") is None else r["achieved"] / r["peak"]
    if traffic is not None:
        r["traffic_GB_per_launch"] = traffic / 1e9
        r["measured_hbm_GB_per_s"] = traffic / (ms / per * 1e-3) / 1e9
    return r


EPSINV_STAGES = ("eps_build", "flags_clear", "gj_diag", "gj_small", "gj_update", "gj_step",
                 "eps_unscale")


def epsinv_roofline(stage, d):
    """eps^-1 by Gauss-Jordan: 8 N^3 flops per frequency (N^3 complex multiply-adds
    of the in-place inverse) over the summed time of the eps build, the
    diagonal-block inverses, the rank updates and the unscaling, against the FP64
    matrix-core peak that the rank updates run on."""
    ms = sum(stage[k][1] for k in EPSINV_STAGES if k in stage)
    if ms <= 0:
        return None
    n, nf = d["neps"], len(d["omega"])
    flops = 8.0 * n ** 3 * nf
    return {"kernel": "epsinv (Gauss-Jordan, all stages)", "ms_per_step": ms, "bound": "mfma",
            "achieved": flops / (ms * 1e-3) / 1e12, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": flops / (ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
            "note": "8 N^3 n_omega flops over the summed stage times"}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sysd, seconds):
    """The oracle on a bounded sample of the same workload, scaled to pairs/s:
    its FFT route (scipy.fft with one worker per host core) and its contraction
    (threaded BLAS) on valence band 0 against growing blocks of conduction
    bands, then its eps^-1 (LAPACK) of every frequency at the full N_eps on the
    chi0 those sampled pairs gave."""
    import oracle
    workers = os.cpu_count() or 1
    try:
        from threadpoolctl import threadpool_info
        info = threadpool_info()
        blas_threads = max([i.get("num_threads", 1) for i in info] + [1])
        blas = ",".join(sorted({i.get("internal_api", "?") for i in info})) or "?"
    except Exception:
        blas_threads, blas = workers, "?"
    nv, nc = sysd["cv"].shape[0], sysd["cc"].shape[0]
    neps = sysd["geps"].shape[0]
    chi = np.zeros((len(sysd["omega"]), neps, neps), dtype=np.complex128)
    t0 = time.perf_counter()
    done, cb, v, c0 = 0, 8, 0, 0
    while time.perf_counter() - t0 < seconds and done < nv * nc:
        cs = slice(c0, min(nc, c0 + cb))
        m = oracle.mtxel_fft(sysd["cv"][v:v + 1], sysd["gv"], sysd["cc"][cs], sysd["gc"],
                             sysd["geps"], sysd["box"], workers=workers)
        chi += oracle.chi0(m, sysd["ev"][v:v + 1], sysd["ec"][cs], sysd["omega"])
        done += cs.stop - cs.start
        c0 = cs.stop
        if c0 >= nc:
            c0, v = 0, v + 1
    t_pairs = time.perf_counter() - t0
    per_pair = t_pairs / done
    t1 = time.perf_counter()
    oracle.epsilon_inverse(chi, sysd["vcoul"])
    t_inv = time.perf_counter() - t1
    P = nv * nc
    step = per_pair * P + t_inv
    return {
        "value": P / step, "unit": "(v,c) pairs/s", "cores": int(workers), "kind": "oracle",
        "cpu_model": _cpu_model(), "blas": blas, "blas_threads": int(blas_threads),
        "sample": (f"oracle FFT route (scipy.fft, {workers} workers) + chi0 (BLAS, "
                   f"{blas_threads} threads) on {done} of {P} pairs in {t_pairs:.1f} s, plus "
                   f"eps^-1 (LAPACK) of all {len(sysd['omega'])} frequencies at N_eps={neps} "
                   f"on the sampled pairs' chi0 in {t_inv:.2f} s; projected full step "
                   f"{step:.1f} s"),
    }


def bench_batch(args):
    """The many-q workload: 64 q-points of a 4x4x4 grid (Gamma replaced by a small
    q0 with FP64 head/wings), per-q eps spheres of 600-2400 G and N_c of 400-1600,
    N_v = 16, box 48^3; complex64 matrix elements, split-BF16 contraction, FP64
    eps^-1; all q in one captured graph."""
    import torch

    import synth
    import paper_2206_00808_amd as P
    from paper_2206_00808_amd import pipeline
    from paper_2206_00808_amd.binding import Plan

    systems = synth.batch_systems()
    ctx = P.Context(0)
    qs = pipeline.upload_batch(systems, dtype="c64")
    plan = Plan(ctx, systems[0]["box"], 2, P.GW_C64, P.GW_PREC_SPLITBF16, systems[0]["omega"],
                1.0, qs)
    t0 = time.perf_counter()
    plan.compile()
    compile_s = time.perf_counter() - t0
    for _ in range(args.warmup):
        plan.launch()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        plan.launch()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    pairs = sum(int(s["cv"].shape[0]) * int(s["nc"]) for s in systems)
    flops = sum(4.0 * s["geps"].shape[0] ** 2 * s["cv"].shape[0] * s["nc"] * len(s["omega"])
                for s in systems)
    result = {
        "metric": METRIC, "value": pairs / (ms * 1e-3), "unit": "(v,c) pairs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64 transforms, split-bf16x3 contraction, f64 eps^-1", "data": "synthetic",
        "config": {"workload": "C4: 64 q-points (4x4x4 grid, Gamma -> q0), N_eps 600-2400, "
                               "N_c 400-1600, N_v 16, box 48^3, one captured graph",
                   "global_batch": len(systems), "pairs": pairs, "parallelism": "single GPU"},
        "chi0_tflops_whole_step": flops / (ms * 1e-3) / 1e12,
        "compile_s": compile_s, "autotune": plan.describe(),
    }
    plan.close()
    ctx.close()
    print(json.dumps(result), flush=True)


def bench_real_axis(ctx, P, d, mtxel, steps, nfreq=9, eta=0.005):
    """Real-frequency chi0 with broadening (gw_chi0_accumulate_real, FP64) on the
    workload's matrix elements at nfreq frequencies in [0, 0.8] Ha, and its
    inverse dielectric matrix by pivoted LU (gw_epsinv_lu)."""
    import torch
    omega = np.linspace(0.0, 0.8, nfreq)
    neps = d["neps"]
    chi = torch.zeros((nfreq, neps, neps), dtype=torch.complex128, device="cuda")
    einv = torch.empty_like(chi)

    def run_chi():
        chi.zero_()
        P.gw_chi0_accumulate_real(ctx, d["nv"], d["nc"], neps, mtxel, d["ev"], d["ec"], omega,
                                  eta, 1.0, P.GW_PREC_FP64, chi)

    def run_inv():
        P.gw_epsinv(ctx, neps, nfreq, chi, d["vcoul"], einv)

    def run_lu():
        P.gw_epsinv_lu(ctx, neps, nfreq, chi, d["vcoul"], einv)

    out = {}
    for name, fn in (("chi0", run_chi), ("epsinv", run_inv), ("epsinv_lu", run_lu)):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name + "_ms"] = e0.elapsed_time(e1) / steps
    pairs = d["nv"] * d["nc"]
    # a general (non-Hermitian) complex rank-P update: 8 N^2 P flops per frequency
    flops = 8.0 * neps * neps * pairs * nfreq
    out["chi0_tflops"] = flops / (out["chi0_ms"] * 1e-3) / 1e12
    out["chi0_frac_of_fp64_peak"] = out["chi0_tflops"] / FP64_PEAK_TFLOPS
    out["config"] = {"nfreq": nfreq, "omega_Ha": [0.0, 0.8], "eta_Ha": eta, "pairs": pairs,
                     "neps": neps}
    out["note"] = ("chi0 includes zeroing the output, the weights, two Hermitian contractions "
                   "(Re and Im of the bracket) and their combination; epsinv is gw_epsinv "
                   "(Gauss-Jordan kept after its residual check, else LU), epsinv_lu is LU "
                   "with partial pivoting throughout")
    return out


def bench_head_dipole(ctx, P, sysd, d, steps):
    """The q -> 0 head from momentum matrix elements (gw_head_dipole) at the
    workload's sizes: N_v bands and N_c bands of the conduction set's sphere at k
    (both at one k-point), q = 1e-3 bohr^-1 along x."""
    import torch
    nv, nc = d["nv"], d["nc"]
    cc = d["cc"]
    cv = cc[:nv].contiguous()
    g = np.asarray(sysd["gc"], dtype=np.int32)
    mh = torch.empty(nv * nc, dtype=torch.complex128, device="cuda")
    args = (ctx, d["nspinor"], g, cv, cc, sysd["cell"], (0.0, 0.0, 0.0), (1e-3, 0.0, 0.0),
            d["ev"], d["ec"], mh)
    P.gw_head_dipole(*args)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        P.gw_head_dipole(*args)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    nbytes = (nv + nc) * d["nspinor"] * g.shape[0] * 16 + nv * nc * 16
    return {"ms": ms, "pairs": nv * nc, "ng": int(g.shape[0]),
            "algorithmic_GB_per_s": nbytes / (ms * 1e-3) / 1e9,
            "note": "includes the G-list upload and the call's final synchronisation; "
                    "algorithmic bytes = both coefficient sets once + the output"}


def bench_w_and_sx(ctx, P, d, mtxel, epsinv, steps):
    """The consumers of eps^-1 at the workload's sizes: W = eps^-1 v over every
    frequency (gw_screened_w, HBM-bound: eps^-1 read once, W written once), and the
    static screened exchange (gw_sigma_sx) with the N_v valence bands as the occupied
    n'' and the N_c conduction bands as n, on the omega = 0 eps^-1."""
    import torch
    nv, nc, neps, nfreq = d["nv"], d["nc"], d["neps"], epsinv.shape[0]
    w = torch.empty_like(epsinv)
    sig = torch.zeros(nc, dtype=torch.complex128, device="cuda")
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    out = {}
    for name, fn in (
            ("screened_w", lambda: P.gw_screened_w(ctx, neps, nfreq, epsinv, d["vcoul"], w)),
            ("sigma_sx", lambda: P.gw_sigma_sx(ctx, nv, nc, neps, mtxel, epsinv[0], d["vcoul"],
                                               1.0, sig))):
        fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name] = {"ms": e0.elapsed_time(e1) / steps}
    wb = 2 * nfreq * neps * neps * 16 + neps * 8
    out["screened_w"]["algorithmic_GB_per_s"] = wb / (out["screened_w"]["ms"] * 1e-3) / 1e9
    fl = 8.0 * nv * nc * neps * neps
    out["sigma_sx"]["TFLOP_per_s"] = fl / (out["sigma_sx"]["ms"] * 1e-3) / 1e12
    out["sigma_sx"]["note"] = ("flops = the U = conj(M) eps^-1 contraction, 8 N_v N_c N_eps^2; "
                               "includes the widening copy and the per-band reduction")
    return out


def bench_unfold(ctx, P, sysd, d, steps):
    """Spinor unfolding (gw_unfold_spinor) of the workload's N_c conduction bands at
    k = 0 under the 2_1 screw {C2z | (0, 0, 1/2)} of its orthorhombic cell, the
    sphere onto itself.  The call's time includes building the index and phase
    tables on the host and the final synchronisation; the kernel's own time comes
    from the library's events around it."""
    import torch
    cc = d["cc"]
    g = np.asarray(sysd["gc"], dtype=np.int32)
    rot = [[-1, 0, 0], [0, -1, 0], [0, 0, 1]]
    tau = (0.0, 0.0, 0.5)
    out = torch.empty_like(cc)
    call = lambda: P.gw_unfold_spinor(ctx, d["nspinor"], g, cc, g, rot, tau, sysd["cell"], out)
    call()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        call()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    ctx.profile_reset()
    ctx.profile(True)
    for _ in range(steps):
        call()
    torch.cuda.synchronize()
    tab = ctx.profile_table()
    ctx.profile(False)
    ctx.profile_reset()
    n, kms = tab.get("unfold", (1, float("nan")))
    kms /= max(n, 1)
    nb, ns, ng = cc.shape
    nbytes = nb * ns * 2 * ng * cc.element_size() + ng * (4 + 16)
    return {"ms_call": ms, "ms_kernel": kms, "bands": nb, "ng": ng,
            "algorithmic_GB_per_s": nbytes / (kms * 1e-3) / 1e9,
            "note": "algorithmic bytes = every coefficient read and written once + the "
                    "index and phase tables; the rate uses the kernel's own time"}


def bench_gpp(ctx, P, sysd, d, epsinv0, steps, nband=8, ne=3):
    """Plasmon-pole SX + COH (gw_gpp_modes, gw_sigma_gpp) at the workload's sizes:
    the static eps^-1 of the timed path, n'' over all N_v + N_c states (N_v
    occupied), Sigma for the `nband` bands at the gap (N_v/2 .. N_v + nband/2),
    three energies per band (E_n and E_n +- 0.02 Ha); synthetic M_{n''n}(G) and a
    synthetic valence density of N_v electrons on the 48^3 box."""
    import torch
    import synth
    nv, nc, neps = d["nv"], d["nc"], d["neps"]
    nn = nv + nc
    rng = np.random.default_rng(77)
    m = (rng.standard_normal((nn, nband, neps)) + 1j * rng.standard_normal((nn, nband, neps)))
    m = torch.from_numpy(m / np.sqrt(2 * neps)).to("cuda")
    en = torch.cat([d["ev"], d["ec"]]).contiguous()
    lo = nv - nband // 2
    e_n = en[lo:lo + nband].cpu().numpy()
    energies = torch.from_numpy(e_n[:, None] + np.array([-0.02, 0.0, 0.02])[None, :ne]).to("cuda")
    rho = torch.from_numpy(synth.charge_density(78, sysd["cell"], sysd["box"], nelec=nv)).to("cuda")
    amp = torch.empty_like(epsinv0)
    wt = torch.empty_like(epsinv0)
    sx = torch.zeros((nband, ne), dtype=torch.complex128, device="cuda")
    coh = torch.zeros_like(sx)
    geps = np.asarray(sysd["geps"], dtype=np.int32)
    modes = lambda: P.gw_gpp_modes(ctx, geps, sysd["cell"], sysd["q"], rho, epsinv0, amp, wt)
    sig = lambda: P.gw_sigma_gpp(ctx, nn, nv, nband, neps, m, en, d["vcoul"], amp, wt, energies,
                                 1.0, sx, coh)
    modes()
    sig()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    out = {}
    for name, fn in (("gpp_modes", modes), ("sigma_gpp", sig)):
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name] = {"ms": e0.elapsed_time(e1) / steps}
    evals = float(nn) * nband * neps * neps * ne
    flops = evals * 21.0 + float(nv) * nband * neps * neps * ne * 23.0
    out["sigma_gpp"].update({
        "element_evaluations_per_s": evals / (out["sigma_gpp"]["ms"] * 1e-3),
        "TFLOP_per_s": flops / (out["sigma_gpp"]["ms"] * 1e-3) / 1e12,
        "states": nn, "occupied": nv, "bands": nband, "energies": ne,
        "note": "flops = 21 per COH element and energy + 23 per SX element and energy "
                "(each also one FP64 reciprocal), counted from the formulas"})
    out["gpp_modes"]["kept_fraction"] = float((amp != 0).float().mean().item())
    return out


def bench_symmetrize(ctx, P, sysd, chi, steps):
    """Little-group average of chi0 (gw_chi0_symmetrize) over the workload's nine
    frequencies at N_eps: the four operations of the orthorhombic cell that keep
    q along x (E, C2x, the mirrors normal to y and z).  The call includes building
    the index and phase tables on the host and the final synchronisation."""
    import torch
    ops = [(np.diag(d), (0.0, 0.0, 0.0)) for d in ((1, 1, 1), (1, -1, -1), (1, -1, 1), (1, 1, -1))]
    out = torch.empty_like(chi)
    geps = np.asarray(sysd["geps"], dtype=np.int32)
    call = lambda: P.gw_chi0_symmetrize(ctx, geps, sysd["q"], ops, chi, out)
    call()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        call()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    ctx.profile_reset()
    ctx.profile(True)
    for _ in range(steps):
        call()
    torch.cuda.synchronize()
    n, kms = ctx.profile_table().get("chi0_symmetrize", (1, float("nan")))
    ctx.profile(False)
    ctx.profile_reset()
    kms /= max(n, 1)
    nf, ne, _ = chi.shape
    nbytes = nf * ne * ne * 16 * (len(ops) + 1)
    return {"ms_call": ms, "ms_kernel": kms, "ops": len(ops),
            "algorithmic_GB_per_s": nbytes / (kms * 1e-3) / 1e9,
            "note": "algorithmic bytes = chi0 read once per operation and written once"}


def bench_bse(ctx, P, d, epsinv0, steps, nc=64):
    """BSE exchange and direct kernels (gw_bse_kernel) for the workload's N_v valence
    bands and its lowest `nc` conduction bands on the N_eps sphere: synthetic
    matrix elements, W = eps^-1 v from the timed path's static eps^-1."""
    import torch
    nv, neps = d["nv"], d["neps"]
    g = torch.Generator(device="cuda").manual_seed(91)
    rnd = lambda *s: torch.randn(*s, dtype=torch.complex128, device="cuda", generator=g) / neps
    mvc, mcc, mvv = rnd(nv, nc, neps), rnd(nc, nc, neps), rnd(nv, nv, neps)
    w = torch.empty_like(epsinv0)
    P.gw_screened_w(ctx, neps, 1, epsinv0, d["vcoul"], w)
    vx = d["vcoul"].clone()
    p = nv * nc
    kx = torch.empty((p, p), dtype=torch.complex128, device="cuda")
    kd = torch.empty_like(kx)
    call = lambda: P.gw_bse_kernel(ctx, mvc, mcc, mvv, vx, w, kx, kd)
    call()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        call()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    flops = 8.0 * (p * p * neps + nc * nc * neps * neps + nc * nc * nv * nv * neps)
    return {"ms": ms, "nv": nv, "nc": nc, "neps": neps, "TFLOP_per_s": flops / (ms * 1e-3) / 1e12,
            "note": "flops = the three complex GEMMs (K^X, conj(M_cc) W, and its product with "
                    "M_vv^T); the time includes widening, transposes and the reordering"}


def bench_lowrank(ctx, P, d, chi, epsinv_full, mtxel, reps=2):
    """eps^-1 in a basis of N_eps/10 static eigenvectors (gw_epsinv_lowrank) for the
    workload's nine frequencies, against the full inverse of the timed path: time
    and the relative Frobenius difference per frequency; then the same with chi0
    built in the basis (each step timed once)."""
    import torch
    nf, neps, _ = chi.shape
    nb = max(1, neps // 10)
    out = torch.empty_like(chi)
    lam = torch.empty(neps, dtype=torch.float64, device="cuda")
    call = lambda: P.gw_epsinv_lowrank(ctx, neps, nf, chi, d["vcoul"], nb, out, lam)
    call()
    torch.cuda.synchronize()
    ctx.profile_reset()
    ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(reps):
        call()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    tab = ctx.profile_table()
    ctx.profile(False)
    ctx.profile_reset()
    jac = tab.get("jacobi_sweep", (0, 0.0))
    diff = (out - epsinv_full).reshape(nf, -1)
    rel = (torch.linalg.vector_norm(diff, dim=1) /
           torch.linalg.vector_norm(epsinv_full.reshape(nf, -1), dim=1)).cpu().numpy()
    lam_h = lam.cpu().numpy()
    # chi0 built in the basis: basis from the static chi0, projected matrix
    # elements, chi_B at every frequency, eps^-1 from chi_B
    import paper_2206_00808_amd as P2
    nv, nc = d["nv"], d["nc"]
    u = torch.empty((neps, nb), dtype=torch.complex128, device="cuda")
    mb = torch.empty((nv, nc, nb), dtype=torch.complex128, device="cuda")
    chib = torch.empty((nf, nb, nb), dtype=torch.complex128, device="cuda")
    proj_out = torch.empty_like(chi)
    steps_ms = {}
    ev = torch.cuda.Event(enable_timing=True)
    ev2 = torch.cuda.Event(enable_timing=True)
    for name, fn in (
            ("basis", lambda: P2.gw_lowrank_basis(ctx, neps, chi[0], d["vcoul"], nb, u)),
            ("project", lambda: P2.gw_mtxel_project(ctx, mtxel, d["vcoul"], u, mb)),
            ("chi0_in_basis", lambda: (chib.zero_(), P2.gw_chi0_accumulate(
                ctx, nv, nc, nb, mb, d["ev"], d["ec"], d["omega"], 1.0, P2.GW_PREC_FP64, chib))),
            ("epsinv_from_basis", lambda: P2.gw_epsinv_from_basis(ctx, chib, d["vcoul"], u,
                                                                   proj_out))):
        torch.cuda.synchronize()
        ev.record()
        fn()
        ev2.record()
        torch.cuda.synchronize()
        steps_ms[name] = ev.elapsed_time(ev2)
    pdiff = (proj_out - out).reshape(nf, -1)
    prel = float((torch.linalg.vector_norm(pdiff) / torch.linalg.vector_norm(out)).item())
    return {"ms": ms, "nb": nb, "chi0_in_basis_route_ms": steps_ms,
            "chi0_in_basis_vs_projected_epst_rel": prel, "jacobi_ms": jac[1] / reps, "jacobi_sweeps": jac[0] / reps,
            "rel_diff_vs_full_inverse": [float(x) for x in rel],
            "kept_eigenvalue_min": float(lam_h[neps - nb]),
            "discarded_eigenvalue_max": float(lam_h[neps - nb - 1]),
            "note": "wall time of the call (it synchronises); the Jacobi sweeps dominate: "
                    "block Jacobi, each sweep N_eps/16 - 1 rounds of a 32 x 32 solve kernel "
                    "and an MFMA update kernel, replayed from a graph"}


def _one_blas_thread():
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:
        pass


def _gen_closure(i):
    import synth
    s = synth.closure_systems([i])[0]
    return i, s


def bench_closure(args):
    """The closure workload: 256 training + 32 held-out systems (box 32^3, N_v 16,
    eps spheres of 300-800 G), chi0 truncated at N_c = 200 and summed to 2000 by
    the GPU path; a 3x256 SiLU network trained by the library's kernels; errors of
    the truncated and corrected chi0 and eps^-1 against the full sum on the
    held-out systems."""
    import multiprocessing as mp

    ntrain, nheld = args.closure_train, args.closure_held
    workers = min(16, os.cpu_count() or 1)
    # the host generator runs in worker processes started before any GPU use
    pool = mp.get_context("spawn").Pool(workers, initializer=_one_blas_thread)
    gen = pool.imap(_gen_closure, range(ntrain + nheld), chunksize=1)
    import torch

    import paper_2206_00808_amd as P
    from paper_2206_00808_amd.binding import Mlp
    from paper_2206_00808_amd.closure import closure_dataset, evaluate, train
    ctx = P.Context(0)
    t0 = time.perf_counter()
    items = []
    for k, (i, s) in enumerate(gen):
        items += closure_dataset(ctx, [s], nc_trunc=200)
        if (k + 1) % 16 == 0:
            print(f"closure data: {k + 1}/{ntrain + nheld} systems, "
                  f"{time.perf_counter() - t0:.0f} s", file=sys.stderr, flush=True)
    pool.close()
    t_data = time.perf_counter() - t0
    net = Mlp(ctx, 7, 256, 3, 2, seed=2026)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    losses = train(ctx, net, items[:ntrain], epochs=args.closure_epochs, lr=1e-3, lr_final=5e-5,
                   log=lambda e, l: print(f"closure epoch {e}: loss {l:.4g}", file=sys.stderr,
                                          flush=True))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    steps = args.closure_epochs * ntrain
    rows = evaluate(ctx, net, items[ntrain:])
    keep = rows  # the prediction's own error, inferred without the full sum
    mean = lambda key, rs: float(np.mean([r[key] for r in rs])) if rs else None  # noqa: E731
    res = {
        "metric": "learned closure: chi0 / eps^-1 rel error vs full band sum (held-out)",
        "value": mean("chi_closure", keep),
        "unit": "rel_F(chi0) mean over held-out systems", "higher_is_better": False,
        "n_gpus": 1, "data": "synthetic",
        "config": {"workload": f"C5: {ntrain} train + {nheld} held-out systems, box 32^3, "
                               "N_v 16, N_c 200 -> 2000, N_eps 300-800, MLP 3x256 SiLU bf16",
                   "epochs": args.closure_epochs},
        "chi0_rel_err_truncated": mean("chi_trunc", rows),
        "chi0_rel_err_closure": mean("chi_closure", keep),
        "epsinv_rel_err_truncated": mean("epsinv_trunc", rows),
        "epsinv_rel_err_closure": mean("epsinv_closure", keep),
        "fallbacks": int(sum(r["fallback"] for r in rows)),
        "train_steps": steps, "train_s": t_train, "train_steps_per_s": steps / t_train,
        "data_s": t_data, "loss_first_epoch": losses[0], "loss_last_epoch": losses[-1],
    }
    net.close()
    ctx.close()
    print(json.dumps(res), flush=True)


def _rel_errors(x, ref):
    """Max over frequencies of rel_F, and max |x - ref| / max |ref| over all."""
    import torch
    nf = ref.shape[0]
    d = (x - ref).reshape(nf, -1)
    r = ref.reshape(nf, -1)
    rel = float((torch.linalg.vector_norm(d, dim=1) / torch.linalg.vector_norm(r, dim=1)).max())
    mx = float(d.abs().max() / r.abs().max())
    return rel, mx


def _workload_name(cfg, sysd, neps):
    kind = {"C1": "small cell", "C2": "Si-like", "C3": "layered Bi2Se3-like cell"}.get(cfg.name,
                                                                                      cfg.name)
    return (f"{cfg.name}: {kind}, spinor chi0 + eps^-1, box {cfg.box[0]}x{cfg.box[1]}x"
            f"{cfg.box[2]}, N_G {sysd['gv'].shape[0]}/{sysd['gc'].shape[0]}, N_v {cfg.nv}, "
            f"N_c {cfg.nc}, N_eps {neps}, {len(cfg.omega_ev)} frequenc"
            f"{'y' if len(cfg.omega_ev) == 1 else 'ies'}")


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                                   "(sharding over GPUs is described in the design notes, "
                                   "not built)"}), flush=True)
        sys.exit(2)
    if args.config == "C5":
        bench_closure(args)
        return
    if args.config == "C4":
        bench_batch(args)
        return
    import torch

    import synth
    import paper_2206_00808_amd as P
    from paper_2206_00808_amd import pipeline

    cfg = synth.CONFIGS[args.config]
    sysd = synth.build_system(cfg)
    ctx = P.Context(0)
    if args.copy_calibration:
        # a plain copy of known size: 1 GiB read + 1 GiB written per launch
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        src.fill_(1.0)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # the roofline kernel of a path: the one with the largest time per step
    heaviest = lambda stage: max(stage.items(), key=lambda kv: kv[1][1])[0]  # noqa: E731

    # ---------------- FP64 path (the headline value)
    d64 = pipeline.upload(sysd, dtype="c128")
    o64 = pipeline.alloc_outputs(d64)
    ms64, wall64, rk64, (rl64, rms64), st64 = time_path(ctx, P, pipeline, d64, o64,
                                                         P.GW_PREC_FP64, args.steps, args.warmup,
                                                         heaviest)
    pairs = d64["nv"] * d64["nc"]
    flops = chi0_flops(d64)
    neps = d64["neps"]
    chi_ms64 = st64.get("chi0_fp64", (0, float("nan")))[1]
    result = {
        "metric": METRIC,
        "value": pairs / (ms64 * 1e-3),
        "unit": "(v,c) pairs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms64,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": _workload_name(cfg, sysd, neps),
                   "global_batch": 1, "pairs": pairs, "parallelism": "single GPU"},
        "chi0_tflops": flops / (chi_ms64 * 1e-3) / 1e12,
        "chi0_tflops_note": "algorithmic 4 N_eps^2 P n_omega over the contraction's time",
        "chi0_tflops_whole_step": flops / (ms64 * 1e-3) / 1e12,
        "stage_ms": {k: round(v[1], 4) for k, v in sorted(st64.items())},
        "stage_ms_note": "per step, from a separate pass with events around every kernel",
        "wall_ms_per_step": wall64 * 1e3 / args.steps,
    }
    result["roofline"] = roofline_of(rk64, rl64, rms64, d64, args.config, "fp64")
    result["roofline"]["timed_over"] = f"{args.steps} timed steps (library events on its stream)"
    others = {}
    for k in ("chi0_fp64", "pair_plane", "pair_xpass"):
        if k in st64 and k != rk64:
            others[k] = roofline_of(k, st64[k][0], st64[k][1], d64, args.config, "fp64")
    others["epsinv"] = epsinv_roofline(st64, d64)
    result["other_rooflines"] = others
    fft_keys = ("band_xpass", "band_plane", "band_zc", "band_zyx", "pair_plane", "pair_xpass")
    fft_ms = sum(st64.get(k, (0, 0))[1] for k in fft_keys)
    work = pair_work(d64)
    bb, pb = fft_stage_bytes(d64, 16)
    result["fft_stage"] = {
        "ms": fft_ms,
        "pair_flop_equivalents": sum(work.values()),
        "alu_TFLOP_per_s": sum(work.values()) / (fft_ms * 1e-3) / 1e12,
        "frac_of_alu_peak": sum(work.values()) / (fft_ms * 1e-3) / 1e12 / VECTOR_PEAK_TFLOPS["f64"],
        "full_field_unit_GB": (bb + pb) / 1e9,
        "note": "bound by the vector ALU: the product and pruned transforms of every pair "
                "(5 n log2 n flop-equivalents per transform) over the band and pair kernels' "
                "time; the full-field byte unit counts conduction planes the kernels never "
                "move, so it is given for reference only; measured HBM traffic per kernel "
                "is in the rooflines when a counter record exists"}
    epsinv64 = o64["epsinv"]

    if args.extras:
        extras = (
            ("lowrank", lambda: bench_lowrank(ctx, P, d64, o64["chi0"], epsinv64, o64["mtxel"])),
            ("real_axis", lambda: bench_real_axis(ctx, P, d64, o64["mtxel"], args.steps)),
            ("head_dipole", lambda: bench_head_dipole(ctx, P, sysd, d64, args.steps)),
            ("w_and_sx", lambda: bench_w_and_sx(ctx, P, d64, o64["mtxel"], epsinv64, args.steps)),
            ("unfold", lambda: bench_unfold(ctx, P, sysd, d64, args.steps)),
            ("gpp", lambda: bench_gpp(ctx, P, sysd, d64, epsinv64[0], args.steps)),
            ("symmetrize", lambda: bench_symmetrize(ctx, P, sysd, o64["chi0"], args.steps)),
            ("bse_kernel", lambda: bench_bse(ctx, P, d64, epsinv64[0], args.steps)))
        for name, fn in extras:
            # an entry point whose size limits this workload exceeds reports
            # its error instead of a timing
            try:
                result[name] = fn()
            except P.GwError as e:
                result[name] = {"error": str(e)}

    # ---------------- mixed path: float transforms, split-BF16 contraction, FP64 eps^-1
    if not args.no_mixed:
        chi64 = o64["chi0"]
        mt64 = o64["mtxel"]
        del o64  # keep only what the comparison needs
        d32 = pipeline.upload(sysd, dtype="c64")
        o32 = pipeline.alloc_outputs(d32)
        ms32, wall32, rk32, (rl32, rms32), st32 = time_path(ctx, P, pipeline, d32, o32,
                                                             P.GW_PREC_SPLITBF16, args.steps,
                                                             args.warmup, heaviest)
        chi_ms32 = st32.get("chi0_bf16x3", (0, float("nan")))[1]
        e_inv, e_inv_max = _rel_errors(o32["epsinv"], epsinv64)
        e_chi, e_chi_max = _rel_errors(o32["chi0"], chi64)
        nf = len(cfg.omega_ev)
        dm = (o32["mtxel"].to(torch.complex128) - mt64).reshape(-1)
        e_m = float(torch.linalg.vector_norm(dm) / torch.linalg.vector_norm(mt64.reshape(-1)))
        bf = roofline_of("chi0_bf16x3", st32["chi0_bf16x3"][0], chi_ms32, d32, args.config,
                         "mixed") if "chi0_bf16x3" in st32 else None
        result["mixed"] = {
            "pairs_per_s": pairs / (ms32 * 1e-3), "ms_per_step": ms32,
            "chi0_tflops": flops / (chi_ms32 * 1e-3) / 1e12,
            "chi0_roofline": bf,
            "epsinv_roofline": epsinv_roofline(st32, d32),
            "roofline": roofline_of(rk32, rl32, rms32, d32, args.config, "mixed"),
            "epsinv_rel_err_vs_fp64": e_inv, "epsinv_max_err_vs_fp64": e_inv_max,
            "chi0_rel_err_vs_fp64": e_chi, "chi0_max_err_vs_fp64": e_chi_max,
            "mtxel_rel_err_vs_fp64": e_m,
            "error_note": f"rel_F max over the {nf} frequenc{'y' if nf == 1 else 'ies'}; max = "
                          "max |x - x_64| / max |x_64|; the FP64 path matches the oracle to "
                          "1e-10 in the parity tests",
            "dtype": "c64 transforms, split-bf16x3 contraction, f64 eps^-1",
            "stage_ms": {k: round(v[1], 4) for k, v in sorted(st32.items())},
        }
        del d32, o32, chi64, mt64
    ctx.close()

    # ---------------- CPU oracle baseline
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(sysd, args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
