"""Device-resident inputs and one pass of the hot path (marshalling only).

`upload` copies a generated system to HIP device memory once; `run_path` then
enqueues mtxel -> chi0 -> eps^-1 through the C ABI with every intermediate
kept in device memory.
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding as B


def upload(sysd, dtype="c128", device="cuda:0", nc=None):
    """Device copies of a system's coefficients, energies and Coulomb potential."""
    cdt = torch.complex128 if dtype == "c128" else torch.complex64
    ncs = sysd["cc"].shape[0] if nc is None else nc
    d = dict(
        box=tuple(int(x) for x in sysd["box"]), nspinor=int(sysd["cv"].shape[1]),
        gv=np.ascontiguousarray(sysd["gv"], dtype=np.int32),
        gc=np.ascontiguousarray(sysd["gc"], dtype=np.int32),
        geps=np.ascontiguousarray(sysd["geps"], dtype=np.int32),
        cv=torch.from_numpy(np.ascontiguousarray(sysd["cv"])).to(device=device, dtype=cdt),
        cc=torch.from_numpy(np.ascontiguousarray(sysd["cc"][:ncs])).to(device=device, dtype=cdt),
        ev=torch.from_numpy(np.ascontiguousarray(sysd["ev"])).to(device),
        ec=torch.from_numpy(np.ascontiguousarray(sysd["ec"][:ncs])).to(device),
        vcoul=torch.from_numpy(np.ascontiguousarray(sysd["vcoul"])).to(device),
        omega=np.asarray(sysd["omega"], dtype=np.float64),
        head_index=int(sysd.get("head_index", -1)),
        dtype=dtype, device=device,
    )
    d["nv"], d["nc"], d["neps"] = d["cv"].shape[0], d["cc"].shape[0], d["geps"].shape[0]
    return d


def alloc_outputs(d, with_head=False):
    cdt = torch.complex128 if d["dtype"] == "c128" else torch.complex64
    nv, nc, neps, nf = d["nv"], d["nc"], d["neps"], len(d["omega"])
    out = dict(
        mtxel=torch.empty((nv, nc, neps), dtype=cdt, device=d["device"]),
        chi0=torch.zeros((nf, neps, neps), dtype=torch.complex128, device=d["device"]),
        epsinv=torch.empty((nf, neps, neps), dtype=torch.complex128, device=d["device"]),
        mhead=None,
    )
    if with_head and d["head_index"] >= 0:
        out["mhead"] = torch.empty((nv * nc,), dtype=torch.complex128, device=d["device"])
    return out


def run_path(ctx, d, out, prec=B.GW_PREC_FP64, prefactor=1.0, stages=("mtxel", "chi0", "epsinv")):
    """One pass of the path on device-resident inputs; outputs stay on device."""
    use_head = out.get("mhead") is not None
    if "mtxel" in stages:
        B.gw_mtxel_spinor(ctx, d["box"], d["nspinor"], d["gv"], d["cv"], d["gc"], d["cc"],
                          d["geps"], out["mtxel"], d["head_index"] if use_head else -1,
                          out["mhead"] if use_head else None)
    if "chi0" in stages:
        out["chi0"].zero_()
        B.gw_chi0_accumulate(ctx, d["nv"], d["nc"], d["neps"], out["mtxel"], d["ev"], d["ec"],
                             d["omega"], prefactor, prec, out["chi0"],
                             out["mhead"] if use_head else None,
                             d["head_index"] if use_head else -1)
    if "epsinv" in stages:
        B.gw_epsinv(ctx, d["neps"], len(d["omega"]), out["chi0"], d["vcoul"], out["epsinv"])
    return out


def upload_batch(systems, dtype="c64", device="cuda:0"):
    """Device copies for a list of per-q systems (synth.batch_systems); the
    conduction coefficients shared by every q are uploaded once."""
    cdt = torch.complex128 if dtype == "c128" else torch.complex64
    shared = {}
    qs = []
    for s in systems:
        key = id(s["cc"])
        if key not in shared:
            shared[key] = torch.from_numpy(np.ascontiguousarray(s["cc"])).to(device=device, dtype=cdt)
        cc = shared[key]
        nc = int(s.get("nc", s["cc"].shape[0]))
        neps = s["geps"].shape[0]
        nf = len(s["omega"])
        qs.append(dict(
            gv=np.ascontiguousarray(s["gv"], dtype=np.int32),
            gc=np.ascontiguousarray(s["gc"], dtype=np.int32),
            geps=np.ascontiguousarray(s["geps"], dtype=np.int32),
            cv=torch.from_numpy(np.ascontiguousarray(s["cv"])).to(device=device, dtype=cdt),
            cc=cc, nc=nc,
            ev=torch.from_numpy(np.ascontiguousarray(s["ev"])).to(device),
            ec=torch.from_numpy(np.ascontiguousarray(s["ec"][:nc])).to(device),
            vcoul=torch.from_numpy(np.ascontiguousarray(s["vcoul"])).to(device),
            head_index=int(s.get("head_index", -1)),
            chi0=torch.zeros((nf, neps, neps), dtype=torch.complex128, device=device),
            epsinv=torch.zeros((nf, neps, neps), dtype=torch.complex128, device=device),
        ))
    return qs
