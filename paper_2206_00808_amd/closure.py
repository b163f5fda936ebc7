"""Training and evaluation driver for the learned band-sum closure.

The training pairs come from the method itself. For each system:

- the spinor matrix elements are computed once on the GPU;
- chi0 is contracted over the first `nc_trunc` conduction bands (truncated sum);
- chi0 is contracted again over all of them (full sum).

The network learns the difference between the two. Every step runs in the
library's kernels: this module only orders the calls.
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding as B
from . import pipeline


def closure_dataset(ctx, systems, nc_trunc, device="cuda:0"):
    """Truncated and full static chi0 for each system, resident on the device."""
    items = []
    for s in systems:
        d = pipeline.upload(s, dtype="c128", device=device)
        m = torch.empty((d["nv"], d["nc"], d["neps"]), dtype=torch.complex128, device=device)
        B.gw_mtxel_spinor(ctx, d["box"], d["nspinor"], d["gv"], d["cv"], d["gc"], d["cc"],
                          d["geps"], m)
        full = torch.zeros((1, d["neps"], d["neps"]), dtype=torch.complex128, device=device)
        B.gw_chi0_accumulate(ctx, d["nv"], d["nc"], d["neps"], m, d["ev"], d["ec"], [0.0], 1.0,
                             B.GW_PREC_FP64, full)
        mt = m[:, :nc_trunc].contiguous()
        trunc = torch.zeros_like(full)
        B.gw_chi0_accumulate(ctx, d["nv"], nc_trunc, d["neps"], mt, d["ev"],
                             d["ec"][:nc_trunc].contiguous(), [0.0], 1.0, B.GW_PREC_FP64, trunc)
        ev, ec = np.asarray(s["ev"]), np.asarray(s["ec"])
        items.append(dict(
            name=s.get("name", ""), neps=d["neps"],
            qg=torch.from_numpy(np.ascontiguousarray(s["qg"])).to(device),
            chi_t=trunc[0].contiguous(), chi_f=full[0].contiguous(),
            gap=float(ec.min() - ev.max()), emax=float(ec[:nc_trunc].max()),
            vcoul=d["vcoul"],
        ))
        del m, mt
    torch.cuda.synchronize()
    return items


def train(ctx, net, items, epochs, lr=1e-3, lr_final=1e-4, seed=0, log=None):
    """One Adam step per system per epoch, systems in a seeded order; the
    learning rate decays geometrically from lr to lr_final."""
    rng = np.random.default_rng(seed)
    losses = []
    total = epochs * len(items)
    k = 0
    for _ in range(epochs):
        ep = []
        for i in rng.permutation(len(items)):
            it = items[i]
            a = lr * (lr_final / lr) ** (k / max(1, total - 1))
            _, loss = B.gw_chi0_closure(ctx, net, B.GW_CLOSURE_TRAIN_STEP, it["neps"], it["qg"],
                                        it["chi_t"], it["gap"], it["emax"], chi0_full=it["chi_f"],
                                        lr=a)
            ep.append(loss)
            k += 1
        losses.append(float(np.mean(ep)))
        if log is not None:
            log(len(losses), losses[-1])
    return losses


def _rel(x, ref):
    return float(torch.linalg.vector_norm(x - ref) / torch.linalg.vector_norm(ref))


def evaluate(ctx, net, items):
    """Per system: relative Frobenius errors against the full sum, for chi0 and
    eps^-1, of the truncated sum and of the network's prediction (inferred
    without the full sum); then the judged call (with the full sum), whether it
    fell back to the full sum and the error of what it returned."""
    rows = []
    for it in items:
        out = torch.empty_like(it["chi_f"])
        B.gw_chi0_closure(ctx, net, B.GW_CLOSURE_INFER, it["neps"], it["qg"], it["chi_t"],
                          it["gap"], it["emax"], chi0_out=out)
        judged = torch.empty_like(it["chi_f"])
        st, _ = B.gw_chi0_closure(ctx, net, B.GW_CLOSURE_INFER, it["neps"], it["qg"],
                                  it["chi_t"], it["gap"], it["emax"], chi0_full=it["chi_f"],
                                  chi0_out=judged)
        n = it["neps"]
        inv = {}
        for key, chi in (("t", it["chi_t"]), ("c", out), ("f", it["chi_f"])):
            e = torch.empty((1, n, n), dtype=torch.complex128, device=chi.device)
            B.gw_epsinv(ctx, n, 1, chi.reshape(1, n, n).contiguous(), it["vcoul"], e)
            inv[key] = e[0]
        torch.cuda.synchronize()
        rows.append(dict(
            name=it["name"], neps=n, fallback=st == B.GW_EFALLBACK,
            chi_judged=_rel(judged, it["chi_f"]),
            chi_trunc=_rel(it["chi_t"], it["chi_f"]), chi_closure=_rel(out, it["chi_f"]),
            epsinv_trunc=_rel(inv["t"], inv["f"]), epsinv_closure=_rel(inv["c"], inv["f"]),
        ))
    return rows
