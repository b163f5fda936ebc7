"""FP64 oracle of the learned band-sum closure.  TEST INFRASTRUCTURE ONLY.

The paper has no learned component.  Its nearest relative is the static
remainder for the Coulomb-hole sum over empty states (Computational Details),
a cheap estimate of what a truncated band sum leaves out.  The closure here
predicts chi0_full - chi0_trunc from per-(G, G') features.  That is a
heuristic, so this oracle is its written-out algorithm:

  features   f(G,G') = [|q+G|, |q+G'|, (q+G).(q+G')/10, Re chi_t/s, Im chi_t/s,
                        10*gap, 2*emax]  for G <= G' (upper triangle, row major),
             s = max_G |chi_t[G][G]|  (per-system scale)
  network    h0 = f (zero-padded to kin), h_l = SiLU(h_{l-1} W_l^T + b_l) for the
             hidden layers, y = h_L W_out^T + b_out;  y = remainder / s
  loss       mean over rows < n and the nout real outputs of (y - t)^2
  update     Adam with bias correction
  result     chi_out = chi_t + s * Hermitise(y): (G,G') gets y, (G',G) its conjugate

What the network should output is not fixed by the paper: the full band sum
is the judge of its error.  The functions themselves are pinned independently:
the forward pass and the gradients by torch's float64 autograd of the same SiLU
network (and the gradients also by central finite differences), the Adam update
by torch.optim.Adam over several steps, and the feature table by a hand-built
three-vector case.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "closure_features", "closure_scale", "mlp_forward", "mlp_loss_and_grads", "adam_step",
    "closure_apply", "closure_target", "init_params", "silu",
]


def closure_scale(chi_t):
    return float(np.abs(np.diag(chi_t)).max())


def closure_features(qg, chi_t, gap, emax):
    """Per-(G <= G') features, row-major over the upper triangle."""
    qg = np.asarray(qg, dtype=np.float64)
    n = qg.shape[0]
    iu, ju = np.triu_indices(n)
    s = closure_scale(chi_t)
    norm = np.linalg.norm(qg, axis=1)
    dot = np.einsum("ij,ij->i", qg[iu], qg[ju])
    c = chi_t[iu, ju]
    f = np.stack([norm[iu], norm[ju], dot / 10.0, c.real / s, c.imag / s,
                  np.full(len(iu), 10.0 * gap), np.full(len(iu), 2.0 * emax)], axis=1)
    return f, (iu, ju), s


def closure_target(chi_t, chi_full, s):
    n = chi_t.shape[0]
    iu, ju = np.triu_indices(n)
    r = (chi_full - chi_t)[iu, ju] / s
    return np.stack([r.real, r.imag], axis=1)


def silu(z):
    return z / (1.0 + np.exp(-z))


def _dsilu(z):
    sg = 1.0 / (1.0 + np.exp(-z))
    return sg * (1.0 + z * (1.0 - sg))


def init_params(rng, dims):
    """Glorot-uniform weights, zero biases: dims = [kin, width, ..., nout]."""
    ps = []
    for a, b in zip(dims[:-1], dims[1:]):
        lim = np.sqrt(6.0 / (a + b))
        ps.append((rng.uniform(-lim, lim, (b, a)), np.zeros(b)))
    return ps


def mlp_forward(params, x):
    """Returns y and the per-layer (input, pre-activation) caches."""
    h = np.asarray(x, dtype=np.float64)
    cache = []
    for l, (w, b) in enumerate(params):
        z = h @ w.T + b
        cache.append((h, z))
        h = silu(z) if l < len(params) - 1 else z
    return h, cache


def mlp_loss_and_grads(params, x, t, nout=None):
    """MSE over the real outputs and its gradients by backpropagation."""
    y, cache = mlp_forward(params, x)
    nout = y.shape[1] if nout is None else nout
    diff = np.zeros_like(y)
    diff[:, :nout] = y[:, :nout] - t[:, :nout]
    count = y.shape[0] * nout
    loss = float((diff ** 2).sum() / count)
    g = 2.0 * diff / count
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        h, z = cache[l]
        if l < len(params) - 1:
            g = g * _dsilu(z)
        w, _ = params[l]
        grads[l] = (g.T @ h, g.sum(axis=0))
        g = g @ w
    return loss, grads


def adam_step(params, grads, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new params, m, v."""
    out_p, out_m, out_v = [], [], []
    for (w, b), (gw, gb), (mw, mb), (vw, vb) in zip(params, grads, m, v):
        new = []
        for p_, g_, m_, v_ in ((w, gw, mw, vw), (b, gb, mb, vb)):
            m2 = b1 * m_ + (1 - b1) * g_
            v2 = b2 * v_ + (1 - b2) * g_ * g_
            mh = m2 / (1 - b1 ** step)
            vh = v2 / (1 - b2 ** step)
            new.append((p_ - lr * mh / (np.sqrt(vh) + eps), m2, v2))
        out_p.append((new[0][0], new[1][0]))
        out_m.append((new[0][1], new[1][1]))
        out_v.append((new[0][2], new[1][2]))
    return out_p, out_m, out_v


def closure_apply(chi_t, y, s):
    """chi_t + s * Hermitise(y) with y the (Re, Im) remainder on the upper triangle."""
    n = chi_t.shape[0]
    iu, ju = np.triu_indices(n)
    r = np.zeros((n, n), dtype=np.complex128)
    r[iu, ju] = (y[:, 0] + 1j * y[:, 1]) * s
    r = r + np.triu(r, 1).conj().T
    d = np.arange(n)
    r[d, d] = r[d, d].real
    return chi_t + r
