"""Pins of the FP64 closure oracle: backprop against central differences, the
closed form of Adam's first step, Hermitian output."""
import numpy as np

import oracle


def _net(rng, dims):
    return oracle.init_params(rng, dims)


def test_backprop_matches_central_differences():
    rng = np.random.default_rng(0)
    dims = [8, 6, 5, 4, 3]
    params = _net(rng, dims)
    params = [(w, rng.normal(size=b.shape) * 0.1) for w, b in params]
    x = rng.normal(size=(11, 8))
    t = rng.normal(size=(11, 3))
    loss, grads = oracle.mlp_loss_and_grads(params, x, t, nout=2)
    h = 1e-6
    for l in range(len(params)):
        w, b = params[l]
        for (arr, g) in ((w, grads[l][0]), (b, grads[l][1])):
            idxs = [tuple(rng.integers(0, s) for s in arr.shape) for _ in range(5)]
            for ix in idxs:
                old = arr[ix]
                arr[ix] = old + h
                lp, _ = oracle.mlp_loss_and_grads(params, x, t, nout=2)
                arr[ix] = old - h
                lm, _ = oracle.mlp_loss_and_grads(params, x, t, nout=2)
                arr[ix] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - g[ix]) <= 1e-7 * max(1.0, abs(fd)), (l, ix, fd, g[ix])


def test_padded_outputs_get_no_gradient():
    rng = np.random.default_rng(1)
    params = _net(rng, [4, 5, 3])
    x = rng.normal(size=(7, 4))
    t = rng.normal(size=(7, 3))
    _, grads = oracle.mlp_loss_and_grads(params, x, t, nout=2)
    assert np.all(grads[-1][0][2] == 0) and grads[-1][1][2] == 0


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(2)
    params = _net(rng, [3, 4, 2])
    grads = [(rng.normal(size=w.shape), rng.normal(size=b.shape)) for w, b in params]
    zeros = [(np.zeros_like(w), np.zeros_like(b)) for w, b in params]
    lr = 1e-2
    new, m, v = oracle.adam_step(params, grads, zeros, zeros, 1, lr)
    for (w, b), (gw, gb), (nw, nb) in zip(params, grads, new):
        # first step: m^ = g, v^ = g^2 -> update = lr g / (|g| + eps)
        assert np.allclose(nw, w - lr * gw / (np.abs(gw) + 1e-8), rtol=0, atol=1e-15)
        assert np.allclose(nb, b - lr * gb / (np.abs(gb) + 1e-8), rtol=0, atol=1e-15)


def test_features_and_hermitian_apply():
    rng = np.random.default_rng(3)
    n = 6
    qg = rng.normal(size=(n, 3))
    a = rng.normal(size=(n, 9)) + 1j * rng.normal(size=(n, 9))
    chi = -(a @ a.conj().T)
    f, (iu, ju), s = oracle.closure_features(qg, chi, 0.05, 0.7)
    assert f.shape == (n * (n + 1) // 2, 7)
    assert np.isclose(s, np.abs(np.diag(chi)).max())
    k = 4
    assert np.isclose(f[k, 2] * 10, qg[iu[k]] @ qg[ju[k]])
    y = rng.normal(size=(f.shape[0], 2))
    out = oracle.closure_apply(chi, y, s)
    assert np.allclose(out, out.conj().T)
    full = chi * 1.7
    t = oracle.closure_target(chi, full, s)
    assert np.allclose(oracle.closure_apply(chi, t, s), full)
