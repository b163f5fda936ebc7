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


# ------------------------------------------------------------------ independent pins
# torch's CPU float64 autograd and its Adam are written independently of the
# oracle: they pin the forward pass, the backward pass and the update rule at
# every step, not only at the first.
import torch  # noqa: E402


def _torch_net(params):
    return [(torch.tensor(w, dtype=torch.float64, requires_grad=True),
             torch.tensor(b, dtype=torch.float64, requires_grad=True)) for w, b in params]


def _torch_forward(tp, x):
    h = torch.as_tensor(x, dtype=torch.float64)
    for l, (w, b) in enumerate(tp):
        h = torch.nn.functional.linear(h, w, b)
        if l < len(tp) - 1:
            h = torch.nn.functional.silu(h)
    return h


def _random_net(seed, dims):
    rng = np.random.default_rng(seed)
    params = [(w, rng.normal(size=b.shape) * 0.2) for w, b in oracle.init_params(rng, dims)]
    return rng, params


def test_forward_matches_torch_silu_mlp():
    rng, params = _random_net(10, [7, 256, 256, 256, 2])
    x = rng.normal(size=(33, 7)) * 2.0
    y, _ = oracle.mlp_forward(params, x)
    want = _torch_forward(_torch_net(params), x).detach().numpy()
    assert np.abs(y - want).max() <= 1e-12 * np.abs(want).max()


def test_backprop_matches_torch_autograd():
    rng, params = _random_net(11, [7, 32, 24, 16, 4])
    x = rng.normal(size=(19, 7))
    t = rng.normal(size=(19, 4))
    loss, grads = oracle.mlp_loss_and_grads(params, x, t, nout=2)
    tp = _torch_net(params)
    y = _torch_forward(tp, x)
    tl = ((y[:, :2] - torch.as_tensor(t[:, :2])) ** 2).mean()
    tl.backward()
    assert abs(loss - tl.item()) <= 1e-13 * abs(tl.item())
    for (gw, gb), (w, b) in zip(grads, tp):
        assert np.abs(gw - w.grad.numpy()).max() <= 1e-12 * max(1e-30, np.abs(w.grad.numpy()).max())
        assert np.abs(gb - b.grad.numpy()).max() <= 1e-12 * max(1e-30, np.abs(b.grad.numpy()).max())


def _adam_gap_to_torch(step_fn, nsteps=5, lr=3e-3, b1=0.9, b2=0.999, eps=1e-8):
    """Largest relative difference between `step_fn` (the oracle's signature) and
    torch.optim.Adam over `nsteps` steps with fresh gradients each step."""
    rng, params = _random_net(12, [5, 7, 3])
    tp = _torch_net(params)
    opt = torch.optim.Adam([p for pair in tp for p in pair], lr=lr, betas=(b1, b2), eps=eps)
    m = [(np.zeros_like(w), np.zeros_like(b)) for w, b in params]
    v = [(np.zeros_like(w), np.zeros_like(b)) for w, b in params]
    gap = 0.0
    for step in range(1, nsteps + 1):
        grads = [(rng.normal(size=w.shape), rng.normal(size=b.shape)) for w, b in params]
        params, m, v = step_fn(params, grads, m, v, step, lr, b1, b2, eps)
        for (w, b), (gw, gb) in zip(tp, grads):
            w.grad = torch.tensor(gw)
            b.grad = torch.tensor(gb)
        opt.step()
        for (w, b), (tw, tb) in zip(params, tp):
            for a, ta in ((w, tw), (b, tb)):
                ta = ta.detach().numpy()
                gap = max(gap, float(np.abs(a - ta).max() / np.abs(ta).max()))
    return gap


def test_adam_matches_torch_over_several_steps():
    assert _adam_gap_to_torch(oracle.adam_step) <= 1e-13


def test_adam_pin_catches_a_wrong_bias_correction_power():
    """A planted mistake in a copy of the oracle's update (the bias corrections
    use the power step - 1 from the second step on) must fail the torch pin."""
    def planted(params, grads, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
        out_p, out_m, out_v = [], [], []
        for (w, b), (gw, gb), (mw, mb), (vw, vb) in zip(params, grads, m, v):
            new = []
            for p_, g_, m_, v_ in ((w, gw, mw, vw), (b, gb, mb, vb)):
                m2 = b1 * m_ + (1 - b1) * g_
                v2 = b2 * v_ + (1 - b2) * g_ * g_
                k = step if step == 1 else step - 1
                mh = m2 / (1 - b1 ** k)
                vh = v2 / (1 - b2 ** k)
                new.append((p_ - lr * mh / (np.sqrt(vh) + eps), m2, v2))
            out_p.append((new[0][0], new[1][0]))
            out_m.append((new[0][1], new[1][1]))
            out_v.append((new[0][2], new[1][2]))
        return out_p, out_m, out_v

    assert _adam_gap_to_torch(planted, nsteps=1) <= 1e-13   # identical at step 1
    assert _adam_gap_to_torch(planted) > 1e-6


def test_features_of_a_hand_built_three_vector_case():
    """Every entry of the feature table written out by hand for three vectors."""
    qg = np.array([[1.0, 0.0, 0.0], [0.0, 2.0, 0.0], [3.0, 4.0, 0.0]])
    chi = np.array([[-4.0, 1 + 2j, -2j], [1 - 2j, -2.0, 0.5], [2j, 0.5, -1.0]])
    gap, emax = 0.05, 0.7
    f, (iu, ju), s = oracle.closure_features(qg, chi, gap, emax)
    assert s == 4.0
    # upper triangle, row major: (0,0) (0,1) (0,2) (1,1) (1,2) (2,2)
    want = np.array([
        [1.0, 1.0, 0.1, -1.0, 0.0, 0.5, 1.4],
        [1.0, 2.0, 0.0, 0.25, 0.5, 0.5, 1.4],
        [1.0, 5.0, 0.3, 0.0, -0.5, 0.5, 1.4],
        [2.0, 2.0, 0.4, -0.5, 0.0, 0.5, 1.4],
        [2.0, 5.0, 0.8, 0.125, 0.0, 0.5, 1.4],
        [5.0, 5.0, 2.5, -0.25, 0.0, 0.5, 1.4],
    ])
    assert list(iu) == [0, 0, 0, 1, 1, 2] and list(ju) == [0, 1, 2, 1, 2, 2]
    assert np.allclose(f, want, rtol=0, atol=1e-15)
