"""Pins of the surrogate MLP oracle (CPU): BF16 rounding against torch's
bfloat16 conversion, backward against central finite differences, the
gradient of a linear layer against the normal equations of least squares,
and Adam's first step in closed form."""
import numpy as np
import pytest
import torch

from oracle import mlp_oracle as M


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 1, 10000), rng.normal(0, 1e-3, 1000), rng.normal(0, 1e4, 1000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 65504.0, 1e-30]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.bf16_round(x), ref)


def test_backward_matches_finite_differences():
    """FP64 network (no rounding): analytic gradients vs central differences."""
    layers = (7, 11, 9, 6, 3)
    rng = np.random.default_rng(1)
    params = M.init_params(2, layers)
    params = [(W, rng.normal(0, 0.1, b.shape)) for W, b in params]
    x = rng.normal(size=(13, 7))
    t = rng.normal(size=(13, 3))

    def loss(p):
        y, _ = M.forward(p, x, bf16=False)
        return M.mse_loss(y, t)[0]

    y, cache = M.forward(params, x, bf16=False)
    _, dy = M.mse_loss(y, t)
    grads, dx = M.backward(params, cache, dy, bf16=False)
    h = 1e-6
    for li, (W, b) in enumerate(params):
        for which, arr in ((0, W), (1, b)):
            for idx in np.ndindex(arr.shape):
                pp = [(a.copy(), c.copy()) for a, c in params]
                pm = [(a.copy(), c.copy()) for a, c in params]
                pp[li][which][idx] += h
                pm[li][which][idx] -= h
                fd = (loss(pp) - loss(pm)) / (2 * h)
                an = grads[li][which][idx]
                assert abs(fd - an) <= 1e-7 * max(1e-3, abs(an)) + 1e-9, (li, which, idx, fd, an)
    # input gradient too
    for idx in np.ndindex(x.shape):
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fp = M.mse_loss(M.forward(params, xp, bf16=False)[0], t)[0]
        fm = M.mse_loss(M.forward(params, xm, bf16=False)[0], t)[0]
        assert abs((fp - fm) / (2 * h) - dx[idx]) <= 1e-7 * max(1e-3, abs(dx[idx])) + 1e-9


def test_linear_layer_gradient_is_normal_equations():
    """One linear layer (no activation after the last layer): the MSE gradient
    is 2 X^T (X W + b - T) / (n m) and vanishes at the least-squares solution."""
    rng = np.random.default_rng(3)
    n, k, m = 200, 6, 4
    x = rng.normal(size=(n, k))
    t = rng.normal(size=(n, m))
    X1 = np.hstack([x, np.ones((n, 1))])
    sol = np.linalg.lstsq(X1, t, rcond=None)[0]
    params = [(sol[:k].copy(), sol[k].copy())]
    y, cache = M.forward(params, x, bf16=False)
    _, dy = M.mse_loss(y, t)
    (gW, gb), = M.backward(params, cache, dy, bf16=False)[0]
    assert np.abs(gW).max() < 1e-13 and np.abs(gb).max() < 1e-13
    W = rng.normal(size=(k, m))
    b = rng.normal(size=m)
    y, cache = M.forward([(W, b)], x, bf16=False)
    _, dy = M.mse_loss(y, t)
    (gW, gb), = M.backward([(W, b)], cache, dy, bf16=False)[0]
    R = x @ W + b - t
    assert np.allclose(gW, 2 * x.T @ R / (n * m), rtol=1e-12, atol=1e-15)
    assert np.allclose(gb, 2 * R.sum(axis=0) / (n * m), rtol=1e-12, atol=1e-15)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(4)
    params = [(rng.normal(size=(5, 3)), rng.normal(size=3))]
    grads = [(rng.normal(size=(5, 3)), rng.normal(size=3))]
    opt = M.Adam(params, lr=1e-3)
    new = opt.step(params, grads)
    for (W, b), (W1, b1), (gW, gb) in zip(params, new, grads):
        assert np.allclose(W1, W - 1e-3 * gW / (np.abs(gW) + 1e-8), rtol=0, atol=1e-15)
        assert np.allclose(b1, b - 1e-3 * gb / (np.abs(gb) + 1e-8), rtol=0, atol=1e-15)


def test_flatten_roundtrip_and_count():
    p = M.init_params(5)
    v = M.flatten(p)
    assert v.size == 96 * 256 + 256 + 2 * (256 * 256 + 256) + 256 * 12 + 12
    q = M.unflatten(v)
    for (a, b), (c, d) in zip(p, q):
        assert np.array_equal(a, c) and np.array_equal(b, d)


def test_silu_matches_torch_and_its_identities():
    """The forward's activation against torch's SiLU (a library routine) in
    FP64 over a wide range, and the identities that fix x * sigmoid(x): it
    vanishes at 0, silu(x) - silu(-x) = x, it tends to x and to 0 in the two
    tails; its derivative against torch's autograd of the same routine."""
    rng = np.random.default_rng(3)
    z = np.concatenate([rng.normal(0, 3, 5000), np.linspace(-40, 40, 801), [0.0, 1e-12, -1e-12, 700.0, -700.0]])
    ref = torch.nn.functional.silu(torch.tensor(z, dtype=torch.float64)).numpy()
    assert np.allclose(M.silu(z), ref, rtol=1e-14, atol=1e-300)
    assert M.silu(0.0) == 0.0
    assert np.allclose(M.silu(z) - M.silu(-z), z, rtol=1e-13, atol=1e-13)
    assert abs(M.silu(50.0) - 50.0) < 1e-15 * 50 * 10 and abs(M.silu(-50.0)) < 1e-19
    t = torch.tensor(z, dtype=torch.float64, requires_grad=True)
    torch.nn.functional.silu(t).sum().backward()
    assert np.allclose(M.dsilu(z), t.grad.numpy(), rtol=1e-13, atol=1e-300)
