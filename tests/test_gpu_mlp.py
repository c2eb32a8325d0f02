"""GPU parity of the surrogate network (BF16 MFMA kernels) against the FP64
oracle with the same BF16 rounding points.

Bars: outputs normwise rel <= 1e-3 (FP32 accumulation vs FP64 sums can flip
an activation's BF16 rounding now and then: one BF16 ulp is 2^-8); weight
gradients Frobenius rel <= 1e-2 per layer (the GPU also rounds dZ to BF16 as
an MFMA input); Adam's first step equals w - lr g / (|g| + eps) to FP32
rounding with the GPU's own gradient."""
import numpy as np
import pytest

from oracle import mlp_oracle as M

pytestmark = pytest.mark.gpu


def _setup(M_rows=256, seed=7):
    import torch
    from paper_2605_13766_amd import rod
    rng = np.random.default_rng(seed)
    params = M.init_params(seed)
    params = [(W, rng.normal(0, 0.05, b.shape)) for W, b in params]
    x = M.bf16_round(rng.normal(0, 1, (M_rows, 96)))
    t = rng.normal(0, 1, (M_rows, 12))
    mask = (rng.uniform(size=(M_rows, 12)) > 0.2).astype(np.float64)
    dev = torch.device("cuda")
    xt = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(dev)
    tt = torch.tensor(t, dtype=torch.float32, device=dev)
    mt = torch.tensor(mask, dtype=torch.float32, device=dev)
    s = rod.Surrogate(k_substeps=32, seed=1, max_rows=1024)
    s.set_params(M.flatten(params))
    return s, params, x, t, mask, xt, tt, mt


def test_params_roundtrip():
    s, params, *_ = _setup()
    got = s.get_params()
    assert np.array_equal(got, M.flatten(params).astype(np.float32))
    s.close()


@pytest.mark.parametrize("rows", [32, 256, 1000 // 32 * 32])
def test_forward_parity(rows):
    import torch
    s, params, x, t, mask, xt, tt, mt = _setup(rows)
    y = torch.empty((rows, 12), dtype=torch.float32, device="cuda")
    s.forward(xt, y)
    torch.cuda.synchronize()
    ref, _ = M.forward(params, x, bf16=True)
    got = y.cpu().numpy().astype(np.float64)
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print("forward normwise rel", rel)
    assert rel < 1e-3
    s.close()


def test_forward_multi_chunk():
    """More rows than the workspace holds: processed in chunks."""
    import torch
    s, params, x, t, mask, xt, tt, mt = _setup(2048 + 96, seed=9)
    y = torch.empty((xt.shape[0], 12), dtype=torch.float32, device="cuda")
    s.forward(xt, y)
    torch.cuda.synchronize()
    ref, _ = M.forward(params, x, bf16=True)
    assert np.linalg.norm(y.cpu().numpy() - ref) / np.linalg.norm(ref) < 1e-3
    s.close()


def test_gradient_parity():
    s, params, x, t, mask, xt, tt, mt = _setup(512, seed=11)
    g, loss = s.gradients(xt, tt, mt)
    y, cache = M.forward(params, x, bf16=True)
    ref_loss, dy = M.mse_loss(y, t, mask)
    grads, _ = M.backward(params, cache, dy, bf16=True)
    assert abs(loss - ref_loss) / ref_loss < 1e-3
    ref = M.flatten(grads)
    gu = M.unflatten(g.astype(np.float64))
    for li, ((gW, gb), (rW, rb)) in enumerate(zip(gu, grads)):
        eW = np.linalg.norm(gW - rW) / np.linalg.norm(rW)
        eb = np.linalg.norm(gb - rb) / np.linalg.norm(rb)
        print(f"layer {li}: dW rel {eW:.2e}, db rel {eb:.2e}")
        assert eW < 1e-2 and eb < 1e-2
    assert np.linalg.norm(g - ref) / np.linalg.norm(ref) < 1e-2
    s.close()


def test_adam_first_step():
    s, params, x, t, mask, xt, tt, mt = _setup(256, seed=13)
    g, _ = s.gradients(xt, tt, mt)
    p0 = s.get_params().astype(np.float64)
    lr = 1e-3
    s.train_step(xt, tt, mt, lr=lr)
    p1 = s.get_params().astype(np.float64)
    exp = p0 - lr * g / (np.abs(g) + 1e-8)
    assert np.abs(p1 - exp).max() < 2e-3 * lr + 1e-7
    s.close()


def test_training_reduces_loss():
    """A few hundred Adam steps on a fixed random regression task."""
    import torch
    s, params, x, t, mask, xt, tt, mt = _setup(1024, seed=15)
    # learnable targets: a smooth function of the inputs
    tgt = np.tanh(x[:, :12] + 0.5 * x[:, 12:24])
    tt = torch.tensor(tgt, dtype=torch.float32, device="cuda")
    first = s.train_step(xt, tt, None, lr=1e-3)
    for _ in range(300):
        last = s.train_step(xt, tt, None, lr=1e-3)
    print("loss", first, "->", last)
    assert last < 0.2 * first
    s.close()
