"""Control-variate MLP on the matrix cores against the FP64 oracle that rounds
to bfloat16 at the same points."""
import numpy as np
import pytest

import oracle
from tests.test_oracle_cv_pins import rand_net

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def W():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_04403_amd import wob
    wob.lib()
    return wob


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def test_forward_matches_bf16_oracle(W):
    params, B = rand_net(11)
    params, B = f32(params), f32(B)
    y = f32(np.random.default_rng(1).uniform(-1.5, 1.5, (1000, 3)))  # ragged: 15 tiles + 40 rows
    net = W.MLP(3, B, params)
    out = net.forward(torch.as_tensor(y, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    g = out.cpu().double().numpy()
    o = oracle.mlp_forward(params, B, y, bf16=True)
    rel = np.abs(g - o) / np.maximum(np.abs(o), 1e-3)
    print(f"forward: median rel {np.median(rel):.2e}, 99% {np.quantile(rel, 0.99):.2e}, "
          f"within 1e-5: {np.mean(rel <= 1e-5):.3f}, normwise {np.linalg.norm(g - o) / np.linalg.norm(o):.2e}")
    # identical rounding points: most outputs agree to binary32 accumulation error;
    # the rest differ by an occasional bfloat16 rounding flip
    assert np.median(rel) < 1e-5
    assert np.linalg.norm(g - o) <= 2e-3 * np.linalg.norm(o)
    net.close()


def test_gradient_matches_bf16_oracle(W):
    params, B = rand_net(12)
    params, B = f32(params), f32(B)
    rng = np.random.default_rng(2)
    y = f32(rng.uniform(-1.5, 1.5, (300, 3)))
    t = f32(rng.standard_normal(300))
    net = W.MLP(3, B, params, max_batch=512)
    loss, grad = net.backward(torch.as_tensor(y, dtype=torch.float32, device="cuda"),
                              torch.as_tensor(t, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    lo, go = oracle.mlp_loss_grad(params, B, y, t, bf16=True)
    gg = grad.cpu().double().numpy()
    assert loss.item() == pytest.approx(lo, rel=2e-3)
    err = np.linalg.norm(gg - go) / np.linalg.norm(go)
    print(f"gradient normwise relative error {err:.2e}")
    assert err <= 1e-2
    # per layer block
    offs = [0, 4096, 4224, 20608, 20736, 37120, 37248, 53632, 53760, 53888, 53889]
    for a, b in zip(offs[:-1], offs[1:]):
        e = np.linalg.norm(gg[a:b] - go[a:b]) / max(np.linalg.norm(go[a:b]), 1e-12)
        assert e <= 2e-2, (a, b, e)
    net.close()


def test_target_map_is_applied_inside_the_loss(W):
    """Raw targets with (shift, scale, clip) on the GPU against the oracle given
    the mapped targets (t - shift) / scale clamped to [-clip, clip]."""
    params, B = rand_net(14)
    params, B = f32(params), f32(B)
    rng = np.random.default_rng(4)
    y = f32(rng.uniform(-1.5, 1.5, (700, 3)))
    t = f32(rng.standard_cauchy(700) * 3.0 + 2.0)
    shift, scale, clip = 2.0, 3.0, 4.0
    net = W.MLP(3, B, params, max_batch=1024)
    loss, grad = net.backward(torch.as_tensor(y, dtype=torch.float32, device="cuda"),
                              torch.as_tensor(t, dtype=torch.float32, device="cuda"),
                              target_map=(shift, scale, clip))
    torch.cuda.synchronize()
    tm = np.clip((t.astype(np.float64) - shift) / scale, -clip, clip)
    assert np.sum(np.abs(tm) == clip) > 20  # the clamp is exercised
    lo, go = oracle.mlp_loss_grad(params, B, y, tm, bf16=True)
    assert loss.item() == pytest.approx(lo, rel=2e-3)
    assert np.linalg.norm(grad.cpu().double().numpy() - go) <= 1e-2 * np.linalg.norm(go)
    with pytest.raises(W.WobError):
        net.backward(torch.as_tensor(y, dtype=torch.float32, device="cuda"),
                     torch.as_tensor(t, dtype=torch.float32, device="cuda"), target_map=(0.0, 0.0, 1.0))
    net.close()


def test_adam_matches_oracle_and_training_reduces_loss(W):
    params, B = rand_net(13)
    params, B = f32(params), f32(B)
    rng = np.random.default_rng(3)
    y = f32(rng.uniform(-1.2, 1.2, (2048, 3)))
    t = f32(np.sin(2 * y[:, 0]) + y[:, 1] * y[:, 2])
    net = W.MLP(3, B, params, max_batch=2048)
    ty = torch.as_tensor(y, dtype=torch.float32, device="cuda")
    tt = torch.as_tensor(t, dtype=torch.float32, device="cuda")
    # one Adam step on a given gradient, against the oracle's
    loss, grad = net.backward(ty, tt)
    net.adam_step(grad, 1, 1e-3)
    torch.cuda.synchronize()
    p_gpu = net.params().astype(np.float64)
    p_o, m_o, v_o = params.copy(), np.zeros_like(params), np.zeros_like(params)
    oracle.adam_step(p_o, m_o, v_o, grad.cpu().double().numpy(), 1, 1e-3)
    np.testing.assert_allclose(p_gpu, p_o, rtol=1e-5, atol=2e-7)
    # and a short training run lowers the loss
    net.set_params(params)
    l0 = net.backward(ty, tt)[0].item()
    lbuf = torch.empty(1, dtype=torch.float32, device="cuda")
    for step in range(1, 201):
        net.train_step(ty, tt, step, 3e-3, loss=lbuf)
    torch.cuda.synchronize()
    l1 = net.backward(ty, tt)[0].item()
    print(f"loss {l0:.4f} -> {l1:.4f}")
    assert l1 < 0.2 * l0
    net.close()
