"""Learned warm start on the GPU: features, forward and gradients of the library's own
kernels against the FP64 NumPy reference; training lowers the loss; a trained network's
x0 never changes the answer (true FP64 residual) and its iteration gain is reported."""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import nn as R
from paper_1305_6653_amd import warmstart as WS

pytestmark = pytest.mark.gpu

TINY = dict(m=15, s=8, conv_ch=(4, 4, 3), fc=(8, 6), nx=4, nt=3)


def _bf16(x):
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _tiny_batch(B, seed):
    import torch
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(seed)
    ps = [W.random_instance(seed * 100 + i, m=TINY["m"], s=TINY["s"], zero_u0=True) for i in range(B)]
    T = rng.standard_normal((B, TINY["s"] * TINY["m"]))
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
    return ps, [d(p.f) for p in ps], [d(p.d_plus) for p in ps], [d(p.d_minus) for p in ps], T, d


def test_features_forward_and_gradients_match_reference():
    import torch
    B = 4
    net = WS.WarmStartNet(max_batch=B, seed=3, **TINY)
    cfg = R.NetConfig(**TINY)
    assert net.num_params == cfg.num_params()
    rng = np.random.default_rng(5)
    theta = (rng.standard_normal(net.num_params) * 0.3).astype(np.float32)
    net.set_params(theta)
    ps, fs, dps, dms, T, d = _tiny_batch(B, 1)
    X = torch.zeros((B, 256, net.cin), dtype=torch.float32, device="cuda:0")
    rms = torch.zeros(B, dtype=torch.float32, device="cuda:0")
    net.features(fs, dps, dms, [p.alpha for p in ps], X, rms)
    Xr, rr = zip(*[R.features(cfg, p.f, p.d_plus, p.d_minus, p.alpha) for p in ps])
    np.testing.assert_allclose(X.cpu().numpy(), np.array(Xr), rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(rms.cpu().numpy(), np.array(rr), rtol=1e-6)
    Td = d(T)
    loss = net.loss_grad(X, Td, rms, None, B)
    g = net.get(1)
    # reference that rounds every product's operands to bf16 as the GPU's GEMMs do (weights,
    # activations, back-propagated gradients, synthesis basis); biases and sums stay wide
    th = theta.astype(np.float64)
    loss_r, g_r = R.loss_and_grad(cfg, th, list(Xr), list(T), list(rr), q=_bf16)
    assert abs(loss - loss_r) <= 1e-2 * loss_r, (loss, loss_r)
    # every parameter tensor (each layer's weights and its bias) against its own norm
    for li, ((gW, gb), (rW, rb)) in enumerate(zip(R.unpack(cfg, g.astype(np.float64)), R.unpack(cfg, g_r))):
        for name, a, b in (("W", gW, rW), ("b", gb, rb)):
            err = np.linalg.norm(a - b) / np.linalg.norm(b)
            assert err <= 1e-2, (li, name, err)
    U = net.output(B)
    Ur = np.array([R.forward(cfg, th, x, q=_bf16)[0] for x in Xr])
    assert np.linalg.norm(U - Ur) <= 1e-2 * np.linalg.norm(Ur)
    net.close()


def test_training_lowers_loss_and_checkpoint_resume():
    """A short training run on real solver data lowers the loss; resuming from a checkpoint
    continues bitwise like the uninterrupted run."""
    make = lambda sd: W.random_instance(sd, m=63, s=32, zero_u0=True)
    net = WS.WarmStartNet(m=63, s=32, max_batch=32, conv_ch=(32, 32, 16), fc=(128, 128), nx=16,
                          nt=8, seed=1)
    data = WS.build_dataset(list(range(256)), net, make, batch=32)
    assert np.all(data["iters"] > 0)
    ck = net.checkpoint()
    h1 = WS.train(net, data, epochs=2, batch=32, lr=1e-3, seed=7)
    p_a = net.get(0)
    net2 = WS.WarmStartNet(m=63, s=32, max_batch=32, conv_ch=(32, 32, 16), fc=(128, 128), nx=16,
                           nt=8, seed=99)
    net2.restore(ck)
    h2 = WS.train(net2, data, epochs=2, batch=32, lr=1e-3, seed=7)
    assert h1 == h2 and np.array_equal(p_a, net2.get(0))
    h3 = WS.train(net, data, epochs=8, batch=32, lr=1e-3, seed=8)
    assert h3[-1] < 0.5 * h1[0], (h1, h3)
    net.close()
    net2.close()


@pytest.mark.slow
@pytest.mark.parametrize("target", ["solution", "lowrank"])
def test_trained_warm_start_keeps_answers_and_reports_gain(target):
    """Train on 2048 solved instances of the warm-start workload (m=255, s=128), evaluate on
    64 held-out seeds: every warm-started solve reaches true residual 1e-10, and the change in
    iterations (which may be a loss) is recorded."""
    if target == "lowrank":
        rows = WS.boundary_rows(2, 3, 128)
        net = WS.WarmStartNet(max_batch=64, seed=0, nx=255, nt=len(rows))
        net.use_boundary_rows(rows)
    else:
        net = WS.WarmStartNet(max_batch=64, seed=0)
    data = WS.build_dataset(list(range(2048)), net, W.warmstart_instance, batch=64, target=target)
    WS.train(net, data, epochs=6, batch=64, lr=1e-3)
    res = WS.evaluate(net, list(range(1_000_000, 1_000_064)), W.warmstart_instance, target=target)
    assert all(r <= 1e-10 for r in res["relres_warm"])
    # a guard, not a gain: the start is projected so that ||r_0|| <= ||b||, and the
    # iteration count of this preconditioned GMRES responds only logarithmically to the
    # start, so a guess with a few per cent of error costs at most a few iterations
    assert np.mean(res["iters_warm"]) <= np.mean(res["iters_zero"]) + 3.0
    out = {k: (float(np.mean(v)) if isinstance(v, list) else v) for k, v in res.items()}
    out_dir = os.environ.get("FDE_EVAL_DIR")  # optional: keep the evaluation as JSON
    if out_dir:
        os.makedirs(out_dir, exist_ok=True)
        with open(os.path.join(out_dir, f"warmstart_small_eval_{target}.json"), "w") as fh:
            json.dump(out, fh)
    print(f"warm start ({target}, 2048 training instances):", out)
