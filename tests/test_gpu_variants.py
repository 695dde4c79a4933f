"""The two training variants on the GPU (tanh hidden activation, heavy-ball
momentum; section 2.2's method is the sigmoid network without momentum)
against the FP64 oracle's variants: the fused small trainer, the layer
kernels behind mlp_forward / mlp_backward / mlp_step, resumability with the
velocity carried across calls, and the trainers that reject them."""
import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import Params
from paper_1908_07847_amd import synth
from paper_1908_07847_amd._lib import MLP_ERR_UNSUPPORTED, MLPError

pytestmark = pytest.mark.gpu
TOL = 1e-5


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def M():
    from paper_1908_07847_amd import mlp
    return mlp


def normwise(got, ref):
    got, ref = np.asarray(got, np.float64).ravel(), np.asarray(ref, np.float64).ravel()
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-30))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("wl,act,mu,lr", [(1, "tanh", 0.0, 0.1), (1, "sigmoid", 0.9, 0.01), (1, "tanh", 0.9, 0.01),
                                          (2, "tanh", 0.0, 0.1), (2, "tanh", 0.5, 0.05)])
def test_fused_trainer_variants_match_the_oracle(M, wl, act, mu, lr):
    w = synth.single(wl)
    say(f"variant: workload {wl}, hidden {act}, momentum {mu}, lr {lr}, {w['epochs']} epochs")
    net = M.Net(w["D"], w["H"], w["K"], w["X"].shape[0], lr=lr, theta=w["theta"], act=act, momentum=mu)
    hist = net.train(dev(w["X"]), dev(w["T"]), w["epochs"])
    torch.cuda.synchronize()
    q, ref_hist, v = oracle.train_var(w["X"], w["T"], Params.of(w["theta"]), lr, w["epochs"], act=act, mu=mu)
    e = normwise(net.flat.detach().cpu().numpy(), q.flat())
    lerr = normwise(hist.cpu().numpy(), ref_hist)
    verr = normwise(net.velocity.cpu().numpy(), v) if mu else 0.0
    say(f"  params {e:.2e}  loss history {lerr:.2e}  velocity {verr:.2e}")
    assert e <= TOL and lerr <= TOL and verr <= TOL


def test_momentum_runs_resume_bitwise(M):
    w = synth.single(1)
    a = M.Net(33, 10, 3, 60, lr=0.02, theta=w["theta"], act="tanh", momentum=0.8)
    b = M.Net(33, 10, 3, 60, lr=0.02, theta=w["theta"], act="tanh", momentum=0.8)
    X, T = dev(w["X"]), dev(w["T"])
    ha = a.train(X, T, 700)
    hb1, hb2 = b.train(X, T, 300), b.train(X, T, 400)
    torch.cuda.synchronize()
    assert torch.equal(a.flat, b.flat) and torch.equal(a.comp, b.comp) and torch.equal(a.velocity, b.velocity)
    assert torch.equal(ha, torch.cat([hb1, hb2]))
    # momentum switched off again: plain descent from there on, like a net that never had it
    b.set_momentum(0.0)
    c = M.Net(33, 10, 3, 60, lr=0.02, theta=b.flat.detach().cpu().numpy(), act="tanh")
    c.comp.copy_(b.comp)
    b.train(X, T, 50), c.train(X, T, 50)
    torch.cuda.synchronize()
    assert torch.equal(b.flat, c.flat)


def test_layer_kernels_with_tanh(M):
    """mlp_forward / mlp_backward with the tanh flag against the oracle's
    tanh network: outputs, hidden activations and the four gradients."""
    w = synth.single(2)
    X, T = w["X"], w["T"]
    net = M.Net(33, 16, 3, 120, theta=w["theta"], act="tanh")
    A, Y = net.forward(dev(X))
    g, _, loss = net.backward(dev(X), A, Y, T=dev(T))
    torch.cuda.synchronize()
    p = Params.of(w["theta"])
    Zr = X.astype(np.float64) @ p.W1.T + p.b1
    Ar = np.tanh(Zr)
    Yr = 1 / (1 + np.exp(-(Ar @ p.W2.T + p.b2)))
    assert normwise(A.cpu().numpy(), Ar) <= 1e-6 and normwise(Y.cpu().numpy(), Yr) <= 1e-6
    L_ref, g_ref = oracle.loss_grad_var(X, T, p, act="tanh")
    assert abs(float(loss.item()) - L_ref) <= 1e-6 * L_ref
    for name in ("W1", "b1", "W2", "b2"):
        assert normwise(getattr(g, name).cpu().numpy(), getattr(g_ref, name)) <= TOL, name


def test_step_with_momentum_two_updates(M):
    """mlp_step with momentum: v = mu v + g, theta -= lr v, twice, against the
    same arithmetic in float64 on the host (plain update, no compensation)."""
    w = synth.single(1)
    net = M.Net(33, 10, 3, 60, theta=w["theta"], compensated=False, momentum=0.7)
    g = net.new_grads()
    rng = np.random.default_rng(4)
    gs = [rng.normal(size=net.flat.numel()).astype(np.float32) for _ in range(2)]
    th = net.flat.detach().cpu().numpy().astype(np.float64)
    v = np.zeros_like(th)
    for gv in gs:
        g.flat.copy_(dev(gv))
        net.step(g, lr=0.05)
        v = 0.7 * v + gv
        th = th - 0.05 * v
    torch.cuda.synchronize()
    assert normwise(net.velocity.cpu().numpy(), v) <= 1e-6
    assert normwise(net.flat.detach().cpu().numpy(), th) <= 1e-6


def test_large_trainer_rejects_the_variants(M):
    w = synth.single(1)
    X, T = dev(w["X"]), dev(w["T"])
    for kw in (dict(act="tanh"), dict(momentum=0.9)):
        net = M.Net(33, 10, 3, 60, batch=32, theta=w["theta"], **kw)   # minibatches: the large-N trainer
        with pytest.raises(MLPError) as ei:
            net.train(X, T, 1)
        assert ei.value.status == MLP_ERR_UNSUPPORTED
