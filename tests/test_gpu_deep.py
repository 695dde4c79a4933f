"""Networks with several hidden layers on the GPU: the dense layer
(mlp_dense_forward / mlp_dense_backward) against float64 on the host at
ragged sizes, and DeepNet training (the layers composed by torch.autograd,
mlp_update) against the FP64 oracle's L-layer training."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1908_07847_amd import synth

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("n,din,dout,act", [(1, 1, 1, 0), (77, 33, 50, 1), (300, 70, 130, 0), (4096, 33, 256, 1)])
def test_dense_layer_forward_and_backward(M, n, din, dout, act):
    g = np.random.default_rng(n + din)
    X = g.normal(size=(n, din)).astype(np.float32)
    W = g.uniform(-0.5, 0.5, (dout, din)).astype(np.float32)
    b = g.uniform(-0.5, 0.5, dout).astype(np.float32)
    dY = g.normal(size=(n, dout)).astype(np.float32)
    Xd = torch.from_numpy(X).cuda().requires_grad_(True)
    Wd = torch.from_numpy(W).cuda().requires_grad_(True)
    bd = torch.from_numpy(b).cuda().requires_grad_(True)
    Y = M.DenseFunction.apply(Xd, Wd, bd, act)
    dX, gW, gb = torch.autograd.grad(Y, [Xd, Wd, bd], torch.from_numpy(dY).cuda())
    torch.cuda.synchronize()
    Z = X.astype(np.float64) @ W.T.astype(np.float64) + b
    Yr = np.tanh(Z) if act == 1 else 1 / (1 + np.exp(-Z))
    dZ = dY * ((1 - Yr * Yr) if act == 1 else Yr * (1 - Yr))
    # float32 contraction of din terms: |dz| <= din u sum|x w| (u = 2^-24); act' <= 1
    zbound = (din + 1) * 2.0 ** -24 * float(np.max(np.abs(X) @ np.abs(W).T + np.abs(b)))
    assert float(np.max(np.abs(Y.detach().cpu().numpy() - Yr))) <= zbound + 1e-7
    assert normwise(gW.cpu().numpy(), dZ.T @ X) <= 1e-5
    assert normwise(gb.cpu().numpy(), dZ.sum(axis=0)) <= 1e-5
    assert normwise(dX.cpu().numpy(), dZ @ W) <= 1e-5


@pytest.mark.parametrize("widths,act,epochs", [([33, 16, 3], "sigmoid", 2000), ([33, 24, 12, 3], "tanh", 1000),
                                               ([33, 16, 16, 3], "sigmoid", 1000), ([33, 20, 10, 6, 1], "tanh", 500)])
def test_deep_net_training_matches_the_oracle(M, widths, act, epochs):
    w = synth.single(2)
    T = w["T"] if widths[-1] == 3 else synth.binary_targets(w)
    g = np.random.default_rng(len(widths))
    theta = g.uniform(-0.5, 0.5, oracle.deep_n_params(widths)).astype(np.float32)
    say(f"deep net {widths} hidden {act}: {epochs} epochs on workload 2's rows")
    net = M.DeepNet(widths, theta=theta, act=act)
    hist = net.train(torch.from_numpy(w["X"]).cuda(), torch.from_numpy(T).cuda(), epochs)
    torch.cuda.synchronize()
    q, ref_hist = oracle.deep_train(w["X"], T, widths, theta, 0.1, epochs, act=act)
    e = normwise(net.flat.detach().cpu().numpy(), q)
    lerr = normwise(hist.cpu().numpy(), ref_hist)
    say(f"  params {e:.2e}  loss history {lerr:.2e}  final loss {ref_hist[-1]:.4f}")
    assert e <= 1e-5 and lerr <= 1e-5


def test_mse_grad_kernel(M):
    from paper_1908_07847_amd._lib import lib
    g = np.random.default_rng(5)
    for n, k in ((1, 1), (120, 3), (5000, 7)):
        Y = g.uniform(0, 1, (n, k)).astype(np.float32)
        T = g.uniform(0, 1, (n, k)).astype(np.float32)
        Yd, Td = torch.from_numpy(Y).cuda(), torch.from_numpy(T).cuda()
        dY, loss = torch.empty_like(Yd), torch.empty(4, device="cuda")
        assert lib.mlp_mse_grad(Yd.data_ptr(), Td.data_ptr(), n, k, dY.data_ptr(), loss.data_ptr(), None) == 0
        torch.cuda.synchronize()
        e = Y.astype(np.float64) - T
        assert abs(float(loss[0]) - np.mean(e * e)) <= 1e-6 * np.mean(e * e) + 1e-12
        assert normwise(dY.cpu().numpy(), 2 * e / (n * k)) <= 1e-6


def test_fused_deep_epochs_match_the_oracle_and_replay_from_a_graph(M):
    """DeepNet.train_fused (the epoch as library calls) against the oracle;
    DeepGraph replays equal the same epochs run eagerly, bitwise, with eager
    work between the replays."""
    w = synth.single(2)
    widths, act = [33, 24, 12, 3], "tanh"
    theta = np.random.default_rng(3).uniform(-0.5, 0.5, oracle.deep_n_params(widths)).astype(np.float32)
    X, T = torch.from_numpy(w["X"]).cuda(), torch.from_numpy(w["T"]).cuda()
    net = M.DeepNet(widths, theta=theta, act=act)
    hist = net.train_fused(X, T, 1000)
    torch.cuda.synchronize()
    q, ref_hist = oracle.deep_train(w["X"], w["T"], widths, theta, 0.1, 1000, act=act)
    e, lerr = normwise(net.flat.detach().cpu().numpy(), q), normwise(hist.cpu().numpy(), ref_hist)
    say(f"  fused deep epochs: params {e:.2e}  loss history {lerr:.2e}")
    assert e <= 1e-5 and lerr <= 1e-5
    G = 25
    a = M.DeepNet(widths, theta=theta, act=act)
    b = M.DeepNet(widths, theta=theta, act=act)
    graph = M.DeepGraph(b, X, T, G)
    assert np.array_equal(b.flat.detach().cpu().numpy(), theta)     # capture left the net as it was
    lbuf = torch.empty(G, device="cuda")
    for rep in range(3):
        a.train_fused(X, T, G, loss_hist=lbuf)
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(a.flat, b.flat) and torch.equal(a.comp, b.comp), rep
        assert torch.equal(graph.loss, lbuf), rep


def _rows(n, d, k, seed):
    g = np.random.default_rng(seed)
    X = g.normal(size=(n, d)).astype(np.float32)
    T = np.zeros((n, k), np.float32)
    T[np.arange(n), g.integers(0, k, n)] = 1.0
    return X, T


@pytest.mark.parametrize("widths,act,epochs,rows,compensated", [
    ([33, 16, 16, 3], "sigmoid", 1000, "w2", True),     # the two-hidden-layer net on workload 2's rows
    ([33, 24, 12, 3], "tanh", 1000, "w2", True),
    ([33, 20, 10, 6, 1], "tanh", 500, "w2", True),      # binary output
    ([33, 10, 3], "sigmoid", 500, "w1", False),         # 60 rows: ragged row segments; plain update
    ([33, 32, 16, 3], "sigmoid", 300, 200, True),       # 200 rows: fewer row segments to fit LDS
    ([1, 1], "sigmoid", 50, 1, True),                   # one row, one unit
    ([7, 5, 4, 3, 2, 2, 3, 2, 1], "tanh", 200, 37, True),  # the most layers
])
def test_one_launch_deep_training_matches_the_oracle(M, widths, act, epochs, rows, compensated):
    """mlp_deep_train (the whole run in one workgroup) against the FP64
    oracle's L-layer training."""
    if rows in ("w1", "w2"):
        w = synth.single(1 if rows == "w1" else 2)
        X, T = w["X"], (w["T"] if widths[-1] == 3 else synth.binary_targets(w))
    else:
        X, T = _rows(rows, widths[0], widths[-1], rows)
    theta = np.random.default_rng(len(widths) + epochs).uniform(-0.5, 0.5,
                                                                 oracle.deep_n_params(widths)).astype(np.float32)
    say(f"one-launch deep net {widths} hidden {act}: {X.shape[0]} rows, {epochs} epochs, "
        f"{'compensated' if compensated else 'plain'} update")
    net = M.DeepNet(widths, theta=theta, act=act, compensated=compensated)
    hist = net.train_kernel(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda(), epochs)
    torch.cuda.synchronize()
    q, ref_hist = oracle.deep_train(X, T, widths, theta, 0.1, epochs, act=act)
    e = normwise(net.flat.detach().cpu().numpy(), q)
    lerr = normwise(hist.cpu().numpy(), ref_hist)
    say(f"  params {e:.2e}  loss history {lerr:.2e}  final loss {ref_hist[-1]:.4f}")
    assert e <= 1e-5 and lerr <= 1e-5


def test_one_launch_deep_training_is_repeatable_and_resumable(M):
    """Two runs are bitwise equal; 300 epochs in one call equal 100 + 200
    (the compensation terms carry across calls)."""
    w = synth.single(2)
    widths, act = [33, 16, 16, 3], "sigmoid"
    theta = np.random.default_rng(11).uniform(-0.5, 0.5, oracle.deep_n_params(widths)).astype(np.float32)
    X, T = torch.from_numpy(w["X"]).cuda(), torch.from_numpy(w["T"]).cuda()
    a, b, c = (M.DeepNet(widths, theta=theta, act=act) for _ in range(3))
    ha = a.train_kernel(X, T, 300)
    hb = b.train_kernel(X, T, 300)
    c.train_kernel(X, T, 100)
    c.train_kernel(X, T, 200)
    torch.cuda.synchronize()
    assert torch.equal(a.flat, b.flat) and torch.equal(a.comp, b.comp) and torch.equal(ha, hb)
    assert torch.equal(a.flat, c.flat) and torch.equal(a.comp, c.comp)
