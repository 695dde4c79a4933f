"""Nets sharing one dataset (mlp_train_shared) against the FP64 oracle.

Every net of the grid is an independent run of the training loop of section
2.2 on the same rows, so each is checked against oracle.train with its own
initial parameters and learning rate: every net at small sizes, sampled nets
at the full 64-net shape on a 65,536-row subset, and properties (bitwise
repeatability, loss descent) on the whole 4,194,304-row workload.
"""
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import oracle
from oracle import Params
from paper_1908_07847_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-5   # float32 path vs float64 oracle, relative to the largest entry


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def M():
    from paper_1908_07847_amd import mlp
    return mlp


def normwise(got, ref):
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-30))


def errors(flat_gpu, q: Params):
    d, h, k = q.shape
    g = synth.Theta.unpack(flat_gpu, d, h, k)
    return dict(W1=normwise(g.W1, q.W1), b1=normwise(g.b1, q.b1), W2=normwise(g.W2, q.W2),
                b2=normwise(g.b2, q.b2))


def gpu_shared(M, w, epochs, batch, prec="fp32", compensated=True, nets=None):
    theta = w["theta"] if nets is None else w["theta"][:nets]
    lrs = w["lrs"][:theta.shape[0]]
    X = torch.from_numpy(np.ascontiguousarray(w["X"])).cuda()
    T = torch.from_numpy(np.ascontiguousarray(w["T"])).cuda()
    th = torch.from_numpy(np.ascontiguousarray(theta)).cuda()
    comp = torch.zeros_like(th) if compensated else None
    hist = torch.empty((th.shape[0], epochs), dtype=torch.float32, device="cuda")
    M.train_shared(X, T, th, lrs, epochs, w["H"], batch=batch, prec=prec, comp=comp, loss_hist=hist)
    torch.cuda.synchronize()
    return th.cpu().numpy(), hist.cpu().numpy()


def oracle_nets(w, idx, epochs, batch):
    """oracle.train of the selected nets, in parallel host threads."""
    d, h, k = w["D"], w["H"], w["K"]

    def one(i):
        p = Params.of(synth.Theta.unpack(w["theta"][i], d, h, k))
        return oracle.train(w["X"], w["T"], p, w["lrs"][i], epochs, batch=batch)

    with ThreadPoolExecutor(max_workers=min(8, len(idx))) as ex:
        return list(ex.map(one, idx))


def check_nets(w, got, hist, idx, epochs, batch, tol, label):
    refs = oracle_nets(w, idx, epochs, batch)
    worst = 0.0
    for i, (q, ref_hist) in zip(idx, refs):
        e = errors(got[i], q)
        lerr = float(np.max(np.abs(hist[i] - ref_hist) / ref_hist))
        worst = max(worst, lerr, *e.values())
        assert max(e.values()) <= tol and lerr <= tol, (label, i, e, lerr)
    say(f"  {label}: {len(idx)} nets, worst relative error {worst:.2e}")


def test_every_net_of_a_shared_grid_matches_the_oracle(M):
    """8 nets, 33-256-3, 8192 rows, minibatch 1024, 2 epochs: one hidden
    block per net, 16 row blocks."""
    w = synth.shared(4, n_nets=8, n_rows=8192)
    say(f"shared fp32: 8 nets N=8192 D=33 H=256 batch=1024 epochs=2 lrs={np.round(w['lrs'], 4).tolist()}")
    got, hist = gpu_shared(M, w, 2, 1024)
    check_nets(w, got, hist, list(range(8)), 2, 1024, TOL, "shared 8 nets")


def test_shared_nets_with_split_hidden_layer_and_row_pieces(M):
    """3 nets, 64-1024-3 (four hidden blocks per net), 20480 rows with a
    minibatch of 16384 (a short second minibatch), 1 epoch: each row block
    is larger than the LDS holds and is staged in pieces."""
    w = synth.shared(5, n_nets=3, n_rows=20480)
    say("shared fp32: 3 nets N=20480 D=64 H=1024 batch=16384 epochs=1")
    got, hist = gpu_shared(M, w, 1, 16384)
    check_nets(w, got, hist, [0, 1, 2], 1, 16384, TOL, "shared split+pieces")


def test_shared_net_equals_the_single_net_trainer(M):
    """Net i of a shared launch and the same net trained alone differ only in
    float32 summation order."""
    w = synth.shared(4, n_nets=4, n_rows=8192)
    got, hist = gpu_shared(M, w, 2, 1024)
    for i in range(4):
        net = M.Net(w["D"], w["H"], w["K"], 8192, batch=1024, lr=w["lrs"][i],
                    theta=synth.Theta.unpack(w["theta"][i], w["D"], w["H"], w["K"]))
        h1 = net.train(torch.from_numpy(w["X"]).cuda(), torch.from_numpy(w["T"]).cuda(), 2)
        torch.cuda.synchronize()
        one = net.flat.cpu().numpy()
        assert normwise(got[i], one) <= 1e-6, i
        assert np.allclose(hist[i], h1.cpu().numpy(), rtol=1e-6)


def test_shared_lr_zero_and_zero_epochs(M):
    w = synth.shared(4, n_nets=2, n_rows=4096)
    w["lrs"] = [0.0, 0.0]
    got, _ = gpu_shared(M, w, 2, 1024)
    assert np.array_equal(got, w["theta"][:2])


@pytest.mark.parametrize("prec,loss_tol,w_tol", [("bf16", 1e-3, 1e-2)])
def test_shared_bf16_error_vs_exact_oracle(M, prec, loss_tol, w_tol):
    """bf16 operands (float32 accumulation and master weights) against the
    exact float64 oracle: the same bounds as the single-net bf16 trainer."""
    w = synth.shared(4, n_nets=4, n_rows=16 * 4096)
    got, hist = gpu_shared(M, w, 2, 4096, prec=prec)
    refs = oracle_nets(w, [0, 1, 2, 3], 2, 4096)
    for i, (q, ref_hist) in enumerate(refs):
        e = errors(got[i], q)
        lerr = float(np.max(np.abs(hist[i] - ref_hist) / ref_hist))
        say(f"  {prec} shared net {i} (lr {w['lrs'][i]:.4f}): params {e} loss {lerr:.2e}")
        assert lerr <= loss_tol and max(e.values()) <= w_tol, (i, e, lerr)


def test_64_nets_full_shape_on_a_65536_row_subset(M):
    """The 64-net grid at its full shape (64-1024-3, minibatch 16384) on the
    first 65,536 rows for one epoch (4 steps); sampled nets (first, one from
    the middle of the grid, last) against the oracle."""
    w = synth.shared(5, n_nets=64, n_rows=65536)
    say("shared fp32: 64 nets N=65536 D=64 H=1024 batch=16384 epochs=1")
    got, hist = gpu_shared(M, w, 1, 16384)
    assert np.all(np.isfinite(got)) and np.all(np.isfinite(hist))
    check_nets(w, got, hist, [0, 37, 63], 1, 16384, TOL, "64 nets sampled")


def test_64_nets_whole_workload_is_repeatable_and_descends(M):
    """All 4,194,304 rows, 64 nets, bf16 operands, 1 epoch, twice: bitwise
    equal results, finite, and every net's loss below its starting loss."""
    w = synth.shared(5, n_nets=64)
    say("shared bf16: 64 nets N=4194304 D=64 H=1024 batch=16384 epochs=1 (twice)")
    a, ha = gpu_shared(M, w, 1, 16384, prec="bf16")
    b, hb = gpu_shared(M, w, 1, 16384, prec="bf16")
    assert np.array_equal(a, b) and np.array_equal(ha, hb)
    assert np.all(np.isfinite(a))
    # loss at the initial parameters on the first minibatch, from the oracle's forward pass
    Xb, Tb = w["X"][:16384], w["T"][:16384]
    for i in (0, 7, 63):
        p = Params.of(synth.Theta.unpack(w["theta"][i], w["D"], w["H"], w["K"]))
        l0 = oracle.mse(oracle.forward(Xb, p)[1], Tb)
        say(f"  net {i} lr {w['lrs'][i]:.4f}: initial minibatch loss {l0:.4f}, epoch-1 mean {ha[i, 0]:.4f}")
        assert ha[i, 0] < l0
