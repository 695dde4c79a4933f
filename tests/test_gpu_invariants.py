"""Invariants of full-batch training on the GPU (the survey's pins for
1/N scaling and indexing): permuting or duplicating the rows changes
nothing, relabelling hidden units, features or outputs permutes the result
the same way, and tied hidden units stay tied.  Each case is also checked
against the FP64 oracle."""
import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import Params
from paper_1908_07847_amd import synth

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
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-30))


def train(M, X, T, th: synth.Theta, epochs, lr=0.1):
    X = np.ascontiguousarray(X, np.float32)
    T = np.ascontiguousarray(T, np.float32)
    net = M.Net(X.shape[1], th.W1.shape[0], T.shape[1], X.shape[0], batch=0, lr=lr, theta=th)
    hist = net.train(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda(), epochs)
    torch.cuda.synchronize()
    d, h, k = X.shape[1], th.W1.shape[0], T.shape[1]
    return synth.Theta.unpack(net.flat.cpu().numpy(), d, h, k), hist.cpu().numpy()


def close(a: synth.Theta, b: synth.Theta, tol=TOL):
    e = max(normwise(a.W1, b.W1), normwise(a.b1, b.b1), normwise(a.W2, b.W2), normwise(a.b2, b.b2))
    assert e <= tol, e
    return e


# the small trainer (120 rows) and the large-N trainer at full batch (2048 rows)
CASES = [("small", 2, None, 16, 400), ("large", 4, 2048, 64, 20)]


def case(kind, wl, n, h):
    w = synth.single(wl, n_rows=n, hidden=h)
    return w["X"], w["T"], w["theta"]


@pytest.mark.parametrize("kind,wl,n,h,epochs", CASES)
def test_row_permutation_changes_nothing(M, kind, wl, n, h, epochs):
    X, T, th = case(kind, wl, n, h)
    perm = np.random.default_rng(5).permutation(X.shape[0])
    a, ha = train(M, X, T, th, epochs)
    b, hb = train(M, X[perm], T[perm], th, epochs)
    e = close(a, b)
    assert np.allclose(ha, hb, rtol=TOL)
    q, _ = oracle.train(X, T, Params.of(th), 0.1, epochs)
    close(a, synth.Theta(q.W1, q.b1, q.W2, q.b2))
    say(f"  {kind}: permuted rows differ by {e:.2e}")


def test_duplicated_rows_change_nothing(M):
    """[X; X] has the same mean loss and gradients as X (full batch)."""
    w = synth.single(1)
    X, T, th = w["X"], w["T"], w["theta"]
    a, ha = train(M, X, T, th, 300)
    b, hb = train(M, np.concatenate([X, X]), np.concatenate([T, T]), th, 300)
    say(f"  duplicated rows differ by {close(a, b):.2e}")
    assert np.allclose(ha, hb, rtol=TOL)


@pytest.mark.parametrize("kind,wl,n,h,epochs", CASES)
def test_relabelling_is_equivariant(M, kind, wl, n, h, epochs):
    X, T, th = case(kind, wl, n, h)
    g = np.random.default_rng(9)
    ph, pd, pk = g.permutation(th.W1.shape[0]), g.permutation(X.shape[1]), g.permutation(T.shape[1])
    a, _ = train(M, X, T, th, epochs)
    # hidden units: rows of W1 and b1, columns of W2
    thh = synth.Theta(th.W1[ph].copy(), th.b1[ph].copy(), th.W2[:, ph].copy(), th.b2.copy())
    b, _ = train(M, X, T, thh, epochs)
    close(synth.Theta(a.W1[ph], a.b1[ph], a.W2[:, ph], a.b2), b)
    # features: columns of X and of W1
    thd = synth.Theta(th.W1[:, pd].copy(), th.b1.copy(), th.W2.copy(), th.b2.copy())
    c, _ = train(M, X[:, pd], T, thd, epochs)
    close(synth.Theta(a.W1[:, pd], a.b1, a.W2, a.b2), c)
    # outputs: columns of T, rows of W2 and b2
    thk = synth.Theta(th.W1.copy(), th.b1.copy(), th.W2[pk].copy(), th.b2[pk].copy())
    d, _ = train(M, X, T[:, pk], thk, epochs)
    close(synth.Theta(a.W1, a.b1, a.W2[pk], a.b2[pk]), d)


@pytest.mark.parametrize("kind,wl,n,h,epochs", CASES)
def test_tied_hidden_units_stay_tied(M, kind, wl, n, h, epochs):
    X, T, th = case(kind, wl, n, h)
    t = th.copy()
    t.W1[1] = t.W1[0]
    t.b1[1] = t.b1[0]
    t.W2[:, 1] = t.W2[:, 0]
    a, _ = train(M, X, T, t, epochs)
    for arr in (a.W1[1] - a.W1[0], a.W2[:, 1] - a.W2[:, 0], np.array([a.b1[1] - a.b1[0]])):
        assert np.max(np.abs(arr)) <= 1e-6 * max(np.max(np.abs(a.W1)), 1.0)
