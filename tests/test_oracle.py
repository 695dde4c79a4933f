"""Pins for the FP64 oracle (arxiv 1908.07847, section 2.2 and Equation 1).

Each check ties the oracle to something other than itself: a hand-derived
worked step (tests/golden/worked_221.json), the scalar chain rule in closed
form, central finite differences of the loss, an independent library
routine (torch float64 autograd and SGD on the CPU), and invariants the
mathematics fixes (lr = 0, linearity in lr, descent, permutation and
duplication invariance, equivariance under relabelling hidden units,
features and outputs).
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from oracle import Params
from paper_1908_07847_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def small_problem(n=12, d=5, h=4, k=3, seed=0, lo=-0.5, hi=0.5):
    g = np.random.default_rng(seed)
    X = g.standard_normal((n, d))
    T = np.eye(k)[g.integers(0, k, n)]
    p = Params(g.uniform(lo, hi, (h, d)), g.uniform(lo, hi, h), g.uniform(lo, hi, (k, h)),
               g.uniform(lo, hi, k))
    return X, T, p


def maxrel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


# ---------------------------------------------------------------- worked example
def test_worked_221_step():
    ref = json.load(open(os.path.join(GOLDEN, "worked_221.json")))
    inp = ref["inputs"]
    X, T = np.array(inp["X"]), np.array(inp["T"])
    p = Params(inp["W1"], inp["b1"], inp["W2"], inp["b2"])
    f = lambda v: np.array(v, dtype=np.float64)
    A, Y = oracle.forward(X, p)
    assert np.allclose(A, f(ref["A"]), rtol=1e-13, atol=0)
    assert np.allclose(Y[:, 0], f(ref["Y"]), rtol=1e-13, atol=0)
    L0, g = oracle.loss_grad(X, T, p)
    assert abs(L0 - float(ref["L0"])) <= 1e-14 * abs(float(ref["L0"]))
    got = {"gW1": g.W1, "gb1": g.b1, "gW2": g.W2, "gb2": g.b2}
    for name, val in got.items():
        assert np.allclose(val, f(ref[name]), rtol=1e-12, atol=1e-17), name
    q, hist = oracle.train(X, T, p, lr=inp["lr"], epochs=1)
    assert np.allclose(q.W1, f(ref["W1_new"]), rtol=1e-14, atol=0)
    assert np.allclose(q.b1, f(ref["b1_new"]), rtol=1e-14, atol=0)
    assert np.allclose(q.W2, f(ref["W2_new"]), rtol=1e-14, atol=0)
    assert np.allclose(q.b2, f(ref["b2_new"]), rtol=1e-14, atol=0)
    assert abs(hist[0] - float(ref["L0"])) <= 1e-14
    _, Y1 = oracle.forward(X, q)
    assert abs(oracle.mse(Y1, T) - float(ref["L1"])) <= 1e-14


# ---------------------------------------------------------------- closed forms
def test_sigmoid_equation_1_values():
    # Equation 1 at points with known values: sigma(0) = 1/2, sigma(ln 3) = 3/4,
    # sigma(-ln 3) = 1/4, and the saturated limits.
    p = Params([[1.0]], [0.0], [[1.0]], [0.0])
    for z, want in [(0.0, 0.5), (np.log(3.0), 0.75), (-np.log(3.0), 0.25), (800.0, 1.0),
                    (-800.0, 0.0)]:
        A, _ = oracle.forward(np.array([[z]]), p)
        assert abs(A[0, 0] - want) <= 1e-15


@pytest.mark.parametrize("seed", range(5))
def test_chain_rule_111_closed_form(seed):
    g = np.random.default_rng(seed)
    x, t = g.normal(), float(g.integers(0, 2))
    w1, b1, w2, b2 = g.uniform(-2, 2, 4)
    h = 1 / (1 + np.exp(-(w1 * x + b1)))
    y = 1 / (1 + np.exp(-(w2 * h + b2)))
    c = 2 * (y - t) * y * (1 - y)          # dL/dz2 for L = (y - t)^2
    want = dict(W2=c * h, b2=c, W1=c * w2 * h * (1 - h) * x, b1=c * w2 * h * (1 - h))
    L, gr = oracle.loss_grad(np.array([[x]]), np.array([[t]]), Params([[w1]], [b1], [[w2]], [b2]))
    assert abs(L - (y - t) ** 2) <= 1e-15
    for k, v in want.items():
        assert abs(getattr(gr, k).ravel()[0] - v) <= 1e-14 * max(1.0, abs(v)), k


# ---------------------------------------------------------------- finite differences
def _flat_loss(X, T, p, v):
    d, h, k = p.shape
    q = Params(v[:h * d].reshape(h, d), v[h * d:h * d + h], v[h * d + h:h * d + h + k * h].reshape(k, h),
               v[-k:])
    A, Y = oracle.forward(X, q)
    return oracle.mse(Y, T)


@pytest.mark.parametrize("seed,lo,hi", [(0, -0.5, 0.5), (1, -0.5, 0.5), (2, -4.0, 4.0)])
def test_gradient_central_fd_every_coordinate(seed, lo, hi):
    X, T, p = small_problem(seed=seed, lo=lo, hi=hi)
    L, g = oracle.loss_grad(X, T, p)
    v = p.flat()
    fd = np.zeros_like(v)
    step = 1e-6
    for i in range(v.size):
        e = np.zeros_like(v); e[i] = step
        fd[i] = (_flat_loss(X, T, p, v + e) - _flat_loss(X, T, p, v - e)) / (2 * step)
    gv = g.flat()
    assert np.max(np.abs(fd - gv)) <= 1e-6 * np.max(np.abs(gv))


def test_gradient_fd_directional_workload2_draws():
    """Workload 2 shapes (N=120, 33-16-3): 100 draws U(-0.5,0.5) + 10 U(-4,4), random directions."""
    w = synth.single(2)
    X, T = w["X"].astype(np.float64), w["T"].astype(np.float64)
    g = np.random.default_rng(7)
    worst = 0.0
    for it in range(110):
        lo, hi = (-0.5, 0.5) if it < 100 else (-4.0, 4.0)
        p = Params(g.uniform(lo, hi, (16, 33)), g.uniform(lo, hi, 16), g.uniform(lo, hi, (3, 16)),
                   g.uniform(lo, hi, 3))
        _, gr = oracle.loss_grad(X, T, p)
        u = g.standard_normal(p.flat().size)
        u /= np.linalg.norm(u)
        h = 1e-6
        fd = (_flat_loss(X, T, p, p.flat() + h * u) - _flat_loss(X, T, p, p.flat() - h * u)) / (2 * h)
        an = float(gr.flat() @ u)
        worst = max(worst, abs(fd - an) / max(np.linalg.norm(gr.flat()), 1e-12))
    assert worst <= 1e-6


# ---------------------------------------------------------------- library special case
def _torch_model(p: Params):
    W1 = torch.tensor(p.W1, dtype=torch.float64, requires_grad=True)
    b1 = torch.tensor(p.b1, dtype=torch.float64, requires_grad=True)
    W2 = torch.tensor(p.W2, dtype=torch.float64, requires_grad=True)
    b2 = torch.tensor(p.b2, dtype=torch.float64, requires_grad=True)
    return W1, b1, W2, b2


def test_gradient_matches_torch_float64_autograd():
    w = synth.single(2)
    X, T = w["X"].astype(np.float64), w["T"].astype(np.float64)
    p = Params.of(w["theta"])
    L, g = oracle.loss_grad(X, T, p)
    W1, b1, W2, b2 = _torch_model(p)
    Xt, Tt = torch.tensor(X), torch.tensor(T)
    Y = torch.sigmoid(torch.sigmoid(Xt @ W1.T + b1) @ W2.T + b2)
    loss = torch.nn.functional.mse_loss(Y, Tt)
    loss.backward()
    assert abs(L - loss.item()) <= 1e-14
    for mine, theirs in [(g.W1, W1.grad), (g.b1, b1.grad), (g.W2, W2.grad), (g.b2, b2.grad)]:
        assert maxrel(mine, theirs.numpy()) <= 1e-12


def test_backward_with_upstream_gradient_and_dx_matches_torch():
    X, T, p = small_problem(n=9, d=6, h=5, k=2, seed=3)
    A, Y = oracle.forward(X, p)
    dY = np.random.default_rng(4).standard_normal(Y.shape)
    g, dX = oracle.backward(X, A, Y, dY, p, want_dx=True)
    W1, b1, W2, b2 = _torch_model(p)
    Xt = torch.tensor(X, requires_grad=True)
    Yt = torch.sigmoid(torch.sigmoid(Xt @ W1.T + b1) @ W2.T + b2)
    Yt.backward(torch.tensor(dY))
    for mine, theirs in [(g.W1, W1.grad), (g.b1, b1.grad), (g.W2, W2.grad), (g.b2, b2.grad),
                         (dX, Xt.grad)]:
        assert maxrel(mine, theirs.numpy()) <= 1e-12


@pytest.mark.parametrize("n,batch,epochs", [(60, 0, 50), (100, 32, 7), (64, 16, 5)])
def test_training_matches_torch_sgd(n, batch, epochs):
    """Plain GD (no momentum) over contiguous minibatches == torch.optim.SGD on the same slices."""
    w = synth.single(1, n_rows=n) if n <= 60 else synth.single(2, n_rows=n)
    X, T = w["X"].astype(np.float64), w["T"].astype(np.float64)
    p = Params.of(w["theta"])
    q, hist = oracle.train(X, T, p, lr=0.1, epochs=epochs, batch=batch)
    params = _torch_model(p)
    opt = torch.optim.SGD(params, lr=0.1, momentum=0.0)
    b = n if batch <= 0 else batch
    th = []
    for _ in range(epochs):
        acc = []
        for r0 in range(0, n, b):
            W1, b1, W2, b2 = params
            xb, tb = torch.tensor(X[r0:r0 + b]), torch.tensor(T[r0:r0 + b])
            loss = torch.nn.functional.mse_loss(torch.sigmoid(torch.sigmoid(xb @ W1.T + b1) @ W2.T + b2), tb)
            opt.zero_grad()
            loss.backward()
            opt.step()
            acc.append(loss.item())
        th.append(np.mean(acc))
    for mine, theirs in zip([q.W1, q.b1, q.W2, q.b2], params):
        assert maxrel(mine, theirs.detach().numpy()) <= 1e-12
    assert np.max(np.abs(hist - np.array(th))) <= 1e-13


# ---------------------------------------------------------------- invariants
def test_lr_zero_leaves_parameters_bitwise():
    X, T, p = small_problem()
    q, _ = oracle.train(X, T, p, lr=0.0, epochs=5)
    for a, b in zip(q.flat(), p.flat()):
        assert a == b


def test_one_step_is_linear_in_lr():
    X, T, p = small_problem(seed=5)
    q1, _ = oracle.train(X, T, p, lr=0.05, epochs=1)
    q2, _ = oracle.train(X, T, p, lr=0.10, epochs=1)
    d1, d2 = q1.flat() - p.flat(), q2.flat() - p.flat()
    assert np.max(np.abs(d2 - 2 * d1)) <= 1e-14


def test_full_batch_descent_is_monotone():
    w = synth.single(1)
    p = Params.of(w["theta"])
    _, hist = oracle.train(w["X"], w["T"], p, lr=0.01, epochs=1000)
    assert np.all(hist[1:] <= hist[:-1] * (1 + 1e-15))
    _, hist = oracle.train(w["X"], w["T"], p, lr=0.1, epochs=1000)
    assert np.all(hist[1:] <= hist[:-1] * (1 + 1e-15))
    assert hist[-1] < hist[0]


def test_permuting_and_duplicating_samples_leave_full_batch_unchanged():
    w = synth.single(1)
    X, T, p = w["X"].astype(np.float64), w["T"].astype(np.float64), Params.of(w["theta"])
    q, h = oracle.train(X, T, p, lr=0.1, epochs=30)
    perm = np.random.default_rng(1).permutation(X.shape[0])
    qp, hp = oracle.train(X[perm], T[perm], p, lr=0.1, epochs=30)
    qd, hd = oracle.train(np.vstack([X, X]), np.vstack([T, T]), p, lr=0.1, epochs=30)
    for other, ho in [(qp, hp), (qd, hd)]:
        assert maxrel(other.flat(), q.flat()) <= 1e-12
        assert np.max(np.abs(ho - h)) <= 1e-13


def test_relabelling_hidden_units_features_and_outputs_is_equivariant():
    X, T, p = small_problem(n=20, d=6, h=5, k=3, seed=9)
    q, hist = oracle.train(X, T, p, lr=0.3, epochs=20)
    g = np.random.default_rng(2)
    ph, pf, po = g.permutation(5), g.permutation(6), g.permutation(3)
    pp = Params(p.W1[ph][:, pf], p.b1[ph], p.W2[po][:, ph], p.b2[po])
    qq, hist2 = oracle.train(X[:, pf], T[:, po], pp, lr=0.3, epochs=20)
    assert np.max(np.abs(qq.W1 - q.W1[ph][:, pf])) <= 1e-14
    assert np.max(np.abs(qq.b1 - q.b1[ph])) <= 1e-14
    assert np.max(np.abs(qq.W2 - q.W2[po][:, ph])) <= 1e-14
    assert np.max(np.abs(qq.b2 - q.b2[po])) <= 1e-14
    assert np.max(np.abs(hist2 - hist)) <= 1e-15


def test_tied_hidden_units_stay_tied():
    X, T, p = small_problem(n=15, d=4, h=3, k=2, seed=11)
    p.W1[2] = p.W1[0]; p.b1[2] = p.b1[0]; p.W2[:, 2] = p.W2[:, 0]
    q, _ = oracle.train(X, T, p, lr=0.5, epochs=25)
    assert np.array_equal(q.W1[2], q.W1[0]) and q.b1[2] == q.b1[0]
    assert np.array_equal(q.W2[:, 2], q.W2[:, 0])


def test_many_nets_equal_their_single_runs():
    w = synth.batched(n_nets=12)
    th, hist = oracle.train_many(w["items"], w["X"], w["T"], w["theta"], 33, 3, epochs=15, threads=2)
    for i, it in enumerate(w["items"]):
        x = w["X"][it["x_off"]:it["x_off"] + it["n_rows"]]
        t = w["T"][it["x_off"]:it["x_off"] + it["n_rows"]]
        p0 = synth.Theta.unpack(w["theta"][it["p_off"]:], 33, it["n_hidden"], 3)
        q, h1 = oracle.train(x, t, Params.of(p0), float(it["lr"]), 15)
        got = th[it["p_off"]:it["p_off"] + synth.n_params(33, it["n_hidden"], 3)]
        assert np.array_equal(got, q.flat())
        assert np.array_equal(hist[i], h1)


# ---------------------------------------------------------------- reduced precision
def test_round_bf16_matches_definition_and_torch():
    assert oracle.round_bf16(1.0 + 2.0 ** -8) == 1.0                 # tie -> even
    assert oracle.round_bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6  # tie -> even (up)
    assert oracle.round_bf16(1.0 + 2.0 ** -7) == 1.0 + 2.0 ** -7      # representable
    v = np.random.default_rng(0).standard_normal(4000).astype(np.float32) * np.float32(3.0)
    t = torch.tensor(v).to(torch.bfloat16).to(torch.float64).numpy()
    mine = np.array([oracle.round_bf16(float(a)) for a in v])
    assert np.array_equal(mine, t)


def test_round_e4m3_matches_definition_and_torch():
    assert oracle.round_e4m3(448.0) == 448.0
    assert oracle.round_e4m3(1000.0) == 448.0 and oracle.round_e4m3(-1e6) == -448.0
    assert oracle.round_e4m3(2.0 ** -9) == 2.0 ** -9                 # smallest subnormal
    assert oracle.round_e4m3(2.0 ** -10) == 0.0                      # tie -> even (0)
    assert oracle.round_e4m3(1.0625) == 1.0                          # tie -> even
    assert oracle.round_e4m3(1.1875) == 1.25
    g = np.random.default_rng(1)
    v = (g.standard_normal(4000) * 60).astype(np.float32)
    v = v[np.abs(v) <= 440]
    t = torch.tensor(v).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    mine = np.array([oracle.round_e4m3(float(a)) for a in v])
    assert np.array_equal(mine, t)


def test_e4m3_scale_exponent():
    assert oracle.e4m3_scale_exp(448.0) == 0
    assert oracle.e4m3_scale_exp(449.0) == -1
    assert oracle.e4m3_scale_exp(1.0) == 8          # 256 <= 448 < 512
    assert oracle.e4m3_scale_exp(0.875) == 9        # exactly 448 at 2^9
    assert oracle.e4m3_scale_exp(0.0) == 0
    for a in np.random.default_rng(3).uniform(1e-6, 1e4, 200):
        e = oracle.e4m3_scale_exp(a)
        assert a * 2.0 ** e <= 448 < a * 2.0 ** (e + 1)


def test_lowp_with_no_rounding_equals_plain_training():
    w = synth.single(4, n_rows=300, hidden=8)
    p = Params.of(w["theta"])
    q0, h0 = oracle.train(w["X"], w["T"], p, lr=0.1, epochs=2, batch=64)
    q1, h1, _ = oracle.train_lowp(w["X"], w["T"], p, lr=0.1, epochs=2, batch=64, prec="fp32")
    assert maxrel(q1.flat(), q0.flat()) <= 1e-14
    assert np.max(np.abs(h1 - h0)) <= 1e-15


@pytest.mark.parametrize("prec,tol", [("bf16", 2e-2), ("e4m3", 2e-1)])
def test_lowp_step_is_close_to_exact_and_rounds_operands(prec, tol):
    w = synth.single(4, n_rows=512, hidden=16)
    p = Params.of(w["theta"])
    q0, h0 = oracle.train(w["X"], w["T"], p, lr=0.1, epochs=1, batch=512)
    q1, h1, slog = oracle.train_lowp(w["X"], w["T"], p, lr=0.1, epochs=1, batch=512, prec=prec)
    d0, d1 = q0.flat() - p.flat(), q1.flat() - p.flat()
    assert not np.array_equal(d0, d1)                  # rounding really happened
    assert np.max(np.abs(d1 - d0)) <= tol * np.max(np.abs(d0))
    assert abs(h1[0] - h0[0]) <= tol * h0[0]
    if prec == "e4m3":
        assert slog[0, 0] == oracle.e4m3_scale_exp(np.max(np.abs(w["X"])))
        assert slog[0, 1] == oracle.e4m3_scale_exp(np.max(np.abs(w["theta"].W1)))


def test_predict_is_the_first_maximum_of_the_outputs():
    """Ties go to the lowest index; equal outputs give class 0; the labels
    equal a plain loop over the rows."""
    g = np.random.default_rng(3)
    X = g.standard_normal((50, 4))
    p = Params(g.uniform(-1, 1, (5, 4)), g.uniform(-1, 1, 5), g.uniform(-1, 1, (3, 5)), g.uniform(-1, 1, 3))
    Y, lab = oracle.predict(X, p)
    for r in range(50):
        best = 0
        for k in range(1, 3):
            if Y[r, k] > Y[r, best]:
                best = k
        assert lab[r] == best
    tie = Params(p.W1, p.b1, np.zeros((3, 5)), np.array([0.2, 0.7, 0.7]))
    _, lab = oracle.predict(X, tie)
    assert np.all(lab == 1)
    # one output (the two-class reading: poor control or not): class 1 above 1/2
    one = Params(p.W1, p.b1, p.W2[:1], p.b2[:1])
    Y1, lab1 = oracle.predict(X, one)
    assert np.array_equal(lab1, np.array([1 if y > 0.5 else 0 for y in Y1[:, 0]]))
    lo = Params(p.W1, p.b1, np.zeros((1, 5)), np.array([0.0]))     # every output exactly 1/2
    assert np.all(oracle.predict(X, lo)[1] == 0)


def test_evaluate_is_the_loss_and_a_count_of_matching_classes():
    g = np.random.default_rng(4)
    X = g.standard_normal((40, 5))
    T = np.eye(3)[g.integers(0, 3, 40)]
    p = Params(g.uniform(-1, 1, (6, 5)), g.uniform(-1, 1, 6), g.uniform(-1, 1, (3, 6)), g.uniform(-1, 1, 3))
    loss, correct = oracle.evaluate(X, T, p)
    sig = lambda z: 1.0 / (1.0 + np.exp(-z))
    Y = sig(sig(X @ p.W1.T + p.b1) @ p.W2.T + p.b2)
    assert abs(loss - np.mean((Y - T) ** 2)) <= 1e-15
    assert correct == sum(int(np.argmax(Y[r]) == np.argmax(T[r])) for r in range(40))


def test_classes_of_one_output_threshold_at_one_half():
    V = np.array([[0.2], [0.5], [0.5000001], [0.99]])
    assert oracle.classes(V).tolist() == [0, 0, 1, 1]
    assert oracle.classes(np.array([[0.1, 0.7, 0.7], [0.3, 0.2, 0.1]])).tolist() == [1, 0]


@pytest.mark.parametrize("prec", [None, "bf16", "e4m3"])
def test_oracle_results_do_not_depend_on_the_thread_count(prec):
    """The shared loops only split independent outputs among threads: one
    thread and several give the same bits (minibatch shape above the
    sharing threshold)."""
    w = synth.single(4, n_rows=4096, hidden=64)
    p = Params.of(w["theta"])
    runs = []
    for threads in (1, max(2, oracle.max_threads())):
        oracle.set_threads(threads)
        if prec is None:
            q, h = oracle.train(w["X"], w["T"], p, lr=0.1, epochs=1, batch=2048)
        else:
            q, h, _ = oracle.train_lowp(w["X"], w["T"], p, lr=0.1, epochs=1, batch=2048, prec=prec)
        runs.append((q.flat(), h))
    oracle.set_threads(0)
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])
