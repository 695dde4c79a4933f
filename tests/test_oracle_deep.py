"""Pins of the oracle's networks with several hidden layers, against
something other than that code: the one-hidden-layer special case (the
pinned core and variant oracles), torch float64 CPU autograd of the same
network (an independent routine), and central finite differences; planted
mistakes in a copy of the source must fail one of them."""
import os

import numpy as np
import pytest
import torch

import oracle
from oracle import Params


def problem(widths, n=20, seed=0):
    g = np.random.default_rng(seed)
    X = g.normal(size=(n, widths[0]))
    T = np.eye(widths[-1])[g.integers(0, widths[-1], size=n)] if widths[-1] > 1 else g.integers(0, 2, (n, 1)) * 1.0
    theta = g.uniform(-0.9, 0.9, oracle.deep_n_params(widths))
    return X, T, theta


def rel(a, b):
    a, b = np.asarray(a, np.float64).ravel(), np.asarray(b, np.float64).ravel()
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def torch_loss(X, T, widths, theta, act):
    th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    a = torch.tensor(X, dtype=torch.float64)
    o = 0
    L = len(widths) - 1
    for l in range(L):
        W = th[o:o + widths[l + 1] * widths[l]].view(widths[l + 1], widths[l])
        o += widths[l + 1] * widths[l]
        b = th[o:o + widths[l + 1]]
        o += widths[l + 1]
        z = a @ W.T + b
        a = torch.sigmoid(z) if (l == L - 1 or act == "sigmoid") else torch.tanh(z)
    loss = torch.nn.functional.mse_loss(a, torch.tensor(T, dtype=torch.float64))
    loss.backward()
    return float(loss.detach()), th.grad.numpy()


def test_one_hidden_layer_is_the_core_oracle():
    widths = [6, 5, 3]
    X, T, th = problem(widths, seed=1)
    L, g = oracle.deep_loss_grad(X, T, widths, th)
    p = Params(th[:30].reshape(5, 6), th[30:35], th[35:50].reshape(3, 5), th[50:53])
    L0, g0 = oracle.loss_grad(X, T, p)
    assert abs(L - L0) <= 1e-15 and rel(g, g0.flat()) <= 1e-13
    Lt, gt = oracle.deep_loss_grad(X, T, widths, th, act="tanh")
    Lv, gv = oracle.loss_grad_var(X, T, p, act="tanh")
    assert abs(Lt - Lv) <= 1e-15 and rel(gt, gv.flat()) <= 1e-13
    q, h = oracle.deep_train(X, T, widths, th, 0.3, 20)
    q0, h0 = oracle.train(X, T, p, 0.3, 20)
    assert rel(q, q0.flat()) <= 1e-13 and rel(h, h0) <= 1e-13


@pytest.mark.parametrize("widths,act", [([5, 7, 4, 3], "sigmoid"), ([5, 7, 4, 3], "tanh"), ([3, 4, 4, 4, 1], "tanh"),
                                        ([8, 6, 2], "sigmoid")])
def test_against_torch_autograd(widths, act):
    X, T, th = problem(widths, seed=len(widths))
    L, g = oracle.deep_loss_grad(X, T, widths, th, act=act)
    Lr, gr = torch_loss(X, T, widths, th, act)
    assert abs(L - Lr) <= 1e-14 * max(Lr, 1) and rel(g, gr) <= 1e-12


def test_two_hidden_layers_against_central_differences():
    widths = [4, 5, 3, 2]
    X, T, th = problem(widths, seed=9)
    _, g = oracle.deep_loss_grad(X, T, widths, th, act="tanh")
    fd = np.zeros_like(th)
    for i in range(th.size):
        a, b = th.copy(), th.copy()
        a[i] += 1e-6
        b[i] -= 1e-6
        fd[i] = (oracle.deep_loss_grad(X, T, widths, a, act="tanh")[0] -
                 oracle.deep_loss_grad(X, T, widths, b, act="tanh")[0]) / 2e-6
    assert rel(g, fd) <= 1e-6


def test_training_descends_and_lr_zero_is_identity():
    widths = [5, 7, 4, 3]
    X, T, th = problem(widths, n=40, seed=2)
    q, h = oracle.deep_train(X, T, widths, th, 0.0, 3)
    assert np.array_equal(q, th)
    q, h = oracle.deep_train(X, T, widths, th, 0.2, 300)
    assert np.all(np.diff(h) <= 1e-15) and h[-1] < h[0]


ODIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")
DMUTANTS = {
    "hidden slope dropped": ("Dl[l][r * w[l] + i] = s * (act == 1 ? 1.0 - a * a : a * (1.0 - a));",
                             "Dl[l][r * w[l] + i] = s;"),
    "output layer uses the hidden activation": ("(l == L - 1 || act == 0) ? sig(z) : tanh(z)",
                                                "(act == 0) ? sig(z) : tanh(z)"),
    "delta propagated with the layer below's weights": ("const double *W = theta + layer_off(w, l);",
                                                        "const double *W = theta + layer_off(w, l > 0 ? l - 1 : 0);"),
    "bias gradient of the wrong layer": ("double *gW = g + layer_off(w, l), *gb = gW + (int64_t)w[l + 1] * w[l];",
                                         "double *gW = g + layer_off(w, l), *gb = gW + (int64_t)w[l + 1] * w[l] - 1;"),
}


def deep_pins_failing() -> list:
    failed = []
    for name, fn in (("core", test_one_hidden_layer_is_the_core_oracle),
                     ("torch 4", lambda: test_against_torch_autograd([5, 7, 4, 3], "sigmoid")),
                     ("torch tanh", lambda: test_against_torch_autograd([3, 4, 4, 4, 1], "tanh"))):
        try:
            fn()
        except AssertionError:
            failed.append(name)
    return failed


@pytest.mark.parametrize("name", sorted(DMUTANTS))
def test_each_planted_deep_mistake_fails_a_pin(name, tmp_path):
    old, new = DMUTANTS[name]
    src = open(oracle.DEEP_SRC).read()
    assert src.count(old) == 1, f"mutation site for {name!r} not found"
    mut = tmp_path / "deep_mut.c"
    mut.write_text(src.replace(old, new))
    lib = oracle.build_variant([os.path.join(ODIR, f) for f in ("mlp_oracle.c", "mlp_oracle_lowp.c",
                                                                  "mlp_oracle_variants.c")] + [str(mut)],
                               str(tmp_path / "libdmut.so"))
    with oracle.use_library(lib):
        failed = deep_pins_failing()
    assert failed, f"planted mistake {name!r} passed every pin"
