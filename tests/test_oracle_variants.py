"""Pins of the oracle's two training variants (tanh hidden activation, heavy-
ball momentum), each against something other than the variant code itself:
the special case that is the paper's method (the pinned core oracle), the
identity tanh(z) = 2 sigma(2z) - 1 that maps a tanh net onto a sigmoid net
with rescaled parameters (loss and, by the chain rule, gradients), central
finite differences, a closed form on a 1-1-1 net, and the momentum
recurrence over two steps written out from gradients of the core oracle."""
import numpy as np
import pytest

import oracle
from oracle import Params
from paper_1908_07847_amd import synth


def small_problem(n=24, d=5, h=4, k=3, seed=7):
    g = np.random.default_rng(seed)
    X = g.normal(size=(n, d))
    T = np.eye(k)[g.integers(0, k, size=n)]
    p = Params(g.uniform(-0.8, 0.8, (h, d)), g.uniform(-0.8, 0.8, h), g.uniform(-0.8, 0.8, (k, h)),
               g.uniform(-0.8, 0.8, k))
    return X, T, p


def rel(a, b):
    a, b = np.asarray(a, np.float64).ravel(), np.asarray(b, np.float64).ravel()
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def test_sigmoid_without_momentum_is_the_core_oracle():
    w = synth.single(1)
    p = Params.of(w["theta"])
    q0, h0 = oracle.train(w["X"], w["T"], p, 0.1, 50)
    q1, h1, v = oracle.train_var(w["X"], w["T"], p, 0.1, 50)
    assert v is None
    assert rel(q1.flat(), q0.flat()) <= 1e-13 and rel(h1, h0) <= 1e-13
    qb0, _ = oracle.train(w["X"], w["T"], p, 0.1, 3, batch=16)
    qb1, _, _ = oracle.train_var(w["X"], w["T"], p, 0.1, 3, batch=16)
    assert rel(qb1.flat(), qb0.flat()) <= 1e-13


def tanh_as_sigmoid(p: Params) -> Params:
    """Parameters of the sigmoid net computing the same outputs as the tanh
    net p: tanh(z) = 2 sigma(2z) - 1."""
    return Params(2 * p.W1, 2 * p.b1, 2 * p.W2, p.b2 - p.W2.sum(axis=1))


def test_tanh_net_equals_a_rescaled_sigmoid_net():
    X, T, p = small_problem()
    L_t, g_t = oracle.loss_grad_var(X, T, p, act="tanh")
    L_s, g_s = oracle.loss_grad(X, T, tanh_as_sigmoid(p))
    assert abs(L_t - L_s) <= 1e-14 * max(1.0, L_s)
    # chain rule through the map p -> p'
    assert rel(g_t.W1, 2 * g_s.W1) <= 1e-12
    assert rel(g_t.b1, 2 * g_s.b1) <= 1e-12
    assert rel(g_t.W2, 2 * g_s.W2 - g_s.b2[:, None]) <= 1e-12
    assert rel(g_t.b2, g_s.b2) <= 1e-12


def test_tanh_gradient_against_central_differences():
    X, T, p = small_problem(seed=11)
    _, g = oracle.loss_grad_var(X, T, p, act="tanh")
    flat = p.flat()
    d, h, k = p.shape
    fd = np.zeros_like(flat)
    eps = 1e-6
    for i in range(flat.size):
        a, b = flat.copy(), flat.copy()
        a[i] += eps
        b[i] -= eps
        La, _ = oracle.loss_grad_var(X, T, Params.of(synth.Theta.unpack(a, d, h, k)), act="tanh")
        Lb, _ = oracle.loss_grad_var(X, T, Params.of(synth.Theta.unpack(b, d, h, k)), act="tanh")
        fd[i] = (La - Lb) / (2 * eps)
    assert rel(g.flat(), fd) <= 1e-6


def test_tanh_one_one_one_closed_form():
    x, t, w1, b1, w2, b2 = 0.7, 1.0, 0.4, -0.2, -0.9, 0.3
    z1 = w1 * x + b1
    hh = np.tanh(z1)
    y = 1 / (1 + np.exp(-(w2 * hh + b2)))
    L_ref = (y - t) ** 2
    dz2 = 2 * (y - t) * y * (1 - y)
    p = Params(np.array([[w1]]), np.array([b1]), np.array([[w2]]), np.array([b2]))
    L, g = oracle.loss_grad_var(np.array([[x]]), np.array([[t]]), p, act="tanh")
    assert abs(L - L_ref) <= 1e-15
    assert abs(g.W2[0, 0] - dz2 * hh) <= 1e-15
    assert abs(g.b2[0] - dz2) <= 1e-15
    assert abs(g.W1[0, 0] - dz2 * w2 * (1 - hh * hh) * x) <= 1e-15
    assert abs(g.b1[0] - dz2 * w2 * (1 - hh * hh)) <= 1e-15


@pytest.mark.parametrize("act", ["sigmoid", "tanh"])
def test_momentum_two_steps_written_out(act):
    X, T, p = small_problem(seed=3)
    lr, mu = 0.3, 0.8
    q2, hist, v = oracle.train_var(X, T, p, lr, 2, act=act, mu=mu)
    _, g0 = oracle.loss_grad_var(X, T, p, act=act)
    q1 = Params.of(synth.Theta.unpack(p.flat() - lr * g0.flat(), *p.shape))   # first step: v = g0
    L1, g1 = oracle.loss_grad_var(X, T, q1, act=act)
    v_ref = mu * g0.flat() + g1.flat()
    assert rel(v, v_ref) <= 1e-13
    assert rel(q2.flat(), q1.flat() - lr * v_ref) <= 1e-13
    assert abs(hist[1] - L1) <= 1e-14


def test_momentum_zero_is_plain_descent_and_resumes():
    X, T, p = small_problem(seed=5)
    qa, ha, _ = oracle.train_var(X, T, p, 0.2, 6, act="tanh")
    qb, hb, vb = oracle.train_var(X, T, p, 0.2, 6, act="tanh", mu=1e-300)   # velocity path, mu ~ 0
    assert rel(qb.flat(), qa.flat()) <= 1e-14
    # a run of 3 + 3 epochs carrying the velocity equals a run of 6
    q6, h6, v6 = oracle.train_var(X, T, p, 0.2, 6, act="tanh", mu=0.9)
    q3, h3, v3 = oracle.train_var(X, T, p, 0.2, 3, act="tanh", mu=0.9)
    q33, h33, v33 = oracle.train_var(X, T, q3, 0.2, 3, act="tanh", mu=0.9, velocity=v3)
    assert np.array_equal(q33.flat(), q6.flat()) and np.array_equal(v33, v6)
    assert np.array_equal(np.concatenate([h3, h33]), h6)


# ---------------------------------------------------------------- planted mistakes
import os

ODIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")
VMUTANTS = {
    "tanh slope as the sigmoid's": ("return act == 1 ? 1.0 - a * a : a * (1.0 - a);",
                                    "return a * (1.0 - a);"),
    "tanh evaluated as the sigmoid": ("return act == 1 ? tanh(z) : sigmoid(z);", "return sigmoid(z);"),
    "velocity updated after the step": ("    *v = mu * *v + g;\n    *w -= lr * *v;",
                                        "    *w -= lr * *v;\n    *v = mu * *v + g;"),
    "learning rate folded into the velocity": ("*v = mu * *v + g;\n    *w -= lr * *v;",
                                               "*v = mu * *v + lr * g;\n    *w -= lr * *v;"),
    "b1 velocity overlaps W1's": ("*vb1 = velocity ? vW1 + (int64_t)h * d : NULL;",
                                  "*vb1 = velocity ? vW1 + (int64_t)h * d - 1 : NULL;"),
}


def variant_pins_failing() -> list:
    failed = []
    for name, fn in (("equivalence", test_tanh_net_equals_a_rescaled_sigmoid_net),
                     ("closed form", test_tanh_one_one_one_closed_form),
                     ("momentum sigmoid", lambda: test_momentum_two_steps_written_out("sigmoid")),
                     ("momentum tanh", lambda: test_momentum_two_steps_written_out("tanh"))):
        try:
            fn()
        except AssertionError:
            failed.append(name)
    return failed


@pytest.mark.parametrize("name", sorted(VMUTANTS))
def test_each_planted_variant_mistake_fails_a_pin(name, tmp_path):
    old, new = VMUTANTS[name]
    src = open(oracle.VARIANTS_SRC).read()
    assert src.count(old) == 1, f"mutation site for {name!r} not found"
    mut = tmp_path / "variants_mut.c"
    mut.write_text(src.replace(old, new))
    lib = oracle.build_variant([os.path.join(ODIR, "mlp_oracle.c"), os.path.join(ODIR, "mlp_oracle_lowp.c"),
                                str(mut)], str(tmp_path / "libvmut.so"))
    with oracle.use_library(lib):
        failed = variant_pins_failing()
    assert failed, f"planted mistake {name!r} passed every pin"


def test_variant_pins_pass_on_the_real_oracle():
    assert variant_pins_failing() == []
