"""Independent pins of the reduced-precision oracle (oracle/mlp_oracle_lowp.c).

The reduced-precision forms are the build's own (the paper trains in float,
section 2.2): the method of section 2.2 with the operands of the two large
contractions rounded -- X and W1 for the hidden pre-activation, delta1 and X
for the input-layer gradient -- while the biases, the sigmoid of Equation 1,
the output layer, both deltas, gb1 (from the unrounded delta1), gW2, gb2, the
loss and the update stay exact.  e4m3 operands carry per-tensor power-of-two
scales: X's from the whole dataset once, W1's from the master W1 of the step,
delta1's from the previous step's amax (the first step from the bound
max_h sum_k |W2| / (8 m K), formed in float32).

Here every step is recomputed in torch float64 on the CPU from that
definition, with the rounding done by torch's own bfloat16 / float8_e4m3fn
casts (an implementation independent of the oracle's), the unrounded
gradients by torch autograd (dL/dZ1 is delta1), and the scale exponents from
the definition "largest e with amax 2^e <= 448".  One and two steps (the
second uses the first step's delta1 amax and the updated W1's scale) must
agree with ora_train_lowp element by element.  Planted mistakes in copies of
the oracle source (delta1 rounded for gb1, X unrounded in gW1, the current
step's delta1 amax, W1 scaled from the previous step, a wrong first-step
bound) must each fail these pins.
"""
import math
import os

import numpy as np
import pytest
import torch

import oracle
from oracle import Params
from paper_1908_07847_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "mlp_oracle.c")
LOWP = os.path.join(ROOT, "oracle", "mlp_oracle_lowp.c")
F64 = torch.float64


def scale_exp(amax: float) -> int:
    """Largest integer e with amax * 2^e <= 448 (0 for amax == 0)."""
    if amax == 0.0:
        return 0
    e = math.floor(math.log2(448.0 / amax))
    while amax * 2.0 ** e > 448.0:
        e -= 1
    while amax * 2.0 ** (e + 1) <= 448.0:
        e += 1
    return e


def q(v: torch.Tensor, prec: str, e: int = 0) -> torch.Tensor:
    """Operand rounding through torch's casts (e4m3: saturate, cast, unscale)."""
    if prec == "bf16":
        return v.to(torch.bfloat16).to(F64)
    s = 2.0 ** e
    return (v * s).clamp(-448.0, 448.0).to(torch.float8_e4m3fn).to(F64) / s


def first_step_bound(W2: torch.Tensor, m: int) -> float:
    """max over hidden units of sum_k |W2[k][h]|, summed left to right in
    float32, divided by 8 m K in float32."""
    a = W2.to(torch.float32).abs()
    col = a[0].clone()
    for k in range(1, a.shape[0]):
        col = col + a[k]
    return float(col.max() / torch.tensor(8 * m * a.shape[0], dtype=torch.float32))


def torch_steps(X, T, p: Params, lr: float, batch: int, steps: int, prec: str):
    """`steps` minibatch steps of the reduced-precision method in torch
    float64; returns (params, losses per step, scale exponents per step)."""
    X, T = torch.tensor(X, dtype=F64), torch.tensor(T, dtype=F64)
    n = X.shape[0]
    W1, b1, W2, b2 = (torch.tensor(a, dtype=F64) for a in (p.W1, p.b1, p.W2, p.b2))
    ex = scale_exp(float(X.abs().max())) if prec == "e4m3" else 0
    Xq = q(X, prec, ex)
    d1_amax_prev = None
    losses, scales = [], []
    for s in range(steps):
        r0 = (s * batch) % n
        m = min(batch, n - r0)
        Xb, Tb = Xq[r0:r0 + m], T[r0:r0 + m]
        ew = ed = 0
        if prec == "e4m3":
            ew = scale_exp(float(W1.abs().max()))
            ed = scale_exp(first_step_bound(W2, m) if d1_amax_prev is None else d1_amax_prev)
        scales.append((ex, ew, ed))
        W1q = q(W1, prec, ew)
        b1l, W2l, b2l = (t.clone().requires_grad_(True) for t in (b1, W2, b2))
        Z1 = Xb @ W1q.T + b1l
        Z1.retain_grad()
        Y = torch.sigmoid(torch.sigmoid(Z1) @ W2l.T + b2l)
        loss = torch.nn.functional.mse_loss(Y, Tb)
        loss.backward()
        d1 = Z1.grad                              # delta1 = dL/dZ1, unrounded
        gW1 = q(d1, prec, ed).T @ Xb               # rounded operands of the gradient contraction
        d1_amax_prev = float(d1.abs().max())
        losses.append(float(loss.detach()))
        W1 = W1 - lr * gW1
        b1 = b1 - lr * b1l.grad
        W2 = W2 - lr * W2l.grad
        b2 = b2 - lr * b2l.grad
    return Params(W1.numpy(), b1.numpy(), W2.numpy(), b2.numpy()), np.array(losses), np.array(scales)


def case(kind: str):
    """Inputs: the large-N workload's generator at a small size.
      'plain'      as generated (weights U(-0.5, 0.5));
      'saturated'  W1 scaled by 8, so some hidden units saturate and delta1
                   spans more than the normal range of e4m3 (its smallest
                   entries then round on the subnormal grid, whose spacing
                   depends on the scale exponent);
      'cross'      W1's largest entry just below 0.875 = 448 / 2^9 with a
                   learning rate that carries it past, so the second step's
                   W1 scale is one power of two lower, and a few tiny W1
                   entries that sit on the subnormal grid of either scale."""
    w = synth.single(4, n_rows=256, hidden=16)
    p = Params.of(w["theta"])
    lr = 0.1
    if kind == "saturated":
        p = Params(p.W1 * 8.0, p.b1, p.W2, p.b2)
    if kind == "cross":
        L, g = oracle.loss_grad(w["X"], w["T"], p)
        j, i = np.unravel_index(np.argmax(np.abs(g.W1)), g.W1.shape)
        W1 = p.W1.copy()
        W1[j, i] = -0.87 * np.sign(g.W1[j, i])      # the update moves it away from 0
        W1[(j + 1) % 16, :3] = [1e-5, -2.3e-5, 3.7e-5]
        p = Params(W1, p.b1, p.W2, p.b2)
        lr = 0.02 / abs(g.W1[j, i])
    return w["X"].astype(np.float64), w["T"].astype(np.float64), p, lr


def compare(prec: str, kind: str, steps: int, batch: int):
    """Max elementwise relative disagreement (per tensor, normwise) between the
    oracle and the torch recomputation, the scale logs of both, and the losses."""
    X, T, p, lr = case(kind)
    n = X.shape[0]
    epochs = steps * batch // n
    qo, ho, slog = oracle.train_lowp(X, T, p, lr, epochs, batch, prec)
    qt, lt, st = torch_steps(X, T, p, lr, batch, steps, prec)
    err = max(float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
              for a, b in [(qo.W1, qt.W1), (qo.b1, qt.b1), (qo.W2, qt.W2), (qo.b2, qt.b2)])
    per_epoch = lt.reshape(epochs, -1).mean(axis=1)
    lerr = float(np.max(np.abs(ho - per_epoch) / per_epoch))
    return err, lerr, (slog if prec == "e4m3" else None), st


CASES = [("bf16", "plain", 1, 256), ("e4m3", "plain", 1, 256), ("bf16", "plain", 2, 128),
         ("e4m3", "plain", 2, 128), ("bf16", "saturated", 2, 128), ("e4m3", "saturated", 2, 128),
         ("e4m3", "cross", 2, 128)]


@pytest.mark.parametrize("prec,kind,steps,batch", CASES)
def test_lowp_steps_equal_torch_recomputation(prec, kind, steps, batch):
    err, lerr, slog, st = compare(prec, kind, steps, batch)
    assert err <= 1e-12 and lerr <= 1e-12, (err, lerr)
    if slog is not None:
        assert np.array_equal(slog, st), (slog, st)


def test_pins_exercise_the_delayed_and_first_step_scales():
    """The two-step e4m3 cases really depend on what they pin: the second
    step's delta1 scale comes from the first step's amax and differs from the
    first step's bound-derived scale, and in the 'cross' case W1's scale
    changes between the steps."""
    _, _, slog, _ = compare("e4m3", "plain", 2, 128)
    assert slog[1, 2] != slog[0, 2]
    _, _, slog, _ = compare("e4m3", "cross", 2, 128)
    assert slog[1, 1] != slog[0, 1]


MUTANTS = {
    "delta1 rounded for gb1": [("for (int64_t r = 0; r < m; ++r) sum += delta1[r * h + j];",
                                "for (int64_t r = 0; r < m; ++r) sum += delta1q[r * h + j];")],
    "X unrounded in gW1": [("sum += delta1q[r * h + j] * Xqb[r * d + i];",
                            "sum += delta1q[r * h + j] * X[(r0 + r) * d + i];")],
    "current step's delta1 amax": [("delta1q[q] = q_op(delta1[q], prec, ed);",
                                    "delta1q[q] = q_op(delta1[q], prec, ora_e4m3_scale_exp(amax_d1));")],
    "W1 scaled from the previous step": [
        ("double amax_d1_prev = -1.0;", "double amax_d1_prev = -1.0; double amax_w1_prev = -1.0;"),
        ("ew = ora_e4m3_scale_exp(amax);",
         "ew = ora_e4m3_scale_exp(amax_w1_prev < 0.0 ? amax : amax_w1_prev); amax_w1_prev = amax;")],
    "first-step bound without the factor 1/8": [("bound = bound / (float)(8 * m * k);",
                                                 "bound = bound / (float)(m * k);")],
    "first step scaled like later steps": [("if (amax_d1_prev < 0.0) {", "if (amax_d1_prev < -2.0) {")],
}


def pins_fail() -> list:
    failed = []
    for prec, kind, steps, batch in CASES:
        try:
            err, lerr, slog, st = compare(prec, kind, steps, batch)
        except Exception as exc:  # a mutant may also crash
            failed.append(f"{prec} {kind} {steps} crashed: {exc}")
            continue
        if err > 1e-12 or lerr > 1e-12 or (slog is not None and not np.array_equal(slog, st)):
            failed.append(f"{prec} {kind} {steps}")
    return failed


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_each_planted_lowp_mistake_fails_a_pin(name, tmp_path):
    src = open(LOWP).read()
    for old, new in MUTANTS[name]:
        assert src.count(old) == 1, f"mutation site for {name!r} not found"
        src = src.replace(old, new)
    mut = tmp_path / "mlp_oracle_lowp_mut.c"
    mut.write_text(src)
    lib = oracle.build_variant([SRC, str(mut)], str(tmp_path / "libmut.so"))
    with oracle.use_library(lib):
        failed = pins_fail()
    assert failed, f"planted mistake {name!r} passed every pin"
