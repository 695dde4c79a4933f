"""Planted mistakes, on the CPU only: each copy of the oracle source carries one
plausible error (a dropped term, a wrong sign, a wrong scale or index), and at
least one of the independent pins must reject it.  This shows the pins are
strong enough to catch mistakes in the oracle they check."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from oracle import Params

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "mlp_oracle.c")
LOWP = os.path.join(os.path.dirname(HERE), "oracle", "mlp_oracle_lowp.c")

MUTANTS = {
    "sigmoid slope dropped from delta2": ("dY[r * k + o] * y * (1.0 - y)", "dY[r * k + o]"),
    "hidden slope a(1-a) dropped": ("delta1[r * h + j] = s * a * (1.0 - a);", "delta1[r * h + j] = s * a;"),
    "hidden bias ignored": ("double z = b1[j];", "double z = 0.0;"),
    "update sign flipped": ("W1[q] -= lr * gW1[q];", "W1[q] += lr * gW1[q];"),
    "loss gradient not divided by outputs": ("dY[r * k + o] = 2.0 * (Y[r * k + o] - T[r * k + o]) / ((double)n * (double)k);",
                                             "dY[r * k + o] = 2.0 * (Y[r * k + o] - T[r * k + o]) / ((double)n);"),
    "gb2 sums the wrong output": ("for (int64_t r = 0; r < n; ++r) s += delta2[r * k + o];\n    gb2[o] = s;",
                                  "for (int64_t r = 0; r < n; ++r) s += delta2[r * k];\n    gb2[o] = s;"),
    "output weight index transposed": ("s += delta2[r * k + o] * W2[(int64_t)o * h + j];",
                                       "s += delta2[r * k + o] * W2[(int64_t)j * k + o];"),
    "gW1 uses the activation instead of the input": ("s += delta1[r * h + j] * X[r * d + i];",
                                                     "s += delta1[r * h + j] * A[r * h + (i % h)];"),
    "short last minibatch dropped": ("int64_t steps = (n + batch - 1) / batch;", "int64_t steps = n / batch;"),
}


def pins_pass() -> list:
    """Run a subset of the independent pins; return the names of those that fail."""
    failed = []
    ref = json.load(open(os.path.join(HERE, "golden", "worked_221.json")))
    inp = ref["inputs"]
    X, T = np.array(inp["X"]), np.array(inp["T"])
    p = Params(inp["W1"], inp["b1"], inp["W2"], inp["b2"])
    q, hist = oracle.train(X, T, p, lr=inp["lr"], epochs=1)
    if not (np.allclose(q.W1, np.array(ref["W1_new"], float), rtol=1e-12) and
            np.allclose(q.b2, np.array(ref["b2_new"], float), rtol=1e-12) and
            abs(hist[0] - float(ref["L0"])) < 1e-12):
        failed.append("worked 2-2-1 step")
    g = np.random.default_rng(0)
    n, d, h, k = 10, 4, 3, 2
    Xr = g.standard_normal((n, d))
    Tr = np.eye(k)[g.integers(0, k, n)]
    pr = Params(g.uniform(-1, 1, (h, d)), g.uniform(-1, 1, h), g.uniform(-1, 1, (k, h)), g.uniform(-1, 1, k))
    try:
        L, gr = oracle.loss_grad(Xr, Tr, pr)
        W1, b1, W2, b2 = (torch.tensor(a, requires_grad=True) for a in (pr.W1, pr.b1, pr.W2, pr.b2))
        loss = torch.nn.functional.mse_loss(torch.sigmoid(torch.sigmoid(torch.tensor(Xr) @ W1.T + b1) @ W2.T + b2),
                                            torch.tensor(Tr))
        loss.backward()
        if abs(L - loss.item()) > 1e-12 or any(np.max(np.abs(a - b.grad.numpy())) > 1e-10 for a, b in
                                               [(gr.W1, W1), (gr.b1, b1), (gr.W2, W2), (gr.b2, b2)]):
            failed.append("torch float64 autograd")
    except Exception:
        failed.append("torch float64 autograd (crashed)")
    # minibatch training against torch SGD on a ragged batch
    qm, _ = oracle.train(Xr, Tr, pr, 0.3, 2, batch=4)
    params = [torch.tensor(a, requires_grad=True) for a in (pr.W1, pr.b1, pr.W2, pr.b2)]
    opt = torch.optim.SGD(params, lr=0.3)
    for _ in range(2):
        for r0 in range(0, n, 4):
            W1, b1, W2, b2 = params
            xb, tb = torch.tensor(Xr[r0:r0 + 4]), torch.tensor(Tr[r0:r0 + 4])
            l = torch.nn.functional.mse_loss(torch.sigmoid(torch.sigmoid(xb @ W1.T + b1) @ W2.T + b2), tb)
            opt.zero_grad(); l.backward(); opt.step()
    if np.max(np.abs(qm.W1 - params[0].detach().numpy())) > 1e-10:
        failed.append("torch SGD minibatches")
    return failed


def test_unmodified_oracle_passes_the_pins():
    assert pins_pass() == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_each_planted_mistake_fails_a_pin(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name!r} not found"
    mut = tmp_path / "mlp_oracle_mut.c"
    mut.write_text(src.replace(old, new, 1))
    lib = oracle.build_variant([str(mut), LOWP], str(tmp_path / "libmut.so"))
    with oracle.use_library(lib):
        failed = pins_pass()
    assert failed, f"planted mistake {name!r} passed every pin"
