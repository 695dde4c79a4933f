"""Writes worked_221.json: one gradient-descent step of a 2-2-1 sigmoid net,
derived scalar by scalar at 40 significant digits with Python's decimal
module (no numpy, no oracle code).  Every quantity below is written out for
this tiny net by hand from the chain rule, so a reader can follow (and
re-derive with pencil and a calculator) each number in the fixture.

Net (section 2.2 of arxiv 1908.07847): two inputs, two sigmoid hidden units
(Equation 1), one sigmoid output, mean squared error over the two samples,
learning rate 0.1, no momentum.

Run:  python tests/golden/make_worked_221.py
"""
import json
import os
from decimal import Decimal as Dm, getcontext

getcontext().prec = 40
one = Dm(1)


def sig(z):
    return one / (one + (-z).exp())


X = [[Dm("0.5"), Dm("-1.0")], [Dm("-0.25"), Dm("0.75")]]
T = [Dm(1), Dm(0)]
W1 = [[Dm("0.1"), Dm("0.3")], [Dm("-0.2"), Dm("0.4")]]   # W1[hidden][input]
b1 = [Dm("0.05"), Dm("-0.05")]
W2 = [Dm("0.6"), Dm("-0.7")]                              # W2[0][hidden]
b2 = Dm("0.1")
lr = Dm("0.1")
m, K = 2, 1


def forward(W1, b1, W2, b2):
    z1 = [[X[r][0] * W1[j][0] + X[r][1] * W1[j][1] + b1[j] for j in range(2)] for r in range(2)]
    a = [[sig(z1[r][j]) for j in range(2)] for r in range(2)]
    z2 = [a[r][0] * W2[0] + a[r][1] * W2[1] + b2 for r in range(2)]
    y = [sig(z2[r]) for r in range(2)]
    loss = ((y[0] - T[0]) ** 2 + (y[1] - T[1]) ** 2) / (m * K)
    return z1, a, y, loss


z1, a, y, L0 = forward(W1, b1, W2, b2)
# dL/dy_r = 2 (y_r - t_r) / (m K);  output delta: times y_r (1 - y_r)
d2 = [Dm(2) * (y[r] - T[r]) / (m * K) * y[r] * (one - y[r]) for r in range(2)]
gW2 = [d2[0] * a[0][j] + d2[1] * a[1][j] for j in range(2)]
gb2 = d2[0] + d2[1]
# hidden delta: d2_r * W2[j] * a_rj (1 - a_rj), with the pre-update W2
d1 = [[d2[r] * W2[j] * a[r][j] * (one - a[r][j]) for j in range(2)] for r in range(2)]
gW1 = [[d1[0][j] * X[0][i] + d1[1][j] * X[1][i] for i in range(2)] for j in range(2)]
gb1 = [d1[0][j] + d1[1][j] for j in range(2)]
W1n = [[W1[j][i] - lr * gW1[j][i] for i in range(2)] for j in range(2)]
b1n = [b1[j] - lr * gb1[j] for j in range(2)]
W2n = [W2[j] - lr * gW2[j] for j in range(2)]
b2n = b2 - lr * gb2
_, _, _, L1 = forward(W1n, b1n, W2n, b2n)

s = lambda v: str(+v)
out = {
    "citation": "arxiv 1908.07847 section 2.2 and Equation 1; hand-derived 2-2-1 step, "
                "MSE mean over rows x outputs, lr 0.1, no momentum",
    "inputs": {"X": [[0.5, -1.0], [-0.25, 0.75]], "T": [[1.0], [0.0]],
               "W1": [[0.1, 0.3], [-0.2, 0.4]], "b1": [0.05, -0.05], "W2": [[0.6, -0.7]],
               "b2": [0.1], "lr": 0.1},
    "Z1": [[s(v) for v in row] for row in z1],
    "A": [[s(v) for v in row] for row in a],
    "Y": [s(v) for v in y],
    "L0": s(L0),
    "delta2": [s(v) for v in d2],
    "gW2": [[s(v) for v in gW2]], "gb2": [s(gb2)],
    "gW1": [[s(v) for v in row] for row in gW1], "gb1": [s(v) for v in gb1],
    "W1_new": [[s(v) for v in row] for row in W1n], "b1_new": [s(v) for v in b1n],
    "W2_new": [[s(v) for v in W2n]], "b2_new": [s(b2n)],
    "L1": s(L1),
}
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "worked_221.json"), "w") as f:
    json.dump(out, f, indent=1)
    f.write("\n")
print(json.dumps({k: out[k] for k in ("L0", "L1")}))
