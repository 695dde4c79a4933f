"""FP64 CPU oracle for one-hidden-layer sigmoid MLP training (arxiv 1908.07847).

TEST INFRASTRUCTURE ONLY.  Only `tests/`, `__graft_entry__.smoke()` and the
CPU-baseline leg of `bench.py` may import this package.  It shares no code
with the HIP library: the C sources here (`mlp_oracle.c`,
`mlp_oracle_lowp.c`, `mlp_oracle_variants.c`, `mlp_oracle_deep.c`) are plain float64 loops
written from the paper's section 2.2 and Equation 1, compiled with gcc into
`liboracle.so`.

Every array argument is converted to float64 here (an exact widening of
float32 inputs), so the oracle sees exactly the values the GPU sees.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRCS = [os.path.join(_HERE, "mlp_oracle.c"), os.path.join(_HERE, "mlp_oracle_lowp.c"),
         os.path.join(_HERE, "mlp_oracle_variants.c"), os.path.join(_HERE, "mlp_oracle_deep.c")]
VARIANTS_SRC = _SRCS[2]
DEEP_SRC = _SRCS[3]
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (portable x86-64, no FMA contraction)."""
    if not force and os.path.exists(_SO):
        return _SO
    tmp = _SO + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-Wall", "-Wextra", "-o", tmp] + _SRCS + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _SO)
    return _SO


def build_timing(out_dir: str) -> str:
    """The same sources compiled for timing on the host that runs them:
    -O3 -march=native (the checker build above stays portable and free of
    FMA contraction).  Built where it runs, never shipped between hosts."""
    out = os.path.join(out_dir, "liboracle_native.so")
    cmd = ["gcc", "-O3", "-march=native", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-w", "-o", out] + \
        _SRCS + ["-lm"]
    subprocess.run(cmd, check=True)
    return out


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build()
    _lib = _bind(_SO)
    return _lib


def _bind(path: str):
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER(ctypes.c_double)
    i64, i32, dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_double
    lib.ora_forward.argtypes = [i64, i32, i32, i32, P, P, P, P, P, P, P]
    lib.ora_mse.argtypes = [i64, i32, P, P]
    lib.ora_mse.restype = dbl
    lib.ora_backward.argtypes = [i64, i32, i32, i32, P, P, P, P, P, P, P, P, P, P, P]
    lib.ora_loss_grad.argtypes = [i64, i32, i32, i32, P, P, P, P, P, P, P, P, P, P]
    lib.ora_loss_grad.restype = dbl
    lib.ora_train.argtypes = [i64, i32, i32, i32, i64, P, P, P, P, P, P, dbl, i32, P]
    lib.ora_train_many.argtypes = [i32, ctypes.c_void_p, ctypes.c_void_p, P, ctypes.c_void_p,
                                   ctypes.c_void_p, i32, i32, P, P, P, i32, P, i32]
    lib.ora_max_threads.restype = i32
    lib.ora_set_threads.argtypes = [i32]
    lib.ora_round_format.argtypes = [dbl, i32, i32, dbl]
    lib.ora_round_format.restype = dbl
    lib.ora_round_bf16.argtypes = [dbl]
    lib.ora_round_bf16.restype = dbl
    lib.ora_round_e4m3.argtypes = [dbl]
    lib.ora_round_e4m3.restype = dbl
    lib.ora_e4m3_scale_exp.argtypes = [dbl]
    lib.ora_e4m3_scale_exp.restype = i32
    lib.ora_train_lowp.argtypes = [i64, i32, i32, i32, i64, P, P, P, P, P, P, dbl, i32, i32, P,
                                   ctypes.c_void_p, P, P]
    lib.ora_round_array.argtypes = [i32, i32, P, P, i64]
    if hasattr(lib, "ora_train_var"):
        lib.ora_train_var.argtypes = [i64, i32, i32, i32, i64, i32, dbl, P, P, P, P, P, P, dbl, i32, P, P]
        lib.ora_loss_grad_var.argtypes = [i64, i32, i32, i32, i32, P, P, P, P, P, P, P, P, P, P]
        lib.ora_loss_grad_var.restype = dbl
    if hasattr(lib, "ora_deep_train"):
        vp = ctypes.c_void_p
        lib.ora_deep_loss_grad.argtypes = [i64, i32, vp, i32, P, P, P, P]
        lib.ora_deep_loss_grad.restype = dbl
        lib.ora_deep_train.argtypes = [i64, i32, vp, i32, P, P, P, dbl, i32, P]
    return lib


def build_variant(sources, out_path: str) -> str:
    """Compile other oracle sources (the tests' planted-mistake copies) with the
    same flags; returns the library path."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-w", "-o",
           out_path] + list(sources) + ["-lm"]
    subprocess.run(cmd, check=True)
    return out_path


class use_library:
    """Context manager: route every oracle call to another compiled copy."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = _load()
        _lib = _bind(self.path)
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved


def _d(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Params:
    """float64 parameters W1 [H][D], b1 [H], W2 [K][H], b2 [K]."""

    def __init__(self, W1, b1, W2, b2):
        self.W1, self.b1, self.W2, self.b2 = _d(W1).copy(), _d(b1).copy(), _d(W2).copy(), _d(b2).copy()

    @classmethod
    def of(cls, theta) -> "Params":
        return cls(theta.W1, theta.b1, theta.W2, theta.b2)

    def copy(self) -> "Params":
        return Params(self.W1, self.b1, self.W2, self.b2)

    def flat(self) -> np.ndarray:
        return np.concatenate([self.W1.ravel(), self.b1, self.W2.ravel(), self.b2])

    @property
    def shape(self):
        h, d = self.W1.shape
        return d, h, self.W2.shape[0]


def forward(X, p: Params):
    """Returns (A [n][H], Y [n][K]) -- section 2.2 feed-forward, Equation 1."""
    X = _d(X)
    d, h, k = p.shape
    n = X.shape[0]
    A = np.zeros((n, h)); Y = np.zeros((n, k))
    _load().ora_forward(n, d, h, k, _p(X), _p(p.W1), _p(p.b1), _p(p.W2), _p(p.b2), _p(A), _p(Y))
    return A, Y


def classes(V) -> np.ndarray:
    """Class of each row of outputs (or one-hot / 0-1 targets) V [n][K]: the
    index of the largest entry, the lowest index on ties (np.argmax returns
    the first maximum); with a single output (K = 1, a two-class net) class 1
    when the entry is above 1/2, else 0."""
    V = np.asarray(V)
    if V.shape[1] == 1:
        return (V[:, 0] > 0.5).astype(np.int32)
    return np.argmax(V, axis=1).astype(np.int32)


def predict(X, p: Params):
    """(Y, labels): the outputs of the forward pass and each row's class
    (section 2.2's network read as a classifier; see `classes`)."""
    _, Y = forward(X, p)
    return Y, classes(Y)


def evaluate(X, T, p: Params):
    """(loss, correct) of a net on rows X, T: the error of section 2.2 (mean
    squared error over rows and outputs) and the number of rows whose class
    (first maximum of the outputs) equals the target's."""
    Y, lab = predict(X, p)
    return mse(Y, T), int(np.sum(lab == classes(_d(T))))


def mse(Y, T) -> float:
    Y, T = _d(Y), _d(T)
    return float(_load().ora_mse(Y.shape[0], Y.shape[1], _p(Y), _p(T)))


def backward(X, A, Y, dY, p: Params, want_dx: bool = False):
    """Backpropagation from dL/dY; returns (gW1, gb1, gW2, gb2[, dX])."""
    X, A, Y, dY = _d(X), _d(A), _d(Y), _d(dY)
    d, h, k = p.shape
    n = X.shape[0]
    g = Params(np.zeros((h, d)), np.zeros(h), np.zeros((k, h)), np.zeros(k))
    dX = np.zeros((n, d)) if want_dx else None
    _load().ora_backward(n, d, h, k, _p(X), _p(A), _p(Y), _p(dY), _p(p.W1), _p(p.W2), _p(g.W1),
                         _p(g.b1), _p(g.W2), _p(g.b2), _p(dX) if want_dx else None)
    return (g, dX) if want_dx else g


def loss_grad(X, T, p: Params):
    """(L, gradient Params) of the mean-squared-error reading."""
    X, T = _d(X), _d(T)
    d, h, k = p.shape
    g = Params(np.zeros((h, d)), np.zeros(h), np.zeros((k, h)), np.zeros(k))
    L = _load().ora_loss_grad(X.shape[0], d, h, k, _p(X), _p(T), _p(p.W1), _p(p.b1), _p(p.W2),
                              _p(p.b2), _p(g.W1), _p(g.b1), _p(g.W2), _p(g.b2))
    return float(L), g


def train(X, T, p: Params, lr: float, epochs: int, batch: int = 0):
    """Gradient-descent training; returns (trained Params, loss_hist [epochs])."""
    X, T = _d(X), _d(T)
    d, h, k = p.shape
    q = p.copy()
    hist = np.zeros(max(epochs, 0))
    _load().ora_train(X.shape[0], d, h, k, int(batch), _p(X), _p(T), _p(q.W1), _p(q.b1), _p(q.W2),
                      _p(q.b2), float(lr), int(epochs), _p(hist))
    return q, hist


def train_many(items, X, T, theta_packed, d: int, k: int, epochs: int, threads: int = 0):
    """Independent full-batch nets in the packed layout; returns (theta, loss_hist)."""
    X, T = _d(X), _d(T)
    th = _d(theta_packed).copy()
    n = len(items)
    nr = np.array([it["n_rows"] for it in items], dtype=np.int32)
    nh = np.array([it["n_hidden"] for it in items], dtype=np.int32)
    lr = np.array([float(it["lr"]) for it in items], dtype=np.float64)
    xo = np.array([it["x_off"] for it in items], dtype=np.int64)
    po = np.array([it["p_off"] for it in items], dtype=np.int64)
    hist = np.zeros((n, max(epochs, 0)))
    _load().ora_train_many(n, nr.ctypes.data, nh.ctypes.data, _p(lr), xo.ctypes.data, po.ctypes.data,
                           d, k, _p(X), _p(T), _p(th), int(epochs), _p(hist), int(threads))
    return th, hist


def max_threads() -> int:
    return int(_load().ora_max_threads())


def set_threads(threads: int) -> None:
    """Threads for the oracle's shared loops (<= 0: all processors).  Results
    do not depend on it."""
    _load().ora_set_threads(int(threads))


def round_bf16(v: float) -> float:
    return float(_load().ora_round_bf16(float(v)))


def round_e4m3(v: float) -> float:
    return float(_load().ora_round_e4m3(float(v)))


def e4m3_scale_exp(amax: float) -> int:
    return int(_load().ora_e4m3_scale_exp(float(amax)))


PREC = {"fp32": 0, "bf16": 1, "e4m3": 2}


def train_lowp(X, T, p: Params, lr: float, epochs: int, batch: int, prec: str, first_step_detail=False):
    """Training with rounded contraction operands; returns (Params, loss_hist, scale_log)
    and, with first_step_detail, also (delta1, delta2 W2) of the first step."""
    X, T = _d(X), _d(T)
    d, h, k = p.shape
    q = p.copy()
    n = X.shape[0]
    b = n if batch <= 0 or batch > n else batch
    steps = -(-n // b) * epochs
    hist = np.zeros(max(epochs, 0))
    slog = np.zeros((steps, 3), dtype=np.int32)
    d1 = np.zeros((b, h)) if first_step_detail else None
    bp = np.zeros((b, h)) if first_step_detail else None
    _load().ora_train_lowp(n, d, h, k, int(batch), _p(X), _p(T), _p(q.W1), _p(q.b1), _p(q.W2),
                           _p(q.b2), float(lr), int(epochs), PREC[prec], _p(hist), slog.ctypes.data,
                           _p(d1) if first_step_detail else None, _p(bp) if first_step_detail else None)
    if first_step_detail:
        return q, hist, slog, d1, bp
    return q, hist, slog


def round_array(values, prec: str, scale_exp: int = 0) -> np.ndarray:
    """Operand rounding of the reduced-precision forms (e4m3: q(v 2^e) 2^-e)."""
    v = _d(values).ravel()
    out = np.empty_like(v)
    _load().ora_round_array(PREC[prec], int(scale_exp), _p(v), _p(out), v.size)
    return out.reshape(np.shape(values))


# ---------------------------------------------------------------- variants (tanh hidden, momentum)
ACT = {"sigmoid": 0, "tanh": 1}


def train_var(X, T, p: Params, lr: float, epochs: int, batch: int = 0, act: str = "sigmoid", mu: float = 0.0,
              velocity=None):
    """Training with the hidden activation `act` ("sigmoid": the paper's,
    "tanh") and heavy-ball momentum mu (0: the paper's plain descent).
    Returns (trained Params, loss_hist [epochs], velocity [P] or None); the
    velocity starts from `velocity` (packed, default zeros) when mu != 0."""
    X, T = _d(X), _d(T)
    d, h, k = p.shape
    q = p.copy()
    hist = np.zeros(max(epochs, 0))
    v = None
    if mu != 0.0:
        v = np.zeros(d * h + h + h * k + k) if velocity is None else _d(velocity).copy()
    _load().ora_train_var(X.shape[0], d, h, k, int(batch), ACT[act], float(mu), _p(X), _p(T), _p(q.W1),
                          _p(q.b1), _p(q.W2), _p(q.b2), float(lr), int(epochs), _p(v) if v is not None else None,
                          _p(hist))
    return q, hist, v


def loss_grad_var(X, T, p: Params, act: str = "sigmoid"):
    """(L, gradient Params) with the hidden activation `act`."""
    X, T = _d(X), _d(T)
    d, h, k = p.shape
    g = Params(np.zeros((h, d)), np.zeros(h), np.zeros((k, h)), np.zeros(k))
    L = _load().ora_loss_grad_var(X.shape[0], d, h, k, ACT[act], _p(X), _p(T), _p(p.W1), _p(p.b1), _p(p.W2),
                                  _p(p.b2), _p(g.W1), _p(g.b1), _p(g.W2), _p(g.b2))
    return float(L), g


# ---------------------------------------------------------------- deeper nets
def deep_n_params(widths) -> int:
    return int(sum(widths[l + 1] * widths[l] + widths[l + 1] for l in range(len(widths) - 1)))


def deep_loss_grad(X, T, widths, theta, act: str = "sigmoid"):
    """(L, gradient [P]) of an L-layer network: widths [w0 .. wL], parameters
    packed layer by layer (W_l [w(l+1)][w(l)], then b_l)."""
    X, T, th = _d(X), _d(T), _d(theta)
    w = np.ascontiguousarray(widths, dtype=np.int32)
    g = np.zeros(deep_n_params(widths))
    L = _load().ora_deep_loss_grad(X.shape[0], len(widths) - 1, w.ctypes.data, ACT[act], _p(X), _p(T), _p(th),
                                   _p(g))
    return float(L), g


def deep_train(X, T, widths, theta, lr: float, epochs: int, act: str = "sigmoid"):
    """Full-batch training of an L-layer network; returns (theta, loss_hist)."""
    X, T = _d(X), _d(T)
    th = _d(theta).copy()
    w = np.ascontiguousarray(widths, dtype=np.int32)
    hist = np.zeros(max(epochs, 0))
    _load().ora_deep_train(X.shape[0], len(widths) - 1, w.ctypes.data, ACT[act], _p(X), _p(T), _p(th), float(lr),
                           int(epochs), _p(hist))
    return th, hist

