"""Seeded synthetic workloads for the one-hidden-layer sigmoid MLP trainer.

The paper's clinical table (120 participants x 33 markers, its Supplementary
Table 1, section 2.1) is not available, so every workload here is synthetic
and seeded.  This module is the only code shared by the GPU path and the
oracle: it draws inputs (features, one-hot targets, initial parameters, the
per-net hyper-parameters of the batched workload) and holds none of the
method's arithmetic -- no sigmoid network, no loss, no gradient.

Recipe (the paper states only that the data were normalised and that the
network predicts the HbA1c class, sections 2.2 and 1):
  * Gaussian feature columns j: mu_j ~ U(0,100), sd_j ~ U(1,20), x ~ N(mu_j, sd_j).
  * Binary feature columns: Bernoulli(0.3) (on-medication style flags).
  * Every column z-scored in float64 with the population std (ddof=0); a
    zero-std column is divided by 1; then cast to float32.
  * Targets: a per-dataset random teacher D->8->1 (tanh hidden layer),
    score standardised (ddof=0), HbA1c-like value 6.0 + score, class
    [value >= 5.7] + [value >= 6.5] in {0,1,2}; T is the one-hot code.
  * Initial parameters ~ U(-0.5, 0.5), drawn in the order W1 ([H][D] row
    major), b1, W2 ([K][H]), b2.
  * Seeds: numpy SeedSequence(190807847, spawn_key=(workload, group, role)).
"""
from __future__ import annotations

import dataclasses
import numpy as np

ROOT_SEED = 190807847
ROLE_DATA, ROLE_TEACHER, ROLE_PERM, ROLE_THETA, ROLE_HPARAMS = 0, 1, 2, 3, 4
N_OUT = 3


def rng(workload: int, group: int, role: int) -> np.random.Generator:
    ss = np.random.SeedSequence(ROOT_SEED, spawn_key=(int(workload), int(group), int(role)))
    return np.random.Generator(np.random.PCG64(ss))


def features(n_rows: int, n_gauss: int, n_bin: int, g: np.random.Generator) -> np.ndarray:
    """Raw (un-normalised) float64 feature matrix [n_rows][n_gauss+n_bin]."""
    mu = g.uniform(0.0, 100.0, size=n_gauss)
    sd = g.uniform(1.0, 20.0, size=n_gauss)
    xg = g.standard_normal((n_rows, n_gauss)) * sd + mu
    xb = (g.random((n_rows, n_bin)) < 0.3).astype(np.float64)
    return np.concatenate([xg, xb], axis=1)


def zscore(x: np.ndarray) -> np.ndarray:
    mean = x.mean(axis=0)
    sd = x.std(axis=0)
    sd = np.where(sd == 0.0, 1.0, sd)
    return (x - mean) / sd


def teacher_classes(xz: np.ndarray, g: np.random.Generator) -> np.ndarray:
    d = xz.shape[1]
    a = g.standard_normal((8, d)) / np.sqrt(d)
    b = g.standard_normal(8) / np.sqrt(8.0)
    score = np.tanh(xz @ a.T) @ b
    sd = score.std()
    score = (score - score.mean()) / (sd if sd > 0 else 1.0)
    hba1c = 6.0 + score
    return (hba1c >= 5.7).astype(np.int64) + (hba1c >= 6.5).astype(np.int64)


def one_hot(cls: np.ndarray, k: int = N_OUT) -> np.ndarray:
    t = np.zeros((cls.shape[0], k), dtype=np.float32)
    t[np.arange(cls.shape[0]), cls] = 1.0
    return t


def dataset(workload: int, group: int, n_rows: int, n_gauss: int, n_bin: int):
    """(X float32 [n][D] z-scored, T float32 [n][3] one-hot, classes int64)."""
    x = zscore(features(n_rows, n_gauss, n_bin, rng(workload, group, ROLE_DATA)))
    cls = teacher_classes(x, rng(workload, group, ROLE_TEACHER))
    return np.ascontiguousarray(x, dtype=np.float32), one_hot(cls), cls


@dataclasses.dataclass
class Theta:
    W1: np.ndarray  # [H][D]
    b1: np.ndarray  # [H]
    W2: np.ndarray  # [K][H]
    b2: np.ndarray  # [K]

    def packed(self) -> np.ndarray:
        return np.concatenate([self.W1.ravel(), self.b1, self.W2.ravel(), self.b2]).astype(np.float32)

    @staticmethod
    def unpack(p: np.ndarray, d: int, h: int, k: int) -> "Theta":
        p = np.asarray(p)
        o = 0
        w1 = p[o:o + h * d].reshape(h, d); o += h * d
        b1 = p[o:o + h]; o += h
        w2 = p[o:o + k * h].reshape(k, h); o += k * h
        b2 = p[o:o + k]
        return Theta(w1.copy(), b1.copy(), w2.copy(), b2.copy())

    def copy(self) -> "Theta":
        return Theta(self.W1.copy(), self.b1.copy(), self.W2.copy(), self.b2.copy())


def n_params(d: int, h: int, k: int) -> int:
    return d * h + h + h * k + k


def theta0(d: int, h: int, k: int, g: np.random.Generator, lo: float = -0.5, hi: float = 0.5) -> Theta:
    w1 = g.uniform(lo, hi, size=(h, d))
    b1 = g.uniform(lo, hi, size=h)
    w2 = g.uniform(lo, hi, size=(k, h))
    b2 = g.uniform(lo, hi, size=k)
    f = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return Theta(f(w1), f(b1), f(w2), f(b2))


# --------------------------------------------------------------------------
# The five workloads.  Each returns a plain dict of numpy arrays and sizes.
# --------------------------------------------------------------------------

WORKLOADS = {
    1: dict(name="plain-small N=60 33-10-3 full-batch 1000 epochs", n=60, g=22, b=11, h=10,
            batch=0, epochs=1000, lr=0.1),
    2: dict(name="differentiation N=120 33-16-3 full-batch 5000 epochs", n=120, g=22, b=11, h=16,
            batch=0, epochs=5000, lr=0.1),
    3: dict(name="batched 4096 nets H~U{4..64} N_i in [40,120] 2000 epochs", nets=4096, g=22, b=11,
            epochs=2000),
    4: dict(name="large-N N=1048576 33-256-3 minibatch 4096 20 epochs", n=1 << 20, g=22, b=11, h=256,
            batch=4096, epochs=20, lr=0.1),
    5: dict(name="wide N=4194304 64-1024-3 minibatch 16384 5 epochs", n=1 << 22, g=48, b=16, h=1024,
            batch=16384, epochs=5, lr=0.1),
}


def single(workload: int, n_rows: int | None = None, hidden: int | None = None, theta_group: int = 0):
    """A single-network workload (1, 2, 4 or 5), optionally with fewer rows.

    Rows are generated for the full size and then truncated, so a reduced
    problem is the leading slice of the full one (z-scoring uses all rows).
    """
    c = WORKLOADS[workload]
    n_full = c["n"]
    x, t, cls = dataset(workload, 0, n_full, c["g"], c["b"])
    if n_rows is not None:
        x, t, cls = x[:n_rows].copy(), t[:n_rows].copy(), cls[:n_rows].copy()
    h = hidden if hidden is not None else c["h"]
    th = theta0(x.shape[1], h, N_OUT, rng(workload, theta_group, ROLE_THETA))
    return dict(X=x, T=t, classes=cls, theta=th, D=x.shape[1], H=h, K=N_OUT, lr=c["lr"],
                epochs=c["epochs"], batch=c["batch"], name=c["name"])


def binary_targets(w: dict) -> np.ndarray:
    """The two-class reading of the targets: one output, 1 for the top class
    (HbA1c at or above the paper's 6.5 % threshold: poor glucose control),
    0 otherwise; shape [N][1], float32."""
    return (w["classes"] == 2).astype(np.float32)[:, None].copy()


def train_test_split(w: dict, train_frac: float = 0.75, workload: int = 1, group: int = 0) -> dict:
    """The paper's split of a dataset into training and test rows (75/25):
    a seeded permutation, the first round(train_frac * M) rows train and the
    rest test (60 rows -> 45/15, 120 -> 90/30).  Returns X_tr, T_tr, X_te,
    T_te and the permutation."""
    m = w["X"].shape[0]
    perm = rng(workload, group, ROLE_PERM).permutation(m)
    n_tr = int(round(train_frac * m))
    tr, te = np.sort(perm[:n_tr]), np.sort(perm[n_tr:])
    return dict(X_tr=np.ascontiguousarray(w["X"][tr]), T_tr=np.ascontiguousarray(w["T"][tr]),
                X_te=np.ascontiguousarray(w["X"][te]), T_te=np.ascontiguousarray(w["T"][te]), perm=perm)


def batched(n_nets: int = 4096, seed_workload: int = 3, heldout: bool = False):
    """The batched workload: net i -> group i//5, fold i%5.

    Each group draws its own dataset (M ~ U{50..150} rows, 22 Gaussian + 11
    binary columns), hidden size H ~ U{4..64} and learning rate 10^U(-2,0);
    its rows are split into 5 folds by a seeded permutation and net i trains
    on the four folds other than fold i%5 (so N_i is in [40, 120]).
    Packed layout: X rows of net i at x_off (in rows), T at the same row
    offset, parameters [W1|b1|W2|b2] at p_off (in floats).  With heldout,
    also X_val / T_val / items_val: net i's held-out fold (the rows it does
    not train on), packed the same way, with the same p_off and n_hidden.
    """
    n_groups = (n_nets + 4) // 5
    xs, ts, items, thetas = [], [], [], []
    xv, tv, items_val = [], [], []
    vrow = 0
    row = 0
    poff = 0
    for gi in range(n_groups):
        hp = rng(seed_workload, gi, ROLE_HPARAMS)
        m = int(hp.integers(50, 151))
        h = int(hp.integers(4, 65))
        lr = float(10.0 ** hp.uniform(-2.0, 0.0))
        x, t, _ = dataset(seed_workload, gi, m, 22, 11)
        perm = rng(seed_workload, gi, ROLE_PERM).permutation(m)
        folds = np.array_split(perm, 5)
        for f in range(5):
            i = gi * 5 + f
            if i >= n_nets:
                break
            keep = np.sort(np.concatenate([folds[j] for j in range(5) if j != f]))
            xi, ti = x[keep], t[keep]
            th = theta0(x.shape[1], h, N_OUT, rng(seed_workload, i, ROLE_THETA))
            items.append(dict(n_rows=len(keep), n_hidden=h, lr=np.float32(lr), x_off=row, p_off=poff))
            xs.append(xi); ts.append(ti); thetas.append(th.packed())
            if heldout:
                held = np.sort(folds[f])
                items_val.append(dict(n_rows=len(held), n_hidden=h, lr=np.float32(0.0), x_off=vrow, p_off=poff,
                                      group=gi, fold=f))
                xv.append(x[held]); tv.append(t[held])
                vrow += len(held)
            row += len(keep)
            poff += n_params(x.shape[1], h, N_OUT)
    out = dict(X=np.ascontiguousarray(np.concatenate(xs)), T=np.ascontiguousarray(np.concatenate(ts)),
               theta=np.concatenate(thetas).astype(np.float32), items=items, D=33, K=N_OUT,
               epochs=WORKLOADS[3]["epochs"], name=WORKLOADS[3]["name"])
    if heldout:
        out.update(X_val=np.ascontiguousarray(np.concatenate(xv)), T_val=np.ascontiguousarray(np.concatenate(tv)),
                   items_val=items_val)
    return out


# learning rates of the nets-sharing-X grid: 10^(-2 + 2j/7), j = 0..7
SHARED_LR_GRID = tuple(float(10.0 ** (-2.0 + 2.0 * j / 7.0)) for j in range(8))


def shared(workload: int = 5, n_nets: int = 64, n_rows: int | None = None, hidden: int | None = None,
           base: dict | None = None):
    """Nets that share one dataset (a hyperparameter grid): the rows of a
    single-network workload, and for net i the learning rate
    SHARED_LR_GRID[i % 8] with initial parameters from seed group i // 8
    (so each group of 8 nets starts from the same weights and differs only
    in the learning rate).  theta is [n_nets][P] float32.  `base`: the
    workload's single-network dict when the caller already generated it
    (its rows are reused, not copied)."""
    if base is None:
        base = single(workload, n_rows=n_rows, hidden=hidden)
    d, h, k = base["D"], base["H"], base["K"]
    thetas = [theta0(d, h, k, rng(workload, 100 + i // 8, ROLE_THETA)).packed() for i in range(n_nets)]
    lrs = [SHARED_LR_GRID[i % 8] for i in range(n_nets)]
    return dict(X=base["X"], T=base["T"], theta=np.stack(thetas).astype(np.float32), lrs=lrs, D=d, H=h, K=k,
                batch=base["batch"], epochs=base["epochs"], name=base["name"] + f", {n_nets} nets sharing X")
