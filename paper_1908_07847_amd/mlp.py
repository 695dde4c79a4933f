"""PyTorch-facing wrapper of libmlp.

PyTorch provides device memory and the stream; the arithmetic of every
step -- forward, error, backpropagation, update -- runs in libmlp's HIP
kernels (arxiv 1908.07847, section 2.2).  Nothing here computes on the
host beyond argument marshalling.
"""
from __future__ import annotations

import ctypes
import weakref
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import BatchItem, Config, LaunchHint, Params, check, lib


def _ptr(t: torch.Tensor | None) -> int | None:
    if t is None:
        return None
    return t.data_ptr()


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def n_params(d: int, h: int, k: int) -> int:
    return d * h + h + h * k + k


def split_packed(flat: torch.Tensor, d: int, h: int, k: int):
    """Views W1 [H][D], b1 [H], W2 [K][H], b2 [K] of a packed [P] tensor."""
    o = 0
    W1 = flat[o:o + h * d].view(h, d); o += h * d
    b1 = flat[o:o + h]; o += h
    W2 = flat[o:o + k * h].view(k, h); o += k * h
    b2 = flat[o:o + k]
    return W1, b1, W2, b2


def _aligned_empty(n: int, device) -> torch.Tensor:
    # torch's caching allocator returns 256-byte aligned blocks; keep sizes >= 1
    return torch.empty(max(n, 4), dtype=torch.float32, device=device)[:n]


@dataclass
class Grads:
    W1: torch.Tensor
    b1: torch.Tensor
    W2: torch.Tensor
    b2: torch.Tensor
    flat: torch.Tensor

    def c(self) -> Params:
        return Params(self.W1.data_ptr(), self.b1.data_ptr(), self.W2.data_ptr(), self.b2.data_ptr())


class Net:
    """One network bound to device parameters, a compensation buffer and a workspace.

    The four parameter tensors are views of one packed float32 buffer
    (`self.flat`, order [W1 | b1 | W2 | b2]).
    """

    def __init__(self, n_in: int, n_hidden: int, n_out: int, n_rows: int, *, batch: int = 0,
                 lr: float = 0.1, prec: str = "fp32", compensated: bool = True, theta=None,
                 act: str = "sigmoid", momentum: float = 0.0, check_finite: bool = False, device="cuda"):
        """act: the hidden activation, "sigmoid" (the paper's) or "tanh";
        momentum: heavy-ball rate mu (0, the paper's plain descent), with a
        zeroed velocity buffer `self.velocity` owned by the net;
        check_finite: MLP_F_CHECK_FINITE (status() reports NaN/Inf after
        training)."""
        self.D, self.H, self.K = int(n_in), int(n_hidden), int(n_out)
        self.n_rows, self.batch, self.lr, self.prec = int(n_rows), int(batch), float(lr), prec
        self.device = torch.device(device)
        P = n_params(self.D, self.H, self.K)
        self.flat = _aligned_empty(P, self.device)
        if theta is not None:
            self.flat.copy_(torch.as_tensor(np.asarray(theta_packed(theta), dtype=np.float32)))
        else:
            self.flat.zero_()
        self.W1, self.b1, self.W2, self.b2 = split_packed(self.flat, self.D, self.H, self.K)
        self.comp = torch.zeros(max(P, 4), dtype=torch.float32, device=self.device)[:P] if compensated else None
        if act not in ("sigmoid", "tanh"):
            raise ValueError(f"unknown hidden activation {act!r}")
        self.act = act
        flags = (_lib.MLP_F_COMPENSATED if compensated else 0) | (_lib.F_TANH_HIDDEN if act == "tanh" else 0) | \
            (_lib.F_CHECK_FINITE if check_finite else 0)
        self.cfg = Config(self.D, self.H, self.K, _lib.PREC[prec], self.n_rows, self.batch, self.lr, flags)
        nbytes = ctypes.c_size_t(0)
        check(lib.mlp_workspace_size(ctypes.byref(self.cfg), ctypes.byref(nbytes)))
        self.ws_bytes = int(nbytes.value)
        self.ws = torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        check(lib.mlp_init(ctypes.byref(h), ctypes.byref(self.cfg), self.params_c(), _ptr(self.comp),
                           _ptr(self.ws), self.ws_bytes))
        self._h = h
        # the handle is released by a finalizer that holds its own reference
        # to mlp_destroy, so it runs (once) at collection or at interpreter
        # exit, before module globals are torn down
        self._finalizer = weakref.finalize(self, lib.mlp_destroy, h)
        self.velocity = None
        if momentum:
            self.set_momentum(momentum)

    def set_momentum(self, mu: float, velocity: torch.Tensor | None = None) -> None:
        """mlp_set_momentum: heavy-ball momentum mu for mlp_step / mlp_train
        (0 turns it off).  The velocity starts at zero unless given."""
        if mu > 0:
            P = self.flat.numel()
            self.velocity = velocity if velocity is not None else torch.zeros(max(P, 4), dtype=torch.float32,
                                                                                device=self.device)[:P]
        else:
            self.velocity = None
        check(lib.mlp_set_momentum(self._h, float(mu), _ptr(self.velocity)))

    def close(self) -> None:
        """Release the library handle now (host memory only); idempotent."""
        fin = getattr(self, "_finalizer", None)
        if fin is not None:
            fin()

    def params_c(self) -> Params:
        return Params(self.W1.data_ptr(), self.b1.data_ptr(), self.W2.data_ptr(), self.b2.data_ptr())

    def set_theta(self, theta) -> None:
        self.flat.copy_(torch.as_tensor(np.asarray(theta_packed(theta), dtype=np.float32)))
        if self.comp is not None:
            self.comp.zero_()

    def new_grads(self) -> Grads:
        flat = _aligned_empty(self.flat.numel(), self.device)
        W1, b1, W2, b2 = split_packed(flat, self.D, self.H, self.K)
        return Grads(W1, b1, W2, b2, flat)

    # ---------------------------------------------------------------- steps
    def forward(self, X: torch.Tensor, want_hidden: bool = True, stream=None):
        n = X.shape[0]
        A = torch.empty((n, self.H), dtype=torch.float32, device=self.device) if want_hidden else None
        Y = torch.empty((n, self.K), dtype=torch.float32, device=self.device)
        check(lib.mlp_forward(self._h, _ptr(X), n, _ptr(A), _ptr(Y), _stream(stream)))
        return A, Y

    def backward(self, X, A, Y, dY=None, T=None, want_dx=False, grads: Grads | None = None, stream=None):
        n = X.shape[0]
        g = grads if grads is not None else self.new_grads()
        dX = torch.empty((n, self.D), dtype=torch.float32, device=self.device) if want_dx else None
        loss = torch.empty(4, dtype=torch.float32, device=self.device)[:1] if dY is None else None
        check(lib.mlp_backward(self._h, _ptr(X), _ptr(A), _ptr(Y), _ptr(dY), _ptr(T), n, g.c(), _ptr(dX),
                               _ptr(loss), _stream(stream)))
        return g, dX, loss

    def step(self, grads: Grads, lr: float | None = None, stream=None) -> None:
        check(lib.mlp_step(self._h, grads.c(), float(self.lr if lr is None else lr), _stream(stream)))

    def predict(self, X: torch.Tensor, T: torch.Tensor | None = None, stream=None):
        """(Y [n][K], labels [n] int32, number correct or None) -- mlp_predict."""
        n = X.shape[0]
        Y = torch.empty((n, self.K), dtype=torch.float32, device=self.device)
        labels = torch.empty(max(n, 4), dtype=torch.int32, device=self.device)[:n]
        correct = torch.empty(4, dtype=torch.int32, device=self.device)[:1] if T is not None else None
        check(lib.mlp_predict(self._h, _ptr(X), n, _ptr(Y), _ptr(labels), _ptr(T), _ptr(correct),
                              _stream(stream)))
        return Y, labels, correct

    def train(self, X: torch.Tensor, T: torch.Tensor, epochs: int, record_loss: bool = True,
              loss_hist: torch.Tensor | None = None, stream=None):
        if record_loss and loss_hist is None:
            loss_hist = torch.empty(max(epochs, 4), dtype=torch.float32, device=self.device)[:epochs]
        check(lib.mlp_train(self._h, _ptr(X), _ptr(T), int(epochs), _ptr(loss_hist) if record_loss else None,
                            _stream(stream)))
        return loss_hist


    def status(self, stream=None) -> int:
        """mlp_query_status: waits for the stream and returns the status of
        the last training launch (MLP_OK, MLP_ERR_TIMEOUT or
        MLP_ERR_NONFINITE) without raising."""
        return int(lib.mlp_query_status(self._h, _stream(stream)))


def workspace_status(workspace: torch.Tensor, stream=None) -> int:
    """mlp_workspace_status of a training workspace (mlp_train_shared)."""
    return int(lib.mlp_workspace_status(_ptr(workspace), int(workspace.numel() * workspace.element_size()),
                                        _stream(stream)))


def mfma_probe(prec: str, A: torch.Tensor, B: torch.Tensor, stream=None) -> torch.Tensor:
    """mlp_mfma_probe: C = A B^T on the trainer's matrix-core instruction for
    operand precision `prec` (A [M][Kd], B [N][Kd] float32 on the device)."""
    M, Kd = A.shape
    N = B.shape[0]
    C = torch.empty((M, N), dtype=torch.float32, device=A.device)
    check(lib.mlp_mfma_probe(_lib.PREC[prec], _ptr(A), _ptr(B), _ptr(C), int(M), int(N), int(Kd), _stream(stream)))
    return C


def set_wait_limit(microseconds: int) -> None:
    """mlp_set_wait_limit: longest grid-barrier wait (negative: the default)."""
    check(lib.mlp_set_wait_limit(int(microseconds)))


class NetEpochs:
    """Full-batch epochs of a one-hidden-layer Net as library calls only:
    per epoch mlp_forward (hidden activations and outputs into fixed
    buffers), mlp_backward with the mean-squared-error reading (dY = NULL,
    the loss written to a device slot) and mlp_step.  `graph(epochs)`
    captures that many epochs in a HIP graph (torch.cuda.CUDAGraph) whose
    replays train the net in place, with no host work between the kernels
    and no torch operation inside the capture."""

    def __init__(self, net: "Net", X: torch.Tensor, T: torch.Tensor):
        self.net, self.X, self.T = net, X, T
        n = X.shape[0]
        self.A = torch.empty((n, net.H), dtype=torch.float32, device=net.device)
        self.Y = torch.empty((n, net.K), dtype=torch.float32, device=net.device)
        self.grads = net.new_grads()
        self.loss = None
        self.cuda_graph = None

    def run(self, epochs: int, loss_hist: torch.Tensor, stream=None) -> None:
        """`epochs` epochs now (eagerly); loss_hist[e] gets epoch e's loss."""
        net, n, st = self.net, self.X.shape[0], _stream(stream)
        for e in range(epochs):
            check(lib.mlp_forward(net._h, _ptr(self.X), n, _ptr(self.A), _ptr(self.Y), st))
            check(lib.mlp_backward(net._h, _ptr(self.X), _ptr(self.A), _ptr(self.Y), None, _ptr(self.T), n,
                                   self.grads.c(), None, loss_hist[e:e + 1].data_ptr(), st))
            check(lib.mlp_step(net._h, self.grads.c(), float(net.lr), st))

    def graph(self, epochs: int) -> "NetEpochs":
        """Capture `epochs` epochs (after one eager epoch that loads every
        kernel; the parameters are restored); `replay()` runs them."""
        if epochs <= 0:
            raise ValueError("epochs must be positive")
        net = self.net
        self.loss = torch.empty(max(epochs, 4), dtype=torch.float32, device=net.device)[:epochs]
        flat0 = net.flat.detach().clone()
        comp0 = net.comp.clone() if net.comp is not None else None
        self.run(1, self.loss)
        torch.cuda.synchronize()
        net.flat.detach().copy_(flat0)
        if comp0 is not None:
            net.comp.copy_(comp0)
        torch.cuda.synchronize()
        self.cuda_graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.cuda_graph, capture_error_mode="thread_local"):
            self.run(epochs, self.loss)
        return self

    def replay(self) -> None:
        self.cuda_graph.replay()


def theta_packed(theta) -> np.ndarray:
    if hasattr(theta, "packed"):
        return theta.packed()
    return np.asarray(theta, dtype=np.float32)


# ---------------------------------------------------------------- batched
class BatchPlan:
    """Host and device copies of the item table for mlp_train_batched.

    `order` lists the nets in launch order: longest first (by N_i * H_i), a
    greedy longest-processing-time schedule over the hardware's workgroup
    dispatcher.  Results are indexed by the caller's net index regardless of
    the order.

    With `buckets=True` the nets are grouped by size -- hidden units in
    16-unit tiles (up to 16, 32 or 64 units) and rows up to 64 or 128 --
    and each group is one launch (largest group cost first, longest first
    inside a group): a launch reserves LDS and registers for its largest
    net, so grouping lets the many smaller nets run more workgroups per CU.
    `groups` lists (start, count, max_rows, max_hidden) in plan order, and
    `threads[g]` (0: the library's choice) is the launch shape of group g,
    set by the autotuner (tune.tune_batched).  `stream_of[g]` is the side
    stream group g is launched on (groups on one stream run one after the
    other): group g on stream g mod 4 unless the autotuner moved it, as it
    does with the groups after the fourth, which wait for the group they
    follow.
    """

    def __init__(self, items, device="cuda", order: str = "lpt", buckets: bool = False):
        n = len(items)
        cost = np.array([it["n_rows"] * it["n_hidden"] for it in items], dtype=np.int64)
        if isinstance(order, str) and order == "lpt":
            lpt = np.argsort(-cost, kind="stable")
            if buckets:
                key = np.array([((it["n_hidden"] + 15) // 16 + 1) // 2 * 2 if it["n_hidden"] > 16 else 1
                                for it in items]) * 2 + np.array([it["n_rows"] > 64 for it in items])
                groups = {}
                for i in lpt:
                    groups.setdefault(int(key[i]), []).append(int(i))
                members = sorted(groups.values(), key=lambda g: -int(cost[g].sum()))
                self.order = np.array([i for g in members for i in g], dtype=np.int64)
                sizes = [len(g) for g in members]
            else:
                self.order = lpt
                sizes = [n]
        elif isinstance(order, str) and order == "given":
            self.order = np.arange(n)
            sizes = [n]
        else:
            self.order = np.asarray(order)
            sizes = [n]
        arr = (BatchItem * n)()
        for pos, i in enumerate(self.order):
            it = items[int(i)]
            arr[pos] = BatchItem(int(it["n_rows"]), int(it["n_hidden"]), float(it["lr"]), 0, int(it["x_off"]),
                                 int(it["p_off"]))
        self.host = arr
        self.n = n
        raw = np.frombuffer(bytes(arr), dtype=np.uint8).copy()
        self.dev = torch.from_numpy(raw).to(device)
        self.max_rows = int(max(it["n_rows"] for it in items))
        self.max_hidden = int(max(it["n_hidden"] for it in items))
        self.groups = []
        self.side_streams = []
        start = 0
        for c in sizes:
            sel = [items[int(i)] for i in self.order[start:start + c]]
            self.groups.append((start, c, int(max(it["n_rows"] for it in sel)),
                                int(max(it["n_hidden"] for it in sel))))
            start += c
        self.threads = [0] * len(self.groups)
        self.stream_of = [g % 4 for g in range(len(self.groups))]
        if len(self.groups) > 1:
            self.side_streams = [torch.cuda.Stream(device=device) for _ in range(min(len(self.groups), 4))]

    def host_at(self, start: int):
        """Pointer to the host item table from position `start`."""
        return ctypes.cast(ctypes.addressof(self.host) + start * ctypes.sizeof(BatchItem), ctypes.POINTER(BatchItem))


def train_batched(plan: BatchPlan, X: torch.Tensor, T: torch.Tensor, theta: torch.Tensor,
                  comp: torch.Tensor | None, epochs: int, n_in: int, n_out: int,
                  loss_hist: torch.Tensor | None = None, stream=None, groups=None):
    """Train every net of the plan, one launch per group of the plan (one
    launch without buckets); loss_hist rows follow the plan order.  `groups`
    (indices) restricts the call to some groups.  Several groups run
    concurrently on the plan's side streams (plan.side_streams, default
    priority), forked from and joined back into the calling stream, so one
    group's last workgroups overlap the next group's."""
    cur = stream if stream is not None else torch.cuda.current_stream()
    item_bytes = ctypes.sizeof(BatchItem)
    todo = [g for g in range(len(plan.groups)) if groups is None or g in groups]
    side = plan.side_streams if len(todo) > 1 else []
    for s_ in side:
        s_.wait_stream(cur)
    for j, g in enumerate(todo):
        start, count, _, _ = plan.groups[g]
        threads = plan.threads[g]
        st = side[plan.stream_of[g] % len(side)] if side else cur
        if threads:
            set_launch_hint(small_threads=threads)
        try:
            lh = None if loss_hist is None else loss_hist.data_ptr() + start * int(epochs) * 4
            check(lib.mlp_train_batched(plan.host_at(start), plan.dev.data_ptr() + start * item_bytes, count, n_in,
                                        n_out, _ptr(X), _ptr(T), X.shape[0], _ptr(theta), _ptr(comp),
                                        theta.numel(), int(epochs), lh, st.cuda_stream))
        finally:
            if threads:
                reset_launch_hint()
    for s_ in side:
        cur.wait_stream(s_)
    return loss_hist


class BatchedGraph:
    """mlp_train_batched captured once in a HIP graph (torch.cuda.CUDAGraph):
    every replay trains all nets of the plan for `epochs` more epochs, in
    place, with one graph launch.  The captured work is the trainer kernel
    of each group of the plan (no memset or copy nodes).  Buffers must stay alive and in place
    for the graph's lifetime."""

    def __init__(self, plan: BatchPlan, X, T, theta, comp, epochs: int, n_in: int, n_out: int,
                 loss_hist=None):
        self.tensors = (X, T, theta, comp, loss_hist)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):   # first launch outside capture (kernel attributes)
            train_batched(plan, X, T, theta.clone(), None if comp is None else comp.clone(), 1, n_in, n_out)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph, capture_error_mode="thread_local"):
            train_batched(plan, X, T, theta, comp, epochs, n_in, n_out, loss_hist=loss_hist)

    def replay(self) -> None:
        self.graph.replay()


def eval_batched(plan: BatchPlan, X: torch.Tensor, T: torch.Tensor, theta: torch.Tensor, n_in: int, n_out: int,
                 stream=None):
    """mlp_eval_batched: (loss [n], correct [n] int32), indexed by the
    caller's net index (the plan's order is undone)."""
    n = plan.n
    loss = torch.empty(max(n, 4), dtype=torch.float32, device=X.device)[:n]
    correct = torch.empty(max(n, 4), dtype=torch.int32, device=X.device)[:n]
    check(lib.mlp_eval_batched(plan.host, _ptr(plan.dev), n, int(n_in), int(n_out), _ptr(X), _ptr(T), X.shape[0],
                               _ptr(theta), theta.numel(), _ptr(loss), _ptr(correct), _stream(stream)))
    inv = torch.as_tensor(np.argsort(plan.order), device=X.device)
    return loss[inv], correct[inv]


def cv_select(loss: torch.Tensor, group: torch.Tensor, n_groups: int, stream=None):
    """mlp_cv_select: (group_mean [n_groups], best [1] int32), both on the
    device -- the mean held-out loss of every group of nets and the group
    with the lowest one (ties to the lower index)."""
    if loss.dtype != torch.float32 or group.dtype != torch.int32 or not loss.is_contiguous() or \
            not group.is_contiguous() or loss.numel() != group.numel():
        raise ValueError("loss (float32) and group (int32) must be contiguous and of one length")
    mean = torch.empty(max(int(n_groups), 4), dtype=torch.float32, device=loss.device)[:int(n_groups)]
    best = torch.empty(4, dtype=torch.int32, device=loss.device)[:1]
    check(lib.mlp_cv_select(_ptr(loss), _ptr(group), loss.numel(), int(n_groups), _ptr(mean), _ptr(best),
                            _stream(stream)))
    return mean, best


# ---------------------------------------------------------------- nets sharing one dataset
def shared_workspace_size(n_in: int, n_hidden: int, n_out: int, n_rows: int, batch: int, n_nets: int,
                          prec: str = "fp32") -> int:
    cfg = Config(n_in, n_hidden, n_out, _lib.PREC[prec], n_rows, batch, 0.1, 0)
    nbytes = ctypes.c_size_t(0)
    check(lib.mlp_shared_workspace_size(ctypes.byref(cfg), int(n_nets), ctypes.byref(nbytes)))
    return int(nbytes.value)


def train_shared(X: torch.Tensor, T: torch.Tensor, theta: torch.Tensor, lrs, epochs: int, n_hidden: int, *,
                 batch: int, prec: str = "fp32", comp: torch.Tensor | None = None,
                 loss_hist: torch.Tensor | None = None, workspace: torch.Tensor | None = None, stream=None,
                 check_finite: bool = False):
    """mlp_train_shared: theta [n_nets][P] (float32, packed per net) trains in
    place on the shared X [N][D], T [N][K]; lrs holds one learning rate per
    net; comp (same shape as theta, or None) selects the compensated update.
    Returns loss_hist [n_nets][epochs] if given (else None)."""
    M = int(theta.shape[0])
    N, D = X.shape
    K = T.shape[1]
    cfg = Config(int(D), int(n_hidden), int(K), _lib.PREC[prec], int(N), int(batch), float(lrs[0]),
                 (_lib.MLP_F_COMPENSATED if comp is not None else 0) | (_lib.F_CHECK_FINITE if check_finite else 0))
    nbytes = ctypes.c_size_t(0)
    check(lib.mlp_shared_workspace_size(ctypes.byref(cfg), M, ctypes.byref(nbytes)))
    ws = workspace if workspace is not None else torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8,
                                                             device=X.device)
    lr_arr = (ctypes.c_float * M)(*[float(v) for v in lrs])
    check(lib.mlp_train_shared(ctypes.byref(cfg), M, lr_arr, _ptr(X), _ptr(T), _ptr(theta), _ptr(comp),
                               int(epochs), _ptr(loss_hist), _ptr(ws), int(ws.numel()), _stream(stream)))
    return loss_hist


def large_plan(n_in: int, n_hidden: int, n_out: int, n_rows: int, *, batch: int = 0, prec: str = "fp32",
               n_nets: int = 1, n_cu: int | None = None) -> dict:
    """The launch shape of the large-N trainer for this shape (host-side
    query, no device call unless n_cu is None): row blocks, hidden blocks,
    waves per workgroup, rows staged per piece, hidden tiles per wave, and
    the name of the kernel instance it launches."""
    if n_cu is None:
        n_cu = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
    cfg = Config(int(n_in), int(n_hidden), int(n_out), _lib.PREC[prec], int(n_rows), int(batch), 0.1, 0)
    out = (ctypes.c_int32 * 5)()
    check(lib.mlp_large_plan(ctypes.byref(cfg), int(n_nets), int(n_cu), out))
    pi = {"fp32": 0, "bf16": 1, "e4m3": 2}[prec]
    return {"row_blocks": out[0], "hidden_blocks": out[1], "waves": out[2], "piece_rows": out[3],
            "tiles_per_wave": out[4],
            "kernel": f"mlpk::k_large_train<{pi}, {3 if n_out <= 3 else 4}, {out[2]}, {out[4]}>"}


def set_launch_hint(small_threads: int = 0, large_grid: tuple[int, int] | None = None, large_waves: int = 0) -> None:
    """Launch-shape override for the autotuner (0 / None: the library's choice)."""
    gi, gj = large_grid if large_grid else (0, 0)
    h = LaunchHint(int(small_threads), int(gi), int(gj), int(large_waves))
    check(lib.mlp_set_launch_hint(ctypes.byref(h)))


def reset_launch_hint() -> None:
    check(lib.mlp_set_launch_hint(None))


# ---------------------------------------------------------------- autograd
class MLPFunction(torch.autograd.Function):
    """Y = sigma(sigma(X W1^T + b1) W2^T + b2) with the hand-written adjoint.

    Usage:  Y = MLPFunction.apply(net, X, net.W1, net.b1, net.W2, net.b2)
    The parameters must be the net's own tensors (the kernels read them from
    the handle); they are passed so autograd can route their gradients.
    """

    @staticmethod
    def forward(ctx, net: Net, X, W1, b1, W2, b2):
        A, Y = net.forward(X)
        ctx.net = net
        ctx.save_for_backward(X, A, Y)
        return Y

    @staticmethod
    def backward(ctx, gY):
        X, A, Y = ctx.saved_tensors
        net: Net = ctx.net
        g, dX, _ = net.backward(X, A, Y, dY=gY.contiguous(), want_dx=ctx.needs_input_grad[1])
        return None, dX, g.W1, g.b1, g.W2, g.b2


# ---------------------------------------------------------------- accuracy during training
def accuracy_curve(net: Net, X_tr: torch.Tensor, T_tr: torch.Tensor, X_te: torch.Tensor | None,
                   T_te: torch.Tensor | None, epochs: int, every: int) -> dict:
    """Train `net` for `epochs` epochs on X_tr, T_tr in launches of `every`
    epochs (a resumed run equals one long run bitwise) and after each launch
    count the correct class predictions (mlp_predict) on the training rows
    and, if given, the test rows.  Returns numpy arrays: epochs done, loss
    history [epochs], train_correct, test_correct (or None)."""
    if every <= 0 or epochs < 0:
        raise ValueError("every must be positive and epochs >= 0")
    hist = torch.empty(max(epochs, 1), dtype=torch.float32, device=net.device)
    done, tr, te = [], [], []
    e = 0
    while e < epochs:
        k = min(every, epochs - e)
        net.train(X_tr, T_tr, k, loss_hist=hist[e:e + k])
        e += k
        done.append(e)
        tr.append(net.predict(X_tr, T_tr)[2])
        if X_te is not None:
            te.append(net.predict(X_te, T_te)[2])
    return dict(epochs=np.array(done), loss=hist[:epochs].cpu().numpy(),
                train_correct=np.array([int(v) for v in tr]),
                test_correct=np.array([int(v) for v in te]) if X_te is not None else None)


# ---------------------------------------------------------------- measurement
def barrier_probe(n_workgroups: int, rounds: int, workspace: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """mlp_barrier_probe: one cooperative launch whose workgroups pass
    `rounds` grid barriers; returns the workspace (its int32 word 16 is
    nonzero if a barrier hit its spin limit)."""
    ws = workspace if workspace is not None else torch.zeros(_lib.BARRIER_PROBE_WS_BYTES // 4, dtype=torch.int32,
                                                              device="cuda")
    check(lib.mlp_barrier_probe(int(n_workgroups), int(rounds), _ptr(ws), ws.numel() * ws.element_size(),
                                _stream(stream)))
    return ws


def barrier_latency_us(n_workgroups: int, rounds: int = 2000) -> float:
    """Time one grid barrier adds (µs): launches of `rounds` and 2 x `rounds`
    barriers timed with HIP events on the current stream, differenced."""
    ws = torch.zeros(_lib.BARRIER_PROBE_WS_BYTES // 4, dtype=torch.int32, device="cuda")
    barrier_probe(n_workgroups, 10, ws)
    times = []
    for r in (rounds, 2 * rounds):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        barrier_probe(n_workgroups, r, ws)
        e1.record()
        torch.cuda.synchronize()
        if int(ws[16].item()) != 0:
            raise RuntimeError("a probe barrier hit its spin limit")
        times.append(e0.elapsed_time(e1) * 1e3)
    return (times[1] - times[0]) / rounds



# ---------------------------------------------------------------- networks with several hidden layers
class DenseFunction(torch.autograd.Function):
    """Y = act(X W^T + b) (mlp_dense_forward, act 0 sigmoid / 1 tanh) with the
    hand-written adjoint (mlp_dense_backward).  When gradient buffers are
    given, the parameter gradients are written into them (views of a packed
    gradient vector) and returned as they are."""

    @staticmethod
    def forward(ctx, X, W, b, act: int, gW_buf=None, gb_buf=None):
        X = X.contiguous()
        n, din = X.shape
        dout = W.shape[0]
        Y = torch.empty((n, dout), dtype=torch.float32, device=X.device)
        check(lib.mlp_dense_forward(_ptr(X), n, din, dout, _ptr(W), _ptr(b), int(act), _ptr(Y), _stream()))
        ctx.save_for_backward(X, W, Y)
        ctx.act, ctx.bufs = int(act), (gW_buf, gb_buf)
        return Y

    @staticmethod
    def backward(ctx, gY):
        X, W, Y = ctx.saved_tensors
        gY = gY.contiguous()
        n, din = X.shape
        dout = W.shape[0]
        gW = ctx.bufs[0] if ctx.bufs[0] is not None else torch.empty_like(W)
        gb = ctx.bufs[1] if ctx.bufs[1] is not None else torch.empty(dout, dtype=torch.float32, device=X.device)
        dX = torch.empty_like(X) if ctx.needs_input_grad[0] else None
        ws = torch.empty(max(n * dout, 4), dtype=torch.float32, device=X.device)
        check(lib.mlp_dense_backward(_ptr(X), _ptr(Y), _ptr(gY), n, din, dout, _ptr(W), ctx.act, _ptr(gW), _ptr(gb),
                                     _ptr(dX), _ptr(ws), ws.numel() * 4, _stream()))
        return dX, gW, gb, None, None, None


def deep_n_params(widths) -> int:
    return int(sum(widths[l + 1] * widths[l] + widths[l + 1] for l in range(len(widths) - 1)))


class DeepNet:
    """A network with several hidden layers (section 2.2's network stacked):
    widths [D, h1, ..., K]; hidden layers apply `act` ("sigmoid" or "tanh"),
    the output layer the sigmoid; parameters packed layer by layer (W_l
    [w(l+1)][w(l)], then b_l) in `flat`.  Trained full batch through
    DenseFunction and torch.autograd (torch's mean squared error), the
    gradients landing in the packed `grad`, and mlp_update."""

    def __init__(self, widths, theta=None, act: str = "sigmoid", lr: float = 0.1, compensated: bool = True,
                 device="cuda"):
        if len(widths) < 2 or act not in ("sigmoid", "tanh"):
            raise ValueError("widths needs at least an input and an output width; act sigmoid or tanh")
        self.widths, self.act, self.lr = [int(v) for v in widths], act, float(lr)
        self.device = torch.device(device)
        P = deep_n_params(self.widths)
        self.flat = _aligned_empty(P, self.device)
        if theta is not None:
            self.flat.copy_(torch.as_tensor(np.asarray(theta, dtype=np.float32)))
        else:
            self.flat.zero_()
        self.grad = _aligned_empty(P, self.device)
        self.comp = torch.zeros(max(P, 4), dtype=torch.float32, device=self.device)[:P] if compensated else None
        self.layers, self.grads = [], []
        o = 0
        for l in range(len(self.widths) - 1):
            din, dout = self.widths[l], self.widths[l + 1]
            W, gW = self.flat[o:o + dout * din].view(dout, din), self.grad[o:o + dout * din].view(dout, din)
            o += dout * din
            b, gb = self.flat[o:o + dout], self.grad[o:o + dout]
            o += dout
            W.requires_grad_(True)
            b.requires_grad_(True)
            self.layers.append((W, b))
            self.grads.append((gW, gb))
        self.params = [t for wb in self.layers for t in wb]

    def forward(self, X: torch.Tensor) -> torch.Tensor:
        a = X
        L = len(self.layers)
        for l, ((W, b), (gW, gb)) in enumerate(zip(self.layers, self.grads)):
            act = 1 if (self.act == "tanh" and l < L - 1) else 0
            a = DenseFunction.apply(a, W, b, act, gW, gb)
        return a

    # ---- the same epoch through the C ABI alone (no autograd): forward layer by
    # layer, the squared-error gradient, backward layer by layer, the update
    def _fused_buffers(self, n: int):
        if getattr(self, "_fb_n", None) != n:
            dev, w = self.device, self.widths
            self._acts = [torch.empty((n, w[l + 1]), dtype=torch.float32, device=dev) for l in range(len(w) - 1)]
            self._dacts = [torch.empty((n, w[l + 1]), dtype=torch.float32, device=dev) for l in range(len(w) - 1)]
            self._dz = torch.empty(max(n * max(w[1:]), 4), dtype=torch.float32, device=dev)
            self._fb_n = n
        return self._acts, self._dacts, self._dz

    def epoch_fused(self, X: torch.Tensor, T: torch.Tensor, loss_out: torch.Tensor, stream=None) -> None:
        """One full-batch epoch (section 2.2's loop over L layers) as library
        calls on the stream; the epoch's loss lands in loss_out[0]."""
        n, w, L = X.shape[0], self.widths, len(self.layers)
        acts, dacts, dz = self._fused_buffers(n)
        s = _stream(stream)
        a = X
        for l, (W, b) in enumerate(self.layers):
            act = 1 if (self.act == "tanh" and l < L - 1) else 0
            check(lib.mlp_dense_forward(_ptr(a), n, w[l], w[l + 1], _ptr(W), _ptr(b), act, _ptr(acts[l]), s))
            a = acts[l]
        check(lib.mlp_mse_grad(_ptr(acts[-1]), _ptr(T), n, w[-1], _ptr(dacts[-1]), _ptr(loss_out), s))
        for l in range(L - 1, -1, -1):
            W, _ = self.layers[l]
            gW, gb = self.grads[l]
            act = 1 if (self.act == "tanh" and l < L - 1) else 0
            xin = X if l == 0 else acts[l - 1]
            check(lib.mlp_dense_backward(_ptr(xin), _ptr(acts[l]), _ptr(dacts[l]), n, w[l], w[l + 1], _ptr(W), act,
                                         _ptr(gW), _ptr(gb), _ptr(dacts[l - 1]) if l > 0 else None, _ptr(dz),
                                         dz.numel() * 4, s))
        check(lib.mlp_update(_ptr(self.flat), _ptr(self.grad), _ptr(self.comp), self.flat.numel(), self.lr, s))

    def train_fused(self, X: torch.Tensor, T: torch.Tensor, epochs: int, loss_hist: torch.Tensor | None = None):
        hist = loss_hist if loss_hist is not None else torch.empty(max(epochs, 1), dtype=torch.float32,
                                                                     device=self.device)
        for e in range(epochs):
            self.epoch_fused(X, T, hist[e:e + 1])
        return hist[:epochs]

    def train_kernel(self, X: torch.Tensor, T: torch.Tensor, epochs: int, loss_hist: torch.Tensor | None = None,
                     stream=None):
        """`epochs` full-batch epochs in one launch (mlp_deep_train: the net
        resident in one workgroup's LDS); the loss of each epoch in the
        returned [epochs] tensor."""
        hist = loss_hist if loss_hist is not None else torch.empty(max(epochs, 1), dtype=torch.float32,
                                                                     device=self.device)
        w = (ctypes.c_int32 * len(self.widths))(*self.widths)
        check(lib.mlp_deep_train(_ptr(X), _ptr(T), X.shape[0], len(self.widths) - 1, w,
                                 1 if self.act == "tanh" else 0, _ptr(self.flat), _ptr(self.comp), self.lr,
                                 int(epochs), _ptr(hist), _stream(stream)))
        return hist[:epochs]

    def train(self, X: torch.Tensor, T: torch.Tensor, epochs: int, loss_hist: torch.Tensor | None = None):
        hist = loss_hist if loss_hist is not None else torch.empty(max(epochs, 1), dtype=torch.float32,
                                                                     device=self.device)
        P = self.flat.numel()
        for e in range(epochs):
            loss = torch.nn.functional.mse_loss(self.forward(X), T)
            torch.autograd.grad(loss, self.params)   # the adjoint writes the packed gradient
            check(lib.mlp_update(_ptr(self.flat), _ptr(self.grad), _ptr(self.comp), P, self.lr, _stream()))
            hist[e:e + 1].copy_(loss.detach())
        return hist[:epochs]


class DeepGraph:
    """`epochs` fused epochs of a DeepNet (library calls only) captured once in
    a HIP graph (torch.cuda.CUDAGraph) and replayed: each replay trains the
    net `epochs` more epochs in place; the loss of each captured epoch lands
    in `loss` [epochs].  X, T and the net's buffers must stay in place."""

    def __init__(self, net: DeepNet, X: torch.Tensor, T: torch.Tensor, epochs: int):
        if epochs <= 0:
            raise ValueError("epochs must be positive")
        self.net, self.X, self.T = net, X, T
        self.loss = torch.empty(max(epochs, 4), dtype=torch.float32, device=net.device)[:epochs]
        net._fused_buffers(X.shape[0])
        # one epoch outside the capture loads every kernel; the parameters are restored
        flat0, comp0 = net.flat.detach().clone(), (net.comp.clone() if net.comp is not None else None)
        net.epoch_fused(X, T, self.loss[:1])
        torch.cuda.synchronize()
        net.flat.detach().copy_(flat0)
        if comp0 is not None:
            net.comp.copy_(comp0)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph, capture_error_mode="thread_local"):
            for e in range(epochs):
                net.epoch_fused(X, T, self.loss[e:e + 1])

    def replay(self) -> None:
        self.graph.replay()

