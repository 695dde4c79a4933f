"""The C ABI of libmlp on the host: the library loads, exports every symbol
that include/mlp.h declares, and rejects bad arguments before any HIP call
(so these run without a GPU; no compute call is made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1908_07847_amd import _lib
    return _lib


def test_header_declarations_are_all_exported():
    L = _lib()
    hdr = open(os.path.join(ROOT, "include", "mlp.h")).read()
    declared = set(re.findall(r"\b(mlp_[a-z_]+)\s*\(", hdr))
    assert declared == set(L.SYMBOLS)
    for name in declared:
        assert hasattr(L.lib, name), name


def test_struct_sizes_match_header():
    L = _lib()
    assert ctypes.sizeof(L.BatchItem) == 32
    assert ctypes.sizeof(L.Config) == 40


def test_status_strings():
    L = _lib()
    for s in range(9):
        assert L.lib.mlp_status_string(s)
    assert L.lib.mlp_status_string(99) == b"unknown status"


def _ws(cfg):
    L = _lib()
    n = ctypes.c_size_t(0)
    st = L.lib.mlp_workspace_size(ctypes.byref(cfg), ctypes.byref(n))
    return st, n.value


def test_workspace_size_and_config_validation():
    L = _lib()
    good = L.Config(33, 16, 3, 0, 120, 0, 0.1, 1)
    st, n = _ws(good)
    assert st == L.MLP_OK and n >= 120 * (16 + 3 + 1) * 4 and n % 256 == 0
    bad = [L.Config(0, 16, 3, 0, 120, 0, 0.1, 1), L.Config(33, 0, 3, 0, 120, 0, 0.1, 1),
           L.Config(33, 16, 0, 0, 120, 0, 0.1, 1), L.Config(33, 16, 3, 0, 0, 0, 0.1, 1),
           L.Config(33, 16, 3, 0, 120, -1, 0.1, 1), L.Config(33, 16, 17, 0, 120, 0, 0.1, 1)]
    for c in bad:
        assert _ws(c)[0] == L.MLP_ERR_SHAPE
    assert _ws(L.Config(33, 16, 3, 7, 120, 0, 0.1, 1))[0] == L.MLP_ERR_ARG        # precision
    assert _ws(L.Config(33, 16, 3, 0, 120, 0, 0.1, 16))[0] == L.MLP_ERR_ARG       # unknown flag bit
    assert _ws(L.Config(33, 16, 3, 0, 120, 0, float("nan"), 1))[0] == L.MLP_ERR_ARG
    assert L.lib.mlp_workspace_size(None, None) == L.MLP_ERR_ARG
    assert b"NULL" in L.lib.mlp_last_error()


def test_init_rejects_before_touching_the_device():
    L = _lib()
    h = ctypes.c_void_p()
    cfg = L.Config(33, 16, 3, 0, 120, 0, 0.1, 1)
    p = L.Params(0x1000, 0x2000, 0x3000, 0x4000)
    # compensated without a buffer
    assert L.lib.mlp_init(ctypes.byref(h), ctypes.byref(cfg), p, None, 0x5000, 1 << 20) == L.MLP_ERR_ARG
    # workspace too small
    assert L.lib.mlp_init(ctypes.byref(h), ctypes.byref(cfg), p, 0x6000, 0x5000, 16) == L.MLP_ERR_WORKSPACE
    # misaligned parameter pointer
    p2 = L.Params(0x1002, 0x2000, 0x3000, 0x4000)
    assert L.lib.mlp_init(ctypes.byref(h), ctypes.byref(cfg), p2, 0x6000, 0x5000, 1 << 20) == L.MLP_ERR_ALIGN
    # NULL parameter
    p3 = L.Params(0x1000, None, 0x3000, 0x4000)
    assert L.lib.mlp_init(ctypes.byref(h), ctypes.byref(cfg), p3, 0x6000, 0x5000, 1 << 20) == L.MLP_ERR_ARG
    assert h.value is None


def test_calls_on_a_null_handle_fail_cleanly():
    L = _lib()
    p = L.Params(0x1000, 0x2000, 0x3000, 0x4000)
    assert L.lib.mlp_forward(None, 0x1000, 4, None, 0x2000, None) == L.MLP_ERR_ARG
    assert L.lib.mlp_backward(None, 0x1000, 0x2000, 0x3000, None, 0x4000, 4, p, None, None, None) == L.MLP_ERR_ARG
    assert L.lib.mlp_step(None, p, 0.1, None) == L.MLP_ERR_ARG
    assert L.lib.mlp_train(None, 0x1000, 0x2000, 5, None, None) == L.MLP_ERR_ARG
    assert L.lib.mlp_destroy(None) == L.MLP_ERR_ARG


def _items(**kw):
    L = _lib()
    base = dict(n_rows=50, n_hidden=8, lr=0.1, reserved=0, x_off=0, p_off=0)
    base.update(kw)
    arr = (L.BatchItem * 1)()
    arr[0] = L.BatchItem(base["n_rows"], base["n_hidden"], base["lr"], base["reserved"], base["x_off"],
                         base["p_off"])
    return arr


@pytest.mark.parametrize("kw,status", [
    (dict(n_rows=0), 2), (dict(n_rows=129), 2), (dict(n_hidden=65), 2), (dict(n_hidden=0), 2),
    (dict(x_off=60), 2), (dict(p_off=10**6), 2), (dict(reserved=1), 1), (dict(lr=-1.0), 1)])
def test_batched_item_validation(kw, status):
    L = _lib()
    st = L.lib.mlp_train_batched(_items(**kw), 0x1000, 1, 33, 3, 0x2000, 0x3000, 100, 0x4000, None,
                                 100000, 10, None, None)
    assert st == status


def test_batched_shape_and_pointer_validation():
    L = _lib()
    it = _items()
    assert L.lib.mlp_train_batched(it, 0x1000, 0, 33, 3, 0x2000, 0x3000, 100, 0x4000, None, 10**5, 1, None,
                                   None) == L.MLP_ERR_SHAPE
    assert L.lib.mlp_train_batched(it, 0x1000, 1, 49, 3, 0x2000, 0x3000, 100, 0x4000, None, 10**5, 1, None,
                                   None) == L.MLP_ERR_SHAPE
    assert L.lib.mlp_train_batched(it, 0x1008, 1, 33, 3, 0x2000, 0x3000, 100, 0x4000, None, 10**5, 1, None,
                                   None) == L.MLP_ERR_ALIGN
    assert L.lib.mlp_train_batched(it, None, 1, 33, 3, 0x2000, 0x3000, 100, 0x4000, None, 10**5, 1, None,
                                   None) == L.MLP_ERR_ARG


def _shared_ws(cfg, n):
    L = _lib()
    b = ctypes.c_size_t(0)
    st = L.lib.mlp_shared_workspace_size(ctypes.byref(cfg), n, ctypes.byref(b))
    return st, b.value


def test_shared_workspace_size():
    L = _lib()
    c5 = L.Config(64, 1024, 3, 1, 1 << 22, 16384, 0.1, 1)
    st, n64 = _shared_ws(c5, 64)
    assert st == L.MLP_OK and n64 % 256 == 0
    P = 64 * 1024 + 1024 + 1024 * 3 + 3
    assert n64 >= 64 * P * 4                       # at least one partial-gradient row per net
    st, n1 = _shared_ws(c5, 1)
    assert st == L.MLP_OK and n1 > 0
    assert _shared_ws(c5, 0)[0] == L.MLP_ERR_SHAPE
    assert _shared_ws(c5, 65)[0] == L.MLP_ERR_SHAPE
    assert _shared_ws(L.Config(65, 1024, 3, 1, 1 << 22, 16384, 0.1, 1), 4)[0] == L.MLP_ERR_UNSUPPORTED
    assert _shared_ws(L.Config(64, 1024, 5, 1, 1 << 22, 16384, 0.1, 1), 4)[0] == L.MLP_ERR_UNSUPPORTED
    assert _shared_ws(L.Config(64, 1024, 3, 1, 1 << 22, 1000, 0.1, 1), 4)[0] == L.MLP_ERR_UNSUPPORTED


def test_train_shared_rejects_before_touching_the_device():
    L = _lib()
    cfg = L.Config(33, 256, 3, 0, 8192, 1024, 0.1, 1)
    st, need = _shared_ws(cfg, 4)
    assert st == L.MLP_OK
    lrs = (ctypes.c_float * 4)(0.1, 0.2, 0.3, 0.4)
    args = lambda **kw: dict(dict(cfg=ctypes.byref(cfg), n=4, lr=lrs, X=0x10000, T=0x20000, th=0x30000,
                                  comp=0x40000, ep=3, lh=None, ws=0x50000, nb=need), **kw)
    call = lambda a: L.lib.mlp_train_shared(a["cfg"], a["n"], a["lr"], a["X"], a["T"], a["th"], a["comp"],
                                            a["ep"], a["lh"], a["ws"], a["nb"], None)
    assert call(args(X=None)) == L.MLP_ERR_ARG
    assert call(args(comp=None)) == L.MLP_ERR_ARG                 # compensated without a buffer
    assert call(args(ep=-1)) == L.MLP_ERR_ARG
    bad = (ctypes.c_float * 4)(0.1, float("nan"), 0.3, 0.4)
    assert call(args(lr=bad)) == L.MLP_ERR_ARG
    assert call(args(X=0x10004)) == L.MLP_ERR_ALIGN
    assert call(args(th=0x30002)) == L.MLP_ERR_ALIGN
    assert call(args(nb=need - 256)) == L.MLP_ERR_WORKSPACE
    assert call(args(ws=None)) == L.MLP_ERR_WORKSPACE
    assert call(args(n=0)) == L.MLP_ERR_SHAPE
    e4 = L.Config(33, 256, 3, 2, 8192, 1024, 0.1, 1)
    assert call(args(cfg=ctypes.byref(e4))) == L.MLP_ERR_UNSUPPORTED   # e4m3 with several nets
    assert call(args(ep=0)) == L.MLP_OK                           # nothing to do, no device work


def test_barrier_probe_rejects_before_touching_the_device():
    L = _lib()
    call = lambda n=64, r=100, ws=0x10000, nb=L.BARRIER_PROBE_WS_BYTES: L.lib.mlp_barrier_probe(n, r, ws, nb, None)
    assert call(r=-1) == L.MLP_ERR_ARG
    assert call(r=1000001) == L.MLP_ERR_ARG
    assert call(ws=None) == L.MLP_ERR_WORKSPACE
    assert call(nb=L.BARRIER_PROBE_WS_BYTES - 4) == L.MLP_ERR_WORKSPACE
    assert call(ws=0x10004) == L.MLP_ERR_ALIGN
    assert call(n=0) == L.MLP_ERR_ARG


def test_variant_flag_and_momentum_arguments():
    L = _lib()
    n = ctypes.c_size_t(0)
    ok = L.Config(33, 16, 3, 0, 120, 0, 0.1, L.MLP_F_COMPENSATED | L.F_TANH_HIDDEN)
    assert L.lib.mlp_workspace_size(ctypes.byref(ok), ctypes.byref(n)) == L.MLP_OK
    bad = L.Config(33, 16, 3, 0, 120, 0, 0.1, 16)
    assert L.lib.mlp_workspace_size(ctypes.byref(bad), ctypes.byref(n)) == L.MLP_ERR_ARG
    assert L.lib.mlp_set_momentum(None, 0.9, 0x1000) == L.MLP_ERR_ARG


def test_deep_train_rejects_before_touching_the_device():
    """mlp_deep_train's argument checks and its LDS-fit check run on the
    host; epochs = 0 launches nothing."""
    L = _lib()

    def call(widths=(33, 16, 16, 3), n=120, act=0, lr=0.1, ep=10, X=0x10000, T=0x20000, th=0x30000, comp=0x40000,
             layers=None):
        w = (ctypes.c_int32 * len(widths))(*widths)
        nl = len(widths) - 1 if layers is None else layers
        return L.lib.mlp_deep_train(X, T, n, nl, w, act, th, comp, lr, ep, None, None)

    assert call(X=None) == L.MLP_ERR_ARG
    assert call(th=None) == L.MLP_ERR_ARG
    assert call(layers=0) == L.MLP_ERR_SHAPE
    assert call(widths=(2,) * 10) == L.MLP_ERR_SHAPE                # 9 weight layers
    assert call(widths=(33, 0, 3)) == L.MLP_ERR_SHAPE
    assert call(widths=(33, 1025, 3)) == L.MLP_ERR_SHAPE
    assert call(n=0) == L.MLP_ERR_SHAPE
    assert call(act=2) == L.MLP_ERR_ARG
    assert call(lr=float("nan")) == L.MLP_ERR_ARG
    assert call(ep=-1) == L.MLP_ERR_ARG
    assert call(th=0x30002) == L.MLP_ERR_ALIGN
    assert call(n=100000) == L.MLP_ERR_UNSUPPORTED                  # rows beyond one workgroup's LDS
    assert call(widths=(64, 512, 64, 3)) == L.MLP_ERR_UNSUPPORTED   # parameters beyond it
    assert call(ep=0) == L.MLP_OK


def test_status_and_check_flags_on_the_host():
    """MLP_F_DETERMINISTIC and MLP_F_CHECK_FINITE are accepted, the status
    query rejects a missing, short or misaligned workspace before any HIP
    call, and the wait limit is a plain host setting."""
    L = _lib()
    n = ctypes.c_size_t(0)
    for flags in (L.F_DETERMINISTIC, L.F_CHECK_FINITE, L.F_COMPENSATED | L.F_CHECK_FINITE | L.F_DETERMINISTIC):
        c = L.Config(33, 16, 3, 0, 120, 0, 0.1, flags)
        assert L.lib.mlp_workspace_size(ctypes.byref(c), ctypes.byref(n)) == L.MLP_OK
        assert n.value >= 2048                     # the status block at the workspace's head
    assert L.lib.mlp_workspace_status(None, 4096, None) == L.MLP_ERR_ARG
    assert L.lib.mlp_workspace_status(0x10000, 1024, None) == L.MLP_ERR_WORKSPACE
    assert L.lib.mlp_workspace_status(0x10004, 4096, None) == L.MLP_ERR_ALIGN
    assert L.lib.mlp_query_status(None, None) == L.MLP_ERR_ARG
    assert L.lib.mlp_set_wait_limit(0) == L.MLP_OK
    assert L.lib.mlp_set_wait_limit(-1) == L.MLP_OK   # back to the default
    assert L.lib.mlp_status_string(L.MLP_ERR_TIMEOUT) == b"a grid-wide wait gave up"
    assert L.lib.mlp_status_string(L.MLP_ERR_NONFINITE) == b"non-finite parameter or loss"


def test_large_plan_on_the_host():
    """mlp_large_plan is host arithmetic: the wide 64-1024-3 net fills 256 CUs
    with 64 row blocks of 256 rows x 4 hidden blocks of 256 units on 8 waves;
    the 33-256-3 net with 4096-row minibatches takes 64-row blocks and 64-unit
    hidden blocks on 4 waves; a launch hint overrides the grid and the waves;
    bad arguments and uncovered shapes are rejected."""
    from paper_1908_07847_amd import mlp
    L = _lib()
    assert mlp.large_plan(64, 1024, 3, 4194304, batch=16384, n_cu=256) == \
        {"row_blocks": 64, "hidden_blocks": 4, "waves": 8, "piece_rows": 256, "tiles_per_wave": 2,
         "kernel": "mlpk::k_large_train<0, 3, 8, 2>"}
    p = mlp.large_plan(33, 256, 3, 1048576, batch=4096, prec="bf16", n_cu=256)
    assert (p["row_blocks"], p["hidden_blocks"], p["waves"], p["tiles_per_wave"]) == (64, 4, 4, 1)
    assert p["kernel"] == "mlpk::k_large_train<1, 3, 4, 1>"
    # a 4-wave block of more than four tiles (here by a launch hint) takes the
    # general instance
    mlp.set_launch_hint(large_grid=(64, 2), large_waves=4)
    try:
        big = mlp.large_plan(33, 256, 4, 1048576, batch=4096, n_cu=256)
        assert (big["waves"], big["tiles_per_wave"], big["kernel"]) == (4, 4, "mlpk::k_large_train<0, 4, 4, 4>")
    finally:
        mlp.reset_launch_hint()
    q = mlp.large_plan(64, 1024, 3, 4194304, batch=16384, n_nets=64, n_cu=256)
    assert q["row_blocks"] * 64 * q["hidden_blocks"] <= 256
    mlp.set_launch_hint(large_grid=(128, 2), large_waves=8)
    try:
        r = mlp.large_plan(33, 256, 3, 1048576, batch=4096, n_cu=256)
        assert (r["row_blocks"], r["hidden_blocks"], r["waves"]) == (128, 2, 8)
    finally:
        mlp.reset_launch_hint()
    out = (ctypes.c_int32 * 5)()
    c = L.Config(64, 1024, 3, 0, 4194304, 16384, 0.1, 0)
    assert L.lib.mlp_large_plan(None, 1, 256, out) == L.MLP_ERR_ARG
    assert L.lib.mlp_large_plan(ctypes.byref(c), 1, 256, None) == L.MLP_ERR_ARG
    assert L.lib.mlp_large_plan(ctypes.byref(c), 1, 0, out) == L.MLP_ERR_ARG
    assert L.lib.mlp_large_plan(ctypes.byref(c), 65, 256, out) == L.MLP_ERR_ARG
    wide_in = L.Config(65, 16, 3, 0, 4096, 64, 0.1, 0)
    assert L.lib.mlp_large_plan(ctypes.byref(wide_in), 1, 256, out) == L.MLP_ERR_UNSUPPORTED
    odd_batch = L.Config(33, 256, 3, 0, 4096, 48, 0.1, 0)
    assert L.lib.mlp_large_plan(ctypes.byref(odd_batch), 1, 256, out) == L.MLP_ERR_UNSUPPORTED


def test_cv_select_rejects_before_touching_the_device():
    L = _lib()
    f = L.lib.mlp_cv_select
    assert f(None, 0x1000, 4, 2, 0x2000, 0x3000, None) == L.MLP_ERR_ARG
    assert f(0x1000, 0x1000, 0, 2, 0x2000, 0x3000, None) == L.MLP_ERR_SHAPE
    assert f(0x1000, 0x1000, 4, 0, 0x2000, 0x3000, None) == L.MLP_ERR_SHAPE
    assert f(0x1000, 0x1000, 4, 65537, 0x2000, 0x3000, None) == L.MLP_ERR_SHAPE
    assert f(0x1002, 0x1000, 4, 2, 0x2000, 0x3000, None) == L.MLP_ERR_ALIGN
