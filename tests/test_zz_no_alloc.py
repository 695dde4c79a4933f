"""The allocation-free entry point (mlp_train_shared_static) against the
entry point it is a variant of (mlp_train_shared with a caller workspace),
through the C ABI: two calls in a row on the static scratch -- the second
with a smaller input (fewer rows, another minibatch, fewer nets) -- each
bitwise equal to the workspace form on the same inputs (same kernels, same
grid, same summation order), and the float32 result within 1e-5 of the
float64 oracle.  A shape whose scratch exceeds the array is rejected before
any device work."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_1908_07847_amd import _lib, mlp, synth
from paper_1908_07847_amd._lib import Config, check, lib

pytestmark = pytest.mark.gpu


def _cfg(D, H, K, N, batch, prec, lr):
    return Config(D, H, K, _lib.PREC[prec], N, batch, float(lr), _lib.MLP_F_COMPENSATED)


def _run(static: bool, w, n_nets, epochs, prec="fp32"):
    D, H, K = w["D"], w["H"], w["K"]
    N, batch = w["X"].shape[0], w["batch"]
    X = torch.from_numpy(w["X"]).cuda()
    T = torch.from_numpy(w["T"]).cuda()
    th = torch.from_numpy(np.ascontiguousarray(w["theta"][:n_nets])).cuda()
    comp = torch.zeros_like(th)
    hist = torch.zeros((n_nets, epochs), device="cuda")
    cfg = _cfg(D, H, K, N, batch, prec, w["lrs"][0])
    lrs = (ctypes.c_float * n_nets)(*[float(v) for v in w["lrs"][:n_nets]])
    if static:
        check(lib.mlp_train_shared_static(ctypes.byref(cfg), n_nets, lrs, X.data_ptr(), T.data_ptr(), th.data_ptr(),
                                          comp.data_ptr(), epochs, hist.data_ptr(), None))
    else:
        nb = ctypes.c_size_t(0)
        check(lib.mlp_shared_workspace_size(ctypes.byref(cfg), n_nets, ctypes.byref(nb)))
        ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
        check(lib.mlp_train_shared(ctypes.byref(cfg), n_nets, lrs, X.data_ptr(), T.data_ptr(), th.data_ptr(),
                                   comp.data_ptr(), epochs, hist.data_ptr(), ws.data_ptr(), nb.value, None))
    torch.cuda.synchronize()
    return th.cpu().numpy(), hist.cpu().numpy()


def test_static_scratch_calls_equal_the_workspace_form():
    big = synth.shared(5, n_nets=2, n_rows=4 * 16384)              # wide net, 2 nets, 4 steps per epoch
    small = synth.shared(4, n_nets=1, n_rows=2 * 4096)             # 33-256-3, 1 net, 2 steps per epoch
    for w, nets, epochs in ((big, 2, 2), (small, 1, 3)):
        a, ha = _run(True, w, nets, epochs)
        b, hb = _run(False, w, nets, epochs)
        assert np.array_equal(a, b) and np.array_equal(ha, hb)
        p0 = oracle.Params.of(synth.Theta.unpack(w["theta"][0], w["D"], w["H"], w["K"]))
        q, ref_hist = oracle.train(w["X"], w["T"], p0, w["lrs"][0], epochs, batch=w["batch"])
        err = np.max(np.abs(a[0] - q.flat())) / np.max(np.abs(q.flat()))
        assert err <= 1e-5, err
        assert np.max(np.abs(ha[0] - ref_hist) / ref_hist) <= 1e-5


def test_static_scratch_rejects_a_shape_beyond_its_size():
    w = synth.shared(5, n_nets=64, n_rows=16384)
    cfg = _cfg(w["D"], w["H"], w["K"], 16384, w["batch"], "bf16", 0.1)
    lrs = (ctypes.c_float * 64)(*([0.1] * 64))
    st = lib.mlp_train_shared_static(ctypes.byref(cfg), 64, lrs, 0x10000, 0x20000, 0x30000, 0x40000, 1, None, None)
    assert st == _lib.MLP_ERR_WORKSPACE
    assert b"static scratch" in lib.mlp_last_error()
