"""Failure reporting of the training launches, forced from the host.

A grid-barrier wait of the minibatch (large-shape) trainer is bounded in
time; with the limit set to 0 (mlp_set_wait_limit) a wait that is not
satisfied at once gives up, so every launch of a grid of several
workgroups fails the same way: the workgroups leave the step loop (no
kernel hangs or faults), the parameters stay untouched (the update phase
follows two barriers that cannot complete), every loss_hist entry is NaN,
and mlp_query_status / mlp_workspace_status return MLP_ERR_TIMEOUT.  The
finite check (MLP_F_CHECK_FINITE) reports a NaN planted in the inputs.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1908_07847_amd import _lib, mlp, synth

pytestmark = pytest.mark.gpu


@pytest.fixture
def zero_wait_limit():
    mlp.set_wait_limit(0)
    try:
        yield
    finally:
        mlp.set_wait_limit(-1)


def _large_case(rows=32768, prec="fp32"):
    w = synth.single(4, n_rows=rows)
    X = torch.from_numpy(w["X"]).cuda()
    T = torch.from_numpy(w["T"]).cuda()
    net = mlp.Net(w["D"], w["H"], w["K"], rows, batch=w["batch"], lr=w["lr"], theta=w["theta"], prec=prec)
    return w, X, T, net


@pytest.mark.parametrize("prec", ["fp32", "e4m3"])
def test_a_barrier_wait_that_gives_up_ends_the_launch_and_is_reported(zero_wait_limit, prec):
    w, X, T, net = _large_case(prec=prec)
    before = net.flat.clone()
    hist = torch.zeros(2, device="cuda")
    net.train(X, T, 2, loss_hist=hist)
    torch.cuda.synchronize()                       # the launch ended (nothing hangs)
    assert net.status() == _lib.MLP_ERR_TIMEOUT
    assert torch.equal(net.flat, before)           # no update was applied
    assert torch.isnan(hist).all()


def test_training_after_a_failed_launch_is_normal_again():
    w, X, T, net = _large_case()
    mlp.set_wait_limit(0)
    try:
        net.train(X, T, 1)
        assert net.status() == _lib.MLP_ERR_TIMEOUT
    finally:
        mlp.set_wait_limit(-1)
    net.set_theta(w["theta"])
    hist = net.train(X, T, 1)
    assert net.status() == _lib.MLP_OK
    ref, ref_hist = oracle.train(w["X"], w["T"], oracle.Params.of(w["theta"]), w["lr"], 1, batch=w["batch"])
    got = net.flat.cpu().numpy()
    err = np.max(np.abs(got - ref.flat())) / np.max(np.abs(ref.flat()))
    assert err <= 1e-5, err
    assert abs(float(hist[0]) - ref_hist[0]) / ref_hist[0] <= 1e-5


def test_shared_trainer_and_probe_report_a_wait_that_gave_up(zero_wait_limit):
    w = synth.shared(4, n_nets=4, n_rows=8192)
    X = torch.from_numpy(w["X"]).cuda()
    T = torch.from_numpy(w["T"]).cuda()
    th = torch.from_numpy(w["theta"]).cuda()
    before = th.clone()
    ws = torch.empty(mlp.shared_workspace_size(w["D"], w["H"], w["K"], 8192, w["batch"], 4, "fp32"),
                     dtype=torch.uint8, device="cuda")
    hist = torch.zeros((4, 1), device="cuda")
    mlp.train_shared(X, T, th, w["lrs"], 1, w["H"], batch=w["batch"], comp=torch.zeros_like(th),
                     loss_hist=hist, workspace=ws)
    assert mlp.workspace_status(ws) == _lib.MLP_ERR_TIMEOUT
    assert torch.equal(th, before) and torch.isnan(hist).all()
    pws = mlp.barrier_probe(64, 10)
    assert mlp.workspace_status(pws) == _lib.MLP_ERR_TIMEOUT


def test_finite_check_reports_a_nan_and_passes_clean_runs():
    # small full-batch trainer
    w = synth.single(1)
    X = torch.from_numpy(w["X"]).cuda()
    T = torch.from_numpy(w["T"]).cuda()
    net = mlp.Net(w["D"], w["H"], w["K"], X.shape[0], lr=w["lr"], theta=w["theta"], check_finite=True)
    net.train(X, T, 5)
    assert net.status() == _lib.MLP_OK
    Xbad = X.clone()
    Xbad[3, 5] = float("nan")
    net.train(Xbad, T, 5)
    assert net.status() == _lib.MLP_ERR_NONFINITE
    # large-shape trainer
    w, X, T, _ = _large_case(rows=8192)
    net = mlp.Net(w["D"], w["H"], w["K"], 8192, batch=w["batch"], lr=w["lr"], theta=w["theta"], check_finite=True)
    net.train(X, T, 1)
    assert net.status() == _lib.MLP_OK
    Xbad = X.clone()
    Xbad[100, 0] = float("inf")
    net.train(Xbad, T, 1)
    assert net.status() == _lib.MLP_ERR_NONFINITE
