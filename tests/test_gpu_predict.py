"""mlp_predict against the FP64 oracle: outputs within float32 rounding,
classes equal wherever the decision is unique (near-ties may go either way
and are checked to be near-ties), ties to the lowest index, and the correct
count equal to a count over the returned labels."""
import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import Params
from paper_1908_07847_amd import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def M():
    from paper_1908_07847_amd import mlp
    return mlp


def net_for(M, th: synth.Theta, n_rows):
    return M.Net(th.W1.shape[1], th.W1.shape[0], th.W2.shape[0], n_rows, theta=th)


def check_predict(M, net, X, T, th_flat):
    d, h, k = net.D, net.H, net.K
    Xd, Td = torch.from_numpy(np.ascontiguousarray(X)).cuda(), torch.from_numpy(np.ascontiguousarray(T)).cuda()
    Y, lab, cor = net.predict(Xd, Td)
    torch.cuda.synchronize()
    Y, lab, cor = Y.cpu().numpy(), lab.cpu().numpy(), int(cor.cpu().numpy()[0])
    # the decision on the kernel's own float32 outputs is exact
    assert np.array_equal(lab, oracle.classes(Y))
    assert cor == int(np.sum(lab == oracle.classes(T)))
    p = Params.of(synth.Theta.unpack(th_flat, d, h, k))
    Yr, labr = oracle.predict(X, p)
    err = float(np.max(np.abs(Y - Yr)))
    assert err <= 1e-6, err
    # where the oracle's class differs, its top two outputs are within the output error
    diff = np.nonzero(lab != labr)[0]
    for r in diff:
        if k == 1:   # one output: the decision is its side of 1/2
            assert abs(Yr[r, 0] - 0.5) <= 4 * err + 1e-7, (r, Yr[r])
        else:
            top = np.sort(Yr[r])[-2:]
            assert top[1] - top[0] <= 4 * err + 1e-7, (r, Yr[r])
    return cor, len(diff), err


def test_predict_after_training_matches_oracle(M):
    w = synth.single(2)
    net = net_for(M, w["theta"], 120)
    net.train(torch.from_numpy(w["X"]).cuda(), torch.from_numpy(w["T"]).cuda(), 2000)
    torch.cuda.synchronize()
    cor, nd, err = check_predict(M, net, w["X"], w["T"], net.flat.cpu().numpy())
    say(f"  workload 2 after 2000 epochs: {cor}/120 correct, {nd} near-tie differences, output error {err:.1e}")


@pytest.mark.parametrize("n", [1, 257, 100_000])
def test_predict_sizes(M, n):
    w = synth.single(4, n_rows=max(n, 1))
    net = net_for(M, w["theta"], n)
    cor, nd, err = check_predict(M, net, w["X"][:n], w["T"][:n], w["theta"].packed())
    say(f"  n={n}: {cor} correct, {nd} near-tie differences, output error {err:.1e}")


def test_predict_ties_go_to_the_lowest_index(M):
    w = synth.single(2)
    th = w["theta"].copy()
    th.W2[:] = 0.0
    th.b2[:] = np.array([0.1, 0.5, 0.5], np.float32)
    net = net_for(M, th, 120)
    Y, lab, _ = net.predict(torch.from_numpy(w["X"]).cuda())
    assert np.all(lab.cpu().numpy() == 1)
    th.b2[:] = 0.25
    net = net_for(M, th, 120)
    Y, lab, _ = net.predict(torch.from_numpy(w["X"]).cuda())
    assert np.all(lab.cpu().numpy() == 0)


def test_binary_output_trains_and_predicts(M):
    """The two-class reading (one sigmoid output: HbA1c at or above 6.5 %,
    poor control, or not) on workload 2's rows: the fused trainer against the
    oracle for 5000 epochs, then the predictions (class 1 above 1/2)."""
    w = synth.single(2)
    T1 = synth.binary_targets(w)
    th = synth.Theta(w["theta"].W1, w["theta"].b1, w["theta"].W2[:1].copy(), w["theta"].b2[:1].copy())
    net = net_for(M, th, 120)
    hist = net.train(torch.from_numpy(w["X"]).cuda(), torch.from_numpy(T1).cuda(), w["epochs"])
    torch.cuda.synchronize()
    q, ref_hist = oracle.train(w["X"], T1, Params.of(th), 0.1, w["epochs"])
    flat = net.flat.cpu().numpy()
    e = float(np.max(np.abs(flat - q.flat())) / np.max(np.abs(q.flat())))
    lerr = float(np.max(np.abs(hist.cpu().numpy() - ref_hist)) / np.max(ref_hist))
    assert e <= 1e-5 and lerr <= 1e-5, (e, lerr)
    cor, nd, err = check_predict(M, net, w["X"], T1, flat)
    say(f"  binary reading: {int(T1.sum())} positive rows, {cor}/120 correct after {w['epochs']} epochs, "
        f"{nd} near-threshold differences, parameter error {e:.1e}")


def _near_tie_rows(Y, margin):
    s = np.sort(Y, axis=1)
    return (s[:, -1] - s[:, -2]) < margin


@pytest.mark.parametrize("wl", [1, 2])
def test_accuracy_curve_on_the_75_25_split(M, wl):
    """Accuracy during training (accuracy_curve): the workload's rows split
    75/25 by a seeded permutation, trained in launches of 100 epochs with
    the correct counts on both parts after each launch.  Against the oracle
    trained to the same epochs: the loss history within 1e-5, and every row
    whose class differs between the two sits at a near-tie of the oracle's
    outputs (a float32 / float64 decision)."""
    w = synth.single(wl)
    sp = synth.train_test_split(w, workload=wl)
    n_tr, n_te = sp["X_tr"].shape[0], sp["X_te"].shape[0]
    assert n_tr + n_te == w["X"].shape[0] and n_tr == int(round(0.75 * w["X"].shape[0]))
    epochs, every = (1000, 100) if wl == 1 else (2000, 250)
    say(f"accuracy curve: workload {wl}, {n_tr} train / {n_te} test rows, {epochs} epochs every {every}")
    net = M.Net(w["D"], w["H"], w["K"], n_tr, lr=w["lr"], theta=w["theta"])
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    cur = M.accuracy_curve(net, dev(sp["X_tr"]), dev(sp["T_tr"]), dev(sp["X_te"]), dev(sp["T_te"]), epochs, every)
    q = Params.of(w["theta"])
    ref_hist = []
    for i, e in enumerate(cur["epochs"]):
        q, h = oracle.train(sp["X_tr"], sp["T_tr"], q, w["lr"], every)
        ref_hist.append(h)
        for part, Xp, Tp, got in (("train", sp["X_tr"], sp["T_tr"], cur["train_correct"][i]),
                                  ("test", sp["X_te"], sp["T_te"], cur["test_correct"][i])):
            Y, lab = oracle.predict(Xp, q)
            ref = int(np.sum(lab == np.argmax(Tp, axis=1)))
            tie = _near_tie_rows(Y, 1e-4)
            assert abs(got - ref) <= int(tie.sum()), (e, part, got, ref, int(tie.sum()))
        say(f"  epoch {e}: train {cur['train_correct'][i]}/{n_tr}, test {cur['test_correct'][i]}/{n_te}")
    ref_hist = np.concatenate(ref_hist)
    assert np.max(np.abs(cur["loss"] - ref_hist)) / np.max(np.abs(ref_hist)) <= 1e-5
