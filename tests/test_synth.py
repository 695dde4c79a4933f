"""The seeded input generator: determinism, shapes, value distributions, folds."""
import numpy as np

from paper_1908_07847_amd import synth


def test_single_workloads_are_seeded_and_shaped():
    a, b = synth.single(1), synth.single(1)
    assert np.array_equal(a["X"], b["X"]) and np.array_equal(a["theta"].W1, b["theta"].W1)
    assert a["X"].shape == (60, 33) and a["X"].dtype == np.float32
    assert a["T"].shape == (60, 3) and np.all(a["T"].sum(1) == 1)
    th = a["theta"]
    assert th.W1.shape == (10, 33) and th.b1.shape == (10,) and th.W2.shape == (3, 10)
    assert th.b2.shape == (3,)
    assert np.all(np.abs(th.packed()) <= 0.5)
    c = synth.single(2)
    assert c["X"].shape == (120, 33) and c["H"] == 16 and c["epochs"] == 5000


def test_columns_are_z_scored_and_binary_columns_two_valued():
    w = synth.single(2)
    x = w["X"].astype(np.float64)
    assert np.allclose(x.mean(0), 0, atol=1e-6)
    assert np.allclose(x.std(0), 1, atol=1e-5)
    for j in range(22, 33):
        assert len(np.unique(w["X"][:, j])) <= 2


def test_raw_feature_distributions():
    g = synth.rng(99, 0, synth.ROLE_DATA)
    x = synth.features(200000, 3, 2, g)
    assert np.all(np.abs(x[:, 3:].mean(0) - 0.3) < 0.01)
    assert np.all((x[:, :3].std(0) > 0.9) & (x[:, :3].std(0) < 20.1))


def test_reduced_rows_are_a_prefix_of_the_full_problem():
    full = synth.single(2)
    part = synth.single(2, n_rows=50)
    assert np.array_equal(part["X"], full["X"][:50])


def test_all_three_classes_present():
    for wl in (1, 2):
        cls = synth.single(wl)["classes"]
        assert set(np.unique(cls)) == {0, 1, 2}


def test_batched_folds_and_hyperparameters():
    w = synth.batched(n_nets=40)
    items = w["items"]
    assert len(items) == 40
    for i, it in enumerate(items):
        assert 40 <= it["n_rows"] <= 120
        assert 4 <= it["n_hidden"] <= 64
        assert 0.01 <= it["lr"] <= 1.0
    # the five folds of a group share H and lr and their row counts sum to 4x the group size
    for g in range(8):
        grp = items[5 * g:5 * g + 5]
        assert len({it["n_hidden"] for it in grp}) == 1 and len({float(it["lr"]) for it in grp}) == 1
        m = sum(it["n_rows"] for it in grp) // 4
        assert 50 <= m <= 150 and sum(it["n_rows"] for it in grp) == 4 * m
    last = items[-1]
    assert w["X"].shape[0] == last["x_off"] + last["n_rows"]
    assert w["theta"].size == last["p_off"] + synth.n_params(33, last["n_hidden"], 3)


def test_theta_pack_roundtrip():
    th = synth.theta0(7, 5, 3, np.random.default_rng(0))
    back = synth.Theta.unpack(th.packed(), 7, 5, 3)
    assert np.array_equal(back.W1, th.W1) and np.array_equal(back.b2, th.b2)


def test_train_test_split_is_a_seeded_75_25_partition():
    for wl, m, n_tr in ((1, 60, 45), (2, 120, 90)):
        w = synth.single(wl)
        a, b = synth.train_test_split(w, workload=wl), synth.train_test_split(w, workload=wl)
        assert np.array_equal(a["perm"], b["perm"])
        assert a["X_tr"].shape == (n_tr, 33) and a["X_te"].shape == (m - n_tr, 33)
        tr, te = np.sort(a["perm"][:n_tr]), np.sort(a["perm"][n_tr:])
        assert len(set(tr) | set(te)) == m and not set(tr) & set(te)
        assert np.array_equal(a["X_tr"], w["X"][tr]) and np.array_equal(a["T_te"], w["T"][te])
