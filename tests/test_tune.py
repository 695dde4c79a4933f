"""The autotuner's host logic: candidate grids, shape keys, the JSON cache."""
import pytest


@pytest.fixture
def tune(monkeypatch, tmp_path):
    monkeypatch.setenv("MLP_TUNE_CACHE", str(tmp_path / "tune.json"))
    from paper_1908_07847_amd import tune as t
    return t


@pytest.mark.parametrize("h,batch", [(256, 4096), (1024, 16384), (100, 1024), (16, 96), (300, 512)])
def test_large_candidates_respect_the_kernel_limits(tune, h, batch):
    cands = tune.large_candidates(h, batch, 256)
    assert cands, "at least one grid"
    for gi, gj in cands:
        hb = -(-h // (64 * gj)) * 64
        assert hb <= 256
        assert batch % gi == 0 and (batch // gi) % 32 == 0
        # one workgroup per CU
        assert gi * gj <= 256


def test_keys_bucket_shapes(tune):
    assert tune.small_key(33, 120, 64, 4096) == tune.small_key(33, 100, 40, 3000)
    assert tune.small_key(33, 120, 64, 4096) != tune.small_key(33, 120, 16, 4096)
    assert tune.large_key(33, 256, 4096, "bf16") != tune.large_key(33, 256, 4096, "fp32")


def test_cache_round_trip(tune):
    tune._store("k", {"grid": [64, 4]})
    tune._store("k2", {"threads": 256})
    c = tune._load_cache()
    assert c["k"]["grid"] == [64, 4] and c["k2"]["threads"] == 256


def test_whole_plan_search_moves_late_groups_and_caches_the_choice(tune, monkeypatch):
    """The whole-plan pass of the batched autotuner: coordinate descent over
    each group's launch shape, then over the stream of every group after the
    fourth, then the shapes again; the choice is cached and re-applied.  The
    plan's time here is a synthetic function of the choices (no device)."""
    import torch

    class Plan:
        groups = [(0, 10, 120, 64), (10, 8, 64, 64), (18, 6, 120, 32), (24, 5, 119, 16), (29, 4, 64, 32),
                  (33, 3, 64, 16)]

        def __init__(self):
            self.threads = [64, 64, 64, 512, 512, 256]
            self.stream_of = [g % 4 for g in range(6)]

    plan = Plan()
    calls = []

    def fake_time(fn, reps=2):
        # the plan is fastest with group 4 behind group 2, group 5 behind
        # group 3, and group 4 at 128 threads once it sits behind group 2
        t = 100.0 + (0.0 if plan.stream_of[4] == 2 else 7.0) + (0.0 if plan.stream_of[5] == 3 else 3.0)
        t += 0.0 if (plan.threads[4] == 128) == (plan.stream_of[4] == 2) else 2.0
        calls.append(t)
        return t

    monkeypatch.setattr(tune, "_time", fake_time)
    th = torch.zeros(8)
    threads = tune._tune_together(plan, None, None, th, 33, 3, 20, force=True)
    assert plan.stream_of == [0, 1, 2, 3, 2, 3]
    assert threads == [64, 64, 64, 512, 128, 256] and plan.threads == threads
    assert min(calls) == 100.0
    # the cached choice is applied to a fresh plan without timing anything
    fresh = Plan()
    calls.clear()
    assert tune._tune_together(fresh, None, None, th, 33, 3, 20, force=False) == threads
    assert fresh.stream_of == [0, 1, 2, 3, 2, 3] and not calls
