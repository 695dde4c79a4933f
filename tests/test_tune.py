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
