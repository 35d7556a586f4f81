"""Host logic of the autotuner: the on-disk cache (atomic replace, lookups
by shape class) without a GPU -- the device name is stubbed."""
import json
import os

import pytest


@pytest.fixture()
def at(tmp_path, monkeypatch):
    monkeypatch.setenv("MSKETCH_TUNE_CACHE", str(tmp_path / "tune.json"))
    from paper_2508_14209_amd import autotune
    monkeypatch.setattr(autotune, "_device_name", lambda device: "gfx950:test:256")
    return autotune


class _T:
    def __init__(self, shape, dtype):
        self.shape = shape
        self.dtype = dtype


def _prob(d, n, adt="torch.float32", gdt="torch.bfloat16"):
    return {"A": _T((d, n), adt), "G": _T((2 * n, 2 * n * n), gdt)}


def test_cache_roundtrip_and_keys(at, tmp_path):
    assert at.cache_path() == str(tmp_path / "tune.json")
    assert at._load() == {}
    at._store("x", {"a": 1})
    at._store("y", {"b": 2})
    data = json.load(open(at.cache_path()))
    assert data == {"x": {"a": 1}, "y": {"b": 2}}
    assert not [f for f in os.listdir(tmp_path) if ".tmp" in f]
    # countsketch key: d rounded to the nearest power of two
    assert at.cs_key(1000, 8, 64, "torch.float64", None) == at.cs_key(1030, 8, 64, "torch.float64", None)
    assert at.cs_key(1000, 8, 64, "torch.float64", None) != at.cs_key(4000, 8, 64, "torch.float64", None)


def test_batch_shape_class(at):
    a = [_prob(100000, 8), _prob(120000, 16)]
    b = [_prob(110000, 16), _prob(100000, 9), _prob(120000, 12)]   # other count, n <= 16
    c = [_prob(110000, 32)]
    assert at.batch_key(a, None) == at.batch_key(b, None)
    assert at.batch_key(a, None) != at.batch_key(c, None)
    assert at.batch_params(a, "cpu") == (0, 0)
    at._store(at.batch_key(a, None), {"rows_log2": 14, "kchunk_log2": 9, "ms": 1.0})
    assert at.lookup_batch(b, "cpu") == (14, 9)
    assert at.batch_params(c, "cpu") == (0, 0)


def test_corrupt_cache_is_ignored(at):
    with open(at.cache_path(), "w") as f:
        f.write("{not json")
    assert at._load() == {}
    at._store("k", {"v": 1})
    assert at._load() == {"k": {"v": 1}}
