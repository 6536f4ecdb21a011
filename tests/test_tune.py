"""Host logic of the routing-threshold autotuner: cache keys and the cached
path (no GPU: the cached record is applied without timing anything)."""
import json
import types

import paper_1508_07953_amd.tune as tune


class FakeIndex:
    def __init__(self):
        self.params = types.SimpleNamespace(patch=8, channels=1, stride=1, n_ref=16384,
                                            n_keys=16, dense_threshold=-1)
        self.set_to = []

    def set_dense_threshold(self, t):
        self.set_to.append(t)
        self.params.dense_threshold = t


def test_cache_key_names_every_table_parameter():
    assert tune.cache_key(FakeIndex(), "gfx950") == "gfx950:p8c1s1:n16384:K16"


def test_cached_threshold_is_applied(tmp_path, monkeypatch):
    path = tmp_path / "tune.json"
    monkeypatch.setenv("RIANN_TUNE_CACHE", str(path))
    idx = FakeIndex()
    tune._store(tune.cache_key(idx, "gfx950"), {"threshold": 96, "ms": {"96": 1.0}})
    assert json.loads(path.read_text())["gfx950:p8c1s1:n16384:K16"]["threshold"] == 96
    r = tune.tune_threshold(idx, [None], [None], arch="gfx950")
    assert r["cached"] and r["threshold"] == 96 and idx.set_to == [96]


def test_unreadable_cache_is_empty(tmp_path, monkeypatch):
    path = tmp_path / "tune.json"
    path.write_text("{not json")
    monkeypatch.setenv("RIANN_TUNE_CACHE", str(path))
    assert tune._load_cache() == {}


class FakeShapeIndex(FakeIndex):
    def __init__(self):
        super().__init__()
        self.shapes_set = []

    def set_dense_shape(self, waves, cols):
        self.shapes_set.append((waves, cols))


def test_cached_shape_is_applied(tmp_path, monkeypatch):
    """A cached block shape is set without timing anything, under its own
    key beside the threshold's."""
    path = tmp_path / "tune.json"
    monkeypatch.setenv("RIANN_TUNE_CACHE", str(path))
    idx = FakeShapeIndex()
    key = tune.cache_key(idx, "gfx950") + ":shape"
    tune._store(key, {"shape": [8, 4], "ms": {"4x4": 1.0, "8x4": 0.9}})
    tune._store(tune.cache_key(idx, "gfx950"), {"threshold": 64, "ms": {"64": 1.0}})
    r = tune.tune_shape(idx, [None], arch="gfx950")
    assert r["cached"] and tuple(r["shape"]) == (8, 4) and idx.shapes_set == [(8, 4)]
    assert json.loads(path.read_text())["gfx950:p8c1s1:n16384:K16"]["threshold"] == 64
