"""Host logic of the batched path's tuning cache (no GPU): the key depends on
everything the search depends on, stored tunings round-trip through the JSON
file, and a hit returns without timing anything (the tensors here are CPU
tensors, which a search could not run on)."""
import json

import torch

from paper_1510_06689_amd import tucker


def _key(**over):
    args = dict(shapes=[(24, 24, 24, 16), (96, 96, 96, 16)], dtype=torch.float32, eps=1e-4,
                options={}, candidates_gram=(8, 16), candidates_ttm=(16, 64),
                device_name="dev", library_id="lib")
    args.update(over)
    return tucker.batch_tuning_key(**args)


def test_key_is_stable_and_sensitive():
    assert _key() == _key()
    base = _key()
    for over in (dict(shapes=[(24, 24, 24, 16), (96, 96, 95, 16)]),
                 dict(shapes=[(96, 96, 96, 16), (24, 24, 24, 16)]),
                 dict(dtype=torch.float64), dict(eps=1e-3),
                 dict(options={"ttm_precision": "bf16"}), dict(candidates_gram=(8, 32)),
                 dict(candidates_ttm=(16,)), dict(device_name="other"),
                 dict(library_id="rebuilt")):
        assert _key(**over) != base, over


def test_store_and_load_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tuning.json")
    assert tucker.load_batch_tuning(path, "k1") is None
    tucker.store_batch_tuning(path, "k1", [16, 8, 32, 64], [64, 64, 256, 256], 2.82)
    tucker.store_batch_tuning(path, "k2", [8], [16], 1.0)
    assert tucker.load_batch_tuning(path, "k1") == ([16, 8, 32, 64], [64, 64, 256, 256], 2.82)
    assert tucker.load_batch_tuning(path, "k2") == ([8], [16], 1.0)
    assert tucker.load_batch_tuning(path, "k3") is None
    assert sorted(json.load(open(path))) == ["k1", "k2"]


def test_unreadable_cache_is_a_miss(tmp_path):
    path = tmp_path / "tuning.json"
    path.write_text("{not json")
    assert tucker.load_batch_tuning(str(path), "k") is None
    tucker.store_batch_tuning(str(path), "k", [1], [2], 3.0)  # replaces the broken file
    assert tucker.load_batch_tuning(str(path), "k") == ([1], [2], 3.0)


def test_hit_returns_the_stored_tuning_without_a_search(tmp_path):
    xs = [torch.zeros((5, 6, 7)), torch.zeros((8, 6, 7))]
    path = str(tmp_path / "tuning.json")
    key = tucker.batch_tuning_key([x.shape for x in xs], xs[0].dtype, 1e-4, {},
                                  (8, 16, 32, 64), (16, 64, 256), "cpu", tucker._library_id())
    tucker.store_batch_tuning(path, key, [32, 8, 32], [64, 64, 256], 2.5)
    info = {}
    got = tucker.autotune_batch(xs, 1e-4, cache=path, info=info)
    assert got == ([32, 8, 32], [64, 64, 256], 2.5)
    assert info == {"cache_hit": True, "key": key}
