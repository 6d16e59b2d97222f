"""The launch-shape cache (paper_1204_1121_amd/tuning.py): size buckets, keys
that keep the output modes and paths apart, a save/load/apply round trip,
and the shipped gfx950 cache.  Host logic only."""
import json

from paper_1204_1121_amd import tuning


class FakeTable:
    """What the cache reads from a table, and a record of blip_set_shape."""

    def __init__(self, storage="f32", norb=768, n=(72, 72, 48)):
        self.storage, self.norb, self.n = storage, norb, n
        self.calls = []

    def set_shape(self, npos, tile_pos, vec, batched=False, ratio=False):
        self.calls.append((npos, tile_pos, vec, batched, ratio))


def test_buckets():
    assert [tuning.bucket(x) for x in (1, 2, 3, 4, 1535, 1536, 2048, 24576, 65289)] == \
        [1, 2, 2, 4, 1024, 1024, 2048, 16384, 32768]


def test_keys_separate_paths_and_modes():
    t = FakeTable()
    keys = {tuning.key(t, 24576, batched, values_only=v, ratio=r)
            for batched in (False, True) for v in (False, True) for r in (False, True)}
    assert len(keys) == 8
    assert tuning.key(t, 24576, True, ratio=True) == "gfx950/f32/L768/72x72x48/batched-ratio/16384"
    assert tuning.key(t, 1536, False) == "gfx950/f32/L768/72x72x48/block/1024"
    # another table never shares an entry
    assert tuning.key(FakeTable(norb=384), 1536, False) != tuning.key(t, 1536, False)


def test_round_trip_and_apply(tmp_path):
    path = str(tmp_path / "tuned.json")
    c = tuning.TuneCache(path)
    t = FakeTable()
    assert c.get(t, 24576, True, ratio=True) is None
    assert not c.apply(t, 24576, batched=True, ratio=True) and t.calls == []
    c.put(t, 24576, True, {"tile_pos": 4, "vec": 4, "us": 459.4}, note="sweep", ratio=True)
    c.put(t, 24576, True, {"tile_pos": 8, "vec": 2, "us": 900.0})
    c.save()
    c2 = tuning.TuneCache(path)
    assert c2.get(t, 20000, True, ratio=True)["tile_pos"] == 4      # same bucket
    assert c2.apply(t, 20000, batched=True, ratio=True)
    assert c2.apply(t, 30000, batched=True)
    # the ratio shape goes to the table's ratio mode, the plain one to the plain mode
    assert t.calls == [(20000, 4, 4, True, True), (30000, 8, 2, True, False)]
    with open(path) as f:
        assert json.load(f) == c2.entries


def test_shipped_cache_has_the_monte_carlo_ratio_shape():
    """The 16-walker TiO2 step (24,576 moves) finds its measured shape."""
    c = tuning.TuneCache()
    e = c.get(FakeTable(), 16 * 2 * 768, True, ratio=True)
    assert e is not None and e["tile_pos"] >= 1 and e["vec"] in (1, 2, 4)
    assert c.get(FakeTable(), 1536, False) is not None
