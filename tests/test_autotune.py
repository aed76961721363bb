"""Host logic of the batch autotuner, with a stand-in context (no GPU)."""
import json

import pytest

from paper_1001_3411_amd import autotune


class FakeCtx:
    """Records settings; run_batch 'takes' a time that depends on them."""

    def __init__(self, clock):
        self.t = {}
        self.clock = clock
        self.runs = 0

    def set_tuning(self, **kw):
        self.t.update(kw)

    def run_batch(self, *a, **kw):
        self.runs += 1
        # fastest at front_cap 512, xcd_queues 1, largest_first 1
        cost = abs(self.t["front_cap"] - 512) / 512 + (1 - self.t["xcd_queues"]) \
            + 0.5 * (1 - self.t["largest_first"])
        self.clock[0] += 0.001 * (1 + cost)


@pytest.fixture
def fake(monkeypatch):
    clock = [0.0]
    monkeypatch.setattr(autotune.time, "perf_counter", lambda: clock[0])
    return FakeCtx(clock)


def test_size_class_rounds_to_powers_of_two():
    assert autotune.size_class([0, 1000, 3000]) == "n2^12_sub2^1"
    assert autotune.size_class([0, 5, 20_000_000]) == autotune.size_class([0, 7, 19_000_000])
    with pytest.raises(ValueError):
        autotune.size_class([0])


def test_picks_fastest_and_caches(fake, tmp_path):
    path = str(tmp_path / "t.json")
    r = autotune.tune_batch(fake, None, [0, 100, 200], None, cache_path=path, sync=lambda: None)
    assert r["tuning"] == {"front_cap": 512, "xcd_queues": 1, "largest_first": 1}
    assert not r["cached"]
    assert len(r["trials"]) == 3 * 2 * 2
    assert fake.t == r["tuning"]
    data = json.load(open(path))
    assert data[autotune.size_class([0, 100, 200])]["tuning"] == r["tuning"]
    # second call: served from the cache, nothing run, settings applied
    runs = fake.runs
    fake.t = {}
    r2 = autotune.tune_batch(fake, None, [0, 100, 200], None, cache_path=path, sync=lambda: None)
    assert r2["cached"] and fake.runs == runs and fake.t == r["tuning"]


def test_corrupt_cache_is_ignored(fake, tmp_path):
    path = tmp_path / "t.json"
    path.write_text("{not json")
    r = autotune.tune_batch(fake, None, [0, 64], None, cache_path=str(path), sync=lambda: None,
                            space={"front_cap": [1024], "xcd_queues": [1], "largest_first": [0, 1]})
    assert r["tuning"]["largest_first"] == 1
