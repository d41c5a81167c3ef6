"""Autotuner logic on the host (no GPU): coordinate descent and the JSON cache,
driven by a mock handle whose step time is a known function of the tuning."""

import json

import pytest

torch = pytest.importorskip("torch")

from paper_2310_16122_amd import tune  # noqa: E402


class MockLeaves:
    """Step time = sum of per-field penalties; the optimum is known."""

    BEST = {"persistent": 0, "waves_per_cu": 16, "kahan_chunk": 4, "block_waves": 4,
            "xcd_groups": 8, "tile_order": 0, "stage16": 1}

    def __init__(self):
        self.t = {"persistent": 1, "waves_per_cu": 32, "kahan_chunk": 1, "block_waves": 1,
                  "xcd_groups": 1, "tile_order": 1, "stage16": 0}
        self.timing_on = False
        self.sets = 0

    def get_tuning(self):
        return dict(self.t)

    def set_tuning(self, **kw):
        self.sets += 1
        self.t.update(kw)

    def timing(self, on=True):
        self.timing_on = on

    def cost(self):
        c = 1.0
        for k, v in self.BEST.items():
            if self.t[k] != v and not (k == "waves_per_cu" and not self.t["persistent"]):
                c += {"tile_order": 4.0, "xcd_groups": 1.0, "persistent": 2.0}.get(k, 0.5)
        return c

    def kernel_times(self):
        return {"accel": (self.cost() * self._steps, self._steps)}

    def step_factory(self):
        self._steps = 0

        def step():
            self._steps += 1
        return step


def run(leaves, **kw):
    step = leaves.step_factory()

    def counting_step():
        step()
    # kernel_times reports cost x number of steps run since timing(True)
    orig = leaves.timing

    def timing(on=True):
        leaves._steps = 0
        orig(on)
    leaves.timing = timing
    return tune.autotune(leaves, counting_step, **kw)


def test_coordinate_descent_finds_the_optimum():
    L = MockLeaves()
    best, ms, tried = run(L, repeats=2)
    for k, v in MockLeaves.BEST.items():
        if k == "waves_per_cu":
            continue
        assert best[k] == v, (k, best)
    assert ms == pytest.approx(1.0)
    assert L.get_tuning() == best
    assert len(tried) > 5


def test_cache_is_written_and_reused(tmp_path):
    path = str(tmp_path / "tune.json")
    L = MockLeaves()
    best, ms, tried = run(L, repeats=1, cache_path=path, key="k1")
    data = json.load(open(path))
    assert data["k1"]["tuning"] == best
    L2 = MockLeaves()
    best2, ms2, tried2 = run(L2, repeats=1, cache_path=path, key="k1")
    assert tried2 == [] and best2 == best and L2.get_tuning()["tile_order"] == best["tile_order"]
