"""Host logic of the autotuner, on stand-in jobs and batches (no device):
which jobs offer a choice of lanes per wheel, that the fastest lanes and
block are chosen and set, and that a cached choice is applied again."""
from paper_0704_3573_amd import autotune
from paper_0704_3573_amd import binding as B


class FakeJob:
    def __init__(self, model, L, NW=64, C=4):
        self.model, self.algo, self.L, self.NW, self.C = model, B.HEATBATH, L, NW, C
        self.lanes = 8 if model in (B.POTTS, B.GPOTTS) and L == 16 else 1

    def set_wheel_lanes(self, lanes, stream=None):
        self.lanes = lanes


class FakeBatch:
    """Launch time = a per-lanes cost + a per-block cost (ms)."""

    def __init__(self, jobs, lane_ms, block_ms):
        self.jobs, self.lane_ms, self.block_ms = jobs, lane_ms, block_ms
        self._block, self.timing, self.runs = 0, False, 0

    def set_timing(self, on):
        self.timing = on

    def set_block(self, b):
        self._block = b

    def block(self):
        return self._block or 512

    def run(self, n, stream=None):
        self.runs += 1

    def sweep_ms(self):
        lanes = {j.lanes for j in self.jobs if j.lanes > 1}
        lane = self.lane_ms[lanes.pop()] if lanes else 0.0
        return lane + self.block_ms.get(self._block, 1.0)


def test_lane_choices_only_for_potts_at_16():
    jobs = [FakeJob(B.ISING, 16), FakeJob(B.POTTS, 32), FakeJob(B.GPOTTS, 16), FakeJob(B.POTTS, 16)]
    js, choices = autotune.lane_choices(jobs)
    assert js == jobs[2:] and choices == [8, 4]
    assert autotune.lane_choices(jobs[:2]) == ([], [])


def test_tune_picks_fastest_lanes_and_block_and_caches(tmp_path):
    path = str(tmp_path / "tune.json")
    jobs = [FakeJob(B.POTTS, 16), FakeJob(B.ISING, 16)]
    blocks = {b: 1.0 for b in autotune.candidates(jobs)}
    blocks[768] = 0.5
    batch = FakeBatch(jobs, {8: 2.0, 4: 1.0}, blocks)
    block, times = autotune.tune(batch, 10, periods=1, cache_path=path)
    assert block == 768 and batch._block == 768 and not batch.timing
    assert jobs[0].lanes == 4 and jobs[1].lanes == 1
    assert set(times) == set(blocks)
    # a new batch of the same signature takes the cached choice without timing
    jobs2 = [FakeJob(B.POTTS, 16), FakeJob(B.ISING, 16)]
    batch2 = FakeBatch(jobs2, {8: 0.1, 4: 9.0}, {})
    block2, _ = autotune.tune(batch2, 10, periods=1, cache_path=path)
    assert block2 == 768 and batch2._block == 768 and batch2.runs == 0
    assert jobs2[0].lanes == 4


def test_tune_without_lane_choice_keeps_lanes(tmp_path):
    jobs = [FakeJob(B.ISING, 32)]
    blocks = {b: 1.0 + b / 1e4 for b in autotune.candidates(jobs)}
    batch = FakeBatch(jobs, {}, blocks)
    block, _ = autotune.tune(batch, 10, periods=1, use_cache=False)
    assert block == min(blocks) and jobs[0].lanes == 1
