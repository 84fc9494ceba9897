"""Host logic of the serving loop (arena, admission, continuous batching,
latency accounting) against a fake executor on a virtual clock, with the real
library's workspace sizes."""
import numpy as np
import pytest

from paper_2107_11627_amd import serving as sv


@pytest.fixture(scope="module")
def p2s():
    from paper_2107_11627_amd import p2s as mod
    mod.lib()
    return mod


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


def make(p2s, budget, n_slots=2, max_frames=8, us_per_mpix=1000.0, launch_s=0.0):
    clk = Clock()

    def ws(shapes):
        return p2s.batch_workspace_bytes(shapes, 35, 100)

    def cost(shapes):
        return launch_s + sum(c * h * w for c, h, w in shapes) / 1e6 * us_per_mpix * 1e-6

    ex = sv.FakeExecutor(clk, cost, ws)
    eng = sv.Engine(ex, budget, n_slots=n_slots, max_batch_frames=max_frames, clock=clk)
    return eng, ex, clk


def test_arena_first_fit_and_merge():
    a = sv.Arena(10 * 256 + 17)
    assert a.capacity == 2560
    x = a.alloc(300)            # 512
    y = a.alloc(256)
    z = a.alloc(1000)           # 1024
    assert (x, y, z) == (0, 512, 768)
    assert a.bytes_in_use == 512 + 256 + 1024
    assert a.alloc(1024) is None            # 768 left
    a.release(y)
    assert a.alloc(512) == 1792             # first fit skips the 256-byte hole
    a.release(x)                            # hole [0, 768) after merging x and y
    assert a.free_blocks[0] == (0, 768)
    assert a.alloc(700) == 0
    a.release(0)
    a.release(z)
    a.release(1792)
    assert a.free_blocks == [(0, 2560)] and a.bytes_in_use == 0


def test_all_requests_finish_within_budget(p2s):
    rng = np.random.default_rng(0)
    shapes = [(int(rng.choice([1, 3])), int(rng.choice([64, 128, 256])), int(rng.choice([64, 192]))) for _ in range(60)]
    budget = 6 * p2s.batch_workspace_bytes([(3, 256, 192)], 35, 100)
    eng, ex, clk = make(p2s, budget)
    arr = sv.poisson_arrivals(len(shapes), 2000.0, 1)
    reqs = [sv.Request(i, s, 1.0, i, float(arr[i])) for i, s in enumerate(shapes)]
    st = sv.run(eng, reqs, sleep=clk.sleep)
    assert st["completed"] == 60 and st["rejected"] == 0
    assert st["peak_hbm_bytes"] <= budget
    for r in reqs:
        assert r.finished >= r.admitted >= r.arrival - 1e-12
        assert r.latency > 0
    # first come, first served: batches take queue prefixes
    order = sorted(reqs, key=lambda r: (r.arrival, r.rid))
    assert [r.batch_id for r in order] == sorted(r.batch_id for r in order)
    assert max(eng.batch_sizes) <= 8
    assert st["latency_ms"]["p50"] <= st["latency_ms"]["p99"] <= st["latency_ms"]["max"]


def test_continuous_batching_overlaps(p2s):
    """A request arriving while a batch runs goes out on the second slot
    before the first batch finishes, instead of waiting for it."""
    eng, ex, clk = make(p2s, 1 << 34, n_slots=2, us_per_mpix=10000.0)
    reqs = [sv.Request(0, (3, 512, 512), 1.0, 0, 0.0), sv.Request(1, (1, 128, 128), 1.0, 1, 0.001)]
    sv.run(eng, reqs, sleep=clk.sleep)
    big, small = reqs
    assert small.batch_id != big.batch_id
    assert small.admitted < big.finished
    assert small.finished < big.finished          # the short one is not stuck behind the long one
    assert eng.overlapped_launches == 1
    # with one slot it has to wait
    eng, ex, clk = make(p2s, 1 << 34, n_slots=1, us_per_mpix=10000.0)
    reqs = [sv.Request(0, (3, 512, 512), 1.0, 0, 0.0), sv.Request(1, (1, 128, 128), 1.0, 1, 0.001)]
    sv.run(eng, reqs, sleep=clk.sleep)
    assert reqs[1].admitted >= reqs[0].finished


def test_admission_waits_for_memory_and_rejects_oversize(p2s):
    one = p2s.batch_workspace_bytes([(3, 256, 256)], 35, 100) + 4 * 3 * 256 * 256
    budget = int(1.5 * one)
    eng, ex, clk = make(p2s, budget, n_slots=4)
    reqs = [sv.Request(i, (3, 256, 256), 1.0, i, 0.0) for i in range(3)]
    reqs.append(sv.Request(3, (3, 1024, 1024), 1.0, 3, 0.0))      # never fits
    st = sv.run(eng, reqs, sleep=clk.sleep)
    assert st["rejected"] == 1 and reqs[3].rejected and reqs[3].finished is None
    assert st["completed"] == 3
    assert eng.batches == 3                    # only one frame fits at a time
    assert reqs[1].admitted >= reqs[0].finished and reqs[2].admitted >= reqs[1].finished
    assert st["peak_hbm_bytes"] <= budget


def test_poisson_arrivals():
    a = sv.poisson_arrivals(20000, 500.0, 3)
    assert a[0] == 0.0 and np.all(np.diff(a) >= 0)
    gaps = np.diff(a)
    assert abs(gaps.mean() - 1 / 500.0) < 0.03 / 500.0
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.03


class FlakyExecutor(sv.FakeExecutor):
    """Fake executor whose launches listed in `fail_on` raise `exc` (by launch
    attempt number, from 0)."""

    def __init__(self, *a, fail_on=(), exc=None, **k):
        super().__init__(*a, **k)
        self.attempts = 0
        self.fail_on = set(fail_on)
        self.exc = exc

    def launch(self, reqs, slot, off, nbytes):
        n = self.attempts
        self.attempts += 1
        if n in self.fail_on:
            raise self.exc
        return super().launch(reqs, slot, off, nbytes)


def flaky(p2s, budget, exc, fail_on, max_frames=4):
    clk = Clock()

    def ws(shapes):
        return p2s.batch_workspace_bytes(shapes, 35, 100)

    def cost(shapes):
        return sum(c * h * w for c, h, w in shapes) * 1e-9

    ex = FlakyExecutor(clk, cost, ws, fail_on=fail_on, exc=exc)
    eng = sv.Engine(ex, budget, n_slots=2, max_batch_frames=max_frames, clock=clk)
    return eng, ex, clk


@pytest.mark.parametrize("kind", ["enomem", "launch_error"])
def test_failed_launch_fails_only_its_batch(p2s, kind):
    exc = (p2s.P2SError(p2s.P2S_ENOMEM, "injected: device allocation failed") if kind == "enomem"
           else RuntimeError("injected: kernel launch failed"))
    budget = 4 * p2s.batch_workspace_bytes([(3, 256, 256)], 35, 100)
    eng, ex, clk = flaky(p2s, budget, exc, fail_on={1}, max_frames=1)
    reqs = [sv.Request(i, (3, 256, 256), 1.0, i, 0.0005 * i) for i in range(6)]
    st = sv.run(eng, reqs, sleep=clk.sleep)
    failed = [r for r in reqs if r.failed]
    assert len(failed) == 1 and failed[0].rid == 1
    assert "injected" in failed[0].error and failed[0].finished is None
    assert st["failed"] == 1 and st["failed_batches"] == 1 and st["completed"] == 5
    for r in reqs:
        if not r.failed:
            assert r.finished is not None and r.latency > 0
    # the failed batch's arena block came back, and so did every other one
    assert eng.arena.bytes_in_use == 0 and eng.arena.free_blocks == [(0, eng.arena.capacity)]
    assert eng.idle() and st["peak_hbm_bytes"] <= budget


def test_every_launch_failing_still_ends(p2s):
    budget = 4 * p2s.batch_workspace_bytes([(1, 128, 128)], 35, 100)
    eng, ex, clk = flaky(p2s, budget, RuntimeError("injected"), fail_on=set(range(100)))
    reqs = [sv.Request(i, (1, 128, 128), 1.0, i, 0.0) for i in range(10)]
    st = sv.run(eng, reqs, sleep=clk.sleep)
    assert st["completed"] == 0 and st["failed"] == 10 and st["frames_per_s"] is None
    assert eng.arena.bytes_in_use == 0 and eng.idle()
