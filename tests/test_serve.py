"""The serving scheduler on the CPU with a fake executor: results, admission
by memory and slots, coalescing, splitting, and the arrival generator."""
import numpy as np
import pytest

from paper_1503_07192_amd import serve


class FakeClock:
    def __init__(self, dt=1e-4):
        self.t, self.dt = 0.0, dt

    def __call__(self):
        self.t += self.dt
        return self.t


class FakeExecutor:
    """Answers f(v1, v2) = 7*v1 + v2 after a delay proportional to the size."""

    def __init__(self, clock, slots, per_pair=1e-6, fixed=5e-4):
        self.clock, self.per_pair, self.fixed = clock, per_pair, fixed
        self.active = set()
        self.max_active = 0
        self.sched = None
        self.max_mem = 0
        self.regions = {}   # slot -> (offset, bytes) of its launch's buffers

    def submit(self, slot, v1, v2, off):
        assert slot not in self.active
        # the launch's buffers lie inside the pool and overlap no running launch
        lo, hi = off, off + 12 * len(v1)
        assert 0 <= lo and hi <= self.sched.arena.size
        for a, b in self.regions.values():
            assert hi <= a or b <= lo
        self.regions[slot] = (lo, hi)
        self.active.add(slot)
        self.max_active = max(self.max_active, len(self.active))
        self.max_mem = max(self.max_mem, sum(b - a for a, b in self.regions.values()))
        ready = self.clock.t + self.fixed + self.per_pair * len(v1)
        return [slot, ready, (7 * v1.astype(np.int64) + v2).astype(np.int32)]

    def done(self, h):
        if self.clock.t >= h[1]:
            self.active.discard(h[0])
            self.regions.pop(h[0], None)
            return True
        return False

    def result(self, h):
        return h[2]


def make(nreq=300, rate=2e6, seed=0, n=1000, max_log2=12.0):
    rng = np.random.default_rng(seed)
    return serve.poisson_stream(rng, rate, nreq, n, max_log2=max_log2)


def run(reqs, slots=3, slot_pairs=4096, mem=10**6):
    clock = FakeClock()
    ex = FakeExecutor(clock, slots)
    sched = serve.Scheduler(ex, slots, slot_pairs, mem)
    ex.sched = sched
    done = serve.run_stream(sched, reqs, clock=clock)
    return sched, ex, done


def test_every_request_gets_its_own_answers():
    reqs = make()
    sched, ex, done = run(reqs)
    assert len(done) == len(reqs)
    for r in reqs:
        assert np.array_equal(r.result, 7 * r.v1 + r.v2)
        assert r.done_at >= r.arrival
    assert ex.max_active <= 3


def test_memory_budget_and_slots_respected_with_splitting():
    reqs = make(nreq=200, max_log2=12.0)
    budget = 12 * 1500          # smaller than many requests: they get cut
    reqs = [r for r in reqs if r.size <= 1500]
    sched, ex, done = run(reqs, slots=2, slot_pairs=2048, mem=budget)
    assert ex.max_mem <= budget
    assert ex.max_active <= 2
    for r in reqs:
        assert np.array_equal(r.result, 7 * r.v1 + r.v2)


def test_requests_split_when_memory_is_short():
    rng = np.random.default_rng(1)
    reqs = [serve.Request(i, 0.0, rng.integers(0, 50, 1000).astype(np.int32),
                          rng.integers(0, 50, 1000).astype(np.int32)) for i in range(4)]
    sched, ex, done = run(reqs, slots=4, slot_pairs=1000, mem=12 * 1600)
    assert any(len(r.launches) > 1 for r in reqs)
    for r in reqs:
        assert np.array_equal(r.result, 7 * r.v1 + r.v2)


def test_small_requests_are_coalesced():
    rng = np.random.default_rng(2)
    reqs = [serve.Request(i, 0.0, rng.integers(0, 9, 10).astype(np.int32),
                          rng.integers(0, 9, 10).astype(np.int32)) for i in range(50)]
    sched, ex, done = run(reqs, slots=1, slot_pairs=4096)
    assert sched.launches < 50
    assert max(sched.launch_sizes) > 10
    for r in reqs:
        assert np.array_equal(r.result, 7 * r.v1 + r.v2)


def test_request_larger_than_a_slot_is_served_in_pieces():
    rng = np.random.default_rng(4)
    r = serve.Request(0, 0.0, rng.integers(0, 99, 5000).astype(np.int32),
                      rng.integers(0, 99, 5000).astype(np.int32))
    sched, ex, done = run([r], slots=2, slot_pairs=1024, mem=10**6)
    assert len(r.launches) == 5 and done == [r]
    assert np.array_equal(r.result, 7 * r.v1 + r.v2)
    with pytest.raises(ValueError):
        serve.Scheduler(ex, 1, 16, 4)


def test_arena_first_fit_free_and_merge():
    a = serve.Arena(10 * 256 + 100)
    assert a.size == 2560 and a.largest() == 2560
    x = a.alloc(1)          # one 256-byte unit
    y = a.alloc(600)        # three units
    z = a.alloc(256)
    assert (x, y, z) == (0, 256, 1024) and a.used == 5 * 256
    assert a.alloc(6 * 256) is None and a.largest() == 5 * 256
    a.free(y)
    assert a.largest() == 5 * 256 and a.alloc(3 * 256) == 256   # first fit reuses the hole
    a.free(256)
    a.free(x)
    a.free(z)
    assert a.used == 0 and a.holes == [(0, 2560)]
    assert a.alloc(2560) == 0 and a.alloc(1) is None


def test_admission_waits_for_pool_memory():
    """A launch is admitted only when its buffers fit in the pool: with room
    for one 1,000-pair launch, four requests run one after another."""
    rng = np.random.default_rng(5)
    reqs = [serve.Request(i, 0.0, rng.integers(0, 50, 1000).astype(np.int32),
                          rng.integers(0, 50, 1000).astype(np.int32)) for i in range(4)]
    sched, ex, done = run(reqs, slots=4, slot_pairs=1000, mem=12 * 1000 + 255)
    assert ex.max_active == 1 and ex.max_mem <= 12 * 1000
    for r in reqs:
        assert np.array_equal(r.result, 7 * r.v1 + r.v2)


def test_poisson_stream_shape():
    rng = np.random.default_rng(3)
    reqs = serve.poisson_stream(rng, 1e6, 4000, 100)
    sizes = np.array([r.size for r in reqs])
    assert sizes.min() >= 1 and sizes.max() <= 65536
    mean_b = (2.0**16 - 1) / (16 * np.log(2))
    assert abs(sizes.mean() / mean_b - 1) < 0.1
    t = np.array([r.arrival for r in reqs])
    assert (np.diff(t) >= 0).all()
    rate_req = len(reqs) / t[-1]
    assert abs(rate_req / (1e6 / mean_b) - 1) < 0.1


def test_autotune_cache_lookup(tmp_path, monkeypatch):
    from paper_1503_07192_amd import autotune
    monkeypatch.setattr(autotune, "device_key", lambda: "gfx950")
    path = tmp_path / "tune.json"
    key = autotune.size_key(65536, 163066, 1024, 0)
    path.write_text('{"gfx950": {"%s": {"best": {"bg_method": 2, "group_comps": 32}}}}' % key)
    assert autotune.lookup(str(path), 65536, 163066, 1024, 0) == {"bg_method": 2, "group_comps": 32}
    assert autotune.lookup(str(path), 1024, 1984, 16, 0) == {}
    assert autotune.lookup(str(tmp_path / "missing.json"), 1, 1, 1) == {}
    c = autotune.candidates(27900, 1024, 0)
    assert {"bg_method": 1, "bg_tile": 128, "inner_kc": 16, "bg_pivot": 256} in c
    assert {"bg_method": 1, "bg_tile": 64, "inner_kc": 32, "bg_pivot": 256} in c
    assert all(o["bg_method"] == 2 for o in autotune.candidates(255422, 4096, 0))


def test_poisson_stream_sources():
    """v1 drawn from a share's vertex list when one is given, v2 from all."""
    import numpy as np
    from paper_1503_07192_amd import serve as SV
    rng = np.random.default_rng(3)
    src = np.array([5, 17, 40], np.int32)
    reqs = SV.poisson_stream(rng, 1e6, 50, 100, max_log2=8.0, sources=src)
    v1 = np.concatenate([r.v1 for r in reqs])
    v2 = np.concatenate([r.v2 for r in reqs])
    assert set(np.unique(v1)) <= set(src.tolist()) and len(np.unique(v1)) == 3
    assert v2.min() >= 0 and v2.max() < 100 and len(np.unique(v2)) > 50
    assert all(r.v1.dtype == np.int32 and len(r.v1) == len(r.v2) >= 1 for r in reqs)
