"""Serving policy on a virtual clock with a fake executor (no GPU):
admission by memory, batching of one geometry, FIFO with bounded backfill,
LRU eviction of idle spectra, rejection, timeouts and cancellation."""

import pytest

from paper_2005_10160_amd.serve import GeometryKey, Request, Scheduler, io_bytes, spectra_bytes


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    """Each launch takes `cost(key, op, models)` virtual seconds."""

    elem = 4

    def __init__(self, clock, cost=lambda k, op, b: 0.010, build=0.0):
        self.clock = clock
        self.cost = cost
        self.build = build            # virtual seconds to build a key's spectra
        self.busy = {}
        self.launched = []
        self.evicted = []
        self.built = {}               # key -> virtual time its spectra are ready
        self.prepared = []

    def prepare(self, key):
        self.prepared.append(key)
        self.built[key] = self.clock() + self.build

    def ready(self, key):
        return self.clock() >= self.built[key]

    def workspace_bytes(self, key, op, batch):
        return 1000 * batch

    def is_resident(self, key):
        return True

    def evict(self, key):
        self.evicted.append(key)
        self.built.pop(key, None)

    def launch(self, slot, reqs):
        models = sum(r.batch for r in reqs)
        self.busy[slot] = self.clock() + self.cost(reqs[0].key, reqs[0].op, models)
        self.launched.append((slot, [r.rid for r in reqs]))

    def poll(self, slot):
        return self.clock() >= self.busy.get(slot, 0.0)


def key(n=64, nz=16, comps=0x3F):
    return GeometryKey(n, n, nz, 20.0, 20.0, 20.0, 10.0, comps)


def req(rid, k, t, batch=1, op="forward"):
    return Request(rid, k, op, batch, t)


def run_until_idle(s, clock, dt=0.001, limit=100.0):
    while not s.idle() and clock.t < limit:
        s.step()
        clock.t += dt
    s.step()


def test_spectra_bytes_matches_quarter_plane():
    k = key(1024, 100, 0x3F)
    assert spectra_bytes(k, 4) == 6 * 100 * 1025 * 1025 * 4
    # gzz alone keeps gxx and gyy resident
    assert spectra_bytes(key(16, 8, 0x40), 8) == 2 * 8 * 17 * 17 * 8


def test_same_geometry_requests_are_batched():
    clock = Clock()
    ex = FakeExecutor(clock)
    s = Scheduler(ex, budget_bytes=1 << 40, n_slots=1, max_models=8, clock=clock)
    k = key()
    rs = [req(i, k, 0.0, batch=3) for i in range(4)]
    for r in rs:
        s.submit(r)
    s.step()
    # 3 + 3 fit in 8 models; the third request would exceed it
    assert ex.launched == [(0, [0, 1])]
    run_until_idle(s, clock)
    assert [l[1] for l in ex.launched] == [[0, 1], [2, 3]]
    assert all(r.status == "done" for r in rs)


def test_arrivals_during_work_use_free_slots():
    """Continuous batching: a request arriving while another runs is started
    on a free slot at once, without waiting for the first to finish."""
    clock = Clock()
    ex = FakeExecutor(clock, cost=lambda k, op, b: 1.0)
    s = Scheduler(ex, budget_bytes=1 << 40, n_slots=2, clock=clock)
    a = req(0, key(64), 0.0)
    s.submit(a)
    s.step()
    clock.t = 0.1
    b = req(1, key(128), 0.1)
    s.submit(b)
    s.step()
    assert [l[0] for l in ex.launched] == [0, 1]
    assert a.status == b.status == "running"
    clock.t = 1.2
    s.step()
    assert a.status == b.status == "done"
    assert a.latency == pytest.approx(1.2) and b.latency == pytest.approx(1.1)


def test_fifo_across_geometries():
    clock = Clock()
    ex = FakeExecutor(clock)
    s = Scheduler(ex, budget_bytes=1 << 40, n_slots=1, clock=clock)
    order = [(0, key(64)), (1, key(128)), (2, key(64)), (3, key(256))]
    for rid, k in order:
        s.submit(req(rid, k, rid * 1e-4))
    clock.t = 1e-3
    run_until_idle(s, clock)
    # the key of the oldest request goes first, taking its later same-key request along
    assert [l[1] for l in ex.launched] == [[0, 2], [1], [3]]


def test_admission_waits_for_memory_and_backfills_then_stops():
    clock = Clock()
    ex = FakeExecutor(clock, cost=lambda k, op, b: 1.0)
    big, small = key(256, 64, 0x3F), key(64, 16, 0x1)
    budget = (io_bytes(big, "forward", 1, 4) + 1000 + spectra_bytes(big, 4)) + 10
    s = Scheduler(ex, budget_bytes=budget, n_slots=3, backfill_limit=0.5, clock=clock)
    first = req(0, big, 0.0)
    s.submit(first)
    s.step()
    assert first.status == "running"
    second = req(1, big, 0.01)      # does not fit while `first` holds memory
    tiny = req(2, small, 0.02)      # small: may pass while `second` waited < 0.5 s
    clock.t = 0.02
    s.submit(second)
    s.submit(tiny)
    s.step()
    assert second.status == "pending"
    # tiny needs its own spectra: only if they fit beside first
    fits = s.free_bytes() >= io_bytes(small, "forward", 1, 4) + 1000 + spectra_bytes(small, 4)
    assert tiny.status == ("running" if fits else "pending")
    clock.t = 0.7                    # second has now waited > backfill limit
    late = req(3, small, 0.7)
    s.submit(late)
    s.step()
    assert late.status == "pending"  # no more backfilling past the starving request
    run_until_idle(s, clock)
    assert first.status == second.status == late.status == "done"
    assert second.t_admit < late.t_admit


def test_idle_spectra_are_evicted_lru():
    clock = Clock()
    ex = FakeExecutor(clock)
    ks = [key(64 * (i + 1), 16, 0x3F) for i in range(3)]
    # room for the spectra of the two largest geometries plus one launch of
    # the largest, but not for all three spectra
    budget = spectra_bytes(ks[1], 4) + spectra_bytes(ks[2], 4) + io_bytes(ks[2], "forward", 1, 4) + 1000
    s = Scheduler(ex, budget_bytes=budget, n_slots=1, clock=clock)
    for i, k in enumerate(ks):
        s.submit(req(i, k, i * 1e-3))
        clock.t = i * 1e-3
        run_until_idle(s, clock)
    assert ex.evicted == [ks[0]]        # least recently used goes first, and only it
    assert ks[1] in s.resident and ks[2] in s.resident
    s.submit(req(9, ks[2], clock.t))
    run_until_idle(s, clock)
    assert s.stats["spectra_hit"] >= 1


def test_never_fitting_request_is_rejected_at_once():
    clock = Clock()
    ex = FakeExecutor(clock)
    s = Scheduler(ex, budget_bytes=10_000, n_slots=1, clock=clock)
    r = req(0, key(512, 128), 0.0)
    assert not s.submit(r)
    assert r.status == "rejected" and "budget" in r.error
    too_many = req(1, key(16, 4), 0.0, batch=1000)
    assert not s.submit(too_many)


def test_admission_timeout_and_cancel():
    clock = Clock()
    ex = FakeExecutor(clock, cost=lambda k, op, b: 10.0)
    s = Scheduler(ex, budget_bytes=1 << 40, n_slots=1, admit_timeout=1.0, clock=clock)
    a, b, c = req(0, key(64), 0.0), req(1, key(128), 0.0), req(2, key(256), 0.0)
    for r in (a, b, c):
        s.submit(r)
    s.step()
    assert a.status == "running"
    assert s.cancel(c) and c.status == "cancelled"
    assert not s.cancel(a)               # running requests cannot be cancelled
    clock.t = 2.0
    s.step()
    assert b.status == "rejected" and "not admitted" in b.error
    clock.t = 10.5
    run_until_idle(s, clock)
    assert a.status == "done"


def test_failed_launch_rejects_its_group_only():
    clock = Clock()

    class Failing(FakeExecutor):
        def launch(self, slot, reqs):
            if reqs[0].key.nx == 128:
                raise RuntimeError("boom")
            super().launch(slot, reqs)

    ex = Failing(clock)
    s = Scheduler(ex, budget_bytes=1 << 40, n_slots=2, clock=clock)
    bad, good = req(0, key(128), 0.0), req(1, key(64), 0.0)
    s.submit(bad)
    s.submit(good)
    run_until_idle(s, clock)
    assert bad.status == "rejected" and "boom" in bad.error
    assert good.status == "done"
    assert s.in_use == 0


def test_level_and_layered_keys():
    """Keys of observation-level plans carry one data plane per level and
    spectra for nz + levels - 1 layer offsets; gx and gy each add a
    spectrum, gzz none beyond gxx and gyy."""
    k = GeometryKey(32, 48, 10, 20.0, 20.0, 20.0, 10.0, 0x1, None, 4)
    assert k.data_shape == (4, 1, 48, 32)
    assert spectra_bytes(k, 4) == 1 * 13 * 33 * 65 * 4     # circulants 64 x 128
    assert io_bytes(k, "forward", 2, 4) == 2 * (10 * 32 * 48 + 4 * 32 * 48) * 4
    one = GeometryKey(32, 48, 10, 20.0, 20.0, 20.0, 10.0, 0x1FF)
    assert one.data_shape == (9, 48, 32) and one.n_spec == 8
    assert GeometryKey(16, 16, 2, 1.0, 1.0, 1.0, 1.0, 0x40).n_spec == 2
    assert GeometryKey(16, 16, 2, 1.0, 1.0, 1.0, 1.0, 0x180).n_spec == 2
    lay = GeometryKey(16, 16, 2, 1.0, 1.0, 1.0, 1.0, 0x1, (0.0, 1.0, 3.0))
    assert lay != GeometryKey(16, 16, 2, 1.0, 1.0, 1.0, 1.0, 0x1, (0.0, 1.0, 4.0))
    assert lay != GeometryKey(16, 16, 2, 1.0, 1.0, 1.0, 1.0, 0x1)


def test_hit_is_admitted_while_a_miss_builds_its_spectra():
    """A request whose spectra are not resident starts their build and waits
    for it off the scheduling loop: a later request of a resident geometry
    is admitted and finishes meanwhile, and the first is admitted as soon
    as its spectra are ready.  Each request records whether it was a hit."""
    clock = Clock()
    ex = FakeExecutor(clock, cost=lambda k, op, b: 0.010, build=0.5)
    s = Scheduler(ex, budget_bytes=1 << 40, n_slots=2, clock=clock)
    warm = key(64)
    s.submit(req(0, warm, 0.0))
    run_until_idle(s, clock)                 # warm's spectra are now resident
    t1 = clock.t
    cold = req(1, key(256), t1)
    s.submit(cold)
    s.step()
    assert ex.prepared[-1] == key(256) and cold.status == "pending"
    clock.t = t1 + 0.05
    hit = req(2, warm, clock.t)
    s.submit(hit)
    s.step()
    assert hit.status == "running" and cold.status == "pending"
    clock.t = t1 + 0.1
    s.step()
    assert hit.status == "done" and cold.status == "pending"
    clock.t = t1 + 0.51
    s.step()
    assert cold.status == "running" and cold.t_admit == pytest.approx(t1 + 0.51)
    run_until_idle(s, clock)
    assert cold.status == "done"
    assert (cold.cache, hit.cache) == ("miss", "hit")
    assert s.stats["spectra_miss"] == 2 and s.stats["spectra_hit"] == 1 and s.stats["launch_after_build"] == 2


def test_requests_arriving_during_a_build_are_misses_and_batched():
    """Requests of a geometry whose spectra are being built wait for that one
    build (no second build starts) and are then launched together."""
    clock = Clock()
    ex = FakeExecutor(clock, build=0.3)
    s = Scheduler(ex, budget_bytes=1 << 40, n_slots=1, max_models=8, clock=clock)
    k = key(128)
    a = req(0, k, 0.0)
    s.submit(a)
    s.step()
    clock.t = 0.1
    b = req(1, k, 0.1)
    s.submit(b)
    s.step()
    assert ex.prepared == [k] and a.status == b.status == "pending"
    clock.t = 0.31
    s.step()
    assert ex.launched[-1][1] == [0, 1]
    assert a.cache == b.cache == "miss"


def test_failed_build_rejects_that_geometry_only():
    clock = Clock()

    class BadBuild(FakeExecutor):
        def ready(self, key):
            if key.nx == 128:
                raise RuntimeError("no memory for spectra")
            return super().ready(key)

    ex = BadBuild(clock)
    s = Scheduler(ex, budget_bytes=1 << 40, n_slots=2, clock=clock)
    bad, good = req(0, key(128), 0.0), req(1, key(64), 0.0)
    s.submit(bad)
    s.submit(good)
    run_until_idle(s, clock)
    assert bad.status == "rejected" and "spectra build failed" in bad.error
    assert good.status == "done"
    assert key(128) not in s.resident and not s.building


def test_failed_launch_drops_the_resident_spectra():
    """After a launch fails, its geometry's spectra are not counted as
    resident: the next request of that geometry is a miss and rebuilds."""
    clock = Clock()

    class FailOnce(FakeExecutor):
        failed = False

        def launch(self, slot, reqs):
            if not self.failed:
                self.failed = True
                raise RuntimeError("boom")
            super().launch(slot, reqs)

    ex = FailOnce(clock)
    s = Scheduler(ex, budget_bytes=1 << 40, n_slots=1, clock=clock)
    k = key(64)
    first = req(0, k, 0.0)
    s.submit(first)
    run_until_idle(s, clock)
    assert first.status == "rejected" and k not in s.resident and ex.evicted == [k]
    second = req(1, k, clock.t)
    s.submit(second)
    assert second.cache == "miss"
    run_until_idle(s, clock)
    assert second.status == "done" and ex.prepared == [k, k]


def test_input_bank_is_bounded_and_seeded_per_request():
    """The served replay's host inputs: one buffer of the largest request
    plus a fixed slack, whatever the trace's length; each request's window
    depends on its own seed only, so requests differ from one another and a
    request is the same on every replay."""
    import numpy as np
    from paper_2005_10160_amd.serve import InputBank, request_shape
    from synth import poisson_trace
    trace = poisson_trace(n_requests=300, rate=200.0, seed=500, n_choices=(16, 32), nz_choices=(4, 8))
    bank = InputBank(trace, "f32", pin=False, slack=1 << 16)
    largest = max(int(np.prod(request_shape(tr))) for tr in trace)
    assert bank.nbytes == 4 * (largest + (1 << 16))
    again = InputBank(trace[:50], "f32", pin=False, slack=1 << 16)
    for tr in trace[:50]:
        x = bank.get(tr)
        assert tuple(x.shape) == request_shape(tr)
        assert float(x.abs().max()) <= 500.0
        if again.largest == bank.largest:
            assert bool((again.get(tr) == x).all())
    offsets = [bank.offset(tr) for tr in trace]
    assert len(set(offsets)) > 0.95 * len(offsets)


def test_latency_summary_splits_hits_and_misses():
    from paper_2005_10160_amd.serve import latency_summary
    recs = [{"status": "done", "cache": "hit", "latency_ms": float(v)} for v in range(1, 101)]
    recs += [{"status": "done", "cache": "miss", "latency_ms": 1000.0 + v} for v in range(10)]
    recs += [{"status": "rejected", "cache": "miss", "latency_ms": None}]
    s = latency_summary(recs)
    assert (s["all"]["n"], s["hit"]["n"], s["miss"]["n"]) == (110, 100, 10)
    assert s["hit"]["p50_ms"] == pytest.approx(50.5) and s["miss"]["p50_ms"] == pytest.approx(1004.5)


def test_latency_summary_device_figures():
    from paper_2005_10160_amd.serve import latency_summary
    recs = [{"status": "done", "cache": "hit", "latency_ms": 10.0 + v, "device_ms": 2.0 + v, "compute_ms": 1.0}
            for v in range(100)]
    recs += [{"status": "rejected", "cache": "miss", "latency_ms": None, "device_ms": None, "compute_ms": None}]
    s = latency_summary(recs)
    assert s["all"]["device_p50_ms"] == pytest.approx(51.5)
    assert s["all"]["compute_p99_ms"] == pytest.approx(1.0)
    # records without device figures (the scheduler's virtual clock) give none
    s = latency_summary([{"status": "done", "cache": "hit", "latency_ms": 1.0}])
    assert "device_p50_ms" not in s["all"]
