"""Scheduler logic of the serving loop, on the CPU with a simulated clock and
a fake executor (no GPU): admission by footprint, FIFO order, continuous
batching over slots, budget accounting, rejection, failure isolation and the
latency statistics."""
import pytest

from paper_2012_06012_amd.serve import Request, Server, Stats

ERANGE, ECANCELED = -2, -6


class Clock:
    def __init__(self):
        self.t = 0.0

    def now(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class FakeExecutor:
    """Service time = fixed + per-cell; marks `bad` request ids as invalid:
    the bad item fails and the rest of its batch is cancelled."""

    def __init__(self, clock, fixed=1e-3, per_cell=1e-9, bad=()):
        self.clock = clock
        self.fixed = fixed
        self.per_cell = per_cell
        self.bad = set(bad)
        self.log = []  # (slot, t_submit, t_done, rids)

    def footprint(self, r):
        r.nnz = r.mat
        return 100 * r.mat

    def submit(self, batch, slot):
        t = self.clock.now()
        done = t + self.fixed + self.per_cell * sum(r.mat for r in batch)
        self.log.append((slot, t, done, [r.rid for r in batch]))
        if any(r.rid in self.bad for r in batch):
            st = [ERANGE if r.rid in self.bad else ECANCELED for r in batch]
        else:
            st = [0] * len(batch)
        return (done, st)

    def poll(self, h):
        return self.clock.now() >= h[0]

    def finish(self, h):
        return h[1]


def _reqs(sizes, arrivals):
    return [Request(rid=i, mat=s, arrival=a) for i, (s, a) in enumerate(zip(sizes, arrivals))]


def test_all_complete_and_latency_stats():
    c = Clock()
    ex = FakeExecutor(c)
    reqs = _reqs([10**6] * 20, [i * 1e-3 for i in range(20)])
    st = Server(ex, budget_bytes=10**12, n_slots=2, clock=c.now, sleep=c.sleep).run(reqs)
    assert st.completed == 20 and st.rejected == 0 and st.failed == 0
    assert all(r.status == 0 and r.latency >= 1e-3 for r in reqs)
    assert st.percentile(50) <= st.percentile(99)
    assert st.cells == 20 * 10**6 and st.cells_per_s > 0


def test_budget_never_exceeded_and_fifo_admission():
    c = Clock()
    ex = FakeExecutor(c, fixed=5e-3)
    sizes = [800, 100, 700, 100, 300, 900]  # footprints 100x
    reqs = _reqs(sizes, [0.0] * 6)
    st = Server(ex, budget_bytes=100_000, n_slots=3, clock=c.now, sleep=c.sleep).run(reqs)
    assert st.completed == 6
    assert st.max_inflight_bytes <= 100_000
    admits = [r.admit_t for r in reqs]
    assert admits == sorted(admits)  # FIFO: nobody admitted before an earlier arrival


def test_over_budget_rejected():
    c = Clock()
    reqs = _reqs([10, 10**9, 10], [0.0, 0.0, 0.0])
    st = Server(FakeExecutor(c), budget_bytes=10**6, clock=c.now, sleep=c.sleep).run(reqs)
    assert st.rejected == 1 and reqs[1].rejected and st.completed == 2


def test_continuous_batching_overlaps_slots():
    c = Clock()
    ex = FakeExecutor(c, fixed=10e-3)
    # first request starts a long batch; later arrivals must start on the other slot
    reqs = _reqs([10] * 6, [0.0, 1e-3, 1.5e-3, 2e-3, 2.5e-3, 30e-3])
    st = Server(ex, budget_bytes=10**9, n_slots=2, max_batch=8, clock=c.now,
                sleep=c.sleep).run(reqs)
    assert st.completed == 6
    (s0, t0, d0, r0), (s1, t1, d1, r1) = ex.log[0], ex.log[1]
    assert s0 != s1 and t1 < d0          # second batch submitted while the first ran
    assert r0 == [0] and set(r1) >= {1}  # arrivals joined the next submit
    assert len(ex.log) <= 4              # batched, not one submit per request


def test_failure_isolation_resubmits_cancelled():
    c = Clock()
    ex = FakeExecutor(c, fixed=2e-3, bad={3})
    reqs = _reqs([10] * 8, [0.0] * 8)
    st = Server(ex, budget_bytes=10**9, n_slots=1, max_batch=8, clock=c.now,
                sleep=c.sleep).run(reqs)
    assert reqs[3].status == ERANGE and st.failed == 1
    assert st.completed == 7 and st.resubmits == 7
    assert all(r.status == 0 for i, r in enumerate(reqs) if i != 3)


def test_stats_percentiles():
    s = Stats(latencies=[float(i) for i in range(1, 101)])
    assert s.percentile(50) == 50.0 and s.percentile(99) == 99.0


def test_batches_respect_the_executors_cell_cap():
    clock = Clock()
    ex = FakeExecutor(clock)
    ex.max_batch_cells = 250
    reqs = _reqs([100, 100, 100, 400, 50, 50], [0.0] * 6)
    st = Server(ex, 10 ** 9, max_batch=8, n_slots=1, clock=clock.now, sleep=clock.sleep).run(reqs)
    assert st.completed == 6
    assert [rids for _, _, _, rids in ex.log] == [[0, 1], [2], [3], [4, 5]]
