"""Scheduler logic of the request server, on the CPU with a simulated device:
admission never exceeds the HBM budget, admission is first-come first-served,
every request completes, batches respect the sample cap, latency is at least
the service time and near it at low load, and queueing grows with load."""
import numpy as np
import pytest

from paper_1909_06374_amd.serving import Backend, Request, Server, make_requests


class SimBackend(Backend):
    """Virtual clock; each slot serves its batch at `rate` sample-iterations/s
    (slots share nothing), plus a fixed launch overhead."""

    def __init__(self, n_slots=2, rate=1e9, overhead=1e-4, bytes_per_sample=80):
        self.n_slots = n_slots
        self.rate = rate
        self.overhead = overhead
        self.bps = bytes_per_sample
        self.t = 0.0
        self.log = []

    def footprint(self, req):
        return self.bps * req.n + 8 * req.iters

    def now(self):
        return self.t

    def idle_wait(self, seconds):
        self.t += max(seconds, 1e-5)

    def launch(self, batch):
        counts = batch.count if batch.count else [r.iters for r in batch.reqs]
        work = sum(r.n * k for r, k in zip(batch.reqs, counts))
        end = self.t + self.overhead + work / self.rate
        self.log.append((batch.bid, batch.slot, self.t, end, [r.rid for r in batch.reqs]))
        return end

    def finished(self, end):
        return end if self.t >= end else None


def _check_common(reqs, st, srv):
    assert st.completed == len(reqs)
    assert st.max_footprint <= srv.budget
    assert all(r.done >= r.launched >= r.admitted >= r.arrival for r in reqs)
    order = sorted(reqs, key=lambda r: (r.arrival, r.rid))
    adm = [r.admitted for r in order]
    assert adm == sorted(adm), "admission must follow arrival order"


def test_low_load_latency_is_service_time():
    be = SimBackend(n_slots=4, rate=1e10)
    reqs = make_requests(rate_hz=20.0, duration_s=2.0, seed=5, k_lo=10, k_hi=14, iters_lo=50, iters_hi=60)
    srv = Server(be, budget_bytes=2**34)
    st = srv.run(reqs)
    _check_common(reqs, st, srv)
    service = np.array([be.overhead + r.n * r.iters / be.rate for r in reqs])
    lat = np.array([r.done - r.arrival for r in reqs])
    assert np.all(lat >= service - 1e-12)
    assert np.median(lat - service) < 1e-3


def test_budget_limits_concurrency_and_is_never_exceeded():
    be = SimBackend(n_slots=8, rate=1e9)
    reqs = [Request(rid=i, n=2**16, iters=10, f_br=0.01, a_low=1.0, a_high=2.0, seed=i, arrival=0.0)
            for i in range(40)]
    budget = 3 * be.footprint(reqs[0]) + 100
    srv = Server(be, budget_bytes=budget)
    st = srv.run(reqs)
    _check_common(reqs, st, srv)
    assert st.max_footprint <= budget
    # never more than 3 requests resident at once
    events = sorted([(r.admitted, 1) for r in reqs] + [(r.done, -1) for r in reqs], key=lambda e: (e[0], e[1]))
    live = 0
    for _, dlt in events:
        live += dlt
        assert live <= 3


def test_sample_cap_and_mixing():
    be = SimBackend(n_slots=1, rate=1e9)
    reqs = make_requests(rate_hz=500.0, duration_s=0.5, seed=6, k_lo=10, k_hi=16)
    srv = Server(be, budget_bytes=2**40, max_batch_samples=2**17)
    st = srv.run(reqs)
    _check_common(reqs, st, srv)
    n_of = {r.rid: r.n for r in reqs}
    for _, _, _, _, rids in be.log:
        assert sum(n_of[i] for i in rids) <= 2**17 or len(rids) == 1
    assert any(len(set(n_of[i] for i in rids)) > 1 for *_, rids in be.log), "batches should mix lengths"


def test_queueing_grows_with_load():
    p99 = []
    for rate in (100.0, 1800.0):  # about 6% and 110% of the simulated capacity
        be = SimBackend(n_slots=2, rate=2e9)
        reqs = make_requests(rate_hz=rate, duration_s=1.0, seed=7, k_lo=12, k_hi=16, iters_lo=50, iters_hi=200)
        st = Server(be, budget_bytes=2**36).run(reqs)
        p99.append(st.latency_p99_s)
    assert p99[1] > 2 * p99[0]


def test_oversized_request_rejected():
    be = SimBackend()
    r = Request(rid=0, n=2**20, iters=10, f_br=0.01, a_low=1.0, a_high=2.0, seed=0, arrival=0.0)
    with pytest.raises(ValueError):
        Server(be, budget_bytes=1000).run([r])


def test_request_generator_matches_recipe():
    reqs = make_requests(rate_hz=2000.0, duration_s=1.0, seed=4)
    assert 1800 < len(reqs) < 2200
    ns = np.array([r.n for r in reqs])
    assert ns.min() >= 2**12 and ns.max() <= 2**22
    its = np.array([r.iters for r in reqs])
    assert its.min() >= 50 and its.max() <= 200
    gaps = np.diff([r.arrival for r in reqs])
    assert abs(gaps.mean() - 1 / 2000.0) < 0.1 / 2000.0


def test_segments_let_a_short_request_overtake_a_long_one():
    """With iteration segments a request that arrives while a long one runs
    joins at the next segment boundary and finishes first; without them it
    waits for the long run to end."""
    def run(seg):
        be = SimBackend(n_slots=1, rate=1e9, overhead=1e-5)
        long_r = Request(rid=0, n=2**20, iters=200, f_br=0.01, a_low=1.0, a_high=2.0, seed=0, arrival=0.0)
        short = Request(rid=1, n=2**12, iters=50, f_br=0.01, a_low=1.0, a_high=2.0, seed=1, arrival=1e-3)
        st = Server(be, budget_bytes=2**36, segment_iters=seg).run([long_r, short])
        assert st.completed == 2
        assert long_r.progress == 200 and short.progress == 50
        return long_r, short, be
    long_r, short, _ = run(None)
    assert short.done > long_r.done
    long_s, short_s, be = run(25)
    assert short_s.done < long_s.done
    assert long_s.segments == 8 and short_s.segments == 2
    # the long run's total work is unchanged; its completion moves only by the
    # short request's share of the shared launches
    assert long_s.done >= long_r.done


def test_segments_keep_budget_and_order():
    be = SimBackend(n_slots=2, rate=2e9)
    reqs = make_requests(rate_hz=300.0, duration_s=1.0, seed=8, k_lo=12, k_hi=18, iters_lo=50, iters_hi=200)
    srv = Server(be, budget_bytes=2**34, segment_iters=30, segment_always=True)
    st = srv.run(reqs)
    _check_common(reqs, st, srv)
    assert all(r.progress == r.iters for r in reqs)
    assert all(r.segments == -(-r.iters // 30) for r in reqs)
    # every launch runs at most 30 iterations of each request
    work = sum(r.n * r.iters for r in reqs)
    assert st.sample_iterations == work


def test_segments_only_under_contention():
    """By default a launch is cut into segments only while the device is
    contended (it takes the last idle stream, or requests wait behind it).
    Requests arriving far apart on a 4-stream device each run whole; the same
    requests all queued at once on one stream run in segments."""
    def reqs(spacing):
        return [Request(rid=i, n=2**16, iters=100, f_br=0.01, a_low=1.0, a_high=2.0, seed=i, arrival=i * spacing)
                for i in range(6)]
    sparse = reqs(1.0)
    st = Server(SimBackend(n_slots=4, rate=1e9), budget_bytes=2**36, segment_iters=25).run(sparse)
    assert st.completed == 6 and all(r.segments == 1 for r in sparse)
    dense = reqs(0.0)
    st = Server(SimBackend(n_slots=1, rate=1e9), budget_bytes=2**36, segment_iters=25).run(dense)
    assert st.completed == 6 and all(r.segments == 4 for r in dense)
