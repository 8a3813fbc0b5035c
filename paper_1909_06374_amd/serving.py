"""Request server for the light-curve generator on one GPU.

Each request asks for one simulated L/L_Edd light curve: a length N, an
iteration count, Eq. 3 PSD parameters and a seed (Sec. 2.1: the user gives
the PSD, the PDF and the number of points; the generator returns the series).
The server

* admits arrived requests first-come first-served while the sum of their HBM
  footprints (workspace + PDF draw + output + convergence history) stays
  within a budget;
* batches admitted requests continuously: whenever one of its launch streams
  is idle it launches every admitted request not yet running (up to a sample
  cap) as one batch on that stream, so several batches of mixed lengths are in
  flight at once and a request never waits for a whole earlier batch to end
  before it is launched;
* optionally works at the granularity of iterations (``segment_iters``): a
  launch runs at most that many iterations of each request in it, and a
  request with iterations left goes back to the end of the queue, so that
  requests that arrive later join the device at the next segment boundary
  instead of waiting for a long request's whole run;
* records, per request, arrival time and completion time on the device clock
  (events), giving latency = completion - arrival.

Batching never changes results: a curve's output depends only on its own
inputs (per-curve Philox keys, per-curve launch groups), so a request served
in a mixed batch is bit-identical to the same request served alone.  A
segment restarts the generator from the request's current series with the
same seed: the Timmer-Koenig moduli are drawn again identically, the series
is a permutation of the draw (the same sorted values), and the iteration's
only state is the series itself (Sec. 2.1), so segmented and uninterrupted
runs are bit-identical too.

The scheduling logic is independent of the GPU (``Backend``), so it is tested
on the CPU with a simulated backend; ``GpuBackend`` drives the C ABI.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np


@dataclass
class Request:
    rid: int
    n: int
    iters: int
    f_br: float
    a_low: float
    a_high: float
    seed: int
    arrival: float          # seconds after the start of the run
    dt: float = 1.0
    footprint: int = 0      # bytes, set at submission
    admitted: float = -1.0
    launched: float = -1.0
    done: float = -1.0      # completion time (seconds after start)
    batch: int = -1
    progress: int = 0       # iterations run so far
    segments: int = 0       # launches the request took part in


@dataclass
class Batch:
    bid: int
    reqs: List[Request]
    slot: int
    handle: object = None
    footprint: int = 0
    # per request: first iteration and iteration count of this launch
    start: List[int] = field(default_factory=list)
    count: List[int] = field(default_factory=list)


class Backend:
    """What the scheduler needs from the device."""

    n_slots = 1

    def footprint(self, req: Request) -> int:
        raise NotImplementedError

    def start_clock(self) -> None:
        """Marks time zero on the device clock."""

    def launch(self, batch: Batch) -> object:
        """Enqueues the batch on its slot: iterations batch.start[i] ..
        batch.start[i] + batch.count[i] - 1 of request batch.reqs[i]; returns
        a handle."""
        raise NotImplementedError

    def finished(self, handle) -> Optional[float]:
        """Completion time (seconds after time zero) if the batch is done, else None."""
        raise NotImplementedError

    def release(self, handle) -> None:
        """Frees what the batch held (after it finished)."""

    def retire(self, req: Request) -> None:
        """The request has run all its iterations: frees what it held."""

    def now(self) -> float:
        raise NotImplementedError

    def idle_wait(self, seconds: float) -> None:
        time.sleep(seconds)


@dataclass
class ServeStats:
    n_requests: int
    completed: int
    wall_s: float
    samples: int
    sample_iterations: int
    latency_p50_s: float
    latency_p99_s: float
    latency_mean_s: float
    max_footprint: int
    budget: int
    batches: int
    mean_batch: float

    def as_dict(self) -> Dict:
        return dict(self.__dict__)


class Server:
    """Continuous-batching scheduler with HBM-footprint admission."""

    def __init__(self, backend: Backend, budget_bytes: int, max_batch_samples: int = 2**26,
                 max_batch_curves: int = 4096, segment_iters: Optional[int] = None,
                 segment_always: bool = False):
        self.be = backend
        self.budget = int(budget_bytes)
        self.max_batch_samples = int(max_batch_samples)
        self.max_batch_curves = int(max_batch_curves)
        if segment_iters is not None and int(segment_iters) < 1:
            raise ValueError("segment_iters must be at least 1")
        self.segment_iters = None if segment_iters is None else int(segment_iters)
        # Segments pay off only while the device is contended: a launch is cut
        # into segments when it takes the last idle stream or requests are
        # still queued behind it; otherwise (light load) it runs the requests'
        # remaining iterations at once.  segment_always cuts every launch.
        self.segment_always = bool(segment_always)

    def run(self, reqs: List[Request]) -> ServeStats:
        be = self.be
        reqs = sorted(reqs, key=lambda r: (r.arrival, r.rid))
        for r in reqs:
            r.progress, r.segments = 0, 0
            r.footprint = int(be.footprint(r))
            if r.footprint > self.budget:
                raise ValueError(f"request {r.rid} needs {r.footprint} bytes, over the {self.budget}-byte budget")
        pending = 0                      # next request not yet admitted (arrival order)
        admitted: List[Request] = []     # admitted, not launched
        inflight: Dict[int, Batch] = {}  # slot -> batch
        used = 0
        max_used = 0
        nb = 0
        sizes = []
        be.start_clock()
        t_wall0 = time.perf_counter()
        done_count = 0
        while done_count < len(reqs):
            progressed = False
            # 1. retire finished batches
            for slot in list(inflight):
                b = inflight[slot]
                t = be.finished(b.handle)
                if t is None:
                    continue
                be.release(b.handle)
                for r, k in zip(b.reqs, b.count):
                    r.progress += k
                    if r.progress >= r.iters:
                        r.done = t
                        done_count += 1
                        used -= r.footprint
                        be.retire(r)
                    else:
                        admitted.append(r)  # next segment, behind what is queued
                del inflight[slot]
                progressed = True
            now = be.now()
            # 2. admit arrived requests, in arrival order, within the budget
            while pending < len(reqs) and reqs[pending].arrival <= now:
                r = reqs[pending]
                if used + r.footprint > self.budget:
                    break
                used += r.footprint
                max_used = max(max_used, used)
                r.admitted = now
                admitted.append(r)
                pending += 1
                progressed = True
            # 3. launch admitted requests on idle slots
            for slot in range(be.n_slots):
                if not admitted:
                    break
                if slot in inflight:
                    continue
                take, samples = [], 0
                while admitted and len(take) < self.max_batch_curves and (
                        not take or samples + admitted[0].n <= self.max_batch_samples):
                    r = admitted.pop(0)
                    take.append(r)
                    samples += r.n
                seg = self.segment_iters
                if seg is not None and not self.segment_always:
                    contended = bool(admitted) or len(inflight) + 1 >= be.n_slots
                    if not contended:
                        seg = None
                b = Batch(nb, take, slot, footprint=sum(r.footprint for r in take),
                          start=[r.progress for r in take],
                          count=[r.iters - r.progress if seg is None else min(seg, r.iters - r.progress)
                                 for r in take])
                for r in take:
                    if r.segments == 0:
                        r.launched = now
                    r.segments += 1
                    r.batch = nb
                b.handle = be.launch(b)
                inflight[slot] = b
                nb += 1
                sizes.append(len(take))
                progressed = True
            if not progressed:
                nxt = reqs[pending].arrival - now if pending < len(reqs) else 0.0
                be.idle_wait(min(max(nxt, 0.0), 2e-4) if inflight else max(nxt, 0.0))
        wall = time.perf_counter() - t_wall0
        lat = np.array([r.done - r.arrival for r in reqs]) if reqs else np.zeros(1)
        return ServeStats(
            n_requests=len(reqs), completed=done_count, wall_s=wall,
            samples=int(sum(r.n for r in reqs)), sample_iterations=int(sum(r.n * r.iters for r in reqs)),
            latency_p50_s=float(np.percentile(lat, 50)), latency_p99_s=float(np.percentile(lat, 99)),
            latency_mean_s=float(lat.mean()), max_footprint=max_used, budget=self.budget, batches=nb,
            mean_batch=float(np.mean(sizes)) if sizes else 0.0)


def make_requests(rate_hz: float, duration_s: float, seed: int, k_lo: int = 12, k_hi: int = 22,
                  iters_lo: int = 50, iters_hi: int = 200) -> List[Request]:
    """Poisson arrivals; N uniform over the 2^a / 3 * 2^a grid in [2^k_lo, 2^k_hi];
    iterations uniform in [iters_lo, iters_hi]; PTF-like Eq. 3 parameters."""
    from . import synth
    t = synth.poisson_arrivals(rate_hz, duration_s, seed)
    m = len(t)
    ns = synth.uneven_sizes(m, seed, k_lo, k_hi) if m else np.zeros(0, dtype=np.int64)
    its = synth.request_iters(m, seed, iters_lo, iters_hi) if m else np.zeros(0, dtype=np.int32)
    a_low, a_high, f_b = synth.curve_params(m, seed) if m else (np.zeros(0),) * 3
    return [Request(rid=i, n=int(ns[i]), iters=int(its[i]), f_br=float(f_b[i]), a_low=float(a_low[i]),
                    a_high=float(a_high[i]), seed=seed * 1000003 + i, arrival=float(t[i])) for i in range(m)]


class GpuBackend(Backend):
    """Runs batches through agn_erdf_draw + agn_lc_generate_batch on
    default-priority streams of one device; completion times from events.
    A request that runs in segments keeps its current series (and its Eq. 4
    history) in buffers of its own between launches; a segment's launch
    starts from that series (as the PDF draw of a generate call with the
    request's seed) and writes the next one back."""

    def __init__(self, ctx, n_slots: int = 4, prec: int = 1, erdf_params=None, keep_outputs: bool = False):
        import torch

        from . import agn_batch_workspace_size, erdf_params as _ep
        self.torch = torch
        self.ctx = ctx
        self.n_slots = int(n_slots)
        self.prec = int(prec)
        self.ep = erdf_params if erdf_params is not None else _ep()
        self.dev = f"cuda:{ctx.device}"
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(self.n_slots)]
        self.keep = keep_outputs
        self.outputs: Dict[int, np.ndarray] = {}
        self.histories: Dict[int, np.ndarray] = {}
        self.state: Dict[int, Dict] = {}
        self._ws_size = agn_batch_workspace_size
        self._t0 = None
        self._wall0 = 0.0

    def footprint(self, req: Request) -> int:
        # workspace (incl. descriptors) + PDF draw + output + history + iteration count,
        # plus the series and history a segmented request keeps between launches
        return int(self._ws_size([req.n], self.prec)) + 24 * req.n + 16 * req.iters + 4

    def start_clock(self) -> None:
        torch = self.torch
        torch.cuda.synchronize(self.dev)
        self._t0 = torch.cuda.Event(enable_timing=True)
        self._t0.record(torch.cuda.current_stream(self.dev))
        torch.cuda.synchronize(self.dev)
        self._wall0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self._wall0

    def launch(self, batch: Batch):
        from . import agn_erdf_draw, agn_lc_generate_batch, psd_params
        torch = self.torch
        st = self.streams[batch.slot]
        reqs = batch.reqs
        counts = list(batch.count) if batch.count else [r.iters for r in reqs]
        starts = list(batch.start) if batch.start else [0] * len(reqs)
        ns = [r.n for r in reqs]
        offs = np.concatenate([[0], np.cumsum(ns)[:-1]]).astype(np.int64)
        tot = int(sum(ns))
        mx = max(max(counts), 1)
        with torch.cuda.stream(st):
            erdf = torch.empty(tot, dtype=torch.float64, device=self.dev)
            x = torch.empty(tot, dtype=torch.float64, device=self.dev)
            d = torch.empty(len(ns) * mx, dtype=torch.float64, device=self.dev)
            done = torch.empty(len(ns), dtype=torch.int32, device=self.dev)
            ws = torch.empty(self._ws_size(ns, self.prec), dtype=torch.uint8, device=self.dev)
            for r, o, s0, k in zip(reqs, offs, starts, counts):
                seg = erdf[int(o):int(o) + r.n]
                if s0 == 0:
                    agn_erdf_draw(self.ctx, self.ep, r.n, r.seed, r.rid, seg, stream=st)
                    if k < r.iters:  # segmented: the request keeps its series between launches
                        self.state[r.rid] = dict(
                            x=torch.empty(r.n, dtype=torch.float64, device=self.dev),
                            hist=torch.zeros(max(r.iters, 1), dtype=torch.float64, device=self.dev))
                else:
                    seg.copy_(self.state[r.rid]["x"])
        agn_lc_generate_batch(self.ctx, ns, offs, [psd_params(0.0, r.f_br, r.a_low, r.a_high) for r in reqs],
                              [r.dt for r in reqs], counts, [r.seed for r in reqs], [r.rid for r in reqs], erdf, -1.0,
                              self.prec, x, d, done, ws, stream=st)
        with torch.cuda.stream(st):
            for i, (r, o, s0, k) in enumerate(zip(reqs, offs, starts, counts)):
                if r.rid in self.state:
                    stt = self.state[r.rid]
                    stt["x"].copy_(x[int(o):int(o) + r.n])
                    if k > 0:
                        stt["hist"][s0:s0 + k].copy_(d[i * mx:i * mx + k])
        ev = torch.cuda.Event(enable_timing=True)
        ev.record(st)
        return dict(ev=ev, bufs=(erdf, x, d, done, ws), batch=batch, offs=offs, starts=starts, counts=counts, mx=mx)

    def finished(self, h) -> Optional[float]:
        if not h["ev"].query():
            return None
        if self.keep:
            x = h["bufs"][1].cpu().numpy()
            d = h["bufs"][2].cpu().numpy()
            for i, (r, o, s0, k) in enumerate(zip(h["batch"].reqs, h["offs"], h["starts"], h["counts"])):
                if s0 + k < r.iters:
                    continue  # more segments to come
                self.outputs[r.rid] = x[int(o):int(o) + r.n].copy()
                if r.rid in self.state:
                    self.histories[r.rid] = self.state[r.rid]["hist"].cpu().numpy()[:r.iters].copy()
                else:
                    self.histories[r.rid] = d[i * h["mx"]:i * h["mx"] + r.iters].copy()
        return self._t0.elapsed_time(h["ev"]) / 1000.0

    def release(self, h) -> None:
        h["bufs"] = None

    def retire(self, req: Request) -> None:
        self.state.pop(req.rid, None)
