"""Continuous-batching request loop for streams of LQR-KKT solves.

Requests of mixed shapes (N, n, m) arrive over time (for example the
per-control-tick MPC subproblems of several robots; each robot is a
*client* whose requests form a stream).  The server:

* admits a request when its memory cost fits the HBM budget (inputs,
  outputs and a batch-of-one workspace; a batch of k requests never needs
  more than the sum of its members' costs, so admitted work always fits);
* groups admitted requests by shape and launches each group as one batched
  solve on one of several HIP streams, so independent batches overlap on
  the device, while requests that arrive meanwhile wait for a free stream
  (continuous batching: a finishing batch frees its stream and budget and
  the next batch is formed from whatever has been admitted by then);
* keeps each client's last solution on the device and passes it as the warm
  start of the client's next request (the solve then refines from it);
* stamps each request's completion with a device event, so latencies are
  measured on the GPU clock from the arrival time.

Each request's result depends only on its own data (and warm start): the
library's per-instance arithmetic does not depend on the batch it runs in.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np

FIELDS = ("A", "B", "c", "Q", "R", "M", "q", "r", "x0")


@dataclasses.dataclass
class Request:
    rid: int
    client: int
    data: dict              # host arrays of one instance (FIELDS)
    arrival: float = 0.0    # seconds after the start of the run
    # filled in by the server
    admitted: float = -1.0
    launched: float = -1.0
    done_ms: float = -1.0   # completion on the device clock, ms after the start
    result: dict | None = None
    warm: bool = False

    @property
    def shape(self):
        N, n, m = self.data["B"].shape
        return int(N), int(n), int(m)


def request_bytes(shape, itemsize: int, workspace_bytes) -> int:
    """Device bytes a request may hold while admitted: its inputs and
    outputs plus the workspace of a batch of one."""
    N, n, m = shape
    inputs = N * (n * n + 2 * n * m + n + m * m + m) + (N + 1) * (n * n + n) + n
    outputs = 2 * (N + 1) * n + N * m
    warm = outputs
    return itemsize * (inputs + outputs + warm) + 8 + int(workspace_bytes(shape))


class Server:
    """Scheduler state; the device work goes through ``backend``:

    backend.workspace_bytes(shape) -> int       (batch of one)
    backend.launch(shape, reqs, warm_list) -> handle   (asynchronous)
    backend.poll(handle) -> bool                  (finished?)
    backend.collect(handle) -> (results list, done_ms, warm_states list)
    backend.nstreams                              (concurrent batches)
    """

    def __init__(self, backend, budget_bytes: int, max_batch: int = 256, warm: bool = True,
                 itemsize: int = 4):
        self.be = backend
        self.budget = int(budget_bytes)
        self.max_batch = max_batch
        self.use_warm = warm
        self.itemsize = itemsize
        self.used = 0
        self.peak_used = 0
        self.waiting = collections.deque()           # submitted, not admitted (FIFO)
        self.pending = collections.OrderedDict()     # shape -> deque of admitted requests
        self.inflight = []                           # (handle, shape, reqs, cost)
        self.warm_state = {}                         # client -> device state of its last solution
        self.busy_clients = set()                    # clients with a request in flight
        self.done = []
        self.launch_log = []                         # (shape, batch size)
        self._cost = {}

    # ------------------------------------------------------------ helpers
    def cost(self, shape) -> int:
        c = self._cost.get(shape)
        if c is None:
            c = self._cost[shape] = request_bytes(shape, self.itemsize, self.be.workspace_bytes)
        return c

    def submit(self, req: Request, now: float):
        if self.cost(req.shape) > self.budget:
            raise ValueError(f"request {req.rid} of shape {req.shape} needs {self.cost(req.shape)} bytes, "
                             f"more than the whole budget ({self.budget})")
        self.waiting.append(req)

    def _admit(self, now: float):
        while self.waiting and self.used + self.cost(self.waiting[0].shape) <= self.budget:
            r = self.waiting.popleft()
            r.admitted = now
            self.used += self.cost(r.shape)
            self.peak_used = max(self.peak_used, self.used)
            self.pending.setdefault(r.shape, collections.deque()).append(r)

    def _dispatch(self, now: float):
        blocked = set()   # shapes whose admitted requests all wait for a client in flight
        while len(self.inflight) < self.be.nstreams:
            # the shape whose oldest admitted request has waited longest
            live = [(q[0].admitted, q[0].rid, s) for s, q in self.pending.items() if q and s not in blocked]
            if not live:
                return
            shape = min(live)[2]
            q = self.pending[shape]
            # at most one request per client per batch, and none for a client
            # with a request in flight: the next request of a client runs
            # after its predecessor and starts from that solution.  A batch
            # holds only warm-started or only cold requests: the solve of a
            # batch with warm starts refines every member from its warm state,
            # so a cold member would otherwise start from zeros and get one
            # refinement sweep fewer than alone.
            batch, keep, seen, kind = [], [], set(), None
            while q and len(batch) < self.max_batch:
                r = q.popleft()
                st = self._warm_of(r, shape)
                if r.client in seen or r.client in self.busy_clients or (kind is not None and (st is not None) != kind):
                    keep.append(r)
                else:
                    batch.append(r)
                    seen.add(r.client)
                    kind = st is not None
            for r in reversed(keep):
                q.appendleft(r)
            if not batch:
                blocked.add(shape)
                continue
            warm = []
            for r in batch:
                st = self._warm_of(r, shape)
                r.warm = st is not None
                warm.append(st)
                r.launched = now
            h = self.be.launch(shape, batch, warm)
            self.busy_clients |= seen
            self.inflight.append((h, shape, batch, sum(self.cost(shape) for _ in batch)))
            self.launch_log.append((shape, len(batch)))

    def _warm_of(self, r: Request, shape):
        """Device state of the client's last solution if it can warm-start
        this request (same shape), else None."""
        st = self.warm_state.get(r.client) if self.use_warm else None
        if st is None or st[0] != shape:
            return None
        return st[1]

    def _retire(self):
        still = []
        for h, shape, reqs, cost in self.inflight:
            if not self.be.poll(h):
                still.append((h, shape, reqs, cost))
                continue
            results, done_ms, states = self.be.collect(h)
            self.busy_clients -= {r.client for r in reqs}
            for r, res, st in zip(reqs, results, states):
                r.result = res
                r.done_ms = done_ms
                if self.use_warm:
                    self.warm_state[r.client] = (shape, st)
                self.done.append(r)
            self.used -= cost
        self.inflight = still

    def step(self, now: float) -> bool:
        """One scheduling round; returns whether anything is still queued."""
        self._retire()
        self._admit(now)
        self._dispatch(now)
        return bool(self.waiting or self.inflight or any(self.pending.values()))

    def run(self, requests, clock=time.perf_counter, idle=lambda: time.sleep(5e-5)):
        """Serve requests (sorted by arrival time, seconds from the start)."""
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        self.be.start()
        t0 = clock()
        i = 0
        busy = True
        while i < len(reqs) or busy:
            now = clock() - t0
            while i < len(reqs) and reqs[i].arrival <= now:
                self.submit(reqs[i], now)
                i += 1
            busy = self.step(now)
            idle()
        return self.done


class GpuBackend:
    """Batched solves on a pool of HIP streams (default priority) through
    the library's C ABI; inputs go host -> device on the launch stream and
    results come back to pinned host buffers on the same stream.

    graphs=True: the solve of a batch is captured into a HIP graph once per
    (shape, batch size, warm or cold, stream) with buffers of its own, and
    replayed for every later batch of that key: a batch then costs its
    copies and one graph launch instead of the whole launch sequence.
    Shapes with an order above `graph_max_order` run eagerly (their
    per-key buffers would be large)."""

    def __init__(self, device: int = 0, nstreams: int = 4, refine: int = 1, dtype=np.float32, graphs: bool = False,
                 graph_max_order: int = 64):
        import torch
        import paper_2506_07823_amd as L
        self.torch, self.L = torch, L
        self.device = device
        self.nstreams = nstreams
        self.refine = refine
        self.np_dtype = dtype
        self.dtype = torch.float32 if dtype == np.float32 else torch.float64
        self.streams = [torch.cuda.Stream(device=device) for _ in range(nstreams)]
        self.free = list(range(nstreams))
        self.ws = [L.Workspace(device) for _ in range(nstreams)]
        self.graphs = graphs
        self.graph_max_order = graph_max_order
        self._graphs = {}
        self.graph_replays = 0
        self.t0 = None

    def workspace_bytes(self, shape) -> int:
        N, n, m = shape
        o = self.L.default_opts(self.dtype)
        o.refine_sweeps = self.refine
        return self.L.workspace_bytes(1, N, n, m, o)

    def start(self):
        torch = self.torch
        self.t0 = torch.cuda.Event(enable_timing=True)
        self.t0.record(torch.cuda.current_stream(self.device))
        torch.cuda.synchronize(self.device)

    def _stage_inputs(self, reqs, dev):
        """host -> device on the current stream, straight from each
        request's buffers (asynchronous when they are pinned)"""
        torch = self.torch
        for f in FIELDS:
            for i, r in enumerate(reqs):
                src = r.data[f]
                if not isinstance(src, torch.Tensor):
                    src = torch.from_numpy(np.ascontiguousarray(src, dtype=self.np_dtype))
                dev[f][i].copy_(src, non_blocking=True)

    def _graph(self, shape, k, warm, sid):
        """Buffers and captured solve of one key (built on first use)."""
        key = (shape, k, warm, sid)
        ent = self._graphs.get(key)
        if ent is not None:
            return ent
        torch, L = self.torch, self.L
        N, n, m = shape
        dn = f"cuda:{self.device}"
        shapes = {"A": (N, n, n), "B": (N, n, m), "c": (N, n), "Q": (N + 1, n, n), "R": (N, m, m),
                  "M": (N, n, m), "q": (N + 1, n), "r": (N, m), "x0": (n,)}
        dev = {f: torch.zeros((k,) + s, dtype=self.dtype, device=dn) for f, s in shapes.items()}
        # a valid problem in every slot for the capture's warm-up solve
        eye_n = torch.eye(n, dtype=self.dtype, device=dn)
        eye_m = torch.eye(m, dtype=self.dtype, device=dn)
        dev["A"][:] = eye_n
        dev["Q"][:] = eye_n
        dev["R"][:] = eye_m
        out = {"x": torch.zeros((k, N + 1, n), dtype=self.dtype, device=dn),
               "u": torch.zeros((k, N, m), dtype=self.dtype, device=dn),
               "lam": torch.zeros((k, N + 1, n), dtype=self.dtype, device=dn),
               "status": torch.zeros((k,), dtype=torch.int32, device=dn),
               "resid": torch.zeros((k,), dtype=torch.float64, device=dn)}
        wbuf = tuple(torch.zeros_like(out[f]) for f in ("x", "u", "lam")) if warm else None
        ws = L.Workspace(self.device)
        s = self.streams[sid]
        s.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(s):
            L.solve(*[dev[f] for f in FIELDS], refine=self.refine, want_resid=True, warm=wbuf, workspace=ws,
                    out=out, stream=s)
        s.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            L.solve(*[dev[f] for f in FIELDS], refine=self.refine, want_resid=True, warm=wbuf, workspace=ws,
                    out=out, stream=s)
        s.synchronize()
        ent = self._graphs[key] = {"dev": dev, "out": out, "warm": wbuf, "ws": ws, "graph": g}
        return ent

    def launch(self, shape, reqs, warm_list):
        torch = self.torch
        sid = self.free.pop()
        s = self.streams[sid]
        k = len(reqs)
        dn = f"cuda:{self.device}"
        has_warm = any(w is not None for w in warm_list)
        if has_warm and not all(w is not None for w in warm_list):
            raise ValueError("a batch holds only warm-started or only cold requests")
        use_graph = self.graphs and max(shape[1], shape[2]) <= self.graph_max_order
        ent = self._graph(shape, k, has_warm, sid) if use_graph else None
        with torch.cuda.stream(s):
            if ent is not None:
                dev, out = ent["dev"], ent["out"]
                self._stage_inputs(reqs, dev)
                if has_warm:
                    for j, f in enumerate(("x", "u", "lam")):
                        for i, w in enumerate(warm_list):
                            ent["warm"][j][i].copy_(w[f], non_blocking=True)
                ent["graph"].replay()
                self.graph_replays += 1
            else:
                dev = {}
                for f in FIELDS:
                    first = reqs[0].data[f]
                    dev[f] = torch.empty((k,) + tuple(first.shape), dtype=self.dtype, device=dn)
                self._stage_inputs(reqs, dev)
                warm = None
                if has_warm:
                    warm = tuple(torch.stack([w[f] for w in warm_list]) for f in ("x", "u", "lam"))
                out = self.L.solve(*[dev[f] for f in FIELDS], refine=self.refine, want_resid=True, warm=warm,
                                   workspace=self.ws[sid], stream=s)
            host_out = {f: torch.empty(tuple(out[f].shape), dtype=out[f].dtype, pin_memory=True)
                        for f in ("x", "u", "lam", "status", "resid")}
            for f, h in host_out.items():
                h.copy_(out[f], non_blocking=True)
            # the device state of each solution (the warm start of the
            # client's next request) outlives the graph's output buffers
            states = [{f: out[f][i].clone() for f in ("x", "u", "lam")} for i in range(k)]
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(s)
        return (sid, ev, states, host_out, dev)

    def poll(self, h) -> bool:
        return h[1].query()

    def collect(self, h):
        sid, ev, states, host_out, _ = h
        done_ms = self.t0.elapsed_time(ev)
        k = host_out["x"].shape[0]
        # copies, not views: a view would pin the whole batch's page-locked
        # block for as long as the request's result lives
        results = [{f: host_out[f][i].numpy().copy() for f in host_out} for i in range(k)]
        self.free.append(sid)
        return results, done_ms, states


def latency_report(done, t_first: float = 0.0) -> dict:
    """p50/p99 latency (ms, arrival -> device completion) and throughput,
    overall and per request shape."""
    lat = np.array([r.done_ms - 1e3 * r.arrival for r in done])
    span = (max(r.done_ms for r in done) - 1e3 * min(r.arrival for r in done)) * 1e-3
    per = {}
    for shape in sorted({r.shape for r in done}):
        ls = np.array([r.done_ms - 1e3 * r.arrival for r in done if r.shape == shape])
        per["N%d_n%d_m%d" % shape] = {"requests": int(ls.size), "p50_ms": float(np.percentile(ls, 50)),
                                      "p99_ms": float(np.percentile(ls, 99))}
    return {"requests": len(done), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "max_ms": float(lat.max()),
            "solves_per_s": len(done) / span if span > 0 else float("inf"), "per_shape": per}
