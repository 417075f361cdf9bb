"""Host-side scheduling logic of the serving loop, with a fake device
backend (no GPU): admission never exceeds the memory budget, every batch has
one shape and at most one request per client, all requests complete in
arrival order per client, and warm starts are handed from a client's
request to its next one."""
import numpy as np
import pytest

from paper_2506_07823_amd.serve import Request, Server, request_bytes


class FakeBackend:
    """Batches finish `delay` polls after launch; results echo the rid."""

    def __init__(self, nstreams=2, delay=2, ws=1000):
        self.nstreams = nstreams
        self.delay = delay
        self.ws = ws
        self.live = []
        self.t = 0

    def workspace_bytes(self, shape):
        return self.ws * shape[1]

    def start(self):
        pass

    def launch(self, shape, reqs, warm):
        h = {"polls": 0, "reqs": reqs, "warm": warm, "shape": shape}
        self.live.append(h)
        return h

    def poll(self, h):
        h["polls"] += 1
        return h["polls"] > self.delay

    def collect(self, h):
        self.t += 1
        self.live.remove(h)
        res = [{"rid": r.rid} for r in h["reqs"]]
        return res, float(self.t), [{"from": r.rid} for r in h["reqs"]]


def _req(rid, client, N, n, m, arrival=0.0):
    data = {"A": np.zeros((N, n, n)), "B": np.zeros((N, n, m))}
    return Request(rid=rid, client=client, data=data, arrival=arrival)


def _drive(server, reqs, steps=10000):
    for r in reqs:
        server.submit(r, 0.0)
    for t in range(steps):
        if not server.step(float(t)):
            break
        assert server.used <= server.budget
    return server.done


def test_budget_and_shapes():
    be = FakeBackend(nstreams=3)
    shapes = [(10, 12, 12), (20, 36, 12), (5, 70, 70)]
    reqs = [_req(i, i % 7, *shapes[i % 3]) for i in range(60)]
    cost = {s: request_bytes(s, 4, be.workspace_bytes) for s in shapes}
    budget = 3 * max(cost.values())
    srv = Server(be, budget, max_batch=8)
    done = _drive(srv, reqs)
    assert len(done) == 60 and all(r.result["rid"] == r.rid for r in done)
    assert srv.peak_used <= budget
    assert srv.used == 0 and not srv.inflight
    for shape, k in srv.launch_log:
        assert shape in shapes and 1 <= k <= 8


def test_one_request_per_client_per_batch_and_warm_handoff():
    be = FakeBackend(nstreams=1, delay=1)
    reqs = [_req(i, i % 2, 10, 12, 12) for i in range(10)]   # two clients, same shape
    srv = Server(be, 10 ** 12, max_batch=64, warm=True)
    done = _drive(srv, reqs)
    assert len(done) == 10
    # two clients -> at most two requests per batch
    assert all(k <= 2 for _, k in srv.launch_log)
    # per client, completion follows submission order and each request after
    # the first is warm-started
    for c in (0, 1):
        mine = [r for r in done if r.client == c]
        assert [r.rid for r in mine] == sorted(r.rid for r in mine)
        assert not mine[0].warm and all(r.warm for r in mine[1:])


def test_client_order_with_parallel_streams():
    """With several streams free, a client's next request still waits for
    the previous one (no overtaking, warm start available)."""
    be = FakeBackend(nstreams=4, delay=3)
    reqs = [_req(i, i % 3, 10, 12, 12) for i in range(30)]
    srv = Server(be, 10 ** 12, max_batch=64, warm=True)
    done = _drive(srv, reqs)
    assert len(done) == 30
    for c in range(3):
        mine = [r for r in done if r.client == c]
        assert [r.rid for r in mine] == sorted(r.rid for r in mine)
        assert all(r.warm for r in mine[1:])
        assert len({r.done_ms for r in mine}) == len(mine)   # never in the same or a parallel batch


def test_oversized_request_rejected():
    be = FakeBackend()
    srv = Server(be, 10)
    with pytest.raises(ValueError):
        srv.submit(_req(0, 0, 10, 12, 12), 0.0)


def test_fifo_across_shapes():
    """The batch launched next is the shape whose oldest admitted request
    has waited longest."""
    be = FakeBackend(nstreams=1, delay=0)
    reqs = [_req(0, 0, 10, 12, 12), _req(1, 1, 20, 36, 12), _req(2, 2, 10, 12, 12)]
    srv = Server(be, 10 ** 12, max_batch=64)
    _drive(srv, reqs)
    assert srv.launch_log[0] == ((10, 12, 12), 2)
    assert srv.launch_log[1] == ((20, 36, 12), 1)


def test_batches_never_mix_warm_and_cold_requests():
    """A client's first request (cold) and another client's later request
    (warm-started) of the same shape are admitted together but launched in
    separate batches, so every member of a batch starts the way it would
    alone."""
    be = FakeBackend(nstreams=1, delay=1)
    srv = Server(be, budget_bytes=10 ** 12, max_batch=64, warm=True, itemsize=4)
    first = [_req(0, 0, 10, 4, 2), _req(1, 1, 10, 4, 2)]
    _drive(srv, first)
    assert len(srv.done) == 2
    # client 0 now has a warm state; client 2 is new (cold)
    later = [_req(2, 0, 10, 4, 2), _req(3, 2, 10, 4, 2), _req(4, 1, 10, 4, 2)]
    launches = []
    orig = be.launch

    def spy(shape, reqs, warm):
        launches.append([w is not None for w in warm])
        return orig(shape, reqs, warm)

    be.launch = spy
    _drive(srv, later)
    assert len(srv.done) == 5
    for kinds in launches:
        assert all(kinds) or not any(kinds), launches
    assert any(all(k) for k in launches) and any(not any(k) for k in launches)
