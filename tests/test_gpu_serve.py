"""Warm start and the continuous-batching serving loop on the GPU.

Warm start: starting the scan's refinement from a nearby solution returns
the same solution (within the FP32 path's tolerance, relative KKT residual
<= 1e-5).  Serving: every request of a mixed Poisson stream gets the result
it gets when solved alone -- bit for bit without warm starts (per-instance
arithmetic does not depend on the batch), and within the FP32 tolerance
with warm starts."""
import numpy as np
import pytest

import synth
from tests.gpuhelp import oracle_check, rel, run, say, to_dev

pytestmark = pytest.mark.gpu

RESID_TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_07823_amd  # noqa: F401


def _solve_dev(dev, **kw):
    import torch
    import paper_2506_07823_amd as L
    out = L.solve(*[dev[k] for k in synth.FIELDS], want_resid=True, **kw)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("N,n,m", [(50, 36, 12), (6, 80, 40)])
def test_warm_start_same_solution(N, n, m):
    import torch
    batch = synth.gen_batch(lambda i: synth.gen_c1_like(N, n, m, [700, N, n, i]), 4, np.float32)
    say(f"[warm start] N={N} n={n} m={m}")
    dev = to_dev(batch, np.float32)
    cold = _solve_dev(dev)
    assert not cold["status"].any()
    g = torch.Generator(device="cpu").manual_seed(7)
    pert = {f: (cold[f].cpu() + 1e-2 * torch.randn(cold[f].shape, generator=g)).to("cuda:0")
            for f in ("x", "u", "lam")}
    warm = _solve_dev(dev, warm=(pert["x"], pert["u"], pert["lam"]))
    assert not warm["status"].any()
    assert warm["resid"].max().item() <= RESID_TOL
    for f in ("x", "u", "lam"):
        assert rel(warm[f].cpu().numpy(), cold[f].cpu().numpy().astype(np.float64)) <= 1e-4, f
    # in place: the warm arrays are the outputs themselves
    out = {f: pert[f].clone() for f in ("x", "u", "lam")}
    out["status"] = torch.empty(4, dtype=torch.int32, device="cuda:0")
    inpl = _solve_dev(dev, warm=(out["x"], out["u"], out["lam"]), out=out)
    for f in ("x", "u", "lam"):
        assert torch.equal(inpl[f], warm[f]), f
    errs, res = oracle_check(batch, {f: warm[f].cpu().numpy() for f in ("x", "u", "lam")}, 2, as_f32=True)
    say(f"  warm-started inst 2: rel err {errs}, oracle resid {res:.2e}")
    assert res <= RESID_TOL


def _clients():
    """(shape generator, seed) per client: SRBD-shaped at N = 25 and 100,
    whole-body-shaped at N = 50 and 100, the multi-robot shape (n = m = 192,
    N = 50) and another large-block shape."""
    gens = []
    for c in range(3):
        gens.append(lambda k, c=c: synth.gen_c2(25, c))
    gens.append(lambda k: synth.gen_c2(100, 5))
    for c in range(2):
        gens.append(lambda k, c=c: synth.gen_c1_like(50, 36, 12, [710, c]))
    gens.append(lambda k: synth.gen_c3(3))
    gens.append(lambda k: synth.gen_c4(0))
    gens.append(lambda k: synth.gen_rand(8, 70, 70, seed=[720]))
    return gens


def _stream(nreq_per_client=5, rate=400.0, seed=0):
    from paper_2506_07823_amd.serve import Request
    rng = np.random.default_rng(seed)
    gens = _clients()
    reqs = []
    t = 0.0
    x0 = {}
    order = rng.permutation(np.repeat(np.arange(len(gens)), nreq_per_client))
    for rid, c in enumerate(order):
        t += rng.exponential(1.0 / rate)
        base = gens[c](0)
        prev = x0.get(c, base["x0"])
        x0[c] = prev + rng.normal(0.0, 1e-2, prev.shape)
        data = {k: np.ascontiguousarray(v, dtype=np.float32) for k, v in base.items()}
        data["x0"] = x0[c].astype(np.float32)
        reqs.append(Request(rid=rid, client=int(c), data=data, arrival=t))
    return reqs


def _alone(req):
    batch = {k: v[None] for k, v in req.data.items()}
    return run(batch, np.float32, want_resid=True)


@pytest.mark.parametrize("warm,graphs", [(False, False), (True, False), (False, True), (True, True)])
def test_serving_mix_equals_alone(warm, graphs):
    from paper_2506_07823_amd.serve import GpuBackend, Server, latency_report
    reqs = _stream()
    say(f"[serving] {len(reqs)} mixed requests, warm={warm}, graph replay={graphs}")
    be = GpuBackend(nstreams=3, refine=1, graphs=graphs)
    srv = Server(be, budget_bytes=16 << 30, max_batch=16, warm=warm)
    done = srv.run(reqs)
    assert len(done) == len(reqs)
    rep = latency_report(done)
    say(f"  {rep}, batches {srv.launch_log[:12]} ...")
    assert srv.peak_used <= srv.budget
    for r in done:
        assert r.result["status"] == 0, (r.rid, r.result["status"])
        assert r.result["resid"] <= RESID_TOL, (r.rid, r.result["resid"])
        a = _alone(r)
        for f in ("x", "u", "lam"):
            if warm:
                assert rel(r.result[f], a[f][0].astype(np.float64)) <= 1e-4, (r.rid, f)
            else:
                assert np.array_equal(r.result[f], a[f][0]), (r.rid, f)
    if warm:
        assert sum(r.warm for r in done) >= len(done) - len(_clients())
    if graphs:
        assert be.graph_replays > 0
