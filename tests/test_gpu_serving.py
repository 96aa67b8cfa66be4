"""GPU tests of the serving loop (slso_server_*) through the C ABI.

A mix of jobs of uneven n and d, FP32 and BF16, is submitted back to back
while earlier jobs are still running. Each job's scores and ordering must
equal those of the same call made alone on a fresh context: every kernel of
the path sums in a fixed order, so the comparison is bit-exact. Admission
by HBM footprint is checked through the server's counters.
"""
import numpy as np
import pytest

import synth
from oracle import leverage as olv
from oracle import metrics as omet

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def slso():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1812_07903_amd as m
    m.load_library()
    return m


def _jobs(n_jobs, seed=7, n_max=60000, d_values=(64, 128, 256), n_min=2000):
    """Serving-shaped jobs: n log-uniform, d from d_values, FP32/BF16 half
    and half, r = d * U{4..8}, k = 32, data like the plain small workload
    with a per-job seed."""
    rng = np.random.default_rng(seed)
    out = []
    for j in range(n_jobs):
        n = int(np.exp(rng.uniform(np.log(n_min), np.log(n_max))))
        d = int(rng.choice(d_values))
        x64 = synth.lowrank_dense(n, d, d // 2,
                                  2.0 ** (-np.arange(d // 2) / 4.0), 1e-3,
                                  1.0, seed=5000 + j)
        if j % 2 == 0:
            x = torch.from_numpy(x64.astype(np.float32)).cuda()
        else:
            b = synth.to_bf16_bits(x64)
            x = torch.from_numpy(b.view(np.int16)).cuda().view(torch.bfloat16)
        r = d * int(rng.integers(4, 9))
        out.append({"x": x, "seed": 9000 + j, "r": r, "k": 32, "n": n, "d": d})
    torch.cuda.synchronize()
    return out


def _alone(slso, jobs):
    ctx = slso.Context(0)
    res = []
    for jb in jobs:
        sc, info = ctx.leverage(jb["x"], jb["seed"], jb["r"], jb["k"])
        pm = ctx.order(sc)
        torch.cuda.synchronize()
        res.append((sc.cpu().numpy(), pm.cpu().numpy(), info["rank"]))
    ctx.close()
    return res


def _check_mix(slso, jobs, slots, budget):
    alone = _alone(slso, jobs)
    srv = slso.Server(0, slots=slots, hbm_budget=budget)
    tickets = [srv.submit(jb["x"], jb["seed"], jb["r"], jb["k"]) for jb in jobs]
    results = [srv.wait(t) for t in tickets]
    stats = srv.stats()
    srv.close()
    print(f"[serving mix d<={max(jb['d'] for jb in jobs)}] "
          f"max_running={stats['max_running']} completed={stats['completed']} "
          f"allocated={stats['allocated_bytes'] >> 20} MiB", flush=True)
    assert stats["completed"] == len(jobs)
    assert stats["max_running"] >= 2          # jobs overlapped on the device
    for jb, t, res, (sc, pm, rank) in zip(jobs, tickets, results, alone):
        assert res["status"] >= 0, res
        assert res["info"]["rank"] == rank
        assert np.array_equal(t.scores.cpu().numpy().view(np.uint32),
                              sc.view(np.uint32))
        assert np.array_equal(t.perm.cpu().numpy(), pm)
    return results


def test_mixed_jobs_wide_equal_alone(slso):
    """Jobs of d up to 1024 (the serving pool's widest), n 20000..60000,
    with one noise-free rank-deficient job among them: the server runs
    its jobs with the decisions on the device, the truncated one is rerun
    on the host path, and every result equals the synchronous call made
    alone, bit for bit."""
    jobs = _jobs(6, seed=19, n_min=20000, d_values=(512, 768, 1024))
    # rank <= 64 in d = 128: each column twice
    half = synth.lowrank_dense(6007, 64, 32, 2.0 ** (-np.arange(32) / 4.0),
                               1e-3, 1.0, seed=23).astype(np.float32)
    x = torch.from_numpy(np.hstack([half, half])).cuda()
    jobs.insert(3, {"x": x, "seed": 77, "r": 512, "k": 32, "n": 6007,
                    "d": 128})
    results = _check_mix(slso, jobs, slots=4, budget=48 << 30)
    assert results[3]["info"]["rank"] <= 64
    assert results[3]["info"]["flags"] & slso.INFO_RERUN


def test_mixed_jobs_equal_alone(slso):
    jobs = _jobs(16)
    alone = _alone(slso, jobs)
    srv = slso.Server(0, slots=4, hbm_budget=32 << 30)
    tickets = [srv.submit(jb["x"], jb["seed"], jb["r"], jb["k"]) for jb in jobs]
    results = [srv.wait(t) for t in tickets]
    stats = srv.stats()
    srv.close()
    print(f"[serving mix] max_running={stats['max_running']} "
          f"completed={stats['completed']}", flush=True)
    assert stats["completed"] == len(jobs)
    assert stats["max_running"] >= 2          # jobs overlapped on the device
    for jb, t, res, (sc, pm, rank) in zip(jobs, tickets, results, alone):
        assert res["status"] >= 0, res
        assert res["info"]["rank"] == rank
        assert res["submit_ms"] <= res["start_ms"] <= res["end_ms"]
        assert np.array_equal(t.scores.cpu().numpy(), sc)
        assert np.array_equal(t.perm.cpu().numpy(), pm)


def test_mixed_job_matches_oracle(slso):
    jobs = _jobs(4, seed=11, n_max=20000)
    srv = slso.Server(0, slots=3)
    tickets = [srv.submit(jb["x"], jb["seed"], jb["r"], jb["k"]) for jb in jobs]
    for jb, t in zip(jobs, tickets):
        srv.wait(t)
        x = jb["x"]
        xv = (x.float() if x.dtype == torch.bfloat16 else x).double().cpu().numpy()
        ref = olv.sketched_leverage(xv, jb["seed"], jb["r"], jb["k"])
        err = omet.max_rel_err(t.scores.cpu().numpy(), ref["scores"])
        print(f"[serving job n={jb['n']} d={jb['d']} {x.dtype}] "
              f"max_rel={err:.2e}", flush=True)
        assert err < 1e-5
    srv.close()


def test_admission_by_hbm_footprint(slso):
    # six jobs of one shape (different data and seeds)
    x64 = synth.lowrank_dense(30000, 128, 64, 2.0 ** (-np.arange(64) / 4.0),
                              1e-3, 1.0, seed=77)
    x = torch.from_numpy(x64.astype(np.float32)).cuda()
    torch.cuda.synchronize()
    jobs = [{"x": x, "seed": 100 + j, "r": 512, "k": 32} for j in range(6)]
    need = slso.workspace_size(x, 512, 32)
    # room for one job's workspace only: the jobs run one at a time
    srv = slso.Server(0, slots=4, hbm_budget=need + (1 << 20))
    tickets = [srv.submit(jb["x"], jb["seed"], jb["r"], jb["k"]) for jb in jobs]
    for t in tickets:
        assert srv.wait(t)["status"] >= 0
    stats = srv.stats()
    srv.close()
    assert stats["max_running"] == 1
    assert stats["allocated_bytes"] <= need + (1 << 20)


def test_oversized_job_rejected_and_poll(slso):
    jobs = _jobs(1, seed=5, n_max=5000)
    jb = jobs[0]
    need = slso.workspace_size(jb["x"], jb["r"], jb["k"])
    srv = slso.Server(0, slots=1, hbm_budget=need - 1)
    with pytest.raises(slso.SlsoError) as e:
        srv.submit(jb["x"], jb["seed"], jb["r"], jb["k"])
    assert e.value.status == slso.ENOMEM
    srv.close()
    srv = slso.Server(0, slots=1, hbm_budget=need)
    t = srv.submit(jb["x"], jb["seed"], jb["r"], jb["k"])
    res = None
    for _ in range(100000):
        res = srv.poll(t)
        if res is not None:
            break
    if res is None:
        res = srv.wait(t)
    assert res["status"] >= 0
    with pytest.raises(slso.SlsoError):
        srv.poll(t)                      # retired ticket
    srv.close()
