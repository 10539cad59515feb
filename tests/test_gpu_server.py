"""Continuous-batching server: results alone equal results in a mix; admission respects the memory budget."""
import time

import numpy as np
import pytest

from gpu_helpers import require_gpu
from oracle import mera as om
from oracle import model
from paper_2007_03638_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    require_gpu()
    from paper_2007_03638_amd import api
    return api.Context(0)


def _jobs():
    out = []
    for k, (chi, kind, par) in enumerate([(4, "tfim", 1.0), (8, "xxz", 0.5), (4, "xxz", -0.3), (8, "tfim", 0.8)]):
        T = 2 if chi == 4 else 3
        dims = om.layer_dims(chi, T)
        init = [m for pair in inputs.mera_init(10 + k, dims) for m in pair]
        h3 = model.tfim_h3(par) if kind == "tfim" else model.xxz_h3(par)
        out.append(dict(T=T, chi=chi, h3=h3, init=init, prec="fp32", m=8, max_iter=6, grad_tol=1e-7,
                        polish_tol=0.0))
    return out


# Grouping needs jobs of one shape to meet at the same program; these tests exercise the grouped launches, so they
# give the leader a fixed 2 ms to wait for its members (the default bound, a tenth of a small program's run time,
# seldom lets the small jobs here meet).
GROUP_WAIT_US = 2000.0


def _wait(srv, ids, timeout=300):
    res = {}
    t0 = time.time()
    while len(res) < len(ids):
        for i in ids:
            if i not in res:
                r = srv.poll(i)
                if r is not None:
                    res[i] = r
        assert time.time() - t0 < timeout
        time.sleep(0.01)
    return [res[i] for i in ids]


def _run_all(ctx, jobs, slots, **opts):
    from paper_2007_03638_amd import api
    srv = api.Server(ctx, hbm_budget=64 << 30, max_slots=slots, **opts)
    ids = [srv.submit(**j) for j in jobs]
    res = _wait(srv, ids)
    st = srv.stats()
    srv.close()
    return res, st


def test_alone_equals_mix(ctx):
    """Each job alone (one slot, every kernel launched eagerly on its own stream) gives bit-identical results
    to the same job in a mix of four (grouped MFMA launches across same-shape jobs, graph replays)."""
    jobs = _jobs()
    alone = []
    for j in jobs:
        r, st = _run_all(ctx, [j], 1, group_launches=False, graph_capture=False)
        assert st["grouped_batches"] == 0 and st["graph_launches"] == 0
        alone += r
    mixed, st = _run_all(ctx, jobs, 4, max_wait_us=GROUP_WAIT_US)
    print("mix stats", st, flush=True)
    for a, b in zip(alone, mixed):
        print(a["energy"], b["energy"], a["iterations"], b["iterations"], flush=True)
        assert a["status"] == b["status"] == 1
        assert a["energy"] == b["energy"]
        assert a["gnorm"] == b["gnorm"]
        assert a["evaluations"] == b["evaluations"]
    # the mix did batch: same-shape jobs shared launches, and repeated programs ran from captured graphs
    assert st["grouped_batches"] > 0
    assert st["graph_captures"] > 0 and st["graph_launches"] > st["graph_captures"]
    assert st["bindings"] > st["batches"]


def test_grouping_and_graphs_separately(ctx):
    """Grouped launches without graphs, and graphs without grouping, each reproduce the eager results."""
    jobs = _jobs()[:2] + _jobs()[:2]       # two pairs of identical jobs
    ref, _ = _run_all(ctx, jobs[:2], 1, group_launches=False, graph_capture=False)
    for opts in (dict(group_launches=True, graph_capture=False), dict(group_launches=False, graph_capture=True)):
        res, st = _run_all(ctx, jobs, 4, max_wait_us=GROUP_WAIT_US, **opts)
        print(opts, st, flush=True)
        for k, r in enumerate(res):
            assert r["energy"] == ref[k % 2]["energy"]
            assert r["gnorm"] == ref[k % 2]["gnorm"]
            assert r["evaluations"] == ref[k % 2]["evaluations"]
        if opts["group_launches"]:
            assert st["grouped_batches"] > 0 and st["graph_launches"] == 0
        else:
            assert st["grouped_batches"] == 0 and st["graph_launches"] > 0


def test_default_wait_policy_mix_equals_alone(ctx):
    """With the default leader wait (bounded by the program's estimated run time) and a zero wait, a mix of two pairs
    of identical jobs still gives each job exactly its result alone, whether or not launches were grouped."""
    jobs = _jobs()[:2] + _jobs()[:2]
    ref, _ = _run_all(ctx, jobs[:2], 1, group_launches=False, graph_capture=False)
    for wait in (None, 0.0):
        res, st = _run_all(ctx, jobs, 4, max_wait_us=wait)
        print("max_wait_us", wait, st, flush=True)
        for k, r in enumerate(res):
            assert r["energy"] == ref[k % 2]["energy"]
            assert r["gnorm"] == ref[k % 2]["gnorm"]
            assert r["evaluations"] == ref[k % 2]["evaluations"]
        assert st["bindings"] >= st["batches"] > 0


def test_admission_budget(ctx):
    from paper_2007_03638_amd import api
    jobs = _jobs()
    fp = max(api.job_footprint(j["T"], j["chi"], "fp32") for j in jobs)
    srv = api.Server(ctx, hbm_budget=fp, max_slots=4)   # room for one job at a time
    ids = [srv.submit(**j) for j in jobs]
    res = _wait(srv, ids)
    srv.close()
    # with room for one job, each job waits for the previous one: queue times grow
    q = [r["queued_seconds"] for r in res]
    assert all(r["status"] == 1 for r in res)
    assert q[-1] > q[0]
    with pytest.raises(Exception):
        small = api.Server(ctx, hbm_budget=1 << 20, max_slots=1)
        small.submit(**jobs[0])


def test_nonfinite_job_fails_alone_in_a_mix(ctx):
    """Two jobs poisoned on the host (a NaN in the local term, a NaN in an initial disentangler) end with
    MERA_ENONFINITE, while the jobs running beside them, grouped with them where the shapes match, give exactly
    their results alone."""
    from paper_2007_03638_amd import api
    jobs = _jobs()
    alone = [_run_all(ctx, [j], 1, group_launches=False, graph_capture=False)[0][0] for j in jobs]
    bad_h = dict(jobs[0])
    bad_h["h3"] = bad_h["h3"].copy()
    bad_h["h3"][5, 5] = np.nan
    bad_u = dict(jobs[1])
    bad_u["init"] = [m.copy() for m in bad_u["init"]]
    bad_u["init"][2][3, 1] = np.nan
    srv = api.Server(ctx, hbm_budget=64 << 30, max_slots=4, max_wait_us=GROUP_WAIT_US)
    ids = [srv.submit(**j) for j in (jobs[0], bad_h, jobs[1], bad_u, jobs[2], jobs[3])]
    t0 = time.time()
    out = {}
    while len(out) < len(ids):
        for i in ids:
            if i in out:
                continue
            try:
                r = srv.poll(i)
            except api.MeraError as e:
                out[i] = e.status
                continue
            if r is not None:
                out[i] = r
        assert time.time() - t0 < 300
        time.sleep(0.01)
    st = srv.stats()
    srv.close()
    print("stats", st, "poisoned:", out[ids[1]], out[ids[3]], flush=True)
    assert out[ids[1]] == -5 and out[ids[3]] == -5
    for k, i in zip((0, 1, 2, 3), (ids[0], ids[2], ids[4], ids[5])):
        r = out[i]
        assert r["status"] == alone[k]["status"] == 1
        assert r["energy"] == alone[k]["energy"]
        assert r["gnorm"] == alone[k]["gnorm"]
        assert r["evaluations"] == alone[k]["evaluations"]


def test_job_arriving_mid_evaluation(ctx):
    """A job submitted while two jobs of its shape are running (their grouped programs under way) joins them and
    computes exactly what it computes alone; so do the two."""
    from paper_2007_03638_amd import api
    jobs = _jobs()
    j8 = [jobs[1], jobs[3], dict(jobs[1])]  # chi = 8 jobs; the third repeats the first
    alone = [_run_all(ctx, [j], 1, group_launches=False, graph_capture=False)[0][0] for j in j8[:2]]
    srv = api.Server(ctx, hbm_budget=64 << 30, max_slots=4, max_wait_us=GROUP_WAIT_US)
    ids = [srv.submit(**j8[0]), srv.submit(**j8[1])]
    t0 = time.time()
    while srv.stats()["grouped_batches"] < 3:  # the two running jobs share launches by now
        assert time.time() - t0 < 120
        time.sleep(0.002)
    assert srv.poll(ids[0]) is None and srv.poll(ids[1]) is None
    ids.append(srv.submit(**j8[2]))
    res = _wait(srv, ids)
    st = srv.stats()
    srv.close()
    print("stats", st, [r["energy"] for r in res], flush=True)
    for r, a in zip(res, [alone[0], alone[1], alone[0]]):
        assert r["energy"] == a["energy"] and r["gnorm"] == a["gnorm"] and r["evaluations"] == a["evaluations"]
    assert res[2]["queued_seconds"] < res[2]["seconds"]


def test_budget_below_one_job(ctx):
    """A job larger than the whole budget is refused at submission with MERA_ENOMEM; the server keeps serving jobs
    that fit."""
    from paper_2007_03638_amd import api
    jobs = _jobs()
    small = jobs[0]
    fp_small = api.job_footprint(small["T"], small["chi"], "fp32")
    fp_big = api.job_footprint(jobs[1]["T"], jobs[1]["chi"], "fp32")
    assert fp_big > fp_small
    srv = api.Server(ctx, hbm_budget=fp_small, max_slots=2)
    with pytest.raises(api.MeraError) as e:
        srv.submit(**jobs[1])
    assert e.value.status == -2
    ids = [srv.submit(**small)]
    res = _wait(srv, ids)
    srv.close()
    ref = _run_all(ctx, [small], 1, group_launches=False, graph_capture=False)[0][0]
    assert res[0]["energy"] == ref["energy"] and res[0]["status"] == 1
