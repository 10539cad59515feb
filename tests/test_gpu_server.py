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
    mixed, st = _run_all(ctx, jobs, 4)
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
        res, st = _run_all(ctx, jobs, 4, **opts)
        print(opts, st, flush=True)
        for k, r in enumerate(res):
            assert r["energy"] == ref[k % 2]["energy"]
            assert r["gnorm"] == ref[k % 2]["gnorm"]
            assert r["evaluations"] == ref[k % 2]["evaluations"]
        if opts["group_launches"]:
            assert st["grouped_batches"] > 0 and st["graph_launches"] == 0
        else:
            assert st["grouped_batches"] == 0 and st["graph_launches"] > 0


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
