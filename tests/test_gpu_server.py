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


def test_alone_equals_mix(ctx):
    from paper_2007_03638_amd import api
    jobs = _jobs()
    alone = []
    for j in jobs:
        srv = api.Server(ctx, hbm_budget=64 << 30, max_slots=1)
        alone += _wait(srv, [srv.submit(**j)])
        srv.close()
    srv = api.Server(ctx, hbm_budget=64 << 30, max_slots=4)
    ids = [srv.submit(**j) for j in jobs]
    mixed = _wait(srv, ids)
    srv.close()
    for a, b in zip(alone, mixed):
        print(a["energy"], b["energy"], a["iterations"], b["iterations"], flush=True)
        assert a["status"] == b["status"] == 1
        assert a["energy"] == b["energy"]
        assert a["gnorm"] == b["gnorm"]
        assert a["evaluations"] == b["evaluations"]


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
