"""Whole-output parity at the benchmark's bond dimension (chi = 24, the scale-invariant layer: a = b = 24), through
the C ABI, in the launch configuration of an evaluation (same tiles, k-walk variants and split-K choices).

The operators are sums of products of one-site matrices, A (x) B (x) C + A^T (x) B^T (x) C^T (symmetric while no
factor is), passed to the GPU as dense FP64 operators: the kernels see dense chi^6 operands, while the oracle
contracts the same networks with the factors in place (oracle.mera.ascend_product, descend_product,
layer_environments_product, pinned against the dense forms), which takes seconds instead of hours. Every element
of every output is compared."""
import numpy as np
import pytest
import torch

from gpu_helpers import require_gpu, to_np
from oracle import mera as om
from paper_2007_03638_amd import inputs

pytestmark = pytest.mark.gpu

T, CHI, LAYER = 3, 24, 3
# Largest elementwise difference relative to the largest reference element. Layer maps: FP64 1e-12; FP32 2e-6 (three
# chained FP32 contractions with K <= chi^3); split-bf16 1e-4 (about 16 mantissa bits per product). The gradient
# chains up to seven FP32 contractions, the longest over K = chi^4 = 331776 terms (split-K partials summed in FP64):
# a random-walk rounding estimate sqrt(K) 2^-24 = 3.4e-5 of the terms' scale, measured 3.1e-6 of max |D|; bound 1e-5.
TOL = {"fp64": 1e-12, "fp32": 2e-6, "bf16x3": 1e-4}
GRAD_TOL = {"fp64": 1e-12, "fp32": 1e-5, "bf16x3": 1e-4}


def _terms(seed, n):
    (f,) = inputs.one_site_factors(seed, n, 1)
    return [f, tuple(x.T for x in f)]


@pytest.fixture(scope="module")
def ctx():
    require_gpu()
    from paper_2007_03638_amd import api
    return api.Context(0)


@pytest.fixture(scope="module")
def case():
    (u, w), = inputs.mera_init(2024, [(CHI, CHI)])
    ht = _terms(2025, CHI)
    rt = _terms(2026, CHI)
    return dict(u=u, w=w, ht=ht, rt=rt, h=om.product_operator(ht), rho=om.product_operator(rt))


@pytest.fixture(scope="module")
def asc_ref(case):
    return om.ascend_product(case["ht"], case["u"], case["w"], CHI, CHI)


@pytest.fixture(scope="module")
def des_ref(case):
    return om.descend_product(case["rt"], case["u"], case["w"], CHI, CHI)


@pytest.fixture(scope="module")
def env_ref(case):
    return om.layer_environments_product(case["ht"], case["rt"], case["u"], case["w"], CHI, CHI)


def _err(got, ref):
    """Largest elementwise difference relative to the largest reference element."""
    g = got.detach().to("cpu", torch.float64).numpy() if torch.is_tensor(got) else got
    return float(np.max(np.abs(g - ref)) / np.max(np.abs(ref)))


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp64"])
def test_ascend_whole_output(ctx, case, asc_ref, prec):
    got = ctx.ascend(T, CHI, LAYER, case["u"], case["w"], case["h"], prec=prec)
    err = _err(got, asc_ref)
    print(f"chi=24 ascend {prec}: max rel err {err:.2e} over {asc_ref.size} elements", flush=True)
    assert err < TOL[prec]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp64"])
def test_descend_whole_output(ctx, case, des_ref, prec):
    got = ctx.descend(T, CHI, LAYER, case["u"], case["w"], case["rho"], prec=prec)
    err = _err(got, des_ref)
    print(f"chi=24 descend {prec}: max rel err {err:.2e} over {des_ref.size} elements", flush=True)
    assert err < TOL[prec]


@pytest.mark.parametrize("split", [False, True])
@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp64"])
def test_layer_grad_whole_output(ctx, case, env_ref, des_ref, asc_ref, prec, split):
    ctx.profile(True)
    Du, Dw, ro, ho = ctx.layer_grad(T, CHI, LAYER, case["u"], case["w"], case["h"], case["rho"], prec=prec,
                                    split=split)
    stats = ctx.kernel_stats()
    ctx.profile(False)
    errs = dict(Du=_err(Du, env_ref[0]), Dw=_err(Dw, env_ref[1]), rho=_err(ro, des_ref))
    if split:
        errs["h"] = _err(ho, asc_ref)
    names = sorted(s["kernel"] for s in stats)
    print(f"chi=24 layer_grad {prec} split={split}: " + " ".join(f"{k} {v:.2e}" for k, v in errs.items())
          + f"; variants {names}", flush=True)
    assert errs["rho"] < TOL[prec] and errs.get("h", 0.0) < TOL[prec]
    assert max(errs["Du"], errs["Dw"]) < GRAD_TOL[prec]
    if prec == "fp32":
        # the benchmark's kernel paths ran: 192 x 192 tiles, four-leg k walks and split-K reductions
        assert any("192x192" in n for n in names)
        assert any(",k4" in n for n in names)
        assert any("splitk" in n for n in names)
