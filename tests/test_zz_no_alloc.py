"""The allocation-free tangent projection stiefel_project_noalloc against stiefel_project, through the C ABI.

Two calls in a row on the same GPU (the second with smaller factors, reusing the fixed scratch array), a call whose
output aliases D, an empty call, and the size limit. Both entry points compute G = D - W (W^T D + D^T W)/2 in FP64
with different summation orders: they agree to 1e-12 of the largest element of G."""
import numpy as np
import pytest
import torch

from gpu_helpers import rel, require_gpu, to_np
from oracle import manifold as mf
from paper_2007_03638_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    require_gpu()
    from paper_2007_03638_amd import api
    return api.Context(0)


def _case(ctx, seed, shapes):
    W = [ctx._dev(x) for x in inputs.haar_params(seed, shapes)]
    D = [ctx._dev(x) for x in inputs.normal_like(seed + 1, [np.zeros(s) for s in shapes])]
    return W, D


def _check(ctx, W, D, tag):
    ref = ctx.stiefel_project(W, D)
    got = ctx.stiefel_project_noalloc(W, D)
    torch.cuda.synchronize()
    for i, (g, r) in enumerate(zip(got, ref)):
        e = rel(to_np(g), to_np(r))
        print(f"{tag} factor {i} {tuple(g.shape)}: rel diff to stiefel_project {e:.2e}", flush=True)
        assert e < 1e-12
        assert rel(to_np(g), mf.project(to_np(W[i]), to_np(D[i]))) < 1e-12


def test_two_calls_second_smaller(ctx):
    # the factor shapes of the chi = 24 binary MERA (T = 3), then a smaller set
    big = [(576, 576), (576, 24), (256, 256), (256, 24), (16, 16), (16, 16), (1024, 32), (13824, 24)]
    W, D = _case(ctx, 40, big)
    _check(ctx, W, D, "call 1")
    W, D = _case(ctx, 41, [(64, 8), (16, 16), (9, 3)])
    _check(ctx, W, D, "call 2")


def test_largest_square_factor_and_aliasing(ctx):
    W, D = _case(ctx, 42, [(1024, 1024), (37, 5)])
    ref = ctx.stiefel_project(W, D)
    out = ctx.stiefel_project_noalloc(W, D, G=D)  # G aliases D
    torch.cuda.synchronize()
    for g, r in zip(out, ref):
        assert g.data_ptr() in [d.data_ptr() for d in D]
        assert rel(to_np(g), to_np(r)) < 1e-12


def test_limits_and_empty_call(ctx):
    from paper_2007_03638_amd import api
    assert ctx.stiefel_project_noalloc([], []) == []
    W, D = _case(ctx, 43, [(1100, 1025)])
    with pytest.raises(api.MeraError) as e:
        ctx.stiefel_project_noalloc(W, D)
    assert e.value.status == -1 and "p <= 1024" in str(e.value)
    W, D = _case(ctx, 44, [(20, 6)])
    with pytest.raises(api.MeraError) as e:
        ctx.stiefel_project_noalloc(W, D, G=W)
    assert e.value.status == -1
    # the context and the entry point keep working
    _check(ctx, W, D, "after errors")
