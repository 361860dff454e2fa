"""Failure reporting forced from the host: non-finite data.

A NaN or an infinity in b (or one that enters x) reaches the first residual
norm; every method reports PFK_ERR_NONFINITE instead of iterating on it,
graph-launched and direct.  Breakdown restarts, breakdown of the initial
direction and maxit exhaustion are covered with the method parity tests.
Each case prints its name before touching the GPU.
"""
import sys

import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu

METHODS = ["fcg", "pipefcg", "pipefcg_naive", "gcr", "pipegcr", "pipegcr_w", "fgmres", "pipefgmres"]


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pfk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1511_07226_amd as pfk
    pfk.lib()
    return pfk


def _dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.mark.parametrize("bad", ["nan_b", "inf_b", "nan_x0"])
@pytest.mark.parametrize("use_graph", [1, 0], ids=["graph", "direct"])
@pytest.mark.parametrize("method", METHODS)
def test_nonfinite_input_is_reported(pfk, method, use_graph, bad):
    _say("nonfinite", method, bad, "graph" if use_graph else "direct")
    p = gen.make_problem(3, 10, 3, 2.0, seed=5, convection=False)
    A = pfk.Operator(3, 10, p.eta, None)
    B = pfk.Precond(A, "jacobi_pcg", 2)
    b = p.b.copy()
    x0 = np.zeros(A.N)
    if bad == "nan_b":
        b[123] = np.nan
    elif bad == "inf_b":
        b[7] = np.inf
    else:
        x0[500] = np.nan
    extra = {"shift_sigma": 1.0} if method == "pipefgmres" else {}
    with pytest.raises(pfk.PfkError) as ei:
        pfk.solve(A, B, method, _dev(b), _dev(x0), rtol=1e-8, maxit=50, mmax=10, use_graph=use_graph, **extra)
    assert ei.value.code == -4                  # PFK_ERR_NONFINITE
