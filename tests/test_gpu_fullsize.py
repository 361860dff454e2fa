"""Full-size checks in the launch configuration bench.py times (256^3 sinker,
nu_max 30, 5-step global Jacobi-PCG, the autotuned geometry of the PIPEFCG
run: 64x8 tiles, 1024 stencil workgroups, 16384 vector workgroups).

The oracle cannot run 256^3 iterations in test time, so these hold the GPU to
properties the oracle can check at any size: after 20 iterations the residual
the method recurred (history) must equal the true residual ||b - A x|| that
the oracle's FP64 operator computes from the GPU's iterate, and the residual
must have decreased.  Each case prints its name first.
"""
import sys

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu


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


@pytest.fixture(scope="module")
def big():
    return gen.config_problem("cfgM", seed=0)


@pytest.mark.parametrize("method,tiling", [("pipefcg", (64, 1024, 16384)), ("fcg", (64, 1024, 4096))])
def test_recurred_residual_is_the_true_residual_at_256(pfk, big, method, tiling):
    import torch
    _say("full size", method, tiling)
    A = pfk.Operator(3, 256, big.eta)
    A.set_tiling(*tiling)
    B = pfk.Precond(A, "jacobi_pcg", 5)
    b = torch.as_tensor(big.b).cuda()
    x = torch.zeros_like(b)
    info = pfk.solve(A, B, method, b, x, rtol=0.0, maxit=20, mmax=30)
    torch.cuda.synchronize()
    xs = x.cpu().numpy()
    del x, b
    Ao = oracle.StencilOperator(3, 256, big.eta)
    true = np.linalg.norm(big.b - Ao.apply(xs))
    rec = info.history[-1]
    print(f"  {method}: recurred {rec:.6e}, true {true:.6e}, ||b|| {np.linalg.norm(big.b):.6e}")
    assert len(info.history) == 21
    assert info.history[-1] < 0.5 * info.history[0]
    bn = np.linalg.norm(big.b)
    assert abs(true - rec) <= 1e-9 * bn
    # the library's own final true-residual check agrees with the oracle's operator
    assert abs(info.true_rel_resid * bn - true) <= 1e-10 * bn
