"""GPU mixed precision on viscosity that varies from node to node.

The sinker fields take two values (1 and the contrast), and at 1e4 the BF16
value is the same whether the FP64 number is rounded to nearest (ties to
even) or truncated.  Here log10(eta) is drawn U(0, 4) at every node, so
almost every coefficient sits between two BF16 numbers and the rounding rule
shows: the mixed inner solves (FP32 sweeps on BF16 viscosity, FP32
velocities) are compared node by node with the FP64 oracle run on the
round-to-nearest-even copy, and must sit far closer to it than to the oracle
run on the truncated copy.  What remains is FP32 arithmetic.

Bounds: every node within 5e-5 of the reference, relative to the larger of
its own magnitude and 1e-3 of the largest (a node near zero is held to the
output's scale; measured 4e-6 to 1.3e-5 -- k FP32 inner steps on
coefficients spanning four decades), the whole vector within 3e-6 in norm,
and at least 1000 times closer to the nearest-even reference than to the
truncated one (measured ratios above 1e4).
"""
import sys

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

NODE_BOUND = 5e-5
NORM_BOUND = 3e-6


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


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def bf16_nearest_even(x):
    """BF16 value nearest to each positive normal FP64 number, ties to even."""
    b = np.asarray(x, dtype=np.float64).view(np.uint64)
    keep = b >> np.uint64(45)
    rem = b & np.uint64((1 << 45) - 1)
    half = np.uint64(1 << 44)
    up = (rem > half) | ((rem == half) & ((keep & np.uint64(1)) == np.uint64(1)))
    return ((keep + up.astype(np.uint64)) << np.uint64(45)).view(np.float64)


def bf16_truncated(x):
    """BF16 value of each positive FP64 number with the low bits dropped."""
    b = np.asarray(x, dtype=np.float64).view(np.uint64)
    return ((b >> np.uint64(45)) << np.uint64(45)).view(np.float64)


def test_rounding_rules_differ_on_the_graded_field():
    p = gen.graded_problem(3, 12, (0.0, 4.0), seed=1)
    rne, tr = bf16_nearest_even(p.eta), bf16_truncated(p.eta)
    assert np.mean(rne != tr) > 0.4            # about half of the nodes round up
    assert np.all(np.abs(rne - p.eta) <= np.abs(tr - p.eta))
    assert np.all(np.abs(rne - p.eta) <= 2.0 ** -8 * p.eta)


def _node_err(y, ref):
    scale = np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
    return float(np.max(np.abs(y - ref) / scale))


CASES = [("jacobi_pcg", 5, 3, 20, False), ("jacobi_gmres", 5, 3, 17, True),
         ("block_jacobi_pcg", 5, 3, 20, False), ("block_jacobi_pcg", 4, 3, 13, True),
         ("jacobi_pcg", 2, 2, 70, False)]


@pytest.mark.parametrize("kind,k,dim,n,conv", CASES, ids=[f"{c[0]}-{c[1]}-{c[2]}d-n{c[3]}" for c in CASES])
def test_mixed_inner_solve_node_by_node(pfk, kind, k, dim, n, conv):
    _say("mixed rounding", kind, k, dim, n, conv)
    p = gen.graded_problem(dim, n, (0.0, 4.0), seed=n, convection=conv)
    vel32 = None if p.vel is None else p.vel.astype(np.float32).astype(np.float64)
    A_rne = oracle.StencilOperator(dim, n, bf16_nearest_even(p.eta), vel32)
    A_tr = oracle.StencilOperator(dim, n, bf16_truncated(p.eta), vel32)
    Ag = pfk.Operator(dim, n, p.eta, p.vel)
    v = np.random.default_rng(n).standard_normal(A_rne.N)
    y = _host(pfk.Precond(Ag, kind, k, precision=pfk.FP32_BF16COEF, block=8).apply(_dev(v)))
    ref = oracle.make_pc(kind, A_rne, k, block=8)(v)
    ref_tr = oracle.make_pc(kind, A_tr, k, block=8)(v)
    e_rne, e_tr = _node_err(y, ref), _node_err(y, ref_tr)
    e_norm = float(np.linalg.norm(y - ref) / np.linalg.norm(ref))
    print(f"  largest node difference: vs nearest-even {e_rne:.2e}, vs truncated {e_tr:.2e}; "
          f"norm-relative {e_norm:.2e}")
    assert e_rne <= NODE_BOUND
    assert e_norm <= NORM_BOUND
    assert e_tr >= 1000 * e_rne
