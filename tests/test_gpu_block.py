"""GPU parity of the block-Jacobi PCG preconditioner and of the solves it drives.

The block form is the inner solve of the paper's experiments (section 6.2):
k Jacobi-PCG steps inside every 8-node block on the block's principal
submatrix.  Each case prints its name, sizes and seed before touching the GPU.
Bars: B(v) within 1e-10 relative (max norm) of the FP64 oracle; outer residual
histories over the first 20 iterations within 1e-9; full solves reach a true
residual <= rtol.  The mixed form is held to the FP64 oracle run on the
BF16-rounded viscosity (only FP32 arithmetic differs).
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


def _dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _bf16_round(x):
    b = np.asarray(x, dtype=np.float64).view(np.uint64)
    keep = b >> np.uint64(45)
    rem = b & np.uint64((1 << 45) - 1)
    half = np.uint64(1 << 44)
    up = (rem > half) | ((rem == half) & ((keep & np.uint64(1)) == np.uint64(1)))
    return ((keep + up.astype(np.uint64)) << np.uint64(45)).view(np.float64)


# (dim, n, convection): multiples of the workgroup span, ragged blocks, a grid
# smaller than one block, and a workgroup whose second block lies outside
SHAPES = [(3, 16, False), (3, 20, False), (3, 13, True), (3, 5, False), (3, 24, True),
          (2, 64, False), (2, 70, False), (2, 9, False)]


@pytest.mark.parametrize("k", [1, 2, 5])
@pytest.mark.parametrize("shape", SHAPES, ids=[f"{d}d-n{n}{'-conv' if c else ''}" for d, n, c in SHAPES])
def test_block_pcg_apply_matches_oracle(pfk, shape, k):
    dim, n, conv = shape
    _say("block pcg apply", dim, n, conv, k)
    p = gen.make_problem(dim, n, 4, 3.0, seed=n + k, convection=conv)
    Ao = oracle.StencilOperator(dim, n, p.eta, p.vel)
    Ag = pfk.Operator(dim, n, p.eta, p.vel)
    v = np.random.default_rng(k).standard_normal(Ao.N)
    y = _host(pfk.Precond(Ag, "block_jacobi_pcg", k, block=8).apply(_dev(v)))
    ref = oracle.make_pc("block_jacobi_pcg", Ao, k, block=8)(v)
    assert np.abs(y - ref).max() <= 1e-10 * np.abs(ref).max()


def test_block_pcg_zero_and_local_input(pfk):
    _say("block pcg zero / local")
    p = gen.make_problem(3, 16, 3, 3.0, seed=2)
    Ag = pfk.Operator(3, 16, p.eta)
    B = pfk.Precond(Ag, "block_jacobi_pcg", 5, block=8)
    assert not np.any(_host(B.apply(_dev(np.zeros(16 ** 3)))))
    # an input supported on one block gives an output supported on that block
    v = np.zeros((16, 16, 16))
    v[8:16, 0:8, 8:16] = np.random.default_rng(0).standard_normal((8, 8, 8))
    y = _host(B.apply(_dev(v.reshape(-1)))).reshape(16, 16, 16)
    mask = np.zeros_like(v, dtype=bool)
    mask[8:16, 0:8, 8:16] = True
    assert not np.any(y[~mask]) and np.any(y[mask])


def test_block_pcg_rejects_other_block_sizes(pfk):
    p = gen.make_problem(2, 16, 2, 2.0, seed=0)
    Ag = pfk.Operator(2, 16, p.eta)
    with pytest.raises(RuntimeError):
        pfk.Precond(Ag, "block_jacobi_pcg", 3, block=4)


@pytest.mark.parametrize("shape", [(3, 20, False), (3, 13, True), (2, 70, False)],
                         ids=["3d-n20", "3d-n13-conv", "2d-n70"])
def test_block_pcg_mixed_matches_rounded_oracle(pfk, shape):
    dim, n, conv = shape
    _say("block pcg mixed", dim, n, conv)
    p = gen.make_problem(dim, n, 6, 4.0, seed=7, convection=conv)
    Ar = oracle.StencilOperator(dim, n, _bf16_round(p.eta),
                                None if p.vel is None else p.vel.astype(np.float32).astype(np.float64))
    Ag = pfk.Operator(dim, n, p.eta, p.vel)
    v = np.random.default_rng(1).standard_normal(Ar.N)
    y = _host(pfk.Precond(Ag, "block_jacobi_pcg", 5, precision=pfk.FP32_BF16COEF, block=8).apply(_dev(v)))
    ref = oracle.make_pc("block_jacobi_pcg", Ar, 5, block=8)(v)
    err = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    print(f"  mixed block PCG vs FP64-on-BF16-eta: {err:.2e}")
    assert err <= 1e-5


def _parity(pfk, method, prob, k, m, its, rtol=0.0, precision=None):
    Ao = oracle.StencilOperator(prob.dim, prob.n, prob.eta, prob.vel)
    Bo = oracle.make_pc("block_jacobi_pcg", Ao, k, block=8)
    sigma = oracle.estimate_sigma(Ao.apply, Bo, Ao.N) if method == "pipefgmres" else None
    ref = oracle.solve(method, Ao, Bo, prob.b, rtol=rtol, maxit=its, nu_max=m, sigma=sigma)
    Ag = pfk.Operator(prob.dim, prob.n, prob.eta, prob.vel)
    kw = {} if precision is None else {"precision": precision}
    Bg = pfk.Precond(Ag, "block_jacobi_pcg", k, block=8, **kw)
    x = _dev(np.zeros(Ao.N))
    opts = {} if sigma is None else {"shift_sigma": float(sigma)}
    info = pfk.solve(Ag, Bg, method, _dev(prob.b), x, rtol=rtol, maxit=its, mmax=m, **opts)
    return ref, info, _host(x), Ao


@pytest.mark.parametrize("method", ["fcg", "pipefcg", "gcr", "pipegcr", "fgmres", "pipefgmres"])
def test_history_parity_first_20(pfk, method):
    conv = method not in ("fcg", "pipefcg")
    prob = gen.make_problem(3, 20, 6, 3.0, seed=11, convection=conv)
    _say("block history", method)
    ref, info, x, _ = _parity(pfk, method, prob, 5, 30, 20)
    h, hr = info.history, np.array(ref.history)
    assert len(h) == len(hr) == 21
    rel = np.abs(h - hr) / np.abs(hr)
    assert rel.max() <= 1e-9, rel


@pytest.mark.parametrize("cfg", ["cfg1", "3d-n24"])
def test_pipefcg_converges_like_oracle(pfk, cfg):
    # with the block form the pipelined CG converges (the global inner CG makes it stagnate)
    prob = gen.config_problem("cfg1", seed=0) if cfg == "cfg1" else gen.make_problem(3, 24, 8, 4.0, seed=3)
    _say("block pipefcg full solve", cfg)
    for method in ("fcg", "pipefcg"):
        ref, info, x, Ao = _parity(pfk, method, prob, 5, 30, 2000, rtol=1e-8)
        true_rel = np.linalg.norm(prob.b - Ao.apply(x)) / np.linalg.norm(prob.b)
        print(f"  {method}: its {info.iterations} (oracle {ref.iterations}), true rel {true_rel:.2e}")
        assert ref.converged and info.converged and info.status == 0
        assert true_rel <= 1e-8
        assert abs(info.iterations - ref.iterations) <= max(3, ref.iterations // 5)


def test_mixed_block_pipefcg_reaches_tolerance(pfk):
    prob = gen.make_problem(3, 24, 8, 4.0, seed=3)
    _say("block pipefcg mixed")
    ref, info, x, Ao = _parity(pfk, "pipefcg", prob, 4, 20, 2000, rtol=1e-8, precision=pfk.FP32_BF16COEF)
    true_rel = np.linalg.norm(prob.b - Ao.apply(x)) / np.linalg.norm(prob.b)
    sol_err = np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x)
    print(f"  mixed pipefcg: its {info.iterations} (FP64 oracle {ref.iterations}), true rel {true_rel:.2e}, "
          f"error vs FP64 solution {sol_err:.2e}")
    assert info.converged and true_rel <= 1e-8
    assert sol_err <= 1e-5
