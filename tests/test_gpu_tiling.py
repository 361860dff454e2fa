"""Launch geometry: the 32 x 16 stencil tile, odd workgroup counts and the
autotuner change performance only.  Every case is held to the FP64 oracle:
operator applies within 1e-12 (max norm), residual histories over the first
20 iterations within 1e-9.
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


SHAPES = [(3, 20, False), (3, 13, True), (2, 70, False), (3, 33, False), (2, 5, False)]
TILINGS = [(32, 8, 1), (32, 2048, 7), (64, 3, 300), (32, 16384, 64)]


@pytest.mark.parametrize("tiling", TILINGS, ids=[f"tx{t[0]}-s{t[1]}-v{t[2]}" for t in TILINGS])
@pytest.mark.parametrize("shape", SHAPES, ids=[f"{d}d-n{n}{'-conv' if c else ''}" for d, n, c in SHAPES])
def test_operator_apply_any_tiling(pfk, shape, tiling):
    dim, n, conv = shape
    _say("tiling apply", shape, tiling)
    p = gen.make_problem(dim, n, 4, 3.0, seed=n, convection=conv)
    Ao = oracle.StencilOperator(dim, n, p.eta, p.vel)
    Ag = pfk.Operator(dim, n, p.eta, p.vel)
    Ag.set_tiling(*tiling)
    assert Ag.tiling()[0] == tiling[0] and Ag.tiling()[2] == tiling[2]
    u = np.random.default_rng(n).standard_normal(Ao.N)
    y = _host(Ag.apply(_dev(u)))
    ref = Ao.apply(u)
    assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()


def test_set_tiling_rejects_bad_values(pfk):
    p = gen.make_problem(2, 16, 2, 2.0, seed=0)
    Ag = pfk.Operator(2, 16, p.eta)
    for bad in [(48, 64, 64), (64, 0, 64), (64, 64, 0), (32, 64, 20000)]:
        with pytest.raises(RuntimeError):
            Ag.set_tiling(*bad)


CASES = [("pipefcg", "block_jacobi_pcg", False), ("fcg", "jacobi_pcg", False),
         ("pipefgmres", "jacobi_gmres", True), ("gcr", "block_jacobi_pcg", True),
         ("pipegcr", "jacobi", True), ("fgmres", "block_jacobi_pcg", True)]


@pytest.mark.parametrize("case", CASES, ids=[f"{m}-{k}" for m, k, _ in CASES])
def test_history_parity_with_narrow_tiles(pfk, case):
    method, kind, conv = case
    _say("tiling history", method, kind)
    prob = gen.make_problem(3, 21, 6, 3.0, seed=5, convection=conv)
    Ao = oracle.StencilOperator(3, 21, prob.eta, prob.vel)
    Bo = oracle.make_pc(kind, Ao, 3, block=8)
    sigma = oracle.estimate_sigma(Ao.apply, Bo, Ao.N) if method == "pipefgmres" else None
    ref = oracle.solve(method, Ao, Bo, prob.b, rtol=0.0, maxit=20, nu_max=30, sigma=sigma)
    Ag = pfk.Operator(3, 21, prob.eta, prob.vel)
    Ag.set_tiling(32, 5, 13)
    Bg = pfk.Precond(Ag, kind, 3, block=8)
    x = _dev(np.zeros(Ao.N))
    opts = {} if sigma is None else {"shift_sigma": float(sigma)}
    info = pfk.solve(Ag, Bg, method, _dev(prob.b), x, rtol=0.0, maxit=20, mmax=30, **opts)
    rel = np.abs(info.history - np.array(ref.history)) / np.abs(np.array(ref.history))
    assert len(info.history) == 21 and rel.max() <= 1e-9, rel


@pytest.mark.parametrize("method", ["pipefcg", "pipefgmres"])
def test_autotune_picks_a_valid_geometry(pfk, method):
    _say("autotune", method)
    prob = gen.make_problem(3, 48, 8, 3.0, seed=2, convection=(method == "pipefgmres"))
    Ag = pfk.Operator(3, 48, prob.eta, prob.vel)
    Bg = pfk.Precond(Ag, "block_jacobi_pcg", 4, block=8)
    res = Ag.autotune(Bg, method, mmax=20, reps=4)
    print("  ", res)
    assert res["tile_x"] in (32, 64) and res["candidates"] >= 5
    assert 0 < res["ms_per_iteration"] <= res["ms_default"]
    assert Ag.tiling() == (res["tile_x"], res["stencil_blocks"], res["vector_blocks"])
    # a solve on the tuned operator still follows the oracle
    Ao = oracle.StencilOperator(3, 48, prob.eta, prob.vel)
    Bo = oracle.make_pc("block_jacobi_pcg", Ao, 4, block=8)
    sigma = oracle.estimate_sigma(Ao.apply, Bo, Ao.N) if method == "pipefgmres" else None
    ref = oracle.solve(method, Ao, Bo, prob.b, rtol=0.0, maxit=20, nu_max=20, sigma=sigma)
    x = _dev(np.zeros(Ao.N))
    opts = {} if sigma is None else {"shift_sigma": float(sigma)}
    info = pfk.solve(Ag, Bg, method, _dev(prob.b), x, rtol=0.0, maxit=20, mmax=20, **opts)
    rel = np.abs(info.history - np.array(ref.history)) / np.abs(np.array(ref.history))
    assert rel.max() <= 1e-9, rel
