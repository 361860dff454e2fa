"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Every case prints its name, sizes and seed before touching the GPU.
Tolerances: the operator and preconditioner agree to rounding (1e-12 relative
to the output's scale; summation orders differ); residual histories over the
first 20 iterations to 1e-9 relative, the bar the solver is held to.
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


OPERATOR_CASES = [
    (2, 64, 8, 3.0, False, 0),
    (2, 100, 8, 3.0, False, 1),     # ragged against the 64 x 4 tile
    (3, 37, 20, 4.0, False, 2),     # ragged in every direction
    (3, 20, 5, 2.0, True, 3),       # convection-diffusion
    (2, 1, 1, 0.0, False, 4),       # a single unknown
    (3, 2, 1, 1.0, True, 5),
]


@pytest.mark.parametrize("dim,n,ninc,contrast,conv,seed", OPERATOR_CASES)
def test_operator_apply_matches_oracle(pfk, dim, n, ninc, contrast, conv, seed):
    _say("operator", dim, n, conv, seed)
    p = gen.make_problem(dim, n, ninc, contrast, seed, convection=conv)
    Ao = oracle.StencilOperator(dim, n, p.eta, p.vel)
    Ag = pfk.Operator(dim, n, p.eta, p.vel)
    u = np.random.default_rng(seed).standard_normal(Ao.N)
    y = _host(Ag.apply(_dev(u)))
    ref = Ao.apply(u)
    assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()
    dinv = _host(Ag.diag_inv())
    assert np.allclose(dinv, 1.0 / Ao.diagonal(), rtol=1e-13)


def test_operator_sampled_at_full_size(pfk):
    # the 256^3 workload operator, checked node by node on sampled outputs
    n = 256
    _say("operator sampled", n)
    p = gen.config_problem("cfgM", seed=0)
    Ao = oracle.StencilOperator(3, n, p.eta)
    Ag = pfk.Operator(3, n, p.eta)
    u = np.random.default_rng(0).standard_normal(Ao.N)
    y = _host(Ag.apply(_dev(u)))
    idx = np.random.default_rng(1).integers(0, Ao.N, 400)
    idx = np.concatenate([idx, [0, Ao.N - 1, n - 1, n * n - 1, n * n * (n - 1)]])
    ref = Ao.apply_at(u, idx)
    assert np.abs(y[idx] - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("kind,k", [("none", 1), ("jacobi", 1), ("jacobi_pcg", 1), ("jacobi_pcg", 2),
                                    ("jacobi_pcg", 5)])
@pytest.mark.parametrize("dim,n", [(2, 64), (3, 33)])
def test_preconditioner_matches_oracle(pfk, kind, k, dim, n):
    _say("precond", kind, k, dim, n)
    p = gen.make_problem(dim, n, 8, 3.0, seed=3)
    Ao = oracle.StencilOperator(dim, n, p.eta)
    Bo = oracle.make_pc(kind, Ao, k)
    Ag = pfk.Operator(dim, n, p.eta)
    Bg = pfk.Precond(Ag, kind, k)
    v = np.random.default_rng(4).standard_normal(Ao.N)
    y = _host(Bg.apply(_dev(v)))
    ref = Bo(v)
    assert np.abs(y - ref).max() <= 1e-11 * np.abs(ref).max()


def test_preconditioner_zero_input(pfk):
    _say("precond zero")
    p = gen.make_problem(2, 16, 2, 2.0, seed=0)
    Ag = pfk.Operator(2, 16, p.eta)
    y = _host(pfk.Precond(Ag, "jacobi_pcg", 3).apply(_dev(np.zeros(256))))
    assert not np.any(y)


def _parity_solve(pfk, method, prob, kind, k, nu, its, rtol=0.0, **kw):
    Ao = oracle.StencilOperator(prob.dim, prob.n, prob.eta, prob.vel)
    ref = oracle.solve(method, Ao, oracle.make_pc(kind, Ao, k), prob.b, rtol=rtol, maxit=its, nu_max=nu,
                       force_breakdown_at=kw.get("force_breakdown_at", -1))
    Ag = pfk.Operator(prob.dim, prob.n, prob.eta, prob.vel)
    Bg = pfk.Precond(Ag, kind, k)
    x = _dev(np.zeros(Ao.N))
    info = pfk.solve(Ag, Bg, method, _dev(prob.b), x, rtol=rtol, maxit=its, mmax=nu, **kw)
    return ref, info, _host(x), Ao


@pytest.mark.parametrize("method", ["fcg", "pipefcg"])
@pytest.mark.parametrize("cfg", ["cfg1", "cfg2_small"])
def test_history_parity_first_20(pfk, method, cfg):
    if cfg == "cfg1":
        prob, k = gen.config_problem("cfg1", seed=0), 2
    else:
        prob, k = gen.config_problem("cfg2", seed=0, n=40), 5
    _say("history", method, cfg, prob.n)
    ref, info, x, _ = _parity_solve(pfk, method, prob, "jacobi_pcg", k, 30, 20)
    h, hr = info.history, np.array(ref.history)
    assert len(h) == len(hr) == 21
    rel = np.abs(h - hr) / np.abs(hr)
    assert rel.max() <= 1e-9, rel
    assert np.allclose(x, ref.x, rtol=0, atol=1e-9 * np.abs(ref.x).max())


@pytest.mark.parametrize("method", ["fcg", "pipefcg"])
def test_full_solve_cfg1(pfk, method):
    prob = gen.config_problem("cfg1", seed=0)
    kind = "jacobi_pcg" if method == "fcg" else "jacobi"
    _say("full solve cfg1", method, kind)
    ref, info, x, Ao = _parity_solve(pfk, method, prob, kind, 2, 30, 2000, rtol=1e-8)
    assert ref.converged and info.converged and info.status == 0
    # the first 20 iterations are held to 1e-9 elsewhere; over a whole solve the
    # two rounding sequences separate near convergence (residual-gap restarts)
    assert abs(info.iterations - ref.iterations) <= max(2, ref.iterations // 5)
    assert np.linalg.norm(prob.b - Ao.apply(x)) <= 1e-8 * np.linalg.norm(prob.b)
    assert info.true_rel_resid <= 1e-8


def test_pipefcg_global_pc_stagnates_like_oracle(pfk):
    # with the global few-step inner CG the pipelined method stagnates (not a
    # faithful preconditioner); the GPU must reproduce the oracle's plateau
    prob = gen.config_problem("cfg1", seed=0)
    _say("pipefcg plateau cfg1")
    ref, info, x, _ = _parity_solve(pfk, "pipefcg", prob, "jacobi_pcg", 2, 30, 300, rtol=1e-8)
    assert not ref.converged and info.status == 1 and info.iterations == 300
    h, hr = info.history, np.array(ref.history)
    assert np.abs(np.log10(h[-50:]) - np.log10(hr[-50:])).max() < 0.5


def test_edge_cases(pfk):
    prob = gen.config_problem("cfg1", seed=1)
    Ag = pfk.Operator(2, 64, prob.eta)
    Bg = pfk.Precond(Ag, "jacobi_pcg", 2)
    _say("edge: b = 0")
    x = _dev(np.ones(4096))
    info = pfk.solve(Ag, Bg, "pipefcg", _dev(np.zeros(4096)), x, rtol=1e-8, maxit=50, mmax=30)
    assert info.status == 0 and info.iterations == 0 and not np.any(_host(x))
    _say("edge: maxit")
    for method in ("fcg", "pipefcg"):
        x = _dev(np.zeros(4096))
        info = pfk.solve(Ag, Bg, method, _dev(prob.b), x, rtol=1e-12, maxit=7, mmax=30)
        assert info.status == 1 and info.iterations == 7 and len(info.history) == 8
    _say("edge: maxit 0")
    info = pfk.solve(Ag, Bg, "fcg", _dev(prob.b), _dev(np.zeros(4096)), rtol=1e-8, maxit=0, mmax=30)
    assert info.status == 1 and info.iterations == 0
    _say("edge: window 1 and 64")
    for nu in (1, 64):
        ref, info, x, _ = _parity_solve(pfk, "pipefcg", prob, "jacobi", 1, nu, 15)
        assert np.allclose(info.history, ref.history, rtol=1e-9)


@pytest.mark.parametrize("method", ["fcg", "pipefcg"])
def test_forced_breakdown_restart(pfk, method):
    prob = gen.config_problem("cfg1", seed=2)
    _say("forced breakdown", method)
    ref, info, x, _ = _parity_solve(pfk, method, prob, "jacobi", 1, 30, 30, rtol=0.0, force_breakdown_at=6)
    assert ref.restarts == 1 and info.restarts == 1
    assert info.iterations == ref.iterations == 30
    n = len(ref.history)
    assert np.allclose(info.history[:n], ref.history[:n], rtol=1e-9)


@pytest.mark.parametrize("truncation", [1, 2])
def test_truncation_rules_parity(pfk, truncation):
    prob = gen.config_problem("cfg1", seed=3)
    rule = {1: "notay", 2: "modp1"}[truncation]
    _say("truncation", rule)
    Ao = oracle.StencilOperator(2, 64, prob.eta)
    ref = oracle.solve("pipefcg", Ao, oracle.make_pc("jacobi", Ao), prob.b, rtol=0.0, maxit=25, nu_max=5,
                       truncation=rule)
    Ag = pfk.Operator(2, 64, prob.eta)
    info = pfk.solve(Ag, pfk.Precond(Ag, "jacobi", 1), "pipefcg", _dev(prob.b), _dev(np.zeros(4096)),
                     rtol=0.0, maxit=25, mmax=5, truncation=truncation)
    assert np.allclose(info.history, ref.history, rtol=1e-9)


def test_deterministic_and_graph_equals_direct(pfk):
    prob = gen.config_problem("cfg2", seed=1, n=24)
    Ag = pfk.Operator(3, 24, prob.eta)
    Bg = pfk.Precond(Ag, "jacobi_pcg", 5)
    _say("determinism")
    hs = []
    for use_graph, gi in ((1, 8), (1, 8), (0, 1), (1, 3)):
        info = pfk.solve(Ag, Bg, "pipefcg", _dev(prob.b), _dev(np.zeros(Ag.N)), rtol=0.0, maxit=40, mmax=30,
                         use_graph=use_graph, graph_iters=gi)
        hs.append(info.history)
    for h in hs[1:]:
        assert np.array_equal(h, hs[0])


@pytest.mark.parametrize("dim,n", [(3, 1), (3, 2), (2, 1), (2, 3), (3, 9)])
@pytest.mark.parametrize("method", ["fcg", "pipefcg", "gcr", "pipegcr", "fgmres", "pipefgmres"])
def test_tiny_grids(pfk, dim, n, method):
    # degenerate sizes: one node, a single ragged tile, fewer nodes than a wave
    _say("tiny grid", dim, n, method)
    prob = gen.make_problem(dim, n, 2, 2.0, seed=n, convection=(dim == 3 and method in ("gcr", "pipegcr",
                                                                                          "fgmres", "pipefgmres")))
    for kind, k in (("jacobi", 1), ("block_jacobi_pcg", 3)):
        Ao = oracle.StencilOperator(prob.dim, n, prob.eta, prob.vel)
        sigma = None
        Bo = oracle.make_pc(kind, Ao, k, block=8)
        if method == "pipefgmres":
            sigma = oracle.estimate_sigma(Ao.apply, Bo, Ao.N)
        ref = oracle.solve(method, Ao, Bo, prob.b, rtol=1e-10, maxit=400, nu_max=30, sigma=sigma)
        Ag = pfk.Operator(prob.dim, n, prob.eta, prob.vel)
        Bg = pfk.Precond(Ag, kind, k, block=8)
        x = _dev(np.zeros(Ao.N))
        opts = {"shift_sigma": float(sigma)} if sigma is not None else {}
        info = pfk.solve(Ag, Bg, method, _dev(prob.b), x, rtol=1e-10, maxit=400, mmax=30, **opts)
        assert ref.converged and info.converged, (kind, info, ref.status)
        # when the Krylov space is exhausted (iteration N), whether a pipelined
        # method sees a breakdown (a restart) or converges is decided by the sign
        # of a rounding-level quantity (PIPEFGMRES's t); iteration counts are
        # compared only when both sides took the same path
        if info.restarts == ref.restarts:
            assert abs(info.iterations - ref.iterations) <= 2, (kind, info.iterations, ref.iterations)
        # histories agree to 1e-8, or to 1e3 times the oracle's own change under
        # a rounding-level perturbation of b where that is larger: as a tiny
        # system's Krylov space runs out, the pipelined recurrences cancel
        # (PIPEFGMRES's t = zeta - sum hbar^2 above all) and a step can amplify
        # rounding by many orders; beyond that point only rounding noise is left
        m = min(len(info.history), len(ref.history), 21)
        hr = np.array(ref.history)[:m]
        sens = np.zeros(m)
        rng = np.random.default_rng(0)
        keep = hr > 1e-6 * hr[0]          # exact zeros (one-node grids) are left out
        safe = np.where(keep, hr, 1.0)
        for _ in range(3):
            b1 = prob.b * (1.0 + 1e-15 * rng.standard_normal(prob.b.shape))
            h1 = np.array(oracle.solve(method, Ao, Bo, b1, rtol=1e-10, maxit=400, nu_max=30,
                                       sigma=sigma).history)[:m]
            k = min(len(h1), m)
            sens[:k] = np.maximum(sens[:k], np.abs(h1[:k] - hr[:k]) / safe[:k])
        rel = np.abs(info.history[:m] - hr) / safe
        assert np.all((rel <= np.maximum(1e-8, 1e3 * sens))[keep]), (rel, sens)
        xs = np.linalg.solve(np.array([Ao.apply(e) for e in np.eye(Ao.N)]).T, prob.b)
        assert np.linalg.norm(_host(x) - xs) <= 1e-8 * np.linalg.norm(xs) * max(1.0, np.linalg.cond(
            np.array([Ao.apply(e) for e in np.eye(Ao.N)]).T))
