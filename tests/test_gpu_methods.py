"""GPU parity for the CR and GMRES families and the inner Jacobi-GMRES solve.

Each case prints its name, sizes and seed before touching the GPU.  The bar:
residual histories over the first 20 iterations within 1e-9 relative of the
FP64 oracle; converged solves reach a true residual <= rtol.
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


def _conv(n=20, seed=0, contrast=2.0):
    return gen.make_problem(3, n, 4, contrast, seed, convection=True)


# k = 6 and 8 run the pass whose basis length is taken at run time (steps 5..7)
@pytest.mark.parametrize("k", [1, 3, 5, 6, 8])
@pytest.mark.parametrize("conv", [False, True])
def test_inner_gmres_matches_oracle(pfk, k, conv):
    _say("inner gmres", k, conv)
    p = _conv(17, seed=k) if conv else gen.make_problem(2, 70, 6, 3.0, seed=k)
    Ao = oracle.StencilOperator(p.dim, p.n, p.eta, p.vel)
    Ag = pfk.Operator(p.dim, p.n, p.eta, p.vel)
    v = np.random.default_rng(k).standard_normal(Ao.N)
    y = _host(pfk.Precond(Ag, "jacobi_gmres", k).apply(_dev(v)))
    ref = oracle.make_pc("jacobi_gmres", Ao, k)(v)
    assert np.abs(y - ref).max() <= 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("k", [1, 2, 5, 7])
@pytest.mark.parametrize("mixed", [False, True])
def test_inner_gmres_exact_breakdown(pfk, k, mixed):
    # one node, eta = 1 (2D, h = 1/2): A = 16 and D^-1 = 1/16 exactly, so for
    # v = 1 the operator A D^-1 is the identity in floating point and the
    # second basis vector is exactly zero: a happy breakdown after one column
    # (found by step 2's pass, or by the finish for k = 1), B(v) = 1/16
    _say("inner gmres exact breakdown", k, mixed)
    p = gen.make_problem(2, 1, 1, 1.0, seed=0)
    eta = np.ones_like(p.eta)
    Ao = oracle.StencilOperator(2, 1, eta)
    ref = oracle.make_pc("jacobi_gmres", Ao, k)(np.array([1.0]))
    assert ref[0] == 0.0625
    Ag = pfk.Operator(2, 1, eta)
    prec = pfk.FP32_BF16COEF if mixed else pfk.FP64
    y = _host(pfk.Precond(Ag, "jacobi_gmres", k, precision=prec).apply(_dev(np.array([1.0]))))
    assert y[0] == 0.0625, y


def test_inner_gmres_zero_input(pfk):
    _say("inner gmres zero")
    p = gen.make_problem(2, 16, 2, 2.0, seed=0)
    Ag = pfk.Operator(2, 16, p.eta)
    assert not np.any(_host(pfk.Precond(Ag, "jacobi_gmres", 4).apply(_dev(np.zeros(256)))))


def test_sigma_estimate_matches_oracle(pfk):
    import ctypes as C
    p = _conv(16, seed=3)
    _say("sigma estimate")
    Ao = oracle.StencilOperator(3, 16, p.eta, p.vel)
    ref = oracle.estimate_sigma(Ao.apply, oracle.make_pc("jacobi_gmres", Ao, 5), Ao.N)
    Ag = pfk.Operator(3, 16, p.eta, p.vel)
    Bg = pfk.Precond(Ag, "jacobi_gmres", 5)
    sig = C.c_double()
    import torch
    code = pfk.lib().pfk_estimate_sigma(Ag.handle, Bg.handle, 10, C.byref(sig), torch.cuda.current_stream().cuda_stream)
    assert code == 0
    assert sig.value == pytest.approx(ref, rel=1e-10)


def _parity(pfk, method, prob, kind, k, m, its, rtol=0.0, sigma=None, **kw):
    Ao = oracle.StencilOperator(prob.dim, prob.n, prob.eta, prob.vel)
    Bo = oracle.make_pc(kind, Ao, k)
    if method == "pipefgmres" and sigma is None:
        sigma = oracle.estimate_sigma(Ao.apply, Bo, Ao.N)
    ref = oracle.solve(method, Ao, Bo, prob.b, rtol=rtol, maxit=its, nu_max=m, sigma=sigma,
                       force_breakdown_at=kw.get("force_breakdown_at", -1))
    Ag = pfk.Operator(prob.dim, prob.n, prob.eta, prob.vel)
    Bg = pfk.Precond(Ag, kind, k)
    x = _dev(np.zeros(Ao.N))
    opts = dict(kw)
    if sigma is not None:
        opts["shift_sigma"] = float(sigma)
    info = pfk.solve(Ag, Bg, method, _dev(prob.b), x, rtol=rtol, maxit=its, mmax=m, **opts)
    return ref, info, _host(x), Ao


CASES = [
    ("cfg1", "jacobi_pcg", 2),
    ("conv20", "jacobi_gmres", 5),
    ("conv20", "jacobi_pcg", 2),
]


@pytest.mark.parametrize("method", ["gcr", "pipegcr", "fgmres", "pipefgmres"])
@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-{c[1]}" for c in CASES])
def test_history_parity_first_20(pfk, method, case):
    name, kind, k = case
    prob = gen.config_problem("cfg1", seed=0) if name == "cfg1" else _conv(20, seed=1)
    _say("history", method, name, kind, k)
    ref, info, x, _ = _parity(pfk, method, prob, kind, k, 30, 20)
    h, hr = info.history, np.array(ref.history)
    assert len(h) == len(hr) == 21
    rel = np.abs(h - hr) / np.abs(hr)
    assert rel.max() <= 1e-9, rel


@pytest.mark.parametrize("method", ["fgmres", "pipefgmres"])
def test_restart_cycles_parity(pfk, method):
    # restart length 4: five cycles in 20 iterations, x updated at each cycle end
    prob = _conv(18, seed=2)
    _say("restart cycles", method)
    ref, info, x, _ = _parity(pfk, method, prob, "jacobi_gmres", 3, 4, 20)
    assert np.allclose(info.history, ref.history, rtol=1e-9)
    assert np.abs(x - ref.x).max() <= 1e-9 * np.abs(ref.x).max()


@pytest.mark.parametrize("method", ["gcr", "fgmres", "pipefgmres", "pipegcr"])
def test_full_solve_convection(pfk, method):
    prob = _conv(20, seed=4)
    kind = "jacobi_gmres" if method != "pipegcr" else "jacobi"
    _say("full solve conv", method, kind)
    ref, info, x, Ao = _parity(pfk, method, prob, kind, 5, 30, 3000, rtol=1e-8)
    assert ref.converged and info.converged and info.status == 0, (ref.status, info.status_name, info.iterations)
    assert abs(info.iterations - ref.iterations) <= max(3, ref.iterations // 5)
    assert np.linalg.norm(prob.b - Ao.apply(x)) <= 1e-8 * np.linalg.norm(prob.b)


def test_pipefgmres_forced_breakdown(pfk):
    prob = _conv(16, seed=5)
    _say("pipefgmres forced breakdown")
    ref, info, x, _ = _parity(pfk, "pipefgmres", prob, "jacobi", 1, 30, 25, force_breakdown_at=7)
    assert ref.restarts == 1 and info.restarts == 1
    assert np.allclose(info.history, ref.history, rtol=1e-9)


def test_ragged_sizes_all_methods(pfk):
    # N not a multiple of the wave width: the in-loop wave reductions must mask lanes
    conv = gen.make_problem(3, 13, 3, 2.0, seed=6, convection=True)   # N = 2197
    sym = gen.make_problem(3, 13, 3, 2.0, seed=6)
    for method in ("fcg", "pipefcg", "gcr", "pipegcr", "fgmres", "pipefgmres"):
        _say("ragged", method)
        kind = "jacobi_gmres" if "gmres" in method else "jacobi_pcg"
        prob = sym if method in ("fcg", "pipefcg") else conv
        ref, info, x, _ = _parity(pfk, method, prob, kind, 3, 30, 15)
        assert np.allclose(info.history, ref.history, rtol=1e-9), method


@pytest.mark.parametrize("method", ["fcg", "gcr", "fgmres"])
def test_host_sync_baseline_matches_device_form(pfk, method):
    # the host-sync form runs the same kernels with the host waiting on every
    # reduction: identical iterates, bit for bit
    prob = _conv(16, seed=8) if method != "fcg" else gen.make_problem(3, 16, 4, 3.0, seed=8)
    kind = "jacobi_gmres" if method != "fcg" else "jacobi_pcg"
    _say("host sync", method)
    Ag = pfk.Operator(prob.dim, prob.n, prob.eta, prob.vel)
    Bg = pfk.Precond(Ag, kind, 3)
    out = []
    for hs in (0, 1):
        x = _dev(np.zeros(Ag.N))
        info = pfk.solve(Ag, Bg, method, _dev(prob.b), x, rtol=1e-8, maxit=400, mmax=30, host_sync=hs)
        out.append((info, _host(x)))
    (i0, x0), (i1, x1) = out
    assert i0.converged and i1.converged and i0.iterations == i1.iterations
    assert np.array_equal(i0.history, i1.history) and np.array_equal(x0, x1)


def test_host_sync_rejected_for_pipelined(pfk):
    prob = gen.make_problem(2, 16, 2, 2.0, seed=0)
    Ag = pfk.Operator(2, 16, prob.eta)
    Bg = pfk.Precond(Ag, "jacobi", 1)
    with pytest.raises(RuntimeError):
        pfk.solve(Ag, Bg, "pipefcg", _dev(prob.b), _dev(np.zeros(256)), host_sync=1)


W_CASES = [("conv20", "jacobi", 1), ("conv20", "jacobi_gmres", 5), ("conv20", "block_jacobi_pcg", 4),
           ("cfg1", "jacobi_pcg", 2)]


@pytest.mark.parametrize("case", W_CASES, ids=[f"{c[0]}-{c[1]}" for c in W_CASES])
def test_pipegcr_w_history_parity_first_20(pfk, case):
    # Alg. 12: PIPEGCR with w recurred; the same windows as PIPEFCG, reductions on w
    name, kind, k = case
    prob = gen.config_problem("cfg1", seed=0) if name == "cfg1" else _conv(20, seed=1)
    _say("pipegcr_w history", name, kind, k)
    Ao = oracle.StencilOperator(prob.dim, prob.n, prob.eta, prob.vel)
    Bo = oracle.make_pc(kind, Ao, k, block=8)
    ref = oracle.solve("pipegcr_w", Ao, Bo, prob.b, rtol=0.0, maxit=20, nu_max=30)
    Ag = pfk.Operator(prob.dim, prob.n, prob.eta, prob.vel)
    Bg = pfk.Precond(Ag, kind, k, block=8)
    x = _dev(np.zeros(Ao.N))
    info = pfk.solve(Ag, Bg, "pipegcr_w", _dev(prob.b), x, rtol=0.0, maxit=20, mmax=30)
    h, hr = info.history, np.array(ref.history)
    assert len(h) == len(hr) == 21
    assert (np.abs(h - hr) / np.abs(hr)).max() <= 1e-9


def test_pipegcr_w_full_solve_and_ragged(pfk):
    prob = _conv(20, seed=4)
    _say("pipegcr_w full solve")
    ref, info, x, Ao = _parity(pfk, "pipegcr_w", prob, "jacobi", 1, 30, 3000, rtol=1e-8)
    assert ref.converged and info.converged and info.status == 0
    assert abs(info.iterations - ref.iterations) <= max(3, ref.iterations // 5)
    assert np.linalg.norm(prob.b - Ao.apply(x)) <= 1e-8 * np.linalg.norm(prob.b)
    conv = gen.make_problem(3, 13, 3, 2.0, seed=6, convection=True)     # N = 2197
    ref, info, x, _ = _parity(pfk, "pipegcr_w", conv, "jacobi_gmres", 3, 30, 15)
    assert np.allclose(info.history, ref.history, rtol=1e-9)
