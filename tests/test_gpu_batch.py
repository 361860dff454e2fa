"""GPU batches: many systems advanced by shared launches.

Every member runs the single-solve device bodies with its own launch
geometry, so a member's residual history, iteration count and solution must be
bit-identical to a single pfk.solve of the same system -- alone or in any mix.
One member per method is also held to the FP64 oracle (first 20 iterations,
1e-9 relative).  Each case prints its name and sizes before touching the GPU.
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


SIZES = [8, 13, 16, 20, 24, 17]


def _members(pfk, kind, prec, conv=False, sizes=SIZES, tilings=None, k=4):
    out = []
    for i, n in enumerate(sizes):
        p = gen.make_problem(3, n, 3 + i, (2.0, 4.0), seed=100 + i, convection=conv)
        A = pfk.Operator(3, n, p.eta, p.vel)
        if tilings:
            A.set_tiling(*tilings[i % len(tilings)])
        B = pfk.Precond(A, kind, k, precision=prec, block=8)
        out.append((p, A, B))
    return out


CASES = [("pipefcg", "block_jacobi_pcg", 0, False), ("pipefcg", "block_jacobi_pcg", 1, False),
         ("fcg", "block_jacobi_pcg", 1, False), ("pipefcg", "jacobi", 0, False),
         ("pipefgmres", "block_jacobi_pcg", 1, True), ("fcg", "none", 0, False)]


FORMS = {0: "phased", 1: "persistent"}


# capacity 256: members from 13^3 up stream with nontemporal accesses (N times
# the capacity >= 2^20) while the single solves of these sizes do not; the
# access hint must not change a bit of the arithmetic
@pytest.mark.parametrize("capacity", [8, 256], ids=["cap8", "cap256"])
@pytest.mark.parametrize("persistent", [0, 1], ids=[FORMS[f] for f in (0, 1)])
@pytest.mark.parametrize("case", CASES, ids=[f"{m}-{k}-{'mixed' if p else 'fp64'}" for m, k, p, _ in CASES])
def test_members_identical_to_single_solves(pfk, case, persistent, capacity):
    method, kind, prec, conv = case
    _say("batch identity", case, FORMS[persistent], "capacity", capacity)
    mem = _members(pfk, kind, prec, conv, tilings=[(64, 2048, 32), (32, 64, 7), (64, 5, 100)])
    sig = {}
    if method == "pipefgmres":
        sig = {i: pfk.estimate_sigma(A, B) for i, (_, A, B) in enumerate(mem)}
    singles = []
    for i, (p, A, B) in enumerate(mem):
        x = _dev(np.zeros(A.N))
        opts = {"shift_sigma": sig[i]} if sig else {}
        info = pfk.solve(A, B, method, _dev(p.b), x, rtol=1e-8, maxit=1500, mmax=20, **opts)
        singles.append((info, _host(x)))
    # PIPEFGMRES members estimate their own shift when they are added (the
    # same estimate pfk.estimate_sigma makes)
    T = pfk.Batch(method, mmax=20, capacity=capacity, graph_iters=5, persistent=persistent)
    xs, slots = {}, {}
    for i in range(len(mem)):
        p, A, B = mem[i]
        xs[i] = _dev(np.zeros(A.N))
        slots[i] = T.add(A, B, _dev(p.b), xs[i], rtol=1e-8, maxit=1500)
    running = len(slots)
    steps = 0
    while running:
        T.step(5)
        _, running = T.poll()
        steps += 1
        assert steps < 2000
    for i, s in slots.items():
        info = T.info(s)
        ref, xref = singles[i]
        assert info.status == ref.status and info.iterations == ref.iterations, (i, info, ref)
        assert np.array_equal(info.history, ref.history), i
        assert np.array_equal(_host(xs[i]), xref), i
        assert info.converged == ref.converged
    T.close()


# the global inner solves (Jacobi-PCG, Jacobi-GMRES) run phase by phase over
# all members, in the phased form only
GLOBAL_CASES = [("pipefgmres", "jacobi_gmres", 1, True), ("pipefgmres", "jacobi_gmres", 0, True),
                ("pipefcg", "jacobi_pcg", 0, False), ("fcg", "jacobi_pcg", 1, False),
                ("fcg", "jacobi_gmres", 1, False)]


# inner step count 4, and 7 for the inner GMRES pass whose basis length is
# taken at run time
@pytest.mark.parametrize("case", GLOBAL_CASES + [("pipefgmres", "jacobi_gmres", 1, True, 7)],
                         ids=[f"{c[0]}-{c[1]}-{'mixed' if c[2] else 'fp64'}" + (f"-k{c[4]}" if len(c) > 4 else "")
                              for c in GLOBAL_CASES + [("pipefgmres", "jacobi_gmres", 1, True, 7)]])
def test_global_inner_members_identical_to_single_solves(pfk, case):
    method, kind, prec, conv = case[:4]
    kin = case[4] if len(case) > 4 else 4
    _say("batch identity, global inner solve", case)
    mem = _members(pfk, kind, prec, conv, tilings=[(64, 2048, 32), (32, 64, 7), (64, 5, 100)], k=kin)
    singles = []
    for p, A, B in mem:
        x = _dev(np.zeros(A.N))
        info = pfk.solve(A, B, method, _dev(p.b), x, rtol=1e-8, maxit=600, mmax=20)
        singles.append((info, _host(x)))
    T = pfk.Batch(method, mmax=20, capacity=8, graph_iters=5)
    xs, slots = {}, {}
    for i, (p, A, B) in enumerate(mem):
        xs[i] = _dev(np.zeros(A.N))
        slots[i] = T.add(A, B, _dev(p.b), xs[i], rtol=1e-8, maxit=600)
    running, steps = len(slots), 0
    while running:
        T.step(5)
        _, running = T.poll()
        steps += 1
        assert steps < 1000
    for i, s in slots.items():
        info = T.info(s)
        ref, xref = singles[i]
        assert info.status == ref.status and info.iterations == ref.iterations, (i, info, ref)
        assert np.array_equal(info.history, ref.history), i
        assert np.array_equal(_host(xs[i]), xref), i
    T.close()


@pytest.mark.parametrize("method,conv,kind,k", [("pipefcg", False, "block_jacobi_pcg", 4),
                                                ("fcg", False, "block_jacobi_pcg", 4),
                                                ("pipefgmres", True, "block_jacobi_pcg", 4),
                                                ("pipefgmres", True, "jacobi_gmres", 5),
                                                ("fcg", False, "jacobi_pcg", 4)])
def test_batch_member_follows_oracle(pfk, method, conv, kind, k):
    _say("batch oracle", method, kind, k)
    p = gen.make_problem(3, 19, 6, 3.0, seed=9, convection=conv)
    Ao = oracle.StencilOperator(3, 19, p.eta, p.vel)
    Bo = oracle.make_pc(kind, Ao, k, block=8)
    sigma = oracle.estimate_sigma(Ao.apply, Bo, Ao.N) if method == "pipefgmres" else None
    ref = oracle.solve(method, Ao, Bo, p.b, rtol=0.0, maxit=20, nu_max=20, sigma=sigma)
    other = gen.make_problem(3, 11, 2, 2.0, seed=3, convection=conv)
    T = pfk.Batch(method, mmax=20, capacity=4, **({"shift_sigma": float(sigma)} if sigma else {}))
    A = pfk.Operator(3, 19, p.eta, p.vel)
    B = pfk.Precond(A, kind, k, block=8)
    A2 = pfk.Operator(3, 11, other.eta, other.vel)
    B2 = pfk.Precond(A2, kind, k, block=8)
    x, x2 = _dev(np.zeros(A.N)), _dev(np.zeros(A2.N))
    s = T.add(A, B, _dev(p.b), x, rtol=0.0, maxit=20)
    T.add(A2, B2, _dev(other.b), x2, rtol=0.0, maxit=20)
    for _ in range(30):
        T.step(1)
        _, running = T.poll()
        if running == 0:
            break
    info = T.info(s)
    rel = np.abs(info.history - np.array(ref.history)) / np.abs(np.array(ref.history))
    assert len(info.history) == 21 and rel.max() <= 1e-9, rel
    T.close()


def test_batch_edge_cases(pfk):
    _say("batch edge cases")
    p = gen.make_problem(3, 12, 3, 3.0, seed=1)
    A = pfk.Operator(3, 12, p.eta)
    B = pfk.Precond(A, "block_jacobi_pcg", 4, block=8)
    Bm = pfk.Precond(A, "block_jacobi_pcg", 4, precision=pfk.FP32_BF16COEF, block=8)
    Bg = pfk.Precond(A, "jacobi_pcg", 4)
    Bg3 = pfk.Precond(A, "jacobi_pcg", 3)
    Bn = pfk.Precond(A, "noisy", eta=0.1, seed=1)
    Tp = pfk.Batch("pipefcg", mmax=10, capacity=2, persistent=1)
    with pytest.raises(RuntimeError):
        Tp.add(A, Bg, _dev(p.b), _dev(np.zeros(A.N)))         # the persistent form has no global inner solve
    Tp.close()
    Tg = pfk.Batch("pipefcg", mmax=10, capacity=2)
    Tg.add(A, Bg, _dev(p.b), _dev(np.zeros(A.N)), rtol=1e-8)
    with pytest.raises(RuntimeError):
        Tg.add(A, Bg3, _dev(p.b), _dev(np.zeros(A.N)))        # another inner step count
    Tg.close()
    T = pfk.Batch("pipefcg", mmax=10, capacity=2)
    with pytest.raises(RuntimeError):
        T.add(A, Bn, _dev(p.b), _dev(np.zeros(A.N)))          # the noisy preconditioner is not batched
    x0 = _dev(np.ones(A.N))
    s0 = T.add(A, B, _dev(np.zeros(A.N)), x0, rtol=1e-8)      # b = 0: x = 0 at once
    with pytest.raises(RuntimeError):
        T.add(A, Bm, _dev(p.b), _dev(np.zeros(A.N)))          # another precision
    x1 = _dev(np.zeros(A.N))
    s1 = T.add(A, B, _dev(p.b), x1, rtol=1e-8, maxit=500)
    with pytest.raises(RuntimeError):
        T.add(A, B, _dev(p.b), _dev(np.zeros(A.N)))           # full
    fin, running = T.poll()
    assert s0 in fin and not np.any(_host(x0))
    info0 = T.info(s0)
    assert info0.converged and info0.iterations == 0
    T.remove(s0)
    x2 = _dev(np.zeros(A.N))
    s2 = T.add(A, B, _dev(p.b), x2, rtol=1e-8, maxit=500)    # the freed slot is reused
    assert s2 == s0
    running = 2
    while running:
        T.step(8)
        _, running = T.poll()
    i1, i2 = T.info(s1), T.info(s2)
    assert i1.converged and i2.converged and i1.iterations == i2.iterations
    assert np.array_equal(_host(x1), _host(x2))
    T.close()
    with pytest.raises(RuntimeError):
        pfk.Batch("gcr", mmax=10, capacity=2)


@pytest.mark.parametrize("persistent", [0, 1], ids=[FORMS[f] for f in (0, 1)])
def test_solve_batched_uneven_systems(pfk, persistent):
    # (a grid of one or two blocks per axis with strong contrast makes the block
    # solve nearly the global few-step CG, under which PIPEFCG stagnates in the
    # oracle too, e.g. n = 8 or 11 with 15 inclusions; FP32 inner sweeps push
    # more systems to that edge, so this check runs the FP64 inner solve, with
    # which all of these sizes converge in the oracle)
    _say("solve_batched 16 systems")
    sizes = [8, 16, 24, 12, 20, 30, 32, 16, 10, 14, 18, 22, 26, 28, 13, 15]
    mem = _members(pfk, "block_jacobi_pcg", 0, sizes=sizes)
    bs = [_dev(p.b) for p, _, _ in mem]
    xs = [_dev(np.zeros(A.N)) for _, A, _ in mem]
    code, infos = pfk.solve_batched([A for _, A, _ in mem], [B for _, _, B in mem], "pipefcg", bs, xs,
                                    rtol=1e-8, maxit=2000, mmax=20, persistent=persistent)
    for n, info in zip(sizes, infos):
        print(f"  n={n}: {info.status_name} its {info.iterations} restarts {info.restarts} "
              f"true rel {info.true_rel_resid:.2e}")
    assert code == 0
    for (p, A, B), info, x in zip(mem, infos, xs):
        Ao = oracle.StencilOperator(3, p.n, p.eta)
        xh = _host(x)
        assert info.converged and np.linalg.norm(p.b - Ao.apply(xh)) <= 1e-8 * np.linalg.norm(p.b)


def test_persistent_barrier_timeout_is_reported(pfk):
    # a grid barrier that may not poll gives up at the first wait: the launch must
    # end (every workgroup leaves) and the next poll must report the failure
    _say("persistent barrier timeout")
    mem = _members(pfk, "block_jacobi_pcg", 0, sizes=[24, 32])
    T = pfk.Batch("pipefcg", mmax=20, capacity=2, persistent=1)
    for p, A, B in mem:
        T.add(A, B, _dev(p.b), _dev(np.zeros(A.N)), rtol=1e-8, maxit=100)
    T.set_barrier_limit(0)
    T.step(3)
    with pytest.raises(RuntimeError):
        T.poll()
    T.close()


@pytest.mark.skip(reason="a persistent form driven by per-system completion counters (work items "
                         "from one ticket counter) did not finish its first launch on the GPU; the "
                         "cause was not found, so the form was taken out and the library refuses "
                         "persistent = 2")
def test_members_identical_dataflow_form(pfk):
    _say("batch identity dataflow")
    raise AssertionError("not built")


def test_unknown_persistent_form_is_refused(pfk):
    _say("persistent form 2 refused")
    with pytest.raises(RuntimeError):
        pfk.Batch("pipefcg", mmax=20, capacity=2, persistent=2)


def test_solve_batched_caller_workspace(pfk):
    _say("solve_batched caller workspace")
    import torch
    mem = _members(pfk, "block_jacobi_pcg", 0, sizes=[12, 20, 16])
    As, Bs = [A for _, A, _ in mem], [B for _, _, B in mem]
    bs = [_dev(p.b) for p, _, _ in mem]
    sizes = [(pfk.workspace_bytes(A, B, "pipefcg", 20, 300) + 255) // 256 * 256 for A, B in zip(As, Bs)]
    ws = torch.empty(sum(sizes), dtype=torch.uint8, device="cuda")
    xa = [_dev(np.zeros(A.N)) for A in As]
    xb = [_dev(np.zeros(A.N)) for A in As]
    ca, ia = pfk.solve_batched(As, Bs, "pipefcg", bs, xa, rtol=1e-8, maxit=300, mmax=20, workspace=ws)
    cb, ib = pfk.solve_batched(As, Bs, "pipefcg", bs, xb, rtol=1e-8, maxit=300, mmax=20)
    assert ca == cb == 0
    for u, v, p, q in zip(xa, xb, ia, ib):
        assert np.array_equal(_host(u), _host(v)) and np.array_equal(p.history, q.history)
    small = torch.empty(sum(sizes) - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(RuntimeError):
        pfk.solve_batched(As, Bs, "pipefcg", bs, xa, rtol=1e-8, maxit=300, mmax=20, workspace=small)
