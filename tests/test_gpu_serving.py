"""GPU serving: requests admitted by memory budget into continuously refilled
batches.  The identity bar: every request's residual history, iteration count
and solution are bit-identical to the same request solved alone (a single
pfk.solve), whatever else is in flight.  Each case prints its name first.
"""
import sys

import numpy as np
import pytest

import gen

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


def _requests(pfk, count, seed=0, mix="block"):
    # mix "block": both methods with the block-Jacobi PCG (4 steps); mix
    # "gmres": PIPEFGMRES requests with the global right-Jacobi GMRES(5)
    # inner solve, as in the serving configuration; all FP32/BF16 inner sweeps
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.choice([12, 16, 20, 24, 28, 32]))
        method = "pipefcg" if i % 2 == 0 else "pipefgmres"
        p = gen.make_problem(3, n, 6, (1.0, 4.0), seed=500 + i)
        A = pfk.Operator(3, n, p.eta)
        if mix == "gmres" and method == "pipefgmres":
            B = pfk.Precond(A, "jacobi_gmres", 5, precision=pfk.FP32_BF16COEF)
        else:
            B = pfk.Precond(A, "block_jacobi_pcg", 4, precision=pfk.FP32_BF16COEF, block=8)
        rtol = 1e-6 if rng.random() < 0.5 else 1e-8
        out.append(dict(p=p, A=A, B=B, method=method, rtol=rtol))
    return out


@pytest.mark.parametrize("mix,direct", [("block", False), ("gmres", False), ("gmres", True)],
                         ids=["block", "gmres", "gmres-direct"])
def test_alone_vs_mix_identical(pfk, mix, direct):
    _say("serving alone vs mix", mix, "direct launches" if direct else "graphs")
    reqs = _requests(pfk, 12, mix=mix)
    alone = []
    for r in reqs:
        x = _dev(np.zeros(r["A"].N))
        info = pfk.solve(r["A"], r["B"], r["method"], _dev(r["p"].b), x, rtol=r["rtol"], maxit=1500, mmax=20)
        alone.append((info, _host(x)))
    # the budget fits only a few requests at a time, so admission queues the rest
    import paper_1511_07226_amd as m
    per = [m.workspace_bytes(r["A"], r["B"], r["method"], 20, 1500) for r in reqs]
    budget = 3 * max(per)
    srv = pfk.Server(hbm_budget=budget, max_active=4, step_iters=5, mmax=20, launch_direct=direct)
    xs, ids, done = {}, {}, set()
    max_active = 0
    # arrivals: half up front, the rest one per round
    for i in range(6):
        xs[i] = _dev(np.zeros(reqs[i]["A"].N))
        ids[i] = srv.submit(reqs[i]["A"], reqs[i]["B"], reqs[i]["method"], _dev(reqs[i]["p"].b), xs[i],
                            rtol=reqs[i]["rtol"], maxit=1500)
    nxt = 6
    rounds = 0
    while len(done) < len(reqs):
        if nxt < len(reqs):
            r = reqs[nxt]
            xs[nxt] = _dev(np.zeros(r["A"].N))
            ids[nxt] = srv.submit(r["A"], r["B"], r["method"], _dev(r["p"].b), xs[nxt], rtol=r["rtol"], maxit=1500)
            nxt += 1
        done.update(srv.progress())
        st = srv.stats()
        max_active = max(max_active, st["active"])
        assert st["bytes_in_use"] <= budget
        rounds += 1
        assert rounds < 5000
    print(f"  {rounds} rounds, at most {max_active} active, budget {budget} bytes")
    assert max_active >= 2
    for i, r in enumerate(reqs):
        info = srv.result(ids[i])
        ref, xref = alone[i]
        assert info.status == ref.status and info.iterations == ref.iterations, (i, info, ref)
        assert np.array_equal(info.history, ref.history), i
        assert np.array_equal(_host(xs[i]), xref), i
    srv.close()


def test_submit_errors(pfk):
    _say("serving errors")
    p = gen.make_problem(3, 16, 3, 2.0, seed=1)
    A = pfk.Operator(3, 16, p.eta)
    B = pfk.Precond(A, "block_jacobi_pcg", 4, block=8)
    srv = pfk.Server(hbm_budget=1 << 20, max_active=2, step_iters=4, mmax=20)
    with pytest.raises(RuntimeError):          # workspace above the whole budget
        srv.submit(A, B, "pipefcg", _dev(p.b), _dev(np.zeros(A.N)))
    srv.close()
    srv = pfk.Server(hbm_budget=1 << 30, max_active=2, step_iters=4, mmax=20)
    with pytest.raises(RuntimeError):
        srv.submit(A, B, "gcr", _dev(p.b), _dev(np.zeros(A.N)))
    with pytest.raises(RuntimeError):
        srv.submit(A, pfk.Precond(A, "noisy", eta=0.1, seed=1), "pipefcg", _dev(p.b), _dev(np.zeros(A.N)))
    srv.close()
