"""The two-stream schedule under a delayed second stream.

The pipelined methods finish each iteration's reduction on a second stream
while the first applies the preconditioner and the operator, and the next
window update waits for it through an event.  The side_delay test hook holds
the second stream back (a bounded sleep kernel before each reduction finish,
about 1 ms here, far longer than these small systems' preconditioner and
operator work), so a missing or misplaced join would let the update read the
previous iteration's scalars.  Results must be bit-identical with and without
the delay, graph-launched and direct.  Each case prints its name before
touching the GPU.
"""
import sys
import time

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


CASES = [("pipefcg", "jacobi_pcg", False), ("pipegcr", "jacobi_pcg", False),
         ("pipegcr_w", "jacobi_gmres", True), ("pipefgmres", "jacobi_gmres", True)]


@pytest.mark.parametrize("use_graph", [1, 0], ids=["graph", "direct"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_delayed_second_stream_changes_nothing(pfk, case, use_graph):
    method, kind, conv = case
    _say("side delay", method, kind, "graph" if use_graph else "direct")
    p = gen.make_problem(3, 14, 4, 2.0, seed=11, convection=conv)
    A = pfk.Operator(3, 14, p.eta, p.vel)
    B = pfk.Precond(A, kind, 3)
    extra = {"shift_sigma": float(pfk.estimate_sigma(A, B))} if method == "pipefgmres" else {}
    out = []
    for delay in (0, 300):
        x = _dev(np.zeros(A.N))
        b = _dev(p.b)
        _host(x)
        t0 = time.perf_counter()
        info = pfk.solve(A, B, method, b, x, rtol=0.0, maxit=25, mmax=10, use_graph=use_graph,
                         graph_iters=5, side_delay=delay, **extra)
        dt = time.perf_counter() - t0
        out.append((info.history.copy(), _host(x), info.iterations, dt))
    (h0, x0, i0, t0), (h1, x1, i1, t1) = out
    print(f"  solve {t0 * 1e3:.1f} ms, with the delayed second stream {t1 * 1e3:.1f} ms")
    assert i0 == i1 == 25
    # the delay sits on the path the join enforces: 25 iterations x 300
    # sleeps of at least 1 us each (about 3.4 us on this clock)
    assert t1 - t0 >= 25 * 300 * 1e-6
    assert np.array_equal(h0, h1)
    assert np.array_equal(x0, x1)


def test_side_delay_range_is_checked(pfk):
    _say("side delay range")
    p = gen.make_problem(3, 8, 2, 2.0, seed=1)
    A = pfk.Operator(3, 8, p.eta, p.vel)
    B = pfk.Precond(A, "jacobi_pcg", 2)
    for bad in (-1, 10001):
        with pytest.raises(pfk.PfkError):
            pfk.solve(A, B, "pipefcg", _dev(p.b), _dev(np.zeros(A.N)), rtol=1e-8, maxit=5, mmax=4,
                      side_delay=bad)


@pytest.mark.parametrize("method", ["pipefcg", "fcg", "pipefgmres"])
def test_device_timestamps(pfk, method):
    # opts.timestamps: the device clock at every history entry, in us from
    # entry 0; non-decreasing, one per entry, spanning about the solve's time
    # (here stretched by the side-stream delay for the pipelined methods)
    _say("timestamps", method)
    p = gen.make_problem(3, 14, 4, 2.0, seed=12, convection=method == "pipefgmres")
    A = pfk.Operator(3, 14, p.eta, p.vel)
    B = pfk.Precond(A, "jacobi_gmres" if method == "pipefgmres" else "jacobi_pcg", 3)
    extra = {"shift_sigma": float(pfk.estimate_sigma(A, B))} if method == "pipefgmres" else {}
    x = _dev(np.zeros(A.N))
    b = _dev(p.b)
    off = pfk.solve(A, B, method, b, x, rtol=0.0, maxit=20, mmax=10, **extra)
    assert off.iter_time_us.size == 0
    x = _dev(np.zeros(A.N))
    delay = 0 if method == "fcg" else 100
    t0 = time.perf_counter()
    info = pfk.solve(A, B, method, b, x, rtol=0.0, maxit=20, mmax=10, timestamps=1, side_delay=delay, **extra)
    wall_us = (time.perf_counter() - t0) * 1e6
    ts = info.iter_time_us
    print(f"  {len(ts)} stamps, last {ts[-1]:.0f} us, host wall {wall_us:.0f} us")
    assert len(ts) == len(info.history) == 21
    assert ts[0] == 0.0 and np.all(np.diff(ts) >= 0.0)
    assert ts[-1] <= wall_us
    if delay:
        # 20 iterations, each holding back the reduction finish by >= 100 us
        assert ts[-1] >= 20 * 100 * 1.0
    assert np.array_equal(info.history, off.history)
    with pytest.raises(pfk.PfkError):
        pfk.solve(A, B, method, b, x, rtol=0.0, maxit=5, mmax=10, timestamps=2, **extra)
