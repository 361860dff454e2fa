"""GPU stagnation restarts (opts.stall_window) against the oracle.

With window K the solve restarts from x at the first iteration i >= K after
the (re)start whose recurred residual is above half of entry i - K.  PIPEFCG
with the global 2-step inner CG on config 1 stalls; the GPU restarts at the
oracle's iterations (its history agrees with the oracle's to 1e-9 up to the
first) and follows the oracle after the restart within the oracle's own
sensitivity to rounding.  Each case prints its name first.
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


@pytest.mark.parametrize("method", ["pipefcg", "fcg", "pipegcr"])
def test_stall_restart_matches_oracle(pfk, method):
    _say("stall restart", method)
    p = gen.config_problem("cfg1", seed=0)
    Ao = oracle.StencilOperator(2, 64, p.eta)
    Bo = oracle.make_pc("jacobi_pcg", Ao, 2)
    K = 20
    h = oracle.solve(method, Ao, Bo, p.b, rtol=0.0, maxit=150, nu_max=30).history
    first = next((i for i in range(K, len(h)) if h[i] > 0.5 * h[i - K]), None)
    if first is None:
        pytest.skip(f"{method} does not stall on this system within 150 iterations")
    its = min(first + 25, 150)
    ref = oracle.solve(method, Ao, Bo, p.b, rtol=0.0, maxit=its, nu_max=30, stall_window=K, max_restarts=50)
    Ag = pfk.Operator(2, 64, p.eta)
    Bg = pfk.Precond(Ag, "jacobi_pcg", 2)
    for maxit, want in ((first - 1, 0), (first, 1)):
        info = pfk.solve(Ag, Bg, method, _dev(p.b), _dev(np.zeros(Ao.N)), rtol=0.0, maxit=maxit, mmax=30,
                         stall_window=K)
        assert info.restarts == want, (maxit, info.restarts)
    info = pfk.solve(Ag, Bg, method, _dev(p.b), _dev(np.zeros(Ao.N)), rtol=0.0, maxit=its, mmax=30,
                     stall_window=K, max_restarts=50)
    hg, hr = np.asarray(info.history), np.array(ref.history)
    # past the stall the method amplifies rounding (see test_gpu_window.py):
    # the bar is 30 times the oracle's own deviation under a 1e-15 change of b
    self_dev = np.zeros_like(hr)
    for seed in (1, 2):
        bp = p.b * (1.0 + 1e-15 * np.random.default_rng(seed).standard_normal(p.b.size))
        hp = np.array(oracle.solve(method, Ao, Bo, bp, rtol=0.0, maxit=its, nu_max=30, stall_window=K,
                                   max_restarts=50).history)
        if len(hp) == len(hr):
            self_dev = np.maximum(self_dev, np.abs(hp - hr) / np.abs(hr))
    bar = np.maximum(1e-9, 30.0 * np.maximum.accumulate(self_dev))
    print(f"  first stall at {first}; restarts oracle {ref.restarts}, GPU {info.restarts}")
    assert info.restarts == ref.restarts and len(hg) == len(hr)
    rel = np.abs(hg - hr) / np.abs(hr)
    print(f"  max relative history difference {rel.max():.2e}, oracle self-deviation {self_dev.max():.2e}")
    assert rel[:first + 1].max() <= 1e-9
    assert np.all(rel <= bar), (rel / bar).max()
