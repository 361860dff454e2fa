"""Writes histories_128.json: the FP64 oracle's first 20 iterations at 128^3
(2,097,152 unknowns, the size from which the GPU path streams vectors with
nontemporal accesses), seed 0, window / restart length 30:

* the 128^3 sinker (20 spheres at viscosity 1e4): FCG and PIPEFCG under the
  5-step global Jacobi-PCG and the 5-step block-Jacobi PCG (8^3 blocks);
* the convection-diffusion sinker (same viscosity recipe, cell Peclet 5) at
  128^3: GCR, PIPEGCR, PIPEGCR_w, FGMRES and PIPEFGMRES under the 5-step
  right-Jacobi GMRES inner solve in FP64, PIPEFGMRES with the oracle's own
  shift estimate (stored and passed to the GPU).

It calls only the oracle and the seeded generators.  The GPU tests compare
against the stored values because these oracle runs take several minutes.

    python tests/golden/make_histories_128.py
"""
import hashlib
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import gen  # noqa: E402
import oracle  # noqa: E402

ITS = 20
SAMPLES = 256


def fingerprint(p) -> str:
    h = hashlib.sha1()
    for a in (p.eta, p.b) + ((p.vel,) if p.vel is not None else ()):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()[:16]


def runs(p, plan, sigma=None):
    A = oracle.StencilOperator(3, p.n, p.eta, p.vel)
    idx = np.random.default_rng(7).integers(0, A.N, SAMPLES)
    idx = np.concatenate([idx, [0, A.N - 1]]).tolist()
    out = {"inputs_sha1": fingerprint(p), "x_index": idx, "runs": {}}
    for kind, methods in plan:
        B = oracle.make_pc(kind, A, 5, block=8)
        if sigma is None and any(m == "pipefgmres" for m in methods):
            sigma = oracle.estimate_sigma(A.apply, B, A.N)
            out["sigma"] = sigma
        for method in methods:
            r = oracle.solve(method, A, B, p.b, rtol=0.0, maxit=ITS, nu_max=30, sigma=sigma)
            out["runs"][f"{method}/{kind}"] = {"history": [float(v) for v in r.history],
                                               "x_at_index": [float(r.x[i]) for i in idx]}
            print(method, kind, r.history[-1] / r.history[0], flush=True)
    return out


def main():
    res = {"what": "oracle residual histories, 20 iterations, 128^3, seed 0, window/restart 30",
           "iterations": ITS}
    res["cfg2"] = runs(gen.config_problem("cfg2", seed=0),
                       [("jacobi_pcg", ("fcg", "pipefcg")), ("block_jacobi_pcg", ("fcg", "pipefcg"))])
    res["cfg3"] = runs(gen.config_problem("cfg3", seed=0, n=128),
                       [("jacobi_gmres", ("gcr", "pipegcr", "pipegcr_w", "fgmres", "pipefgmres"))])
    with open(os.path.join(HERE, "histories_128.json"), "w") as f:
        json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
