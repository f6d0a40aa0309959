"""Write the whole-mesh oracle values that the full-size GPU tests compare
against, where the oracle takes minutes on the host:

* fullsize_norms.json: ||D^-1 f^|| over all interior faces (the scale of a
  solve's residual bound) for the uneven-level mesh, instance 0;
* c2_lambda_direct.npy: lam = S^-1 f^ on the 8192-macro mesh (r = 3, p = 3,
  kappa = 1e-2, a = (1, 0.5), u = exp(x) sin(2 pi y)) by a sparse direct
  solve of the assembled condensed system (eq. global_problem).

Only the oracle computes these (through tests/oracle_parallel.py, which
imports numpy, scipy and oracle/ alone).  Run from the repository root:

    python tests/golden/make_fullsize.py [--workers N] [--only NAME]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

from oracle import hdg  # noqa: E402
from paper_2302_10917_amd import inputs  # noqa: E402

import oracle_parallel  # noqa: E402


def mixed_inst0_norm(workers):
    xy, tri = inputs.structured_mesh(64)
    r = inputs.random_levels(len(tri), (1, 2, 3, 4), seed=3)
    kap_i, beta_i = inputs.coefficient_instances(64, seed=33)
    kap = np.full(len(tri), float(kap_i[0]))
    beta = tuple(float(x) for x in beta_i[0])
    orc = hdg.Oracle(xy, tri, r, 3, kap, beta, 1.0)
    fo, go = orc.sample(inputs.exp_sin(float(kap_i[0]), beta))
    lamD = orc.dirichlet_trace(go)
    return oracle_parallel.preconditioned_rhs_norm(xy, tri, r, 3, kap, beta, 1.0, fo, lamD,
                                                   workers=workers)


def c2_direct(workers):
    xy, tri = inputs.structured_mesh(64)
    kappa, beta = 1e-2, (1.0, 0.5)
    kap = np.full(len(tri), kappa)
    orc = hdg.Oracle(xy, tri, 3, 3, kap, beta, 1.0)
    fo, go = orc.sample(inputs.exp_sin(kappa, beta))
    return oracle_parallel.direct_solve(xy, tri, 3, 3, kap, beta, 1.0, fo, go, workers=workers)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--only", choices=["norms", "c2"], default=None)
    a = ap.parse_args()
    if a.only in (None, "norms"):
        t = time.time()
        norms = {"mixed_r1to4_8192macro_p3_inst0": mixed_inst0_norm(a.workers)}
        with open(os.path.join(HERE, "fullsize_norms.json"), "w") as fh:
            json.dump(norms, fh, indent=1)
        print(f"norms {norms} ({time.time() - t:.0f} s)", flush=True)
    if a.only in (None, "c2"):
        t = time.time()
        lam, pf = c2_direct(a.workers)
        np.save(os.path.join(HERE, "c2_lambda_direct.npy"), lam)
        print(f"c2 direct solve: n = {len(lam)}, ||D^-1 f^|| = {pf:.6e} ({time.time() - t:.0f} s)",
              flush=True)


if __name__ == "__main__":
    main()
