"""Write the oracle's potential for the finite-difference study of the
differentiable loss (64 x 64, k = 3 triangle, the loss workload's generator
at that size): `fd_potential_64x64_k3.npz` holds Phi = dV/drho0 (m x n x k,
mean removed per mass class; dual problem, Sec. 3.2) of the FP64 oracle run
to a relative residual of 1e-7 (fixed-point residual of Sec. 6.1), with the
run's iteration count, V and residual.  Calls only `oracle/`; takes about
17 minutes on one core.

    python tests/golden/make_fd_potential.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from paper_1712_10279_amd import inputs as I  # noqa: E402

SIDE = 64
TOL = 1e-7


def main():
    d = I.loss_512(0, m=SIDE, n=SIDE)
    tau = I.tuned_tau(SIDE, SIDE)
    r = O.solve_pair(d["rho0"], d["rho1"], d["edges"], alpha=d["alpha"], tau=tau, max_iters=20_000_000, tol=TOL)
    assert r["converged"], r["residual"]
    out = os.path.join(HERE, f"fd_potential_{SIDE}x{SIDE}_k3.npz")
    np.savez_compressed(out, Phi=r["Phi"], iters=r["iters"], V=r["primal"], residual=r["residual"],
                        tau=tau, tol=TOL)
    print(json.dumps({"file": out, "iters": r["iters"], "V": r["primal"], "residual": r["residual"],
                      "rel_gap": r["rel_gap"], "wall_s": r["wall_s"]}))


if __name__ == "__main__":
    main()
