"""Write spiral_4096_iterations.json: iteration counts of the CPU oracle's
Krylov solvers on the N = 4096 Archimedean spiral (theta in [pi, 6 pi], one
plane wave at pi/6, block preconditioner with leaves of 64, relres 1e-6).

Only the oracle runs here (dense FP64 operator, dense block substitutions).
The GPU solver's iteration counts on the same system are compared with these
(its operator differs from the dense one by the compression tolerance, so
counts agree to a few per cent, not exactly).

Run: python tests/golden/make_spiral_iterations.py   (about two minutes)
"""
import json
import math
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import scipy.linalg as sla  # noqa: E402

from oracle import efie  # noqa: E402
from paper_1901_11371_amd import inputs  # noqa: E402

N = 4096
ANGLE = math.pi / 6
TOL = 1e-6


def main():
    c = inputs.archimedean_spiral(N)
    rho, w = efie.segments(c.xy, c.node_off)
    A = efie.dense_A(rho, w, inputs.KAPPA)
    b = inputs.plane_wave_rhs(c, [ANGLE])[0]
    D, Al, Au = efie.block_parts(A, 64)
    L = sla.lu_factor(D + Al)
    U = sla.lu_factor(D + Au)
    M = lambda r: sla.lu_solve(U, D @ sla.lu_solve(L, r))
    out = {"n": N, "angle": ANGLE, "tol": TOL, "leaf": 64}
    _, it, _ = efie.gmres(lambda v: A @ v, M, b, tol=TOL, restart=300, maxiter=1000)
    out["gmres_full"] = it
    _, it, _ = efie.gmres(lambda v: A @ v, M, b, tol=TOL, restart=30, maxiter=2000)
    out["gmres30"] = it
    _, it, _ = efie.tfqmr(lambda v: A @ v, M, b, tol=TOL, maxiter=2000)
    out["tfqmr"] = it
    with open(os.path.join(HERE, "spiral_4096_iterations.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(out)


if __name__ == "__main__":
    main()
