"""Write precond_spiral_16384.npz: z = P^{-1} r and z = P^{-H} r for two seeded
vectors r on the N = 2^14 Archimedean spiral (theta in [pi, 6 pi], leaves of
64), in both preconditioner readings, from the CPU oracle's dense
definitions (block substitutions with the exact leaf blocks; the paper's
point-wise triangular factors of the rescaled matrix).

At this size the GPU sweeps run three block levels above the default
subtree programs, so these values check the big-block sweep launches, which
the N = 4096 references cannot reach.

Run: python tests/golden/make_precond_2p14.py   (about 5 minutes, ~30 GB RAM)
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import efie  # noqa: E402
from paper_1901_11371_amd import inputs  # noqa: E402

N = 1 << 14
SEED = 190111371 + 500
NVEC = 2


def main():
    c = inputs.archimedean_spiral(N)
    rho, w = efie.segments(c.xy, c.node_off)
    A = efie.dense_A(rho, w, inputs.KAPPA)
    R = inputs.random_complex((NVEC, N), SEED)
    out = {"r": R}
    for adj in (False, True):
        tag = "adj" if adj else "fwd"
        out[f"block_{tag}"] = efie.precond_block_apply(A, R.T, 64, adjoint=adj).T
        out[f"paper_{tag}"] = efie.precond_paper_apply(A, R.T, adjoint=adj).T
        print(tag, "done", flush=True)
    np.savez_compressed(os.path.join(HERE, "precond_spiral_16384.npz"), **out)


if __name__ == "__main__":
    main()
