#!/usr/bin/env python3
"""Write the oracle's solution of the 2048 x 2048 periodic multi-circle
extension at a strided sample of nodes, for the GPU parity test of that
configuration.

The problem is ``workloads.periodic_circles_problem(2048, seed=3)``: [0, 1)^2
periodic, 20 seeded circles (centres uniform, radii U[0.05, 0.15]), F a sum of
8 seeded Fourier modes, known inside the circles.  The solution comes from
``oracle.extend_direct`` alone (SuperLU factorisation of A_UU plus two
long-double refinement steps); nothing here runs or reads the GPU library.
The full solve takes about ten minutes and some 20 GiB of host memory.

Sampled nodes: linear indices k * STRIDE (k = 0, 1, ...) that are unknown.
Output: ``periodic_circles_2048_sample.txt`` beside this script, one
"index value" pair per line (value printed with 17 significant digits),
after a header that records the problem, the norms of the whole solution and
the oracle's refinement residuals.

    python3 tests/golden/make_periodic_2048_sample.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

N_SIDE = 2048
SEED = 3
STRIDE = 1021          # prime: the sample visits every row and column phase
OUT = os.path.join(HERE, "periodic_circles_2048_sample.txt")


def main():
    import oracle as O
    from paper_1704_08897_amd import workloads as W
    p = W.periodic_circles_problem(N_SIDE, seed=SEED)
    known = O.known_mask(p.phi)
    t0 = time.time()
    ref, info = O.extend_direct(p.phi, p.F, p.bcx, p.bcy)
    secs = time.time() - t0
    relres = O.true_relative_residual(known, p.F, ref, p.bcx, p.bcy)
    flat = ref.ravel()
    unk = ~known.ravel()
    idx = np.arange(0, flat.size, STRIDE)
    idx = idx[unk[idx]]
    with open(OUT, "w") as f:
        f.write("# oracle solution of periodic_circles_problem(2048, seed=3) at sampled unknown nodes\n")
        f.write("# written by tests/golden/make_periodic_2048_sample.py (oracle.extend_direct: SuperLU + 2 long-double refinement steps)\n")
        f.write(f"nx = {p.nx}\nny = {p.ny}\nseed = {SEED}\nstride = {STRIDE}\n")
        f.write(f"n_unknown = {int(unk.sum())}\n")
        f.write(f"norm_all = {np.linalg.norm(flat):.17e}\n")
        f.write(f"norm_unknown = {np.linalg.norm(flat[unk]):.17e}\n")
        f.write(f"true_rel_residual = {relres:.3e}\n")
        f.write(f"refine_residuals = {' '.join(f'{r:.3e}' for r in info['refine_residuals'])}\n")
        f.write(f"oracle_seconds = {secs:.1f}\n")
        f.write(f"samples = {idx.size}\n")
        for i in idx:
            f.write(f"{int(i)} {flat[i]:.17e}\n")
    print(f"wrote {idx.size} samples to {OUT} ({secs:.0f} s; true rel residual {relres:.2e})")


if __name__ == "__main__":
    main()
