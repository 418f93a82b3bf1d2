"""Write the stored expected values under tests/golden/ from the CPU oracle alone.

The paper prints no numerical worked example (its results are figures), so
the stored values here are the oracle's own outputs on the smallest
workload: a 4^4 periodic SU(3) lattice, Wilson action at beta 5.7, theta 0,
the perturbed start with sigma_x 0.3, sigma_y 0.05 and seed 1, then 20
complex Langevin steps (section *Preliminary results for 4d SU(3)
Yang-Mills theory with a theta-term*, action eq. (eq:st)) at fixed
eps = 1e-3, each followed by 5 gauge cooling steps (eq. (eq:24)) at
alpha_gf = 1 (fixed alpha, eps_c = 1e-3).  Per step the distance d of
eq. (d) before and after the cooling steps and the plaquette; after the
last step the sum of |U_ij|^2 over all links and sampled link entries.

Run from the repository root after building the oracle:

    python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402

from tests.golden.fixture import (ALPHA, BETA, DIMS, EPS, EPS_C, FILE, MODE, N_COOL, N_STEPS,  # noqa: E402
                                  SAMPLES, SEED, SIGMA_X, SIGMA_Y, THETA)


def compute():
    """(obs rows [step, d_pre, d_post, plaq_re, plaq_im], final links (V, 4, 3, 3) complex)."""
    U = oracle.init_links(DIMS, SEED, SIGMA_X, SIGMA_Y)
    obs, _ = oracle.run(DIMS, U, BETA, THETA, SEED, N_STEPS, EPS, False, N_COOL, EPS_C, ALPHA, MODE)
    rows = [(n, *(float(obs[n, k]) for k in range(4))) for n in range(N_STEPS)]
    return rows, oracle.to_complex(U)


def write(path=FILE):
    rows, Uc = compute()
    lines = [
        "# 4^4 SU(3) complex Langevin with gauge cooling, written by tests/golden/make_golden.py",
        "# from the CPU oracle alone: beta 5.7, theta 0, seed 1, start sigma_x 0.3 sigma_y 0.05,",
        "# 20 steps at fixed eps 1e-3, after each 5 cooling steps (fixed alpha_gf 1, eps_c 1e-3).",
        "# step d_before_cooling d_after_cooling plaquette_re plaquette_im   (d: eq. (d))",
    ]
    for n, dp, d, pr, pi in rows:
        lines.append(f"step {n} {dp!r} {d!r} {pr!r} {pi!r}")
    lines.append("# after the last step: sum over all links of sum_ij |U_ij|^2")
    lines.append(f"norm2 {float(np.sum(np.abs(Uc) ** 2))!r}")
    lines.append("# sampled final entries: site (lexicographic, x0 fastest) mu row col re im")
    for s, mu, i, j in SAMPLES:
        z = Uc[s, mu, i, j]
        lines.append(f"link {s} {mu} {i} {j} {float(z.real)!r} {float(z.imag)!r}")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    write()
    print(FILE)
