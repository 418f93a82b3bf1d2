"""The stored 4^4 workload under tests/golden/: its parameters and a reader.

The values were written by make_golden.py from the CPU oracle; this module
holds no arithmetic of the method and imports neither the oracle nor the
HIP binding, so GPU tests read the file through it.
"""
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))

DIMS = (4, 4, 4, 4)
BETA, THETA, SEED = 5.7, 0.0, 1
SIGMA_X, SIGMA_Y = 0.3, 0.05
N_STEPS, EPS = 20, 1e-3
N_COOL, EPS_C, ALPHA, MODE = 5, 1e-3, 1.0, 0
# (site, mu, row, col) of the sampled final link entries
SAMPLES = [(0, 0, 0, 0), (0, 3, 2, 1), (17, 1, 1, 2), (100, 2, 0, 2), (128, 0, 2, 2),
           (200, 3, 1, 0), (255, 1, 2, 0), (255, 3, 0, 1)]
FILE = os.path.join(HERE, "cl_4x4x4x4_beta5.7_seed1.txt")


def read(path=FILE):
    """{'steps': array (N, 5), 'norm2': float, 'links': [(s, mu, i, j, complex)]}."""
    steps, links, norm2 = [], [], None
    with open(path) as f:
        for line in f:
            t = line.split()
            if not t or t[0].startswith("#"):
                continue
            if t[0] == "step":
                steps.append([float(x) for x in t[1:]])
            elif t[0] == "norm2":
                norm2 = float(t[1])
            elif t[0] == "link":
                s, mu, i, j = (int(x) for x in t[1:5])
                links.append((s, mu, i, j, complex(float(t[5]), float(t[6]))))
    return {"steps": np.array(steps), "norm2": norm2, "links": links}
