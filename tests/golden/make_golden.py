"""Write the stored expected values of the 64 x 64 x 3 x 16 parity workload.

Runs only the FP64 oracle (Algorithm 1, tau = 10, sigma = 0.099, theta = 1,
cold start) on the seeded FP32-rounded inputs of synth.inputs.cfg2_pair and
stores summary values plus the density at a seeded sample of interior nodes.
Usage: python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import grid as G  # noqa: E402
from oracle import pdhg  # noqa: E402
from synth import inputs  # noqa: E402

TAU, SIGMA, ITERS = 10.0, 0.099, 2000
X, Y, C, P = 64, 64, 3, 16
N_SAMPLE = 4096


def main():
    f0, f1 = inputs.cfg2_pair()
    g = G.Grid(X, Y, C, P)
    st = pdhg.solve(g, f0.astype(np.float64), f1.astype(np.float64), TAU, SIGMA, ITERS,
                    record_every=ITERS)
    h = st.hist[-1]
    f = st.x[3]
    rng = np.random.default_rng(2024)
    idx = rng.choice(f.size, size=N_SAMPLE, replace=False)
    out = {
        "source": "oracle.pdhg.solve, cold start, cfg2_pair seeds 201/202",
        "grid": [X, Y, C, P], "tau": TAU, "sigma": SIGMA, "iters": ITERS,
        "cost": h["cost"], "r_prim": h["r_prim"], "r_dual": h["r_dual"],
        "r_div": h["r_div"], "e_mass": h["e_mass"],
        "f_norm": float(np.linalg.norm(f)),
        "frame_norms": [float(np.linalg.norm(f[k])) for k in range(P - 1)],
        "m_norms": [float(np.linalg.norm(st.x[a])) for a in range(3)],
        "sample_index": [int(i) for i in idx],
        "sample_f": [float(v) for v in f.ravel()[idx]],
    }
    with open(os.path.join(HERE, "cfg2_2000.json"), "w") as fh:
        json.dump(out, fh, indent=0)
    print({k: out[k] for k in ("cost", "r_prim", "r_dual", "r_div", "e_mass", "f_norm")})


if __name__ == "__main__":
    main()
