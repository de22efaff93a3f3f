"""Write the stored expected values of the parity tests (FP64 oracle only).

* cfg2_2000.json, cfg2_2000_f.npy: the 64 x 64 x 3 x 16 workload after 2000
  iterations of Algorithm 1 (tau = 10, sigma = 0.099, theta = 1, cold start)
  on the seeded FP32-rounded inputs of synth.inputs.cfg2_pair: summary
  values, a seeded sample of the density, and the whole interior density
  f[1..P-1] (stored in FP32: its rounding, 6e-8 relative, is far below the
  1e-5 parity tolerance).
* cfg1_converged.json, cfg1_converged.npz: the 16 x 16 x 3 x 8 workload
  (synth.inputs.cfg1_pair) iterated by the same Algorithm 1 until max(r_prim,
  r_dual) < 1e-12, i.e. the minimiser of the discrete model to FP64 accuracy,
  and the distance between it and the iterate at the first residual check
  (every 100 iterations) where the certificate max(r_prim, r_dual) < 1e-6,
  r_div < 1e-6 holds: the distance the certificate implies on this problem.

Usage: python tests/golden/make_golden.py [cfg2] [cfg1]
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


def _rel(a, b):
    a, b = np.ravel(a), np.ravel(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def cfg2():
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
    np.save(os.path.join(HERE, "cfg2_2000_f.npy"), f.astype(np.float32))
    print({k: out[k] for k in ("cost", "r_prim", "r_dual", "r_div", "e_mass", "f_norm")})


def cfg1(tol_exact=1e-12, tol_cert=1e-6, check=100, max_iters=200000):
    f0, f1 = inputs.cfg1_pair()
    a0, a1 = f0.astype(np.float64), f1.astype(np.float64)
    g = G.Grid(16, 16, 3, 8)
    st, it, cert = None, 0, None
    while it < max_iters:
        st = pdhg.solve(g, a0, a1, TAU, SIGMA, check, state=st, record_every=check)
        it += check
        h = st.hist[-1]
        res = max(h["r_prim"], h["r_dual"])
        if cert is None and res < tol_cert and h["r_div"] < tol_cert:
            cert = {"iterations": it, "x": tuple(np.copy(a) for a in st.x), "cost": h["cost"]}
        if res < tol_exact:
            break
    h = st.hist[-1]
    assert max(h["r_prim"], h["r_dual"]) < tol_exact, h
    out = {
        "source": "oracle.pdhg.solve, cold start, cfg1_pair seeds 101/102, until "
                  f"max(r_prim, r_dual) < {tol_exact:g}",
        "grid": [16, 16, 3, 8], "tau": TAU, "sigma": SIGMA,
        "iterations": it, "cost": h["cost"], "r_prim": h["r_prim"], "r_dual": h["r_dual"],
        "r_div": h["r_div"],
        "certified_at": cert["iterations"], "certified_cost": cert["cost"],
        "certified_f_distance": _rel(cert["x"][3], st.x[3]),
        "certified_m_distance": [_rel(cert["x"][a], st.x[a]) for a in range(3)],
    }
    with open(os.path.join(HERE, "cfg1_converged.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    np.savez_compressed(os.path.join(HERE, "cfg1_converged.npz"), m_x=st.x[0], m_y=st.x[1],
                        m_c=st.x[2], f=st.x[3])
    print(out)


if __name__ == "__main__":
    which = sys.argv[1:] or ["cfg2", "cfg1"]
    for w in which:
        {"cfg2": cfg2, "cfg1": cfg1}[w]()
