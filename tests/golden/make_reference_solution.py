"""Writes tests/golden/reference_solution_16x32.json: sampled entries of the
oracle's solution x* of D(m0) x = b on the 16^3x32 lattice of the
poorly conditioned single-solve workload (eps = 0.6 links, gauge seed 0,
m0 just above the critical mass, one Gaussian right-hand side).

x* comes from the FP64 oracle alone: FGMRES-DR (Alg. 4) preconditioned by
the oracle's SAP (Alg. 2), run to a relative residual well below the one
the GPU test asks for, and its true residual is recomputed with the
oracle's D (eq. 1). The whole solution (25 MB) is not stored: a seeded
sample of its entries, with their flat indices into the canonical
[t][z][y][x][spin][colour] array, and its 2-norm are.

Usage: python tests/golden/make_reference_solution.py [delta]
  delta: m0 = m_c + delta (default 0.001), m_c from critical_mass.json
  (the 16^3x32 entry when present, else the 12^4 one, recorded as m0_from).
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import fgmresdr as F  # noqa: E402
from oracle import sap as S  # noqa: E402
from oracle import wilson as W  # noqa: E402

OUT = os.path.join(HERE, "reference_solution_16x32.json")
L = (16, 16, 16, 32)
EPS, GAUGE_SEED, RHS_SEED = 0.6, 0, 2024
BLOCK, NCYC, NMR = (4, 4, 4, 4), 1, 4
M, K, TOL = 30, 10, 1e-13
NSAMPLE, SAMPLE_SEED = 2048, 77


def main(delta):
    crit = json.load(open(os.path.join(HERE, "critical_mass.json")))
    src = "16^3x32_eps0.6" if "16^3x32_eps0.6" in crit else "12^4_eps0.6"
    m0 = crit[src]["m_c"] + delta
    U = synth.gauge_field(L, EPS, GAUGE_SEED)
    b = synth.gaussian_spinor(L, RHS_SEED)
    shp = b.shape

    def A(v):
        return W.apply_D(U, m0, v.reshape(shp)).reshape(-1)

    def Mp(v):
        return S.sap(U, m0, L, BLOCK, NCYC, NMR, v.reshape(shp)).reshape(-1)

    t0 = time.time()
    x, info = F.fgmresdr(A, Mp, b.reshape(-1), M, K, tol=TOL, max_iter=20000)
    secs = time.time() - t0
    r = b.reshape(-1) - A(x)
    relres = float(np.linalg.norm(r) / np.linalg.norm(b))
    rng = np.random.default_rng(SAMPLE_SEED)
    idx = np.sort(rng.choice(x.size, size=NSAMPLE, replace=False))
    out = {
        "L": list(L), "eps": EPS, "gauge_seed": GAUGE_SEED, "rhs_seed": RHS_SEED,
        "m0": m0, "m0_from": f"m_c({src}) + {delta}",
        "oracle_solver": {"method": "FGMRES-DR", "m": M, "k": K, "tol": TOL,
                          "sap": {"block": list(BLOCK), "ncycles": NCYC, "nmr": NMR}},
        "converged": bool(info.converged), "iterations": int(info.iterations), "cycles": int(info.cycles),
        "true_relres": relres, "seconds": round(secs, 1),
        "x_norm": float(np.linalg.norm(x)),
        "sample_seed": SAMPLE_SEED,
        "sample_index": idx.tolist(),
        "sample_re": x[idx].real.tolist(),
        "sample_im": x[idx].imag.tolist(),
    }
    with open(OUT, "w") as fh:
        json.dump(out, fh)
    print(f"{OUT}: m0 {m0:.6f} ({src}), {info.iterations} iterations, {info.cycles} cycles, "
          f"true relres {relres:.2e}, {secs:.0f} s")


if __name__ == "__main__":
    main(float(sys.argv[1]) if len(sys.argv) > 1 else 0.001)
