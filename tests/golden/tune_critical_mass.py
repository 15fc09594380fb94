"""Writes tests/golden/critical_mass.json: the leftmost eigenvalues of the
massless Wilson-Dirac operator D(0) (with the clover term where a
coefficient is given) for the seeded synthetic gauge fields,
from which the near-critical masses of the workloads are set.

Uses only the FP64 oracle's operator (and SciPy's ARPACK). Since
D(m0) = D(0) + m0 I exactly, the eigenvalue of D(m0) closest to the left
edge is lambda_edge + m0; the critical mass is m_c = -Re(lambda_edge) and
a near-critical mass is m0 = m_c + delta.

Usage: python tests/golden/tune_critical_mass.py [--quick] [name ...]
  --quick: 4 Ritz values, ncv 24, tol 1e-7 (enough for the critical mass
           to about 1e-5; for lattices where the default settings take hours)
"""
import fcntl
import json
import os
import sys
import time

import numpy as np
import scipy.sparse.linalg as sla

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import clover as Cl  # noqa: E402
from oracle import wilson as W  # noqa: E402

OUT = os.path.join(HERE, "critical_mass.json")

# name: (L, eps, gauge seed[, clover coefficient[, ARPACK settings]])
FIELDS = {
    "8^4_eps0.3": ((8, 8, 8, 8), 0.3, 0),
    "8^4_eps0.7": ((8, 8, 8, 8), 0.7, 0),
    "12^4_eps0.7": ((12, 12, 12, 12), 0.7, 0),
    "8^4_eps0.6": ((8, 8, 8, 8), 0.6, 0),
    "12^4_eps0.6": ((12, 12, 12, 12), 0.6, 0),
    "16^3x32_eps0.6": ((16, 16, 16, 32), 0.6, 0),
    "16^3x32_eps0.7": ((16, 16, 16, 32), 0.7, 0),
    "8^4_eps0.7_csw1.9": ((8, 8, 8, 8), 0.7, 0, 1.9),
    "12^4_eps0.7_csw1.9": ((12, 12, 12, 12), 0.7, 0, 1.9),
    # 25.2M unknowns: fewer Ritz values and a looser tolerance keep the basis
    # (ncv vectors of 403 MB) in host memory and the matvec count bounded;
    # the critical mass is needed to about 1e-5
    "32^3x64_eps0.7": ((32, 32, 32, 64), 0.7, 0, 0.0, dict(nev=4, ncv=24, tol=1e-7)),
    "24^3x48_eps0.6": ((24, 24, 24, 48), 0.6, 0, 0.0, dict(nev=4, ncv=32, tol=1e-7)),
    "32^3x64_eps0.6": ((32, 32, 32, 64), 0.6, 0, 0.0, dict(nev=4, ncv=24, tol=1e-7)),
}


def leftmost(L, eps, seed, csw=0.0, nev=12, ncv=64, tol=1e-9):
    U = synth.gauge_field(L, eps, seed)
    C = Cl.clover_term(U, csw) if csw else None
    shp = synth.lattice_shape(L) + (4, 3)
    n = int(np.prod(shp))
    count = [0]

    def mv(v):
        count[0] += 1
        return W.apply_D(U, 0.0, v.reshape(shp).astype(np.complex128), C).reshape(-1)

    op = sla.LinearOperator((n, n), matvec=mv, dtype=np.complex128)
    v0 = synth.gaussian_spinor(L, 4242).reshape(-1)
    t0 = time.time()
    ev = sla.eigs(op, k=nev, which="SR", ncv=ncv, tol=tol, v0=v0, return_eigenvectors=False, maxiter=5000)
    ev = ev[np.argsort(ev.real)]
    return ev, count[0], time.time() - t0


QUICK = dict(nev=4, ncv=24, tol=1e-7)


def main(names, quick=False):
    for name in names:
        L, eps, seed = FIELDS[name][:3]
        csw = FIELDS[name][3] if len(FIELDS[name]) > 3 else 0.0
        opts = dict(nev=12, ncv=64, tol=1e-9)
        opts.update(FIELDS[name][4] if len(FIELDS[name]) > 4 else {})
        if quick:
            opts.update(QUICK)
        ev, nmv, secs = leftmost(L, eps, seed, csw, **opts)
        # several runs may finish at once: read-modify-write under a lock
        lock = open(OUT + ".lock", "w")
        fcntl.flock(lock, fcntl.LOCK_EX)
        data = json.load(open(OUT)) if os.path.exists(OUT) else {}
        data[name] = {
            "L": list(L), "eps": eps, "seed": seed, "csw": csw,
            "leftmost_eigenvalues_D0": [[float(e.real), float(e.imag)] for e in ev],
            "m_c": float(-ev[0].real),
            "matvecs": nmv, "seconds": round(secs, 1),
            "method": f"scipy.sparse.linalg.eigs(which='SR', k={opts['nev']}, ncv={opts['ncv']}, tol={opts['tol']:g}) "
                      "on oracle.wilson.apply_D(U, 0, ., C) (C = oracle.clover.clover_term(U, csw) when csw != 0)",
        }
        with open(OUT + ".tmp", "w") as fh:
            json.dump(data, fh, indent=1)
        os.replace(OUT + ".tmp", OUT)
        fcntl.flock(lock, fcntl.LOCK_UN)
        lock.close()
        print(name, "m_c", -ev[0].real, "edge", ev[:4], nmv, "matvecs", round(secs), "s", flush=True)


if __name__ == "__main__":
    args = [a for a in sys.argv[1:] if a != "--quick"]
    main(args or list(FIELDS), quick="--quick" in sys.argv[1:])
