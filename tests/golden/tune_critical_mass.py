"""Writes tests/golden/critical_mass.json: the leftmost eigenvalues of the
massless Wilson-Dirac operator D(0) (with the clover term where a
coefficient is given) for the seeded synthetic gauge fields,
from which the near-critical masses of the workloads are set.

Uses only the FP64 oracle's operator (and SciPy's ARPACK). Since
D(m0) = D(0) + m0 I exactly, the eigenvalue of D(m0) closest to the left
edge is lambda_edge + m0; the critical mass is m_c = -Re(lambda_edge) and
a near-critical mass is m0 = m_c + delta.

Usage: python tests/golden/tune_critical_mass.py [--quick | --arnoldi K] [name ...]
  --quick: 4 Ritz values, ncv 24, tol 1e-7 (enough for the critical mass
           to about 1e-5; for lattices where the default settings take hours)
  --arnoldi K: the leftmost Ritz value of K steps of a plain (unrestarted)
           Arnoldi process on D(0) instead of ARPACK, for lattices where the
           edge of the spectrum is too dense for the restarted method to
           converge in hours. The Ritz value approaches the edge from inside
           the spectrum: on the 12^4 eps = 0.6 field 150 steps give 0.86627
           against ARPACK's 0.86591, so such an m_c lies below the true one by
           a few 1e-4 and a mass m_c + delta is that much closer to critical.
           The basis is kept in complex64 for lattices above 2^20 sites (the
           Ritz values agree with a complex128 basis to 6 digits on 12^4).
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


def arnoldi_leftmost(L, eps, seed, steps, csw=0.0):
    """Ritz values of D(0) from `steps` Arnoldi steps (classical Gram-Schmidt
    applied twice), sorted by real part; the start vector is the same seeded
    Gaussian spinor as for ARPACK."""
    import scipy.linalg as sla_dense
    U = synth.gauge_field(L, eps, seed)
    C = Cl.clover_term(U, csw) if csw else None
    v = synth.gaussian_spinor(L, 4242)
    shp, n = v.shape, v.size
    dt = np.complex64 if synth.volume(L) > (1 << 20) else np.complex128
    V = np.zeros((steps + 1, n), dtype=dt)
    H = np.zeros((steps + 1, steps), dtype=np.complex128)
    V[0] = v.reshape(-1) / np.linalg.norm(v)
    t0 = time.time()
    for j in range(steps):
        w = W.apply_D(U, 0.0, V[j].astype(np.complex128).reshape(shp), C).reshape(-1)
        for _ in range(2):
            h = (V[:j + 1].conj() @ w.astype(dt)).astype(np.complex128)
            w = w - (V[:j + 1].T @ h.astype(dt)).astype(np.complex128)
            H[:j + 1, j] += h
        H[j + 1, j] = np.linalg.norm(w)
        V[j + 1] = w / H[j + 1, j]
    ev = sla_dense.eigvals(H[:steps, :steps])
    return ev[np.argsort(ev.real)][:12], steps, time.time() - t0


def main(names, quick=False, arnoldi=0):
    for name in names:
        L, eps, seed = FIELDS[name][:3]
        csw = FIELDS[name][3] if len(FIELDS[name]) > 3 else 0.0
        opts = dict(nev=12, ncv=64, tol=1e-9)
        opts.update(FIELDS[name][4] if len(FIELDS[name]) > 4 else {})
        if quick:
            opts.update(QUICK)
        if arnoldi:
            ev, nmv, secs = arnoldi_leftmost(L, eps, seed, arnoldi, csw)
            method = (f"leftmost Ritz value of {arnoldi} unrestarted Arnoldi steps (CGS twice) on "
                      "oracle.wilson.apply_D(U, 0, .); approaches the edge from inside the spectrum")
        else:
            ev, nmv, secs = leftmost(L, eps, seed, csw, **opts)
            method = (f"scipy.sparse.linalg.eigs(which='SR', k={opts['nev']}, ncv={opts['ncv']}, tol={opts['tol']:g}) "
                      "on oracle.wilson.apply_D(U, 0, ., C) (C = oracle.clover.clover_term(U, csw) when csw != 0)")
        # several runs may finish at once: read-modify-write under a lock
        lock = open(OUT + ".lock", "w")
        fcntl.flock(lock, fcntl.LOCK_EX)
        data = json.load(open(OUT)) if os.path.exists(OUT) else {}
        data[name] = {
            "L": list(L), "eps": eps, "seed": seed, "csw": csw,
            "leftmost_eigenvalues_D0": [[float(e.real), float(e.imag)] for e in ev],
            "m_c": float(-ev[0].real),
            "matvecs": nmv, "seconds": round(secs, 1),
            "method": method,
        }
        with open(OUT + ".tmp", "w") as fh:
            json.dump(data, fh, indent=1)
        os.replace(OUT + ".tmp", OUT)
        fcntl.flock(lock, fcntl.LOCK_UN)
        lock.close()
        print(name, "m_c", -ev[0].real, "edge", ev[:4], nmv, "matvecs", round(secs), "s", flush=True)


if __name__ == "__main__":
    argv = sys.argv[1:]
    steps = 0
    if "--arnoldi" in argv:
        i = argv.index("--arnoldi")
        steps = int(argv[i + 1])
        del argv[i:i + 2]
    args = [a for a in argv if a != "--quick"]
    main(args or list(FIELDS), quick="--quick" in argv, arnoldi=steps)
