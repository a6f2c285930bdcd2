"""Writes tests/golden/spectrum_c{1,3}.json: brute-force spectra of the complex-symmetric pencils.

The stated circles (radius 0.3 around 0.5+0.2i at n = 4096, radius 0.5 around
0 at n = 8192) enclose several hundred to thousands of eigenvalues, far more
than the subspace sizes 64 and 128 can hold (the convergence properties of
Section 4 need p >= m').  The workloads therefore keep the pencil, center,
node count and subspace size and place the radius in the middle of a gap in
the sorted distances |lambda - c| near the m*-th eigenvalue (m* = 48 and 100):
the widest relative gap among counts m* - 6 .. m* + 6, so that no eigenvalue
sits close to the contour.

Calls only the oracle on the seeded pencils: the eigenvalues nearest the
center by shift-invert Arnoldi (pinned against QZ in the oracle tests).
Usage:
    python tests/golden/make_spectra.py c1 [n]     # n = 4096 by default
    python tests/golden/make_spectra.py c3 [n]     # n = 8192 by default
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import pencils  # noqa: E402
from oracle import brute  # noqa: E402

CASES = {"c1": (pencils.c1, 48, 0.3), "c3": (pencils.c3, 100, 0.5)}


def main(name, n=None):
    build, m_star, stated_radius = CASES[name]
    P = build() if n is None else build(n=n)
    t0 = time.time()
    near = brute.nearest_eigenvalues(P.A, P.B, P.center, m_star + 24)
    secs = time.time() - t0
    R, m, lo, hi = brute.widest_gap_radius(near, P.center, m_star)
    out = dict(
        workload=name, n=P.n, center=[P.center.real, P.center.imag], m_star=m_star, m=m, radius=R,
        gap=[lo, hi], stated_radius=stated_radius,
        nearest=[[float(z.real), float(z.imag)] for z in near],
        seconds=secs,
        source="oracle.brute.nearest_eigenvalues (shift-invert Arnoldi) on pencils.%s()" % name,
    )
    path = os.path.join(HERE, "spectrum_%s%s.json" % (name, "" if n is None else "_n%d" % n))
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path, "m =", m, "R* =", R, "gap", lo, hi, round(secs, 1), "s")


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else None)
