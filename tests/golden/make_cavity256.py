"""Writes cavity256_oracle.npz: the FP64 oracle's lid-driven cavity (256^2, tanh
stretching beta = 1.5, Re = 1000, dt from CFL 0.8 on the finest cell; App. B.2 set-up)
at steps 100 and 500 from rest, with direct sparse solves.  Calls only the oracle and
the seeded case generator; about 1.5 hours on one core.

    python tests/golden/make_cavity256.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import cases  # noqa: E402
from oracle.piso import Geometry, step  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cavity256_oracle.npz")
KEEP = (100, 500)


def main():
    c = cases.lid_cavity(256)
    geo = Geometry(c.domain)
    u, p = c.u0, c.p0
    keep = {}
    t0 = time.time()
    for n in range(1, max(KEEP) + 1):
        r = step(geo, u, p, c.nu, c.S, c.dt, c.u_b)
        u, p = r.u2, r.p2
        if n in KEEP:
            keep["u%d" % n] = u.copy()
            keep["p%d" % n] = p.copy()
        if n % 10 == 0:
            print("step %d  %.0f s" % (n, time.time() - t0), flush=True)
    np.savez_compressed(OUT, dt=c.dt, steps=np.array(KEEP), **keep)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
