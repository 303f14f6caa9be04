"""Writes the tiny brute-force fixtures in this folder.

The paper prints no worked numeric example, so these fixtures hold dense
least-squares solutions (oracle.dense only: assembled face-flux operators and
numpy.linalg) of tiny channel problems built from the seeded generator. They
freeze the reading of the discretisation (MAC staggering, Neumann and
Dirichlet walls, tanh faces, mean pin) so that a later change to it shows up.

Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import dense  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    cases = []
    for (nx, ny, nz, beta, seed) in [(4, 4, 3, 1.5, 0), (6, 2, 5, 2.0, 1), (3, 3, 4, 1.0, 2)]:
        f, zf = synth.channel_rhs(seed, nx, ny, nz, beta=beta)
        p = dense.poisson_dense(f, zf, 2 * np.pi, np.pi)
        cases.append(dict(kind="poisson", nx=nx, ny=ny, nz=nz, beta=beta, seed=seed,
                          lx=2 * np.pi, ly=np.pi, lz=2.0,
                          p=[float(v) for v in p.reshape(-1)]))
    for (nz, bc, s, seed) in [(6, 1, 0.05, 3), (6, 2, 0.05, 4), (9, 1, 9.615e-9, 5)]:
        zf = synth.tanh_faces(nz, 2.0, 1.5)
        n = nz if bc == 1 else nz - 1
        r = synth.normal01(seed, (n, 2, 2))
        u = dense.helmholtz_dense(r, zf, s, bc)
        cases.append(dict(kind="helmholtz", nz=nz, bc=bc, s=s, seed=seed, beta=1.5, lz=2.0,
                          nx=2, ny=2, u=[float(v) for v in u.reshape(-1)]))
    with open(os.path.join(HERE, "bruteforce_tiny.json"), "w") as fh:
        json.dump(dict(source="oracle.dense least-squares / dense solve; "
                              "discretisation of Sec. 2.1 (MAC grid) and eq. fijk_eq",
                       cases=cases), fh, indent=1)


if __name__ == "__main__":
    main()
