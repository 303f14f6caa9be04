"""Oracle against the frozen brute-force fixtures in tests/golden/."""
import json
import os

import numpy as np

import synth
from oracle import poisson

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_bruteforce_fixtures():
    with open(os.path.join(HERE, "bruteforce_tiny.json")) as fh:
        data = json.load(fh)
    for c in data["cases"]:
        if c["kind"] == "poisson":
            f, zf = synth.channel_rhs(c["seed"], c["nx"], c["ny"], c["nz"], beta=c["beta"])
            p = poisson.solve_poisson(f, zf, c["lx"], c["ly"])
            ref = np.array(c["p"]).reshape(p.shape)
            assert poisson.rel_l2(p, ref) < 1e-12
        else:
            zf = synth.tanh_faces(c["nz"], c["lz"], c["beta"])
            n = c["nz"] if c["bc"] == 1 else c["nz"] - 1
            r = synth.normal01(c["seed"], (n, c["ny"], c["nx"]))
            u = poisson.solve_helmholtz(r, zf, c["s"], c["bc"])
            assert poisson.rel_l2(u, np.array(c["u"]).reshape(u.shape)) < 1e-13
