"""Writes the stored expected values under tests/golden/ from the oracle alone.

Each fixture is a small seeded case: the right-hand side (or state) comes from numpy's
PCG64 with the seed named in the file, the expected values from ``oracle/``.  The files
pin the oracle against unintended change and give the GPU tests a reference that needs
no oracle run.  Usage: ``python tests/golden/make_golden.py`` (rewrites the files).
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import Grid, poisson  # noqa: E402
from oracle import substep as ss  # noqa: E402
from paper_1705_01423_amd.synth import zfaces  # noqa: E402

CASES = {
    # Poisson solve (Sec. 2.2): nx, ny, nz, lx, ly, alpha, seed
    "poisson_8x6x4": dict(kind="poisson", nx=8, ny=6, nz=4, lx=1.0, ly=0.75, alpha=3.0, seed=11),
    "poisson_12x8x5": dict(kind="poisson", nx=12, ny=8, nz=5, lx=2.0, ly=1.0, alpha=2.0, seed=12),
    # explicit terms H of u, v, w, T (Sec. 2.1): nu, kappa
    "explicit_8x4x4": dict(kind="explicit", nx=8, ny=4, nz=4, lx=1.0, ly=1.0, alpha=3.0, seed=13,
                           nu=1e-2, kappa=7e-3),
}


def case_inputs(c):
    g = Grid(c["nx"], c["ny"], c["nz"], c["lx"], c["ly"], zfaces(c["nz"], c["alpha"]))
    rng = np.random.default_rng(c["seed"])
    if c["kind"] == "poisson":
        f = torch.as_tensor(rng.standard_normal((c["nz"], c["ny"], c["nx"])))
        return g, (f,)
    cs = (c["nz"], c["ny"], c["nx"])
    fs = (c["nz"] + 1, c["ny"], c["nx"])
    u = torch.as_tensor(rng.standard_normal(cs))
    v = torch.as_tensor(rng.standard_normal(cs))
    w = torch.as_tensor(rng.standard_normal(fs))
    t = torch.as_tensor(rng.standard_normal(fs))
    w[0] = 0.0
    w[-1] = 0.0
    return g, (u, v, w, t)


def expected(c):
    g, ins = case_inputs(c)
    if c["kind"] == "poisson":
        return [poisson.solve(ins[0], g)]
    return list(ss.explicit_terms(*ins, g, c["nu"], c["kappa"]))


def main():
    for name, c in CASES.items():
        out = {"case": c, "generated_by": "tests/golden/make_golden.py (oracle only)",
               "values": [x.reshape(-1).tolist() for x in expected(c)]}
        with open(os.path.join(HERE, name + ".json"), "w") as fh:
            json.dump(out, fh)
            fh.write("\n")
        print("wrote", name)


if __name__ == "__main__":
    main()
