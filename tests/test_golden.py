"""Stored expected values (tests/golden/, written from the oracle by make_golden.py):
the oracle still reproduces them, and the GPU library matches them."""
import json
import os

import pytest
import torch

from golden.make_golden import CASES, case_inputs, expected

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
F64 = torch.float64


def _stored(name):
    with open(os.path.join(HERE, name + ".json")) as fh:
        rec = json.load(fh)
    assert rec["case"] == CASES[name]
    return [torch.tensor(v, dtype=F64) for v in rec["values"]]


def _rel(a, b):
    return float((a.reshape(-1) - b.reshape(-1)).norm() / b.norm())


@pytest.mark.parametrize("name", sorted(CASES))
def test_oracle_reproduces_stored(name):
    got = expected(CASES[name])
    for g, s in zip(got, _stored(name)):
        assert _rel(g, s) < 1e-13


@pytest.mark.gpu
@pytest.mark.parametrize("name", sorted(CASES))
def test_library_matches_stored(name):
    from paper_1705_01423_amd.api import Plan
    from paper_1705_01423_amd.synth import zfaces
    c = CASES[name]
    print(f"[gpu-test] golden {name}", flush=True)
    g, ins = case_inputs(c)
    plan = Plan(c["nx"], c["ny"], c["nz"], c["lx"], c["ly"], zfaces(c["nz"], c["alpha"]), precision="fp64")
    stored = _stored(name)
    if c["kind"] == "poisson":
        phi, _ = plan.solve(ins[0].to("cuda"))
        assert _rel(phi.cpu(), stored[0]) < 1e-12
    else:
        u, v, w, t = [x.to("cuda") for x in ins]
        p = torch.zeros_like(u)
        h = [torch.empty_like(x) for x in (u, v, w, t)]
        plan.substep(1, 1e-3, c["nu"], c["kappa"], u, v, w, t, p, h_out=h)
        for got, s in zip(h, stored):
            assert _rel(got.cpu(), s) < 1e-13
