"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a copy of an oracle module (a dropped term, a wrong sign,
a shifted index, a swapped metric), built from the module's source text in memory, installs
that copy wherever the oracle and its pin tests refer to the original, and checks that at
least one of the named pins then fails.  Nothing on disk changes and no GPU is involved.
"""
import importlib
import pathlib
import sys
import types

import pytest

import oracle
import test_oracle_adjoint as t_adj
import test_oracle_cn_substep as t_cn
import test_oracle_multires as t_mr
import test_oracle_poisson as t_po
import test_oracle_timestep as t_ts

ORACLE_DIR = pathlib.Path(oracle.__file__).parent
PIN_MODULES = (t_adj, t_cn, t_mr, t_po, t_ts)


def _mutant(name, old, new):
    """A fresh module built from oracle/<name>.py with ``old`` replaced by ``new`` once."""
    path = ORACLE_DIR / f"{name}.py"
    text = path.read_text()
    if old:
        assert text.count(old) == 1, f"mutation site not unique in {name}: {old!r}"
        text = text.replace(old, new)
    mod = types.ModuleType(f"oracle.{name}")
    mod.__package__ = "oracle"
    mod.__file__ = str(path)
    exec(compile(text, f"<oracle/{name}.py with a planted mistake>", "exec"), mod.__dict__)
    return mod


def _install(monkeypatch, name, mod):
    """Point every reference to the original module, or to a function or class defined in it,
    at the mutant's counterpart (oracle package, its modules and the pin test modules)."""
    orig = importlib.import_module(f"oracle.{name}")
    own = dict(vars(orig))
    holders = [m for k, m in list(sys.modules.items())
               if (k == "oracle" or k.startswith("oracle.")) and m is not orig]
    holders += list(PIN_MODULES)
    for holder in holders:
        for attr, val in list(vars(holder).items()):
            if val is orig:
                monkeypatch.setattr(holder, attr, mod)
            elif (callable(val) and getattr(val, "__module__", None) == orig.__name__
                  and own.get(getattr(val, "__name__", "")) is val):
                monkeypatch.setattr(holder, attr, getattr(mod, val.__name__))


def _fails(pin):
    try:
        pin()
    except (AssertionError, FloatingPointError, ZeroDivisionError, RuntimeError, ValueError):
        return True
    return False


# (module, original text, planted mistake, pins expected to catch it)
CASES = {
    # Poisson solve, Sec. 2.2 (Eqs. (1)-(3) give the equations it serves)
    "z-solve: first-row excess from the wrong cell": (
        "poisson", "e = lam * dz[0]", "e = lam * dz[1]",
        [lambda: t_po.test_manufactured_stretched((16, 12, 10)), lambda: t_po.test_brute_force_dense((6, 12, 5))]),
    "z-solve: sign of the eliminated right-hand side": (
        "poisson", "y = -dz[k] * F[k] + m * y", "y = -dz[k] * F[k] - m * y",
        [lambda: t_po.test_closed_form_eigenvector_uniform((16, 12, 10)), t_po.test_zsolve_vs_banded]),
    "z-solve: back-substitution couples through the wrong face": (
        "poisson", "x = (ys[k] + o[k + 1] * x) / pivots[k]", "x = (ys[k] + o[k] * x) / pivots[k]",
        [lambda: t_po.test_manufactured_stretched((16, 12, 10)), t_po.test_zsolve_vs_banded]),
    "(0,0) column: compatibility mean not removed": (
        "poisson", "fixed = [v - mean_plane for v in vals]", "fixed = list(vals)",
        [t_po.test_residual_and_gauge, lambda: t_po.test_brute_force_dense((6, 12, 5))]),
    "(0,0) column: cell width in place of the centre spacing": (
        "poisson", "dzc[k] * q[k] for k in range(1, g.nz)", "dz[k] * q[k] for k in range(1, g.nz)",
        [lambda: t_po.test_brute_force_dense((6, 12, 5)), t_po.test_residual_and_gauge]),
    "(0,0) column: unweighted gauge": (
        "poisson", "shift = math.fsum(d * p for d, p in zip(dz, phi)) / total_dz",
        "shift = math.fsum(phi) / g.nz",
        [t_po.test_residual_and_gauge, lambda: t_po.test_brute_force_dense((6, 12, 5))]),
    "projection: wrong sign of the velocity correction": (
        "poisson", "wn = w - s * gw", "wn = w + s * gw",
        [t_po.test_projector_identities]),
    "pressure update: wrong sign of the implicit correction": (
        "poisson", "pn = p + phi - c * op.dzz_centre_neumann(phi, g)",
        "pn = p + phi + c * op.dzz_centre_neumann(phi, g)",
        [t_adj.test_projection_transpose_dense, lambda: t_cn.test_rest_state()]),
    # Grid metrics and modified wavenumbers
    "modified wavenumber with 2/dx^2": (
        "grid", "self.lamx = (4.0 / self.dx ** 2)", "self.lamx = (2.0 / self.dx ** 2)",
        [lambda: t_po.test_closed_form_eigenvector_uniform((16, 12, 10))]),
    "y wavenumber over the x length": (
        "grid", "torch.sin(math.pi * ky / ny)", "torch.sin(math.pi * ky / self.nx)",
        [lambda: t_po.test_closed_form_eigenvector_uniform((16, 12, 10))]),
    "face coupling over the cell width": (
        "grid", "o[1:nz] = 1.0 / dzc[1:nz]", "o[1:nz] = 1.0 / self.dz[1:nz]",
        [lambda: t_po.test_manufactured_stretched((16, 12, 10)), lambda: t_po.test_brute_force_dense((6, 12, 5))]),
    "wall distance of the first centre": (
        "grid", "dzw[0] = 0.5 * self.dz[0]", "dzw[0] = self.dz[0]",
        [t_cn.test_dzz_linear_profiles, t_cn.test_dzz_centre_convergence]),
    # Discrete operators
    "gradient: forward instead of backward difference in x": (
        "operators", "gu = (phi - torch.roll(phi, 1, dims=2)) / g.dx", "gu = (torch.roll(phi, -1, dims=2) - phi) / g.dx",
        [t_po.test_summation_by_parts, lambda: t_po.test_closed_form_eigenvector_uniform((16, 12, 10))]),
    "divergence: z difference over the centre spacing": (
        "operators", "+ (w[1:] - w[:-1]) / g.dz[:, None, None])", "+ (w[1:] - w[:-1]) / g.dzc[1:, None, None])",
        [t_po.test_summation_by_parts, lambda: t_po.test_second_order_convergence(3.0)]),
    # Crank-Nicolson solves, Sec. 2.1-2.2
    "CN centre matrix: upper coupling from the lower wall distance": (
        "cn", "ap[k] = 1.0 / (g.dzw[k + 1] * g.dz[k])", "ap[k] = 1.0 / (g.dzw[k] * g.dz[k])",
        [t_cn.test_cn_centre_dense]),
    "Thomas: sign of the forward elimination": (
        "cn", "dp[k] = (rhs[k] - sub[k] * dp[k - 1]) / den", "dp[k] = (rhs[k] + sub[k] * dp[k - 1]) / den",
        [t_cn.test_cn_centre_dense, t_cn.test_cn_face_dense]),
    # Explicit terms, RK3 substep, Sec. 2.1
    "RK3: the two rho coefficients swapped": (
        "substep", "RHO = (0.0, -17.0 / 60.0, -5.0 / 12.0)", "RHO = (0.0, -5.0 / 12.0, -17.0 / 60.0)",
        [t_cn.test_rk3_coefficients, t_ts.test_step_rk3_amplification]),
    "CN: full instead of half implicit weight": (
        "substep", "bnu = alp * dt * nu / 2.0", "bnu = alp * dt * nu",
        [lambda: t_cn.test_substep_crank_nicolson_modes(2)]),
    "CN: explicit half without alpha": (
        "substep", "r = gam * h - alp * gp + alp * lapz", "r = gam * h - alp * gp + lapz",
        [lambda: t_cn.test_substep_crank_nicolson_modes(1)]),
    "buoyancy dropped": (
        "substep", "nu * (op.dxx(w, g) + op.dyy(w, g)) + t", "nu * (op.dxx(w, g) + op.dyy(w, g))",
        [t_cn.test_rest_state, lambda: t_cn.test_explicit_terms_second_order(0.0)]),
    "temperature advection with the wrong sign": (
        "substep", "ht = -adv_face(t, u, v, w, g)", "ht = adv_face(t, u, v, w, g)",
        [lambda: t_cn.test_explicit_terms_second_order(0.0)]),
    "side-face transport weights swapped": (
        "substep", "uw = (dzm * u[:-1] + dzp * u[1:]) / den", "uw = (dzp * u[:-1] + dzm * u[1:]) / den",
        [t_cn.test_advection_conserves_energy, lambda: t_cn.test_explicit_terms_second_order(2.0)]),
    "u advection: y flux interpolated from the wrong neighbour": (
        "substep", "fy = (0.5 * (v + _xm(v))) * (0.5 * (u + _ym(u)))", "fy = (0.5 * (v + _xp(v))) * (0.5 * (u + _ym(u)))",
        [t_cn.test_advection_conserves_energy, lambda: t_cn.test_explicit_terms_second_order(0.0)]),
    "temperature advected with the corrected velocity": (
        "substep",
        "    tn = t + cn.solve_face(rt, g, bka)\n    s = alp * dt\n"
        "    un, vn, wn, pn, _ = poisson.project(us, vs, ws, p, g, s=s, c=bnu,\n"
        "                                        differentiable=differentiable)\n",
        "    s = alp * dt\n"
        "    un, vn, wn, pn, _ = poisson.project(us, vs, ws, p, g, s=s, c=bnu,\n"
        "                                        differentiable=differentiable)\n"
        "    ht = _zero_walls(-adv_face(t, un, vn, wn, g) + kappa * (op.dxx(t, g) + op.dyy(t, g)), g)\n"
        "    rt = _zero_walls(comb(ht, hpt, torch.zeros_like(t), kappa * op.dzz_face(t, g)), g)\n"
        "    tn = t + cn.solve_face(rt, g, bka)\n",
        [t_ts.test_step_third_order_in_time]),
    "CFL: y neighbour on the wrong side": (
        "substep", "+ torch.abs(v + _yp(v)) / g.dy", "+ torch.abs(v + _ym(v)) / g.dy",
        [t_cn.test_cfl_brute_force]),
    # Multiple-resolution temperature grid, Sec. 6
    "prolongation: local divergence correction dropped": (
        "multires", "M = -G @ np.linalg.pinv(L) if ncell > 1", "M = 0.0 * G @ np.linalg.pinv(L) if ncell > 1",
        [lambda: t_mr.test_prolonged_velocity_is_divergence_free((2, 2, 2)),
         t_mr.test_uniform_temperature_stays_uniform]),
    "prolongation: transverse slope with the wrong sign": (
        "multires", "uf[k * rz + m, b::ry, ::rx] = u[k] + syu[k] * ey[b]",
        "uf[k * rz + m, b::ry, ::rx] = u[k] - syu[k] * ey[b]",
        [lambda: t_mr.test_prolongation_second_order(0.0, (2, 2, 2))]),
    "prolongation: zero-gradient wall in place of the no-slip value": (
        "multires", "qm = torch.cat([zero, q[:-1]], dim=0)", "qm = torch.cat([q[:1], q[:-1]], dim=0)",
        [lambda: t_mr.test_prolongation_second_order(1.5, (2, 2, 2))]),
    "prolongation: sub-face offsets not centred on the coarse face": (
        "multires", "return torch.tensor([((b + 0.5) / r - 0.5) * h for b in range(r)], dtype=F64)",
        "return torch.tensor([(b / r - 0.5) * h for b in range(r)], dtype=F64)",
        [lambda: t_mr.test_coarse_face_fluxes_are_kept((2, 2, 2)),
         lambda: t_mr.test_prolongation_second_order(0.0, (3, 2, 3))]),
    "restriction: one sub-column instead of the column mean": (
        "multires", "return at_faces.reshape(n, g.ny, ry, g.nx, rx).mean(dim=(2, 4))",
        "return at_faces.reshape(n, g.ny, ry, g.nx, rx)[..., 0].mean(dim=2)",
        [t_mr.test_restriction_keeps_plane_means_and_converges]),
    "temperature step: every stage advected with the end-of-step velocity": (
        "multires", "th = (s + STAGE_START[l - 1]) / nsub", "th = (s + 1.0) / nsub",
        [t_mr.test_temperature_step_third_order_in_substep]),
    "temperature substep: diffusion weighted by gamma instead of alpha": (
        "multires", "rt = gam * h + alp * (kappa * op.dzz_face(t, gf))", "rt = gam * h + gam * (kappa * op.dzz_face(t, gf))",
        [lambda: t_mr.test_temperature_substep_is_the_single_grid_one(2)]),
    # Full step and statistics, Sec. 2.1 and Sec. 5 (Table 3)
    "heat flux: conduction term with the wrong sign": (
        "timestep", "cond = kappa * (tm[1:] - tm[:-1]) / g.dz", "cond = kappa * (tm[:-1] - tm[1:]) / g.dz",
        [t_ts.test_heat_flux_conduction]),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_pins_catch_planted_mistake(case, monkeypatch):
    name, old, new, pins = CASES[case]
    _install(monkeypatch, name, _mutant(name, old, new))
    caught = [_fails(pin) for pin in pins]
    assert any(caught), f"no pin caught: {case}"


def test_pins_pass_on_unmodified_copies(monkeypatch):
    """Control: the same machinery with no change leaves every listed pin passing."""
    for name in sorted({c[0] for c in CASES.values()}):
        _install(monkeypatch, name, _mutant(name, "", ""))
    for case in sorted(CASES):
        for pin in CASES[case][3]:
            assert not _fails(pin), case
