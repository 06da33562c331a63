#!/usr/bin/env python3
"""Benchmark: direct pressure-Poisson solves on the 1024 x 1024 x 512 wall-bounded slab.

One step = one FP64 ``poisson_solve`` (x FFT, y FFT, z solves, inverse y FFT,
inverse x FFT) on the plane-Couette-like slab (Lx = Ly = 4, tanh stretching 3),
right-hand side = divergence of a seeded 64-mode k^-5/3 velocity field with
noise and the Couette base flow.  Inputs are resident in HBM before timing.

Also reported on the same input: the FP32-refined solve (solves/s, iterations,
difference from the FP64 result), per-stage kernel times measured with HIP
events, the roofline position of the dominant kernel, a same-run device copy
rate, full-size parity against the CPU oracle, and the oracle's own rate on the
host (CPU baseline).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HBM_PEAK_GBS = 8000.0
ROOT = os.path.dirname(os.path.abspath(__file__))


def kernel_source_hash():
    """sha256 (first 16 hex) of the HIP sources, in the form the traffic record stores."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1705_01423_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h")):
            h.update(name.encode())
            with open(os.path.join(csrc, name), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(stage):
    """HBM bytes per launch of ``stage`` from the committed counter record, or None when the
    kernels have changed since the counters were taken (hash mismatch) or no record exists."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except OSError:
        return None
    if rec.get("source_hash") != kernel_source_hash():
        return None
    k = rec.get("kernels", {}).get(stage)
    return None if k is None else k["traffic_bytes"]


def cpu_model():
    """The host CPU's model name (lscpu), or None."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
    except (OSError, subprocess.SubprocessError):
        return None
    for line in out.splitlines():
        if line.startswith("Model name:"):
            return line.split(":", 1)[1].strip()
    return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="couette1024x1024x512")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-single-thread", action="store_true", help="skip the single-thread oracle solve")
    ap.add_argument("--no-refined", action="store_true")
    ap.add_argument("--stage-reps", type=int, default=10)
    ap.add_argument("--no-extra", action="store_true", help="skip the projection/adjoint/substep legs")
    ap.add_argument("--only-extra", nargs="?", const="all", default=None,
                    help="run only the other workloads and print their JSON (profiling); optionally a "
                         "comma-separated subset of " + ",".join(EXTRA_LEGS))
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this library runs one box on one GPU; runs on more than one GPU are not supported",
              file=sys.stderr)
        sys.exit(2)
    if args.only_extra:
        legs = EXTRA_LEGS if args.only_extra == "all" else tuple(args.only_extra.split(","))
        bad = [x for x in legs if x not in EXTRA_LEGS]
        if bad:
            ap.error(f"unknown workloads {bad}; choose from {EXTRA_LEGS}")
        print(json.dumps(other_workloads(args, legs)), flush=True)
        return

    import numpy as np
    import torch

    from paper_1705_01423_amd import synth
    from paper_1705_01423_amd.api import Plan

    cfg = synth.CONFIGS[args.config]
    nx, ny, nz = cfg.nx, cfg.ny, cfg.nz
    npts = nx * ny * nz
    zf = synth.zfaces(nz, cfg.alpha)
    log(f"generating inputs {nx}x{ny}x{nz}")
    t0 = time.time()
    u, v, w = synth.mode_velocity(cfg)
    log(f"inputs ready in {time.time() - t0:.1f}s")
    dev = torch.device("cuda")
    # Right-hand side: discrete divergence of the synthetic field (input preparation with
    # plain torch ops, outside the timed region).
    dx, dy = cfg.lx / nx, cfg.ly / ny
    dzt = torch.as_tensor(np.diff(zf)).to(dev)
    ug = torch.as_tensor(u).to(dev)
    f = (torch.roll(ug, -1, 2) - ug) / dx
    del ug
    vg = torch.as_tensor(v).to(dev)
    f += (torch.roll(vg, -1, 1) - vg) / dy
    del vg
    wg = torch.as_tensor(w).to(dev)
    f += (wg[1:] - wg[:-1]) / dzt[:, None, None]
    del wg
    f = f.contiguous()
    torch.cuda.synchronize()

    plan = Plan(nx, ny, nz, cfg.lx, cfg.ly, zf, precision="fp64")
    phi = torch.empty_like(f)
    stream = torch.cuda.current_stream()
    log("fp64 warmup")
    for _ in range(args.warmup):
        plan.solve_nosync(f, phi)
    torch.cuda.synchronize()
    log(f"fp64 timing {args.steps} solves")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.solve_nosync(f, phi)
    torch.cuda.synchronize()
    t_fp64 = (time.perf_counter() - t0) / args.steps
    _, info64 = plan.solve(f, phi)
    torch.cuda.synchronize()

    # per-stage kernel times (HIP events on the launch stream)
    log("stage timing")
    names = ["x_fft_fwd", "y_fft_fwd", "z_solve", "y_fft_inv", "x_fft_inv"]
    stage_ms = {}
    for s, name in enumerate(names):
        ins = f if s == 0 else None
        outs = phi if s == 4 else None
        for _ in range(2):
            plan.debug_stage(s, ins, outs)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.stage_reps):
            plan.debug_stage(s, ins, outs)
        e1.record(stream)
        torch.cuda.synchronize()
        stage_ms[name] = e0.elapsed_time(e1) / args.stage_reps
    # restore phi after the stage runs overwrote the plan buffers
    plan.solve_nosync(f, phi)
    torch.cuda.synchronize()

    # practical ceiling: the library's streaming copy (read + write one field), and torch's copy_
    from paper_1705_01423_amd.api import stream_copy
    tmp = torch.empty_like(f)
    stream_copy(tmp, f)
    copy_ms = _event_ms(lambda: stream_copy(tmp, f), 5)
    copy_gbs = 2 * f.numel() * 8 / (copy_ms * 1e-3) / 1e9
    torch_copy_gbs = 2 * f.numel() * 8 / (_event_ms(lambda: tmp.copy_(f), 5) * 1e-3) / 1e9
    del tmp

    dominant = max(stage_ms, key=stage_ms.get)
    alg_bytes = 16.0 * npts        # one read + one write of the field's spectral/physical data
    achieved = alg_bytes / (stage_ms[dominant] * 1e-3) / 1e9
    stage_frac = {k: {"gbs": round(alg_bytes / (x * 1e-3) / 1e9, 1),
                      "frac_peak": round(alg_bytes / (x * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                      "frac_copy": round(alg_bytes / (x * 1e-3) / 1e9 / copy_gbs, 4)} for k, x in stage_ms.items()}
    roofline = {"bound": "hbm", "kernel": dominant, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": recorded_traffic(dominant),
                "alg_bytes_per_launch": alg_bytes}
    solve_bytes = 80.0 * npts
    total_gbs = solve_bytes / t_fp64 / 1e9

    refined = None
    if not args.no_refined:
        log("fp32-refined timing")
        # refinement target of this workload: rel-L2 <= 1e-11 (the stop rule estimates the error left)
        plan32 = Plan(nx, ny, nz, cfg.lx, cfg.ly, zf, precision="fp32_refined", tol=1e-11)
        phi32 = torch.empty_like(f)
        for _ in range(max(1, args.warmup)):
            plan32.solve(f, phi32)
        torch.cuda.synchronize()
        nref = max(3, args.steps // 2)
        t0 = time.perf_counter()
        for _ in range(nref):
            _, inf32 = plan32.solve(f, phi32)
        torch.cuda.synchronize()
        t_ref = (time.perf_counter() - t0) / nref
        diff = float((phi32 - phi).norm() / phi.norm())
        refined = {"solves_per_s": round(1.0 / t_ref, 3), "ms_per_solve": round(t_ref * 1e3, 3),
                   "gpoints_per_s": round(npts / t_ref / 1e9, 3), "iterations": inf32["iterations"],
                   "rel_update": inf32["rel_update"], "rel_l2_vs_fp64_gpu": diff,
                   "speedup_vs_fp64": round(t_fp64 / t_ref, 3)}
        plan32.close()
        del phi32
        torch.cuda.empty_cache()

    cpu_baseline = None
    parity = None
    if not args.no_cpu_baseline:
        import torch as _t
        from oracle import Grid, operators as op, poisson
        log("oracle (CPU) divergence and solve at full size")
        g = Grid(nx, ny, nz, cfg.lx, cfg.ly, zf)
        fo = op.divergence(_t.as_tensor(u), _t.as_tensor(v), _t.as_tensor(w), g)
        del u, v, w
        # three full-size solves on all host threads (median), then one on a single thread
        times = []
        for _ in range(3):
            t0 = time.perf_counter()
            ref = poisson.solve(fo, g)
            times.append(time.perf_counter() - t0)
        t_cpu = sorted(times)[1]
        nthreads = _t.get_num_threads()
        t_single = None
        if not args.no_single_thread:
            _t.set_num_threads(1)
            t0 = time.perf_counter()
            poisson.solve(fo, g)
            t_single = time.perf_counter() - t0
            _t.set_num_threads(nthreads)
        cpu_baseline = {"value": round(1.0 / t_cpu, 5), "unit": "solves/s", "cores": nthreads,
                        "kind": "oracle", "gpoints_per_s": round(npts / t_cpu / 1e9, 4),
                        "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
                        "single_thread_solves_per_s": None if t_single is None else round(1.0 / t_single, 5),
                        "sample": f"median of 3 full {nx}x{ny}x{nz} FP64 solves of the same input on {nthreads} "
                                  f"threads ({', '.join(f'{x:.2f}' for x in times)} s)"
                                  + ("" if t_single is None else f"; one solve on 1 thread: {t_single:.1f} s")}
        phih = phi.cpu()
        parity = {"fp64_rel_l2_vs_oracle": float((phih - ref).norm() / ref.norm()),
                  "rhs_rel_diff_gpu_vs_oracle": float((f.cpu() - fo).norm() / fo.norm())}
        log(f"parity {parity}")

    del f, phi, plan
    torch.cuda.empty_cache()
    extra = {} if args.no_extra else other_workloads(args)

    out = {
        "metric": "Poisson solves/s at 1024x1024x512 (FP64)",
        "value": round(1.0 / t_fp64, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_fp64 * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"poisson_solve {nx}x{ny}x{nz} Lx={cfg.lx} Ly={cfg.ly} tanh-stretched z "
                               f"(alpha={cfg.alpha}); rhs = divergence of seeded 64-mode k^-5/3 field + "
                               f"N(0,1e-2) + Couette profile", "nx": nx, "ny": ny, "nz": nz},
        "gpoints_per_s": round(npts / t_fp64 / 1e9, 3),
        "model_bytes_per_solve": solve_bytes,
        "model_gbs": round(total_gbs, 1),
        "model_frac_hbm": round(total_gbs / HBM_PEAK_GBS, 4),
        "stages_ms": {k: round(x, 4) for k, x in stage_ms.items()},
        "copy_gbs": round(copy_gbs, 1),
        "torch_copy_gbs": round(torch_copy_gbs, 1),
        "stages_roofline": stage_frac,
        "fp32_refined": refined,
        "roofline": roofline,
        "cpu_baseline": cpu_baseline,
        "parity": parity,
        "compat_defect": info64["compat_defect"],
        "other_workloads": extra,
    }
    print(json.dumps(out), flush=True)


def _event_ms(fn, reps):
    import torch
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        fn()
    e1.record(st)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


EXTRA_LEGS = ("projection", "adjoint", "substep", "step", "multires")


def other_workloads(args, legs=EXTRA_LEGS):
    """Projection (512^2 x 384), adjoint/forward ratio (256^2 x 192), RK3 substep and its
    adjoint (768^2 x 512, FP32-refined and FP64 Poisson), the full RK3 step and its adjoint,
    and the multiple-resolution step, each on its own seeded input."""
    res = {}
    if "projection" in legs:
        res.update(_projection_workload())
    if "adjoint" in legs:
        res.update(_adjoint_workload())
    if "substep" in legs or "step" in legs:
        res.update(_substep_workloads("substep" in legs, "step" in legs))
    if "multires" in legs:
        res.update(multires_workload())
    return res


def _projection_workload():
    import torch

    from paper_1705_01423_amd import synth
    from paper_1705_01423_amd.api import Plan

    res = {}
    # ---- projection + pressure update, 512 x 512 x 384 ----
    cfg = synth.CONFIGS["slab512x512x384"]
    zf = synth.zfaces(cfg.nz, cfg.alpha)
    log("projection 512x512x384")
    u, v, w = (torch.as_tensor(a).to("cuda") for a in synth.mode_velocity(cfg))
    plan = Plan(cfg.nx, cfg.ny, cfg.nz, cfg.lx, cfg.ly, zf, precision="fp64")
    us, vs, ws = u.clone(), v.clone(), w.clone()
    p = torch.zeros_like(u)

    def proj():
        u.copy_(us)
        v.copy_(vs)
        w.copy_(ws)
        plan.project(u, v, w, p, None, 1.0, 0.0, want_info=False)

    proj()
    copy_ms = _event_ms(lambda: (u.copy_(us), v.copy_(vs), w.copy_(ws)), 3)
    t = _event_ms(proj, 5) - copy_ms
    npts = cfg.nx * cfg.ny * cfg.nz
    res["project_512x512x384"] = {"ms": round(t, 3), "gpoints_per_s": round(npts / t / 1e6, 3),
                                  "model_bytes_per_point": 184, "model_gbs": round(184 * npts / t / 1e6, 1)}
    del u, v, w, us, vs, ws, p, plan
    torch.cuda.empty_cache()
    return res


def _adjoint_workload():
    import torch

    from paper_1705_01423_amd import synth
    from paper_1705_01423_amd.api import Plan

    res = {}
    # ---- adjoint / forward cost, 256 x 256 x 192 ----
    cfg = synth.CONFIGS["slab256x256x192"]
    zf = synth.zfaces(cfg.nz, cfg.alpha)
    log("projection adjoint 256x256x192")
    u, v, w = (torch.as_tensor(a).to("cuda") for a in synth.mode_velocity(cfg))
    om = [torch.as_tensor(a).to("cuda") for a in synth.face_weights(cfg)]
    plan = Plan(cfg.nx, cfg.ny, cfg.nz, cfg.lx, cfg.ly, zf, precision="fp64")
    us, vs, ws = u.clone(), v.clone(), w.clone()
    fwd = _event_ms(lambda: plan.project(us, vs, ws, None, None, 1.0, 0.0, want_info=False), 10)
    adj = _event_ms(lambda: plan.project_adjoint(om[0], om[1], om[2], None, 1.0, 0.0), 10)
    res["adjoint_256x256x192"] = {"forward_ms": round(fwd, 3), "adjoint_ms": round(adj, 3),
                                  "adjoint_over_forward": round(adj / fwd, 3)}
    del u, v, w, us, vs, ws, om, plan
    torch.cuda.empty_cache()
    return res


def _substep_workloads(substeps=True, steps=True):
    import math
    import torch

    from paper_1705_01423_amd import synth
    from paper_1705_01423_amd.api import Plan

    res = {}
    # ---- RK3 substep and its adjoint, 768 x 768 x 512, Ra = 1e8, Pr = 1 ----
    cfg = synth.CONFIGS["rb768x768x512"]
    zf = synth.zfaces(cfg.nz, cfg.alpha)
    log("rk3 substep 768x768x512")
    ra, pr = cfg.extra["ra"], cfg.extra["pr"]
    nu, ka = math.sqrt(pr / ra), 1.0 / math.sqrt(ra * pr)
    saved = [torch.as_tensor(a).to("cuda") for a in synth.rb_state(cfg)]
    st = [a.clone() for a in saved]
    plan = Plan(cfg.nx, cfg.ny, cfg.nz, cfg.lx, cfg.ly, zf, precision="fp32_refined")
    dt = 1.3 / float(plan.cfl(saved[0], saved[1], saved[2]).item())   # CFL 1.3 (Listing 1 number)

    def reset():
        for a, b in zip(st, saved):
            a.copy_(b)

    infos = []

    def step():
        reset()
        infos.append(plan.substep(1, dt, nu, ka, *st))

    reset_ms = _event_ms(reset, 3)
    cot = [torch.randn_like(a) for a in saved]
    for c in (cot[2], cot[3]):
        c[0] = 0
        c[-1] = 0
    npts = cfg.nx * cfg.ny * cfg.nz
    if substeps:
        step()
        fwd = _event_ms(step, 3) - reset_ms
        plan.substep_adjoint(dt, nu, ka, *saved, cot)
        adj = _event_ms(lambda: plan.substep_adjoint(dt, nu, ka, *saved, cot), 3)
        res["rk3_substep_768x768x512"] = {"dt": dt, "forward_ms": round(fwd, 3), "adjoint_ms": round(adj, 3),
                                          "adjoint_over_forward": round(adj / fwd, 3),
                                          "poisson_iterations": infos[-1]["iterations"],
                                          "gpoints_per_s": round(npts / fwd / 1e6, 3)}
    plan.close()
    # the same substep with the FP64 solve (one pass instead of three FP32 ones)
    plan = Plan(cfg.nx, cfg.ny, cfg.nz, cfg.lx, cfg.ly, zf, precision="fp64")
    if substeps:
        step()
        fwd64 = _event_ms(step, 3) - reset_ms
        plan.substep_adjoint(dt, nu, ka, *saved, cot)
        adj64 = _event_ms(lambda: plan.substep_adjoint(dt, nu, ka, *saved, cot), 3)
        res["rk3_substep_768x768x512_fp64_poisson"] = {"forward_ms": round(fwd64, 3), "adjoint_ms": round(adj64, 3),
                                                       "gpoints_per_s": round(npts / fwd64 / 1e6, 3)}
    if steps:
        # one full RK3 step (three substeps, Courant-limited dt) and the heat-flux statistics
        used = []

        def full_step():
            reset()
            used.append(plan.step(nu, ka, *st, dt=0.0, cfl=1.3)[0])

        full_step()
        step_ms = _event_ms(full_step, 3) - reset_ms
        hf_ms = _event_ms(lambda: plan.heat_flux(st[2], st[3], ka), 5)
        mean_t, flux = plan.heat_flux(st[2], st[3], ka)
        nu_prof = (flux / ka).cpu()
        # the whole step's adjoint (fixed dt: the intermediate states recomputed, three substep adjoints)
        plan.step_adjoint(used[-1], nu, ka, *saved, cot)
        sadj_ms = _event_ms(lambda: plan.step_adjoint(used[-1], nu, ka, *saved, cot), 3)
        res["rk3_step_768x768x512_fp64_poisson"] = {
            "ms": round(step_ms, 3), "dt": used[-1], "adjoint_ms": round(sadj_ms, 3),
            "adjoint_over_forward": round(sadj_ms / step_ms, 3), "heat_flux_ms": round(hf_ms, 3),
            "nusselt_wall_mean": round(float(0.5 * (nu_prof[0] + nu_prof[-1])), 6)}
    plan.close()
    del st, saved, cot
    torch.cuda.empty_cache()
    return res


def multires_workload(nsub=2):
    """One coupled step with the momentum on the 384^2 x 256 grid and the temperature on a grid
    refined twice in every direction (768^2 x 512 points), nsub temperature steps per step."""
    import math

    import numpy as np
    import torch

    from paper_1705_01423_amd import synth
    from paper_1705_01423_amd.api import MultiRes, Plan

    cfg = synth.CONFIGS["rb384x384x256"]
    log("multiple-resolution step 384x384x256 / 768x768x512")
    zf = synth.zfaces(cfg.nz, cfg.alpha)
    ra, pr = cfg.extra["ra"], cfg.extra["pr"]
    nu, ka = math.sqrt(pr / ra), 1.0 / math.sqrt(ra * pr)
    u, v, w, _, p = (torch.as_tensor(a).to("cuda") for a in synth.rb_state(cfg))
    plan = Plan(cfg.nx, cfg.ny, cfg.nz, cfg.lx, cfg.ly, zf, precision="fp64")
    m = MultiRes(plan, 2, 2, 2, nsub=nsub)
    zff = np.concatenate([[zf[k] + (q / 2) * (zf[k + 1] - zf[k]) for k in range(cfg.nz) for q in range(2)], [zf[-1]]])
    tf = torch.as_tensor(synth.rb_temperature(cfg, zff, m.nxf, m.nyf)).to("cuda")
    saved = [a.clone() for a in (u, v, w, p, tf)]
    st = [a.clone() for a in saved]
    dt = 1.3 / float(plan.cfl(u, v, w).item())

    def reset():
        for a, b in zip(st, saved):
            a.copy_(b)

    def step():
        reset()
        m.step(nu, ka, *st, dt=dt)

    step()
    reset_ms = _event_ms(reset, 3)
    step_ms = _event_ms(step, 3) - reset_ms
    vel = m.prolong_velocity(*saved[:3])
    prol_ms = _event_ms(lambda: m.prolong_velocity(*saved[:3], out=vel), 5)
    tt = saved[4].clone()
    t_ms = _event_ms(lambda: m.temperature_step(dt, ka, vel, vel, tt), 3)
    nf = m.nxf * m.nyf * m.nzf
    out = {"rk3_step_mr_384x384x256_T768x768x512": {
        "ms": round(step_ms, 3), "dt": dt, "nsub": nsub, "prolongation_ms": round(prol_ms, 3),
        "prolongation_gbs": round(27.0 * nf / (prol_ms * 1e-3) / 1e9, 1),
        "temperature_step_ms": round(t_ms, 3)}}
    m.close()
    plan.close()
    torch.cuda.empty_cache()
    return out


if __name__ == "__main__":
    main()
