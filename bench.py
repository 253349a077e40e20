#!/usr/bin/env python3
"""Benchmark of the finite-T orbital-free DFT hot path on one MI355X.

Headline: F[n] + gradient evaluations per second at 128^3 (1024 H atoms,
4.0 g/cm^3, T = 100 kK, VT84F + PZ81, mixed precision: FP32 FFTs and gradient
terms, FP64 Fermi-Dirac inversion and sums).  One step = one evaluation of
every stage of the evaluation path on the cell (density, forward FFT, Hartree
and pseudopotential in reciprocal space, gradient, pointwise free energy and
XC, divergence term, potential, Euler multiplier and energy reductions),
launched back to back on the library's stream.

Also reported: the same rate in FP64, per-kernel HIP-event durations with the
roofline of the dominant kernel, milliseconds per converged MD step (128 H,
1.0 g/cm^3, 64^3, 50 kK, VT84F, warm-started velocity Verlet) in mixed and FP64
precision with the stress tensor timed at the last step, one density optimisation
of the static fcc-Al workload (2048 ions on 128^3 and 16384 ions on 256^3, 100 K,
Heine-Abarenkov Al pseudopotential) in mixed and FP64 with its forces and pressure, and the FP64
CPU oracle timed on the host as a baseline.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--md-steps M] [--no-md] [--no-al] [--no-cpu]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Vector ALU peak for the pointwise kernel: 256 CUs x 4 SIMDs x 16 lanes x 2 flop (FMA) x 2.4 GHz.
# FP64 runs at this rate; FP32 without packed math (not used here) runs at the same lane rate.
VALU_PEAK_TFLOPS = 78.6
# Algorithmic flops per grid point of the pointwise GGA kernel (VT84F + PZ81), counting an FMA
# as 2 and every add, multiply, reciprocal, square root, exp or log as 1, with one pass over
# the t-factor tables: FP64 239 (ln n and l: 3; piece abscissa: 2; Chebyshev recurrence
# T_2..T_13: 24; 8 series of 14 terms: 208; energy sums: 2) + FP32 151 (density powers and
# s^2: 16; two VT84F enhancement factors: 64; f, df/dn, df/dsigma, T s: 37; PZ81: 24; W and
# v_loc: 5; sums: 5).
POINTWISE_GGA_FLOP_PER_POINT = 390
WORKLOAD = "1024 H, 4.0 g/cm^3, 128^3 grid, T=100 kK, VT84F+PZ81 ftGGA, Gaussian LPP rc=0.5"


def log(msg: str):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def host_threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def kernel_bytes(name: str, n1: int, n2: int, n3: int, rsize: int) -> float:
    """Algorithmic HBM bytes of one launch: compulsory reads + writes of whole arrays."""
    N = n1 * n2 * n3
    CS = (n3 // 2 + 1) * n1 * n2 * 2 * rsize      # one half-spectrum array (complex R)
    RR = N * rsize                               # one real R array
    P = N * 8                                    # phi (FP64)
    table = {
        "rpass_fwd_density": P + CS,
        "cpass_x2_fwd": 2 * CS,
        "x1_density_gradient": 6 * CS,
        "x1_density_hartree": 3 * CS,
        "cpass_x2_inv3": 6 * CS,
        "rpass_inv_grad3": 3 * CS + 3 * RR,
        "pointwise_gga": P + 7 * RR,
        "rpass_fwd_w3": 3 * CS + 3 * RR,
        "cpass_x2_fwd3": 6 * CS,
        "x1_divergence": 5 * CS,
        "cpass_x2_inv": 2 * CS,
        "rpass_final": CS + P + 2 * RR,
        "rpass_tf_final": CS + P + RR,
        "plane_fwd_density": P + CS,
        "plane_inv_grad3": 3 * CS + 3 * RR,
        "plane_fwd_w3": 3 * CS + 3 * RR,
        "plane_final": CS + P + 2 * RR,
        "plane_tf_final": CS + P + RR,
        "reduce_scalars": 0,
    }
    return float(table.get(name, 0))


def source_digest() -> str:
    """SHA-256 over the HIP sources; a counter record applies only to the kernels it measured."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1406_0835_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE, each scaled by the same counter on a copy kernel of known size),
    or None when there is none or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_128cubed_counters.md")
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as f:
        for line in f:
            if line.startswith("- ") and ":" in line:
                k, v = line[2:].split(":", 1)
                rec[k.strip()] = v.strip().strip("`")
    if rec.get("source_sha256") != source_digest():
        return None
    try:
        return float(rec["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def sync():
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.synchronize()
    except Exception:
        pass


def make_context(P, cell, functional, precision, **kw):
    ctx = P.Context(functional=functional, precision=precision, **kw)
    ctx.set_cell(cell.lattice, cell.grid)
    ctx.set_ions(cell.positions, cell.charges)
    ctx.set_temperature(cell.temperature_K)
    return ctx


def eval_rate(ctx, steps, warmup):
    ctx.time_evals(max(warmup, 1), 0)
    sync()
    t0 = time.perf_counter()
    dev_ms, _ = ctx.time_evals(steps, 0)
    sync()
    t1 = time.perf_counter()
    return steps / (t1 - t0), 1e3 * (t1 - t0) / steps, dev_ms / steps


def host_api_rate(ctx, steps):
    """Evaluations per second through the C ABI's ofdft_eval, which returns its report (and
    optionally the FP64 potential, N doubles over PCIe) in host memory."""
    out = {}
    for name, pot in (("report_only", False), ("with_potential", True)):
        ctx.eval(potential=pot)
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.eval(potential=pot)
        out[name] = steps / (time.perf_counter() - t0)
    return out


def md_run(P, wl, precision, n_steps):
    from paper_1406_0835_amd import md
    cell = wl.md_cell()
    ctx = make_context(P, cell, "VT84F", precision, tol_energy=1e-8, max_iter=400)
    masses = [md.H_MASS_ME] * cell.nat
    v0 = md.maxwell_boltzmann(cell.nat, cell.temperature_K, md.H_MASS_ME, seed=wl.SEED_BASE + 4)
    dt = 0.2 * md.FS_AU
    recs = md.velocity_verlet(ctx, cell.positions, v0, cell.charges, masses, dt, n_steps)
    steps = recs[1:]
    e = [r.F_total + r.kinetic for r in recs]
    # stress tensor at the last converged density (ofdft_stress), timed
    ctx.stress()
    t0 = time.perf_counter()
    for _ in range(5):
        sig = ctx.stress()
    stress_ms = (time.perf_counter() - t0) / 5 * 1e3
    ctx.close()
    return {
        "stress_ms": stress_ms,
        "pressure_Ha_per_bohr3": -float(sig[0][0] + sig[1][1] + sig[2][2]) / 3.0,
        "ms_per_step": sum(r.wall_ms for r in steps) / len(steps),
        "evals_per_step": sum(r.evaluations for r in steps) / len(steps),
        "first_minimization_ms": recs[0].wall_ms,
        "E_cons_span_Ha": max(e) - min(e),
        "steps": n_steps,
    }


def al_static(P, wl, precision, n_rep=8):
    """The static fcc-Al workload: n_rep^3 conventional cells (2048 ions on 128^3 for n_rep = 8,
    16384 ions on 256^3 for 16; 16 grid points per cell edge), 2.70 g/cm^3, 100 K, VT84F + PZ81,
    Heine-Abarenkov Al pseudopotential; one density optimisation from the uniform density,
    then forces and stress.  setup_ms covers set_ions (the structure factor on the device; the
    Ewald sum starts on a host thread and overlaps the optimisation)."""
    cell = wl.fcc_al_cell(n_rep, 16 * n_rep)
    lpp = wl.AL_HA_LPP
    ctx = P.Context(functional="VT84F", precision=precision, xc="pz81", tol_energy=1e-9 * cell.nat,
                    max_iter=2000, lpp="ha", lpp_rc=lpp["rc"], lpp_A=lpp["A"], lpp_qc=lpp["qc"])
    ctx.set_cell(cell.lattice, cell.grid)
    ctx.set_temperature(cell.temperature_K)
    sync()
    t0 = time.perf_counter()
    ctx.set_ions(cell.positions, cell.charges)
    sync()
    t_set = time.perf_counter() - t0
    t0 = time.perf_counter()
    rep = ctx.minimize_density()
    sync()
    t_min = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, _, f = ctx.free_energy_and_forces(forces=True)
    P_el = ctx.pressure()
    t_fs = time.perf_counter() - t0
    ctx.close()
    return {"atoms": cell.nat, "grid": list(cell.grid), "precision": precision,
            "minimize_ms": 1e3 * t_min, "iterations": rep.iterations, "evaluations": rep.evaluations,
            "F_per_atom_Ha": rep.F_total / cell.nat, "max_force_Ha_bohr": float(abs(f).max()),
            "pressure_Ha_per_bohr3": P_el, "forces_and_stress_ms": 1e3 * t_fs, "setup_ms": 1e3 * t_set}


def batch_run(P, wl, n_cells, precision):
    """Heterogeneous batch: all cells minimised concurrently vs one after another."""
    import numpy as np
    cells = wl.batch_cells(n_cells)
    def build():
        out = []
        for c in cells:
            out.append(make_context(P, c, "VT84F", precision, tol_energy=1e-8, max_iter=2000))
        return out
    seq = build()
    sync()
    t0 = time.perf_counter()
    seq_reps = [c.minimize_density() for c in seq]
    sync()
    t_seq = time.perf_counter() - t0
    bat = build()
    sync()
    t0 = time.perf_counter()
    bat_reps = P.batch_minimize(bat)
    sync()
    t_bat = time.perf_counter() - t0
    pts = sum(int(np.prod(c.grid)) for c in cells)
    evals = sum(r.evaluations for r in bat_reps)
    pt_evals = sum(int(np.prod(c.grid)) * r.evaluations for c, r in zip(cells, bat_reps))
    dF = max(abs(a.F_total - b.F_total) / abs(b.F_total) for a, b in zip(bat_reps, seq_reps))
    for c in seq + bat:
        c.close()
    return {"cells": n_cells, "precision": precision, "batched_s": t_bat, "sequential_s": t_seq,
            "speedup": t_seq / t_bat, "grid_points": pts, "evaluations": evals,
            "grid_points_per_s": pt_evals / t_bat, "max_rel_dF_batch_vs_sequential": dF,
            "all_converged": all(r.converged for r in bat_reps)}


def md_long(P, wl, n_steps):
    """NVE drift (Ha/atom/ps) of the mixed and FP64 paths, and mixed-vs-FP64 forces."""
    import numpy as np
    from paper_1406_0835_amd import md
    out = {}
    cell = wl.md_cell()
    check = make_context(P, cell, "VT84F", "fp64", tol_energy=1e-10, max_iter=2000)
    for precision in ("mixed", "fp64"):
        ctx = make_context(P, cell, "VT84F", precision, tol_energy=1e-8, max_iter=400)
        masses = [md.H_MASS_ME] * cell.nat
        v0 = md.maxwell_boltzmann(cell.nat, cell.temperature_K, md.H_MASS_ME, seed=wl.SEED_BASE + 4)
        dt = 0.2 * md.FS_AU
        ferr = {}

        def cb(rec, x, v, f):
            if precision == "mixed" and rec.step in (n_steps // 2, n_steps):
                _, f64, _ = md.step_forces(check, x, cell.charges)
                ferr[rec.step] = float(np.max(np.abs(f - f64)))
            if rec.step % 20 == 0:
                log(f"MD {precision} step {rec.step}")
        recs = md.velocity_verlet(ctx, cell.positions, v0, cell.charges, masses, dt, n_steps, callback=cb)
        if precision == "mixed":
            ctx.set_ions(cell.positions, cell.charges)
            ctx.minimize_density()
            _, _, f0 = ctx.free_energy_and_forces(forces=True)
            _, f64, _ = md.step_forces(check, cell.positions, cell.charges)
            ferr[0] = float(np.max(np.abs(f0 - f64)))
        e = np.array([r.F_total + r.kinetic for r in recs])
        tps = np.arange(len(recs)) * dt / md.FS_AU * 1e-3       # ps
        slope = float(np.polyfit(tps, e, 1)[0]) / cell.nat
        out[precision] = {"steps": n_steps, "ms_per_step": float(np.mean([r.wall_ms for r in recs[1:]])),
                          "drift_Ha_per_atom_per_ps": slope, "E_cons_std_Ha": float(np.std(e)),
                          "evals_per_step": float(np.mean([r.evaluations for r in recs[1:]]))}
        if ferr:
            out[precision]["max_force_diff_vs_fp64_Ha_bohr"] = ferr
        ctx.close()
    check.close()
    return out


def cpu_baseline(wl, cell, phi):
    os.environ.setdefault("OFDFT_ORACLE_THREADS", str(host_threads()))
    import numpy as np
    import oracle
    sysm = oracle.System(cell.lattice, cell.grid, cell.positions[:1], cell.charges[:1] * cell.nat,
                         cell.temperature_K, functional="VT84F", with_ions=False)
    sysm.vext_hat = np.zeros(sysm.grid.shape, dtype=complex)
    t0 = time.perf_counter()
    oracle.evaluate(phi, sysm)
    dt = time.perf_counter() - t0
    from oracle import fermi_dirac
    return {"value": 1.0 / dt, "unit": "evals/s", "cores": fermi_dirac._THREADS, "kind": "oracle",
            "sample": "one FP64 oracle F+gradient evaluation of the 128^3 VT84F+PZ81 cell at the benchmark "
                      "phi (numpy/scipy, threaded Fermi-Dirac quadrature); the ionic setup (structure factor, "
                      "Ewald) is outside the timed region",
            "seconds": dt}


def copy_probe(mib: float):
    """A plain device-to-device copy kernel of known size (FETCH_SIZE/WRITE_SIZE calibration)."""
    import torch
    n = int(mib * 1024 * 1024 / 4)
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_MiB": mib, "bytes_read_per_copy": 4 * n, "bytes_written_per_copy": 4 * n}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--md-steps", type=int, default=4)
    ap.add_argument("--no-md", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-al", action="store_true", help="skip the static fcc-Al line (--no-md skips it too)")
    ap.add_argument("--kernel-steps", type=int, default=50)
    ap.add_argument("--no-tune", action="store_true", help="keep the default FFT tiles")
    ap.add_argument("--batch", type=int, default=0, help="also run the heterogeneous batch of this many cells")
    ap.add_argument("--md-long", type=int, default=0, help="also run an NVE trajectory of this many steps")
    ap.add_argument("--copy-probe", type=float, default=0.0,
                    help="only run a plain device copy of this many MiB (counter calibration) and exit")
    args = ap.parse_args()
    if args.copy_probe > 0:
        copy_probe(args.copy_probe)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(sharding is described in DESIGN.md); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import paper_1406_0835_amd as P
    import workloads as wl

    cell = wl.gga_128_cell(1.0e5)
    n1, n2, n3 = cell.grid
    nbar = cell.nat / abs(np.linalg.det(cell.lattice))
    phi = wl.trial_phi(cell.grid, nbar, seed=wl.SEED_BASE + 2, contrast=0.6)

    log("setting up the 128^3 cell (structure factor, Ewald)")
    ctx = make_context(P, cell, "VT84F", "mixed")
    ctx.set_density(phi)
    tiles = None
    if not args.no_tune:
        tiles = ctx.autotune(5)
        log(f"autotuned tiles (tr, tc, rb) = {tiles}")
    log(f"timing {args.steps} mixed-precision evaluations")
    value, ms_per_step, dev_ms = eval_rate(ctx, args.steps, args.warmup)
    log(f"{value:.1f} evals/s; per-kernel events over {args.kernel_steps} evaluations")
    _, kern = ctx.time_evals(args.kernel_steps, 16)
    host_api = host_api_rate(ctx, max(10, args.steps // 10))
    ctx.close()

    per_kernel = []
    for name, ms in kern:
        b = kernel_bytes(name, n1, n2, n3, 4)
        per_kernel.append({"kernel": name, "avg_us": 1e3 * ms, "alg_bytes": b,
                           "GB_s": (b / (ms * 1e-3) / 1e9) if ms > 0 and b > 0 else None})
    dom = max(per_kernel, key=lambda k: k["avg_us"])
    traffic = measured_traffic(dom["kernel"])
    if dom["kernel"] == "pointwise_gga":
        flops = POINTWISE_GGA_FLOP_PER_POINT * n1 * n2 * n3
        achieved = flops / (dom["avg_us"] * 1e-6) / 1e12
        roofline = {"bound": "alu", "kernel": dom["kernel"], "achieved": achieved, "peak": VALU_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": achieved / VALU_PEAK_TFLOPS, "traffic": traffic,
                    "alg_flop_per_launch": float(flops), "alg_bytes_per_launch": dom["alg_bytes"],
                    "hbm_GB_s": dom["GB_s"], "avg_launch_us": dom["avg_us"]}
    else:
        achieved = dom["GB_s"] or 0.0
        roofline = {"bound": "hbm", "kernel": dom["kernel"], "achieved": achieved, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                    "alg_bytes_per_launch": dom["alg_bytes"], "avg_launch_us": dom["avg_us"]}
    total_alg = sum(k["alg_bytes"] for k in per_kernel)
    eval_gbs = total_alg / (dev_ms * 1e-3) / 1e9

    fp64 = None
    if not args.no_fp64:
        log("FP64 evaluation rate")
        c64 = make_context(P, cell, "VT84F", "fp64")
        c64.set_density(phi)
        tiles64 = c64.autotune(3) if not args.no_tune else None
        v64, ms64, _ = eval_rate(c64, max(20, args.steps // 4), max(2, args.warmup // 2))
        c64.close()
        fp64 = {"evals_per_s": v64, "ms_per_eval": ms64, "tiles": tiles64}

    md_res = None
    if not args.no_md and args.md_steps > 0:
        log(f"MD: {args.md_steps} steps mixed and FP64")
        md_res = {"mixed": md_run(P, wl, "mixed", args.md_steps), "fp64": md_run(P, wl, "fp64", args.md_steps),
                  "workload": "128 H, 1.0 g/cm^3, 64^3 grid, T=50 kK, VT84F+PZ81, CG to 1e-8 Ha, dt=0.2 fs"}

    al = None
    if not args.no_al and not args.no_md:
        log("static fcc-Al: 2048 ions, 128^3, mixed and FP64")
        al = {"mixed": al_static(P, wl, "mixed"), "fp64": al_static(P, wl, "fp64")}
        log("static fcc-Al: 16384 ions, 256^3, mixed and FP64")
        al["16384"] = {"mixed": al_static(P, wl, "mixed", 16), "fp64": al_static(P, wl, "fp64", 16)}

    batch = None
    if args.batch > 0:
        log(f"batch of {args.batch} cells")
        batch = batch_run(P, wl, args.batch, "mixed")

    mdl = None
    if args.md_long > 0:
        mdl = md_long(P, wl, args.md_long)

    cpu = None
    if not args.no_cpu:
        log("CPU oracle baseline (one 128^3 evaluation)")
        cpu = cpu_baseline(wl, cell, phi)

    out = {
        "metric": "F[n]+gradient evals/s at 128^3",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "grid_points": n1 * n2 * n3, "precision": "mixed",
                   "step": "one F+gradient evaluation", "fft_tiles_tr_tc_rb": tiles},
        "grid_points_per_s": value * n1 * n2 * n3,
        "device_ms_per_eval": dev_ms,
        "eval_alg_GB_s": eval_gbs,
        "host_api_evals_per_s": host_api,
        "roofline": roofline,
        "kernels": per_kernel,
        "fp64": fp64,
        "md_step": md_res,
        "al_static": al,
        "batch": batch,
        "md_trajectory": mdl,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
