#!/usr/bin/env python3
"""Benchmark of the SPME stochastic-Lanczos MBD hot path on one MI355X.

One step = one full E_MBD evaluation of the 24,000-atom water box (8000 rigid
molecules at 1 g/cm^3, 62.09 A cube): device setup at the step's positions,
128 Rademacher probes as one block of right-hand sides, 50 Lanczos steps
(6400 probe-vector matvecs through the pair kernel and SPME on a 96^3 grid,
order-6 B-splines, 9 A real-space cutoff), the tridiagonal quadrature and the
energy sum. SPME and the pair kernel run in float32, the Lanczos recurrence,
quadrature and energy in float64 ("mixed"). The plan's launch shape is measured
on the box at plan creation (outside the timed region) and replayed from a HIP graph.

Prints one JSON line on stdout; progress goes to stderr.
  value   probe-vector SPME matvecs per second (batched, mixed precision)
  extra   E_MBD + forces wall time at the same box (median of graph replays), the
          plain one-vector float64 rate on the same GPU and the speedup, per-stage
          times, the dominant kernel's roofline, errors against stored oracle values,
          the CPU oracle rate (all threads and one thread, CPU model), and the
          E + F legs of the 12k-atom organic box and of the batch of 32 water boxes.
"""
import argparse
import json
import math
import os
import statistics
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E
FP32_PEAK_TFLOPS = 157.3         # MI355X published FP32 peak (packed FMA and matrix cores)
FP32_NONPACKED_TFLOPS = 78.6     # 256 CU x 64 FMA lanes x 2 flop x 2.4 GHz, no packed FP32
GOLDEN = os.path.join(ROOT, "tests", "golden")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Kernel instance behind each grid stage at the 24k workload (float, p = 6, 64-wide
# chunks); the pair stage's instance depends on the shape (pair_kernel_name).
STAGE_KERNEL = {
    "spread": "k_spread<float, 6, 64>",
    "fft_x": "k_fft_x_real<96, true>", "fft_y": "k_fft_reg<96, 1>",
    "fft_z_conv": "k_fft_reg<96, 2>", "ifft_y": "k_fft_reg<96, 3>",
    "ifft_x": "k_fft_x_real<96, false>", "gather": "k_gather_epilogue<float, 6, 64>",
}


def pair_kernel_name(shape, B, n_atoms):
    """Instance of the direct-space list kernel that a float plan with this shape launches
    for B right-hand sides (the launcher's rules in pair.hip)."""
    ngroups = (n_atoms + 15) // 16
    ns_given = shape.get("pair_subsets", 0)
    mode = shape.get("pair_mode", 0)
    if mode in (1, 2) and B % 64 == 0 and B <= 256:
        wide = 128 if (mode == 1 and B % 128 == 0) else 64
        nn, nk = B // wide, ns_given or 1
        while nk > 1 and nn * nk > 4:
            nk //= 2
        nt = 8 if wide == 128 else 4
        nn_t = 2 if (nk == 2 and nn == 2) else 1
        return f"k_pair_mfma<{nk}, {nt}, {nn_t}>"
    ns = 1 if B >= 64 else 64 // B
    if ns_given > 0:
        ns = max(ns, min(4, ns_given))
    else:
        while ns < 4 and ngroups * B * ns / 64 < 4096:
            ns *= 2
    return f"k_pair_list<float, {ns}, {B * ns // 64}>"


def measured_traffic(kernel):
    """HBM-side bytes per launch (scaled FETCH_SIZE + WRITE_SIZE) recorded in
    profiles/traffic_water24k.md, or None when absent or when the kernel's source file
    has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_water24k.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        f = [x.strip() for x in line.split("|")]
        if len(f) == 7 and f[0] == kernel:
            src = os.path.join(ROOT, f[1])
            if not os.path.exists(src):
                return None
            sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
            return float(f[5]) + float(f[6]) if sha == f[2] else None
    return None


def stage_bytes(stage, K, N, B):
    """Algorithmic HBM bytes of one launch of a grid stage (B right-hand sides, float32)."""
    K1, K2, K3 = K
    real = 4.0 * K1 * K2 * K3
    cplx = 8.0 * K2 * K3 * (K1 // 2 + 1)
    per = {
        "spread": real + 12.0 * N,                  # write the real grid, read the dipoles
        "fft_x": real + cplx,                       # read real lines, write half spectrum
        "fft_y": 2 * cplx,
        "fft_z_conv": 2 * cplx,
        "ifft_y": 2 * cplx,
        "ifft_x": cplx + real,
        "gather": real + 12.0 * N + 48.0 * N,       # read phi, E_dir, w; write l
    }.get(stage)
    return None if per is None else per * B


def golden(name):
    path = os.path.join(GOLDEN, name + ".npz")
    return np.load(path) if os.path.exists(path) else None


def quadrature_error(plan, gold, sys=0, prefix=""):
    """Largest relative error of the plan's per-probe quadrature values against stored
    oracle values (the probes the golden file lists)."""
    if gold is None:
        return None
    q = plan.quadrature(sys).numpy()
    probes = [int(x) for x in gold[prefix + "probes"]]
    ref = gold[prefix + "q"]
    return float(np.max(np.abs(q[probes] - ref) / np.abs(ref)))


def median_ms(fn, reps, torch):
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        ts.append(1000.0 * (time.perf_counter() - t0))
    return statistics.median(ts), out


TUNE_CACHE = None  # --tune-cache: JSON-lines file of measured shapes (read and appended)


def plan_for(P, synth, wl, forces, graph, tune, precision=None, shape=None, systems=None):
    A = synth.ANGSTROM_BOHR
    systems = systems or wl.systems
    ds = [P.DeviceSystem(x.pos, x.cell, x.alpha, x.omega, x.rvdw) for x in systems]
    grid = tuple(wl.grid) * 3 if wl.grid else (0, 0, 0)
    prm = P.Params(real_cutoff=wl.real_cutoff_angstrom * A, grid=grid, n_probes=wl.n_probes,
                   n_steps=wl.n_steps, block=wl.block,
                   precision=P.PREC_MIXED if precision is None else precision,
                   seed=wl.probe_seed, want_forces=forces, store_grids=forces, graph=graph,
                   tune=(P.TUNE_GIVEN if shape else (P.TUNE_MEASURE if tune else P.TUNE_OFF)),
                   shape=shape, tune_cache=TUNE_CACHE if tune else None)
    return ds, P.Plan(ds, prm)


def shape_of(P, plan, sys=0):
    inf = plan.info(sys)
    d = {k: int(getattr(inf.shape, k)) for k, _ in P.MbdShape._fields_}
    d["source"] = P.SHAPE_SOURCES[inf.shape_source]
    return d


def energy_forces_leg(P, torch, synth, name, graph, reps, fp64_check=False, golden_name=None):
    """E_MBD + forces wall time (set_positions + execute with forces) for one workload:
    median of `reps` runs after a warm-up, next to the energy-only median of the same
    plan; errors of the per-probe quadrature against stored oracle values; optionally
    the largest force difference against the float64 GPU path."""
    wl = synth.workload(name)
    t0 = time.perf_counter()
    ds, plan = plan_for(P, synth, wl, forces=True, graph=graph, tune=True)
    t_plan = time.perf_counter() - t0
    pos = [d.pos.clone() for d in ds]

    def run(forces):
        for k, p in enumerate(pos):
            plan.set_positions(p, k)
        return plan.execute(forces=forces, energy_sd=True)

    run(True)
    run(False)
    torch.cuda.synchronize()
    plan.check()
    t_ef, (e, f, sd) = median_ms(lambda: run(True), reps, torch)
    t_e, _ = median_ms(lambda: run(False), reps, torch)
    plan.check()
    out = {"workload": name, "systems": len(wl.systems), "atoms": sum(x.n for x in wl.systems),
           "probes": wl.n_probes, "lanczos_steps": wl.n_steps, "block": wl.block,
           "execution": "hip_graph_replay" if graph else "eager", "replays": reps,
           "energy_forces_ms": round(t_ef, 2), "energy_only_ms": round(t_e, 2),
           "plan_create_s": round(t_plan, 2), "forces_finite": bool(torch.isfinite(f).all()),
           "shape": shape_of(P, plan), "store_grids": True,
           "workspace_gib": round(sum(plan.info(k).workspace_bytes
                                      for k in range(len(wl.systems))) / 2**30, 2)}
    if len(wl.systems) == 1:
        out["energy_ha"] = float(e[0])
        out["energy_sd_ha"] = float(sd[0])
    gold = golden(golden_name) if golden_name else None
    if gold is not None:
        if "probes" in gold:
            out["quadrature_rel_err_vs_oracle"] = quadrature_error(plan, gold)
        else:
            errs = [quadrature_error(plan, gold, int(gold[t + "_system"]), t + "_")
                    for t in ("smallest", "median", "largest")]
            out["quadrature_rel_err_vs_oracle"] = max(errs)
        out["oracle_reference"] = f"tests/golden/{golden_name}.npz"
    if fp64_check:
        _, p64 = plan_for(P, synth, wl, forces=True, graph=False, tune=False,
                          precision=P.PREC_FP64)
        for k, p in enumerate(pos):
            p64.set_positions(p, k)
        e64, f64 = p64.execute(forces=True)
        p64.check()
        out["forces_max_err_vs_fp64_gpu"] = float((f - f64).abs().max() / f64.abs().max())
        out["energy_rel_err_vs_fp64_gpu"] = float((e - e64).abs().max() / e64.abs().max())
        p64.close()
    # per-stage times from one more eager, event-timed run
    plan.stage_times()
    plan.set_timing(True)
    run(True)
    plan.set_timing(False)
    out["stage_ms"] = {k: round(v[0], 2) for k, v in plan.stage_times().items() if v[1] > 0}
    plan.close()
    log(f"{name}: E+F {t_ef:.1f} ms, E only {t_e:.1f} ms (median of {reps}, "
        f"{'graph' if graph else 'eager'})")
    return out


def cpu_info():
    model, cores = None, os.cpu_count()
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in txt.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except Exception:
        pass
    return model, cores


def probe_vector(P, seed, system, probe, n):
    """Probe `probe` of `system` as the library defines it: sign of bit 63 of SplitMix64
    output (probe 3N + 3i + a) of the stream seeded with output `system` of the stream
    seeded with `seed`, scaled by 1/sqrt(3N) (computed with the library's host build)."""
    from paper_2307_02278_amd import _lib
    h = _lib.hostcheck()
    zs = h.mbdh_splitmix(seed, system)
    D = 3 * n
    bits = np.array([h.mbdh_splitmix(zs, probe * D + k) >> 63 for k in range(D)], dtype=float)
    return ((1.0 - 2.0 * bits) / math.sqrt(D)).reshape(n, 3)


def delta11_study(P, torch, synth):
    """Delta_11 = v^T C v for one fixed Rademacher probe (the first Lanczos diagonal),
    by SPME-Ewald as a function of the grid and by the replica sum as a function of the
    spherical cutoff, with the time of one evaluation (execute with m = 1). The replica
    sum tends to the vacuum limit, which exceeds the tin-foil Ewald value by
    (4 pi / 3V) |sum_i g_i v_i|^2; that corrected SPME value is reported beside it."""
    A = synth.ANGSTROM_BOHR
    out = {}
    for name, s in (("water216", synth.water_box(216, seed=7)),
                    ("diamond512", synth.diamond_box(4))):
        ds = P.DeviceSystem(s.pos, s.cell, s.alpha, s.omega, s.rvdw)
        V = float(abs(np.linalg.det(s.cell)))

        def d11(**kw):
            plan = P.Plan([ds], P.Params(n_probes=1, n_steps=1, block=1,
                                         precision=P.PREC_FP64, seed=12345, **kw))
            plan.execute()
            torch.cuda.synchronize()
            reps = 3
            t0 = time.perf_counter()
            for _ in range(reps):
                plan.execute()
            torch.cuda.synchronize()
            ms = 1000.0 * (time.perf_counter() - t0) / reps
            plan.check()
            a, _, _ = plan.tridiagonal()
            plan.close()
            return float(a[0, 0]), ms

        spme = []
        for K in (12, 16, 18, 20, 24, 30, 32, 36, 40, 48):
            val, ms = d11(real_cutoff=7.0 * A, grid=(K, K, K))
            spme.append([K, val, round(ms, 3)])
        rep = []
        for rc in (10.0, 15.0, 20.0, 30.0, 40.0, 60.0, 80.0, 100.0):
            val, ms = d11(real_cutoff=7.0 * A, grid=(16, 16, 16), replica_cutoff=rc * A)
            rep.append([rc, val, round(ms, 3)])
        # surface term of the vacuum limit for this probe
        g = s.omega * np.sqrt(s.alpha)
        v = probe_vector(P, 12345, 0, 0, s.n)
        surf = 4.0 * math.pi / (3.0 * V) * float(((g[:, None] * v).sum(0) ** 2).sum())
        k18 = [r for r in spme if r[0] == 18][0]
        out[name] = {"atoms": s.n, "box_angstrom": round(float(s.cell[0, 0]) / A, 3),
                     "spme_vs_K": spme, "replica_vs_Rcut_angstrom": rep,
                     "spme_plus_surface_at_K48": spme[-1][1] + surf,
                     "cost_ratio_replica100A_over_spme_K18": round(rep[-1][2] / k18[2], 1)}
        log(f"delta11 {name}: SPME K=48 {spme[-1][1]:.10f}, +surface {spme[-1][1] + surf:.10f}, "
            f"replica 100 A {rep[-1][1]:.10f}; cost ratio {rep[-1][2] / k18[2]:.1f}")
    return out


def scs_timing(plan, torch, s, n_pairs, n_freq=15):
    """Range-separated SCS of the 24k water box at its current positions (static point +
    n_freq nodes, 3 (n_freq + 1) right-hand sides in one float64 conjugate gradient):
    wall time of one call after a warm-up call, iterations, and the rate of
    (pair, frequency) tensor evaluations of the operator kernel."""
    plan.scs(n_freq=n_freq)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    a, o, r, info = plan.scs(n_freq=n_freq)
    torch.cuda.synchronize()
    ms = 1000.0 * (time.perf_counter() - t0)
    ratio = a.cpu().numpy() / s.alpha
    it = info["iterations"]
    log(f"scs: {ms:.1f} ms, {it} iterations, residual {info['max_rel_residual']:.2e}")
    return {"workload": "water box N=24000 (the headline box)", "n_freq": n_freq,
            "ms": round(ms, 2), "iterations": it, "ms_per_iteration": round(ms / max(it, 1), 3),
            "max_rel_residual": info["max_rel_residual"],
            "pair_frequency_evals_per_s": round(n_pairs * (n_freq + 1) * it / (ms * 1e-3), 1),
            "alpha_scs_over_alpha": [round(float(ratio.min()), 4), round(float(ratio.max()), 4)]}


def block_study(P, torch, synth):
    """Quadrature error per probe at a fixed number of matvecs: single-probe Lanczos
    against block Lanczos (krylov_block 4 and 8) with the same probes and the same m,
    on the 24k water box in mixed precision; the reference is single-probe Lanczos with
    full re-orthogonalization at m = 120. Also the wall time of one execute."""
    wl = synth.workload("batched24k")
    s = wl.systems[0]
    A = synth.ANGSTROM_BOHR
    K = tuple(wl.grid) * 3 if len(wl.grid) == 1 else tuple(wl.grid)
    ds = P.DeviceSystem(s.pos, s.cell, s.alpha, s.omega, s.rvdw)
    R = 64

    def run(m, kb=1, reorth=P.REORTH_NONE):
        plan = P.Plan([ds], P.Params(real_cutoff=wl.real_cutoff_angstrom * A, grid=K,
                                     n_probes=R, n_steps=m, block=R, precision=P.PREC_MIXED,
                                     seed=wl.probe_seed, reorth=reorth, krylov_block=kb))
        plan.execute()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.execute()
        torch.cuda.synchronize()
        ms = 1000.0 * (time.perf_counter() - t0)
        plan.check()
        q = plan.quadrature()
        plan.close()
        return q, ms

    qref, _ = run(120, 1, P.REORTH_FULL)
    rows = []
    for m in (3, 4, 6, 8, 12, 16):
        for kb in (1, 4, 8):
            q, ms = run(m, kb)
            rel = ((q - qref).abs() / qref.abs())
            rows.append({"m": m, "krylov_block": kb, "max_rel_err": float(rel.max()),
                         "mean_rel_err": float(rel.mean()),
                         "trace_rel_err": float(abs(q.sum() - qref.sum()) / qref.sum()),
                         "execute_ms": round(ms, 2)})
            log(f"block study m={m} kb={kb}: max rel err {float(rel.max()):.2e}, "
                f"{ms:.1f} ms")
    return {"workload": "water box N=24000, 64 probes, mixed precision",
            "reference": "single-probe Lanczos, full re-orthogonalization, m = 120",
            "rows": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--plain-probes", type=int, default=2)
    ap.add_argument("--reps", type=int, default=10,
                    help="graph replays per energy + forces median")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON-lines shape cache: measured shapes are stored there and later "
                         "runs with the same key reuse them (e.g. counter runs, whose "
                         "serialised dispatches would distort a fresh measurement)")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain FP64 B=1 leg")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a 1 GiB device copy first (reference for HBM byte counters)")
    ap.add_argument("--no-forces", action="store_true",
                    help="skip every energy + forces leg")
    ap.add_argument("--no-uneven", action="store_true",
                    help="skip the uneven batch (32 water boxes, energy + forces)")
    ap.add_argument("--eager", action="store_true",
                    help="launch every kernel from the host instead of replaying HIP graphs")
    ap.add_argument("--no-scs", action="store_true",
                    help="skip the self-consistent screening leg on the 24k box")
    ap.add_argument("--block-study", action="store_true",
                    help="also compare single-probe and block Lanczos quadrature errors at "
                         "equal matvec counts on the 24k box")
    ap.add_argument("--delta11", action="store_true",
                    help="also run the Delta_11 convergence study (SPME vs grid, replica vs "
                         "cutoff) on a 216-water box and a 512-atom diamond box")
    args = ap.parse_args()
    global TUNE_CACHE
    TUNE_CACHE = args.tune_cache
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(probes would shard across GPUs with one final all-reduce).", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_2307_02278_amd as P

    wl = synth.workload("batched24k")
    s = wl.systems[0]
    A = synth.ANGSTROM_BOHR
    K = tuple(wl.grid) * 3 if len(wl.grid) == 1 else tuple(wl.grid)
    R, m, B = wl.n_probes, wl.n_steps, wl.block
    graph = not args.eager
    log(f"workload: water N={s.n} L={s.cell[0, 0] / A:.2f} A K={K} R={R} m={m} B={B}")
    t0 = time.perf_counter()
    _, plan = plan_for(P, synth, wl, forces=False, graph=graph, tune=True)
    t_plan = time.perf_counter() - t0
    info = plan.info(0)
    shape = shape_of(P, plan)
    n_pairs = int(info.n_pairs)
    log(f"tau={info.tau:.6f}/bohr r_pair={info.r_pair / A:.3f} A cells={list(info.cells)} "
        f"pairs={n_pairs} workspace={info.workspace_bytes / 2**30:.2f} GiB shape={shape} "
        f"(plan {t_plan:.2f} s)")
    pos = torch.as_tensor(s.pos, dtype=torch.float64, device="cuda")

    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration: 3 x 1 GiB device-to-device copies")

    def step():
        plan.set_positions(pos)
        return plan.execute(energy_sd=True)

    for w in range(args.warmup):
        e, sd = step()
        torch.cuda.synchronize()
        plan.check()
        log(f"warmup {w}: E = {float(e[0]):.10e} Ha")

    def timed(n):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(n):
            out = step()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, out

    # The timed steps: execute replayed from its captured HIP graph (the plan's
    # production mode), or launched eagerly with --eager.
    dt, (e, sd) = timed(args.steps)
    plan.check()
    energy, energy_sd = float(e[0]), float(sd[0])
    ms_per_step = 1000.0 * dt / args.steps
    value = R * m * args.steps / dt
    log(f"timed {args.steps} steps ({'eager' if args.eager else 'graph replay'}): "
        f"{ms_per_step:.2f} ms/step, {value:.1f} matvecs/s, E = {energy:.10e} "
        f"+- {energy_sd:.3e} Ha")
    errors = {"quadrature_rel_err_8_probes": quadrature_error(plan,
                                                              golden("water24k_quadrature"))}
    rows = golden("water24k_rows")
    if rows is not None:
        v = torch.from_numpy(synth.gaussian_block(int(rows["block_seed"]), B, s.n)).cuda()
        got = plan.matvec(v).cpu().numpy()[[int(c) for c in rows["columns"]]]
        got = got[:, [int(i) for i in rows["sample"]]]
        want = rows["rows"]
        num = np.abs(got - want).reshape(len(want), -1).max(1)
        den = np.abs(want).reshape(len(want), -1).max(1)
        errors["matvec_elementwise_err_sampled_rows"] = float((num / den).max())
    errors["oracle_reference"] = "tests/golden/water24k_quadrature.npz, water24k_rows.npz"
    log(f"errors vs oracle: {errors}")
    plan.close()

    # Per-stage times: the same steps launched eagerly with HIP events around every
    # stage, on one stream (the tuned shape without the side stream), so that each
    # kernel's time is its own; not part of the value.
    sh1 = {k: v for k, v in shape.items() if k != "source"}
    sh1["overlap"] = 0
    _, splan = plan_for(P, synth, wl, forces=False, graph=False, tune=False, shape=sh1)
    splan.set_positions(pos)
    splan.execute()
    torch.cuda.synchronize()
    splan.stage_times()
    splan.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        splan.set_positions(pos)
        ee = splan.execute()
    torch.cuda.synchronize()
    te = time.perf_counter() - t0
    splan.set_timing(False)
    splan.check()
    stages = splan.stage_times()
    splan.close()
    eager_rate = R * m * args.steps / te
    log(f"eager one-stream with stage events: {1000 * te / args.steps:.2f} ms/step, "
        f"{eager_rate:.1f} matvecs/s")

    # Per-stage averages and the dominant kernel's roofline.
    stage_ms = {k: v[0] / args.steps for k, v in stages.items() if v[1] > 0}
    kernel_stages = {k: v for k, v in stages.items()
                     if v[1] > 0 and k not in ("lanczos", "setup")}
    dom = max(kernel_stages, key=lambda k: kernel_stages[k][0])
    dom_ms_avg = kernel_stages[dom][0] / kernel_stages[dom][1]
    pair_kernel = pair_kernel_name(shape, B, s.n)
    if dom == "pair":
        flops = 18.0 * n_pairs * B
        achieved = flops / (dom_ms_avg * 1e-3) / 1e12
        mfma = pair_kernel.startswith("k_pair_mfma")
        roof = {"kernel": pair_kernel, "bound": "mfma" if mfma else "alu",
                "achieved": round(achieved, 3),
                "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
                "traffic": measured_traffic(pair_kernel),
                "avg_launch_ms": round(dom_ms_avg, 4),
                "algorithmic_per_launch": f"18 flop x {n_pairs} pairs x {B} rhs"}
        if mfma:
            # the matrix cores also multiply the list's zero tensors (out-of-range
            # target-candidate pairs of a 16-target group)
            roof["peak_note"] = "FP32 matrix-core peak; algorithmic flops exclude zero tensors"
        else:
            roof["peak_nonpacked_fp32"] = FP32_NONPACKED_TFLOPS
            roof["frac_of_nonpacked_fp32"] = round(achieved / FP32_NONPACKED_TFLOPS, 4)
    else:
        by = stage_bytes(dom, K, s.n, B // 2)
        achieved = by / (dom_ms_avg * 1e-3) / 1e9
        roof = {"kernel": STAGE_KERNEL.get(dom, dom), "bound": "hbm",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(STAGE_KERNEL.get(dom, "")),
                "avg_launch_ms": round(dom_ms_avg, 4),
                "algorithmic_per_launch": f"{by:.4g} B"}
    # The pair kernel alone in its fastest stand-alone shape (matrix cores, four
    # wavefronts per group, every group resident), timed the same way; the timed shape
    # may run it narrower, to leave room for the grid stages beside it.
    alone = None
    if B % 64 == 0 and B <= 256:
        sh_alone = dict(sh1, pair_mode=1, pair_subsets=4, pair_wg_per_cu=0, overlap=0)
        _, aplan = plan_for(P, synth, wl, forces=False, graph=False, tune=False,
                            shape=sh_alone)
        aplan.set_positions(pos)
        aplan.execute()
        torch.cuda.synchronize()
        aplan.stage_times()
        aplan.set_timing(True)
        for _ in range(args.steps):
            aplan.set_positions(pos)
            aplan.execute()
        torch.cuda.synchronize()
        aplan.set_timing(False)
        aplan.check()
        pst = aplan.stage_times()["pair"]
        aplan.close()
        a_ms = pst[0] / pst[1]
        a_tf = 18.0 * n_pairs * B / (a_ms * 1e-3) / 1e12
        alone = {"kernel": pair_kernel_name(sh_alone, B, s.n), "achieved": round(a_tf, 3),
                 "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                 "frac": round(a_tf / FP32_PEAK_TFLOPS, 4), "avg_launch_ms": round(a_ms, 4),
                 "shape": sh_alone}
        log(f"pair kernel alone: {alone}")
    roof["pair_kernel_alone"] = alone
    # Whole-matvec algorithmic bytes 24 K^3 + 48 N per probe-vector.
    bmv = 24.0 * K[0] * K[1] * K[2] + 48.0 * s.n

    scs_leg = None
    if not args.no_scs:
        _, sp = plan_for(P, synth, wl, forces=False, graph=False, tune=False)
        scs_leg = scs_timing(sp, torch, s, n_pairs)
        sp.close()

    # Plain form: one probe vector at a time in float64, same kernels, same GPU,
    # launched eagerly and replayed from a graph.
    plain = None
    if not args.no_plain:
        plain = {}
        Rp = args.plain_probes
        for g in (False, True):
            ds = P.DeviceSystem(s.pos, s.cell, s.alpha, s.omega, s.rvdw)
            pp = P.Plan([ds], P.Params(real_cutoff=wl.real_cutoff_angstrom * A, grid=K,
                                       n_probes=Rp, n_steps=m, block=1,
                                       precision=P.PREC_FP64, seed=wl.probe_seed, graph=g))
            pp.execute()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pp.execute()
            torch.cuda.synchronize()
            tp = time.perf_counter() - t0
            pp.check()
            plain["graph" if g else "eager"] = Rp * m / tp
            pp.close()
        log(f"plain fp64 B=1: {plain}")
    plain_rate = max(plain.values()) if plain else None

    # E_MBD + forces: the headline box (the metric's second half), the 12k organic box
    # and the uneven batch.
    ef24 = ef12 = ef_uneven = None
    if not args.no_forces:
        ef24 = energy_forces_leg(P, torch, synth, "batched24k", graph, args.reps,
                                 golden_name="water24k_quadrature")
        ef12 = energy_forces_leg(P, torch, synth, "forces12k", graph, args.reps,
                                 fp64_check=True, golden_name="organic12k_quadrature")
        if not args.no_uneven:
            ef_uneven = {"eager": energy_forces_leg(P, torch, synth, "uneven", False, 3,
                                                    golden_name="uneven_quadrature")}
            if graph:
                ef_uneven["graph"] = energy_forces_leg(P, torch, synth, "uneven", True, 3)

    d11 = delta11_study(P, torch, synth) if args.delta11 else None
    bstudy = block_study(P, torch, synth) if args.block_study else None

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import method as om
        model, ncpu = cpu_info()
        op = om.Operator(s, om.MethodParams(tau=info.tau, r_pair=info.r_pair, grid=K,
                                            order=info.spline_order))
        y = torch.randn(s.n, 3, 1, dtype=torch.float64, generator=torch.Generator().manual_seed(0))
        threads = torch.get_num_threads()

        def rate(nmv):
            t0 = time.perf_counter()
            for _ in range(nmv):
                op(y)
            return nmv / (time.perf_counter() - t0), time.perf_counter() - t0

        r_all, t_all = rate(12)
        torch.set_num_threads(1)
        r_one, t_one = rate(2)
        torch.set_num_threads(threads)
        cpu = {"value": round(r_all, 4), "unit": "matvecs/s", "cores": threads, "kind": "oracle",
               "sample": f"12 single-vector float64 SPME matvecs of the 24k box (same N, K, p, "
                         f"tau, r_pair) with the CPU oracle on {threads} threads, {t_all:.1f} s",
               "cpu_model": model, "host_logical_cpus": ncpu,
               "single_thread_value": round(r_one, 4),
               "single_thread_sample": f"2 matvecs on 1 thread, {t_one:.1f} s"}
        log(f"cpu oracle: {r_all:.3f} matvecs/s on {threads} threads, {r_one:.3f} on 1 ({model})")

    out = {
        "metric": "probe-vector SPME matvecs/s and E_MBD+forces ms at N=24k, batched vs plain",
        "value": round(value, 1),
        "unit": "matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "water box N=24000, L=62.09 A, K=96^3, p=6, r_c=9 A, "
                               "128 probes x 50 Lanczos steps as one RHS block, mixed precision",
                   "n_atoms": s.n, "grid": list(K), "probes": R, "lanczos_steps": m,
                   "block": B, "pairs": n_pairs, "shape": shape},
        "execution": "eager" if args.eager else "hip_graph_replay",
        "energy_ms": round(ms_per_step, 3),
        "energy_ha": energy,
        "energy_sd_ha": energy_sd,
        "energy_forces_ms_24k": ef24["energy_forces_ms"] if ef24 else None,
        "errors_vs_oracle": errors,
        "plain_matvecs_per_s": {k: round(v, 2) for k, v in plain.items()} if plain else None,
        "speedup_vs_plain": round(value / plain_rate, 2) if plain_rate else None,
        "path_algorithmic_GBps": round(bmv * value / 1e9, 1),
        "path_roofline_frac": round(bmv * value / 1e9 / HBM_PEAK_GBS, 4),
        "eager_one_stream_matvecs_per_s": round(eager_rate, 1),
        "stage_ms_per_step": {k: round(v, 3) for k, v in stage_ms.items()},
        "stage_timing": "eager, one stream (tuned shape without the side stream), HIP events "
                        "around every stage",
        "roofline": roof,
        "cpu_baseline": cpu,
        "energy_forces_24k": ef24,
        "energy_forces": ef12,
        "energy_forces_uneven": ef_uneven,
        "scs": scs_leg,
    }
    if d11 is not None:
        out["delta11"] = d11
    if bstudy is not None:
        out["block_study"] = bstudy
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
