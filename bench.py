#!/usr/bin/env python3
"""Benchmark of the KPM energy + gradient hot path on one MI355X.

Workload (the 100x100 configuration): 100 x 100 torus (10^4 sites, BdG
dimension 2 x 10^4) with two vortices (two superconducting flux quanta, Landau
gauge Peierls phases) and a period-8 checkerboard pair/charge-density seed of
amplitude 0.02, doping 0.125, t'/t = -0.3, J/t = 0.3, T = 0.005 t; M = 4096
Chebyshev moments with Jackson damping; 256 colored Z4 probes (8 x 8 coloring,
Nambu-split, two independent phase draws of weight 1/2); FP32 recurrence
vectors with FP64 moments, bounds, coefficients and density-matrix sums;
alpha checkpoints every 64 steps for the reversible adjoint.

One step = one energy + gradient evaluation: build h from the order
parameters, Gershgorin bounds, expansion coefficients, forward recursion with
moments and Omega, adjoint recursion with the density matrix, the order-
parameter map and the builder VJP (dOmega/dtheta for all ~1e5 parameters).
Inputs are resident in HBM before the timed region; nothing is skipped.

Prints ONE JSON line.  ``value`` is Chebyshev vector-steps per second: a
vector-step is one application of H~ to one 2N-dimensional probe vector; one
energy + gradient costs R (M - 1) forward and 2 R (M - 2) adjoint vector-steps.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0
PMC_ARGS = ("--moments 256 --steps 1 --warmup 1 --no-cpu-baseline --no-fp64-form --no-batched-form --no-rmft-form "
            "--no-direct-form --no-supercell-form --no-kernel-timing")
METRIC = "Chebyshev vector-steps/s + HBM GB/s; s per KPM energy+gradient at 100x100"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the recursion kernels' source with comments and whitespace
    removed: a counter record stays valid across comment-only edits and goes
    stale with any change to the code."""
    import re
    src = open(os.path.join(ROOT, "paper_2212_05685_amd", "csrc", "kpm_cheb.hip")).read()
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    src = " ".join(src.split())
    return hashlib.sha256(src.encode()).hexdigest()[:16]


def halves_used(R: int, N: int, streams: int) -> bool:
    """Whether a single-lattice call runs as two probe halves on two streams
    (kpm_set_streams: 2 forced, 1 never, 0 the library's automatic rule)."""
    return streams == 2 or (streams == 0 and R >= 128 and R * N >= 2 ** 19)


def traffic_record(kernel: str):
    """HBM bytes per recursion step (all launches of one step) from the
    committed rocprofv3 counter summary, if it was taken on the current kernel
    source; else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_c5_fp32_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_step")


def _pmc_rows(d, counter):
    """Per-dispatch (grid size, value) of one counter from a rocprofv3 --pmc CSV
    directory, keyed by kernel name."""
    import csv
    import glob
    vals = {}
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] == counter:
                vals.setdefault(r["Kernel_Name"], []).append((int(r["Grid_Size"]), float(r["Counter_Value"])))
    if not vals:
        raise SystemExit(f"no {counter} rows under {d}")
    return vals


def _modal_grid(rows):
    """Values of the dispatches with the most common grid size: the kernel in
    the configuration the run used, without the tuner's trial launches."""
    import collections
    grid = collections.Counter(g for g, _ in rows).most_common(1)[0][0]
    return grid, [v for g, v in rows if g == grid]


def traffic_summary(base: str, copy_bytes: int) -> None:
    """Turn the four rocprofv3 --pmc runs under ``base`` (fetch/, write/: the
    workload; copyf/, copyw/: one plain copy of ``copy_bytes``) into the
    traffic record of the recursion kernels (written under profiles/)."""
    fetch, write = _pmc_rows(os.path.join(base, "fetch"), "FETCH_SIZE"), _pmc_rows(os.path.join(base, "write"), "WRITE_SIZE")
    cf, cw = _pmc_rows(os.path.join(base, "copyf"), "FETCH_SIZE"), _pmc_rows(os.path.join(base, "copyw"), "WRITE_SIZE")
    kib_f = max(v for rows in cf.values() for _, v in rows)   # the copy is the largest dispatch of its run
    kib_w = max(v for rows in cw.values() for _, v in rows)
    f_fetch, f_write = copy_bytes / (kib_f * 1024.0), copy_bytes / (kib_w * 1024.0)
    import workloads as wl
    c5 = wl.C5("fp32")
    R = sum(p.nprobes() for p in c5.probes)
    # the counter runs use the library's default streams: a step is then the two
    # equal probe halves' launches (same kernel, same grid)
    per_step = 2 if halves_used(R, c5.N, 0) else 1
    out = {}
    # the plain step launches (not the checkpoint-storing forward nor the last adjoint step)
    for short, tags in (("k_adj", (">::adj<false>(",)), ("k_fwd", (">::fwdp<false, false>(",))):
        fr = [x for k, vs in fetch.items() if any(t in k for t in tags) for x in vs]
        wr = [x for k, vs in write.items() if any(t in k for t in tags) for x in vs]
        if not fr or not wr:
            raise SystemExit(f"no dispatches of {short} in the counter runs")
        grid, fr = _modal_grid(fr)
        wr = [v for g, v in wr if g == grid]
        fk, wk = sum(fr) / len(fr), sum(wr) / len(wr)
        out[short] = {
            "kernel_source_sha256_16": kernel_source_hash(),
            "kernel_source_hash_rule": "sha256 of kpm_cheb.hip with comments and whitespace removed "
                                       "(bench.kernel_source_hash)",
            "dispatches": len(fr),
            "grid_size": grid,
            "FETCH_SIZE_KiB_per_dispatch": fk,
            "WRITE_SIZE_KiB_per_dispatch": wk,
            "copy_calibration": {"bytes": copy_bytes, "FETCH_SIZE_KiB": kib_f, "WRITE_SIZE_KiB": kib_w,
                                 "fetch_factor": f_fetch, "write_factor": f_write},
            "hbm_bytes_per_launch": fk * 1024.0 * f_fetch + wk * 1024.0 * f_write,
            "launches_per_step": per_step,
            "hbm_bytes_per_step": per_step * (fk * 1024.0 * f_fetch + wk * 1024.0 * f_write),
            "note": "bytes leaving L2 for the memory fabric (Infinity Cache hits included), "
                    "scaled by what the same counters read for a plain copy of known size; a step of "
                    "the 100x100 workload is the launches of its two probe halves (128 probes each)",
            "commands": [
                "cd /tmp && export TMPDIR=/tmp",
                "export KPM_TUNE_CACHE=<file>   # the kernel configuration tuned at the benchmark's M, "
                "reused by the counter runs (the shape key does not include M)",
                "python3 bench.py --steps 1 --warmup 0 --no-cpu-baseline --no-fp64-form --no-batched-form "
                "--no-rmft-form --no-direct-form --no-supercell-form",
                f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d {base}/fetch -o fetch -- python3 bench.py {PMC_ARGS}",
                f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d {base}/write -o write -- python3 bench.py {PMC_ARGS}",
                f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d {base}/copyf -o copyf -- python3 bench.py "
                f"--copy-calibration {copy_bytes}",
                f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d {base}/copyw -o copyw -- python3 bench.py "
                f"--copy-calibration {copy_bytes}",
                f"python3 bench.py --traffic-summary {base}",
            ],
        }
    for short, rec in out.items():
        path = os.path.join(ROOT, "profiles", f"{short}_c5_fp32_traffic.json")
        with open(path, "w") as fh:
            json.dump(rec, fh, indent=1)
        print(f"{path}: {rec['hbm_bytes_per_step'] / 1e6:.1f} MB per step")


def make_problem(cfg, precision):
    import torch
    from paper_2212_05685_amd import kpm
    from paper_2212_05685_amd.solver import KPMProblem
    import workloads as wl

    kinds = {"unit": kpm.KPM_PROBE_UNIT, "dense_z4": kpm.KPM_PROBE_DENSE_Z4,
             "colored_z4": kpm.KPM_PROBE_COLORED_Z4}
    specs = [kpm.ProbeSpec(kinds[p.kind], p.count, p.seed, p.px, p.py, p.split_nambu, p.first, p.weight)
             for p in cfg.probes]
    prec = kpm.KPM_FP32 if precision == "fp32" else kpm.KPM_FP64
    prob = KPMProblem(cfg.Lx, cfg.Ly, cfg.n_v, cfg.t, cfg.tp, cfg.J, cfg.mu, cfg.T, cfg.M, specs,
                      prec, cfg.ckpt_k)
    n, chi, dlt = wl.make_theta(cfg)
    th = (torch.from_numpy(n).cuda(), torch.from_numpy(chi).cuda(), torch.from_numpy(dlt).cuda())
    return prob, th


def energy_grad(prob, th):
    """One full energy + gradient evaluation (every row of the hot path)."""
    n, chi, dlt = th
    h = prob.build_H(n, chi, dlt)
    ab = prob.bounds(h)
    C = prob.coefficients(ab)
    out = prob.density_matrix(h, ab, C)
    grads = prob.build_H_vjp(n, chi, dlt, out["rho"])
    return out, grads


def timed(prob, th, steps, warmup, profile):
    """`warmup` untimed steps, then exactly `steps` steps between two device
    synchronisations; each step is bracketed by HIP events on the stream the
    library launches on (torch's current stream).  Returns the median event
    time per step (s), the per-step times, the wall-clock mean, the last
    outputs and the sampled kernel durations."""
    import statistics

    import torch
    from paper_2212_05685_amd import kpm

    for w in range(warmup):
        energy_grad(prob, th)
        torch.cuda.synchronize()
        log(f"{'fp32' if prob.precision else 'fp64'} warmup {w + 1}/{warmup} done")
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    if profile:
        kpm.kpm_profile_begin(128)
    t0 = time.perf_counter()
    for s in range(steps):
        ev[s][0].record()
        out, grads = energy_grad(prob, th)
        ev[s][1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = kpm.kpm_profile_end() if profile else None
    if prob.status() != 0:
        raise RuntimeError(f"device status {prob.status()}")
    per = [a.elapsed_time(b) * 1e-3 for a, b in ev]
    med = statistics.median(per)
    log(f"{'fp32' if prob.precision else 'fp64'} timed {steps} steps: median {med * 1e3:.1f} ms/step "
        f"(events), wall mean {(t1 - t0) / steps * 1e3:.1f} ms")
    return med, per, (t1 - t0) / steps, out, grads, prof


def batched_form(steps: int):
    """48 uneven lattices (24..64 sites on a side, doping 0.05-0.25, 2 or 4
    vortices, M = 1024, 64 colored probes each): one batched FP32 energy +
    gradient replayed as hipGraphs (the plan's instance groups one after
    another, each group's two halves side by side), against the plain FP64
    single-lattice form run lattice by lattice on the same inputs."""
    import numpy as np
    import torch
    from paper_2212_05685_amd import kpm
    import workloads as wl

    cfgs = wl.C4_instances(48)
    probs, hs, abs_, Cs = [], [], [], []
    for cfg in cfgs:
        q, th = make_problem(cfg, "fp32")
        h = q.build_H(*th)
        ab = q.bounds(h)
        probs.append(q)
        hs.append(h)
        abs_.append(ab)
        Cs.append(q.coefficients(ab))
    M, k = cfgs[0].M, cfgs[0].ckpt_k
    plan = kpm.kpm_batch_create([q.lat for q in probs], [q.probes for q in probs], M, kpm.KPM_FP32, k)
    try:
        omega = torch.zeros(len(cfgs), dtype=torch.float64, device="cuda")
        rhos = [torch.zeros_like(h) for h in hs]
        kpm.kpm_batch_energy_grad(plan, hs, abs_, Cs, omega, rhos, use_graph=True)   # tune + capture
        torch.cuda.synchronize()
        tune = kpm.kpm_batch_tuning(plan)
        streams = kpm.kpm_batch_streams(plan)
        groups = kpm.kpm_batch_groups(plan)
        t0 = time.perf_counter()
        for _ in range(steps):
            kpm.kpm_batch_energy_grad(plan, hs, abs_, Cs, omega, rhos, use_graph=True)
        torch.cuda.synchronize()
        dt32 = (time.perf_counter() - t0) / steps
        om32 = omega.cpu().numpy()
        r32 = [r.cpu().numpy() for r in rhos]
        # kernel durations: the same sequence launched directly (a graph replay
        # cannot carry the library's timing events), same kernels and configuration
        kpm.kpm_profile_begin(32)
        t0 = time.perf_counter()
        for _ in range(2):
            kpm.kpm_batch_energy_grad(plan, hs, abs_, Cs, omega, rhos, use_graph=False)
        torch.cuda.synchronize()
        dt_direct = (time.perf_counter() - t0) / 2
        fwd_ms, n_fwd, adj_ms, n_adj = kpm.kpm_profile_end()
    finally:
        kpm.kpm_batch_destroy(plan)
    RN = sum(q.R * c.N for q, c in zip(probs, cfgs))
    NS = sum(c.N for c in cfgs)
    # bytes of one recursion step of all 48 lattices; with instance groups a
    # launch covers one group (the groups hold nearly equal sum R N), so the
    # bytes per launch are the step's bytes over the group count
    fwd_bytes = 3 * 16 * RN + 288 * NS
    adj_bytes = 6 * 16 * RN + 288 * NS
    fwd_launch = fwd_bytes / groups
    adj_launch = adj_bytes / groups
    fwd_s = fwd_ms / max(n_fwd, 1) * 1e-3
    adj_s = adj_ms / max(n_adj, 1) * 1e-3
    log(f"batched FP32: {dt32 * 1e3:.1f} ms per energy + gradient of 48 lattices ({groups} groups)")
    p64 = []
    for cfg in cfgs:
        q, _ = make_problem(cfg, "fp64")
        p64.append(q)

    def fp64_pass():
        out = []
        for q, h, ab, C in zip(p64, hs, abs_, Cs):
            om = q.grand_potential(h, ab, C)
            out.append((om, q.grand_potential_grad(h, ab, C)))
        return out

    fp64_pass()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out64 = fp64_pass()
    torch.cuda.synchronize()
    dt64 = time.perf_counter() - t0
    om64 = np.array([float(o.item()) for o, _ in out64])
    e_om = float(np.max(np.abs(om32 - om64) / np.abs(om64)))
    e_rho = max(float(np.max(np.abs(r32[q] - out64[q][1].cpu().numpy())) /
                      np.max(np.abs(out64[q][1].cpu().numpy()))) for q in range(len(cfgs)))
    vsteps = sum(q.R for q in probs) * (3 * M - 5)
    log(f"FP64 lattice by lattice: {dt64 * 1e3:.1f} ms")
    return {
        "workload": "48 lattices L in {24..64}, doping U(0.05, 0.25), 2 or 4 vortices, M=1024, "
                    "64 colored Z4 probes (8x8) each, checkpoints every 64",
        "sites_total": int(sum(c.N for c in cfgs)),
        "ms_per_step_fp32_batched_graph": dt32 * 1e3,
        "ms_per_step_fp64_lattice_by_lattice": dt64 * 1e3,
        "speedup_fp32_batched_over_fp64": dt64 / dt32,
        "vector_steps_per_s_fp32_batched": vsteps / dt32,
        "fp32_vs_fp64_max_rel_err_omega": e_om,
        "fp32_vs_fp64_max_rel_err_rho": e_rho,
        "ms_per_step_fp32_batched_direct_launches": dt_direct * 1e3,
        "tuning": tune,
        "streams": streams,
        "groups": groups,
        "roofline": {
            "kernel": "k_adj (fused adjoint step)",
            "launch": (f"one recursion step of one of {groups} instance groups (run one after another, "
                       "each sized to the Infinity Cache, bytes averaged over the groups)"
                       if groups > 1 else "one recursion step of all 48 lattices")
                      + ("; the group's two instance halves run side by side on two streams, timed on "
                         "the first stream while the second's overlaps it" if streams == 2 else ""),
            "bound": "hbm",
            "achieved": adj_launch / adj_s / 1e9,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": adj_launch / adj_s / 1e9 / HBM_PEAK_GBS,
            "traffic": None,
            "algorithmic_bytes_per_launch": adj_launch,
            "avg_launch_us": adj_s * 1e6,
            "launches_timed": n_adj,
        },
        "forward_kernel": {"algorithmic_bytes_per_launch": fwd_launch, "avg_launch_us": fwd_s * 1e6,
                           "achieved_GBs": fwd_launch / fwd_s / 1e9, "launches_timed": n_fwd},
        "hbm_GBs_algorithmic_whole_step": ((M - 1) * fwd_bytes + (M - 2) * adj_bytes) / dt32 / 1e9,
    }


def rmft_form(iters: int, warmup: int):
    """Self-consistent iteration on the plain-vortex workload of the Results
    section (48 x 96, two vortices, mean hole density 0.16, M = 1024, 128
    colored probes, FP32 recursion): every iteration runs the chemical-
    potential search (density-matrix evaluations) and the mixing update.
    After `warmup` iterations, the same state is iterated `iters` times with
    each search, and with the Illinois search on the direct estimate of rho;
    the fused adjoint kernel is timed live on two more Illinois iterations
    (so that the timing events do not weigh on the timed iterations), and the
    oracle's cost per evaluation is sampled on one probe."""
    import torch
    from paper_2212_05685_amd import kpm
    import workloads as wl

    cfg = wl.RMFT("fp32")
    prob, th = make_problem(cfg, "fp32")
    n, chi, dlt = th

    def params(search, estimator=kpm.KPM_RMFT_ADJOINT):
        return kpm.rmft_params(cfg.doping, mix=0.1, tol_n=1e-5, tol_mu=1e-9, mu_step=0.004,
                               max_evals=60, search=search, estimator=estimator)

    mu_w, _, st = prob.rmft_iterate(n, chi, dlt, cfg.mu, params(kpm.KPM_RMFT_ILLINOIS), warmup)
    if st != kpm.KPM_OK:
        raise RuntimeError(f"rmft warmup status {st}")
    torch.cuda.synchronize()
    log(f"rmft warmup {warmup} iterations done, mu = {mu_w:.6f}")
    out = {}
    for name, search, est in (("illinois", kpm.KPM_RMFT_ILLINOIS, kpm.KPM_RMFT_ADJOINT),
                              ("bisection", kpm.KPM_RMFT_BISECTION, kpm.KPM_RMFT_ADJOINT),
                              ("illinois_direct", kpm.KPM_RMFT_ILLINOIS, kpm.KPM_RMFT_DIRECT)):
        n2, chi2, dlt2 = n.clone(), chi.clone(), dlt.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mu, hist, st = prob.rmft_iterate(n2, chi2, dlt2, mu_w, params(search, est), iters)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if st != kpm.KPM_OK or len(hist) != iters:
            raise RuntimeError(f"rmft status {st}")
        evals = sum(h["evals"] for h in hist)
        log(f"rmft {name}: {iters} iterations, {dt / iters * 1e3:.1f} ms/iteration, "
            f"{evals / iters:.1f} evaluations each")
        out[name] = {"s_per_iteration": dt / iters, "evaluations_per_iteration": evals / iters,
                     "ms_per_density_matrix_evaluation": dt / evals * 1e3,
                     "residual_first": hist[0]["residual"], "residual_last": hist[-1]["residual"],
                     "mu_last": mu}
    # the spin-polarised loop (SDW builder, per-spin map, 34 N Anderson vector) on the same lattice,
    # from a spin-symmetric seed with small spin-dependent noise (the path's cost, not an SDW state)
    th6 = [torch.from_numpy(x).cuda() for x in wl.make_theta_sdw(cfg, m_amp=0.0, spin_noise=0.005)]
    try:
        mu6, _, st = prob.rmft_iterate_sdw(*th6, cfg.mu, params(kpm.KPM_RMFT_ILLINOIS), warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mu6, hist6, st6 = prob.rmft_iterate_sdw(*th6, mu6, params(kpm.KPM_RMFT_ILLINOIS), iters)
        torch.cuda.synchronize()
        dt6 = time.perf_counter() - t0
        ev6 = sum(h["evals"] for h in hist6)
        out["illinois_spin_polarised"] = {
            "s_per_iteration": dt6 / max(len(hist6), 1), "evaluations_per_iteration": ev6 / max(len(hist6), 1),
            "ms_per_density_matrix_evaluation": dt6 / max(ev6, 1) * 1e3, "status": st6,
            "iterations": len(hist6), "residual_last": hist6[-1]["residual"] if hist6 else None}
        log(f"rmft spin-polarised: {dt6 / max(len(hist6), 1) * 1e3:.1f} ms/iteration, "
            f"{ev6 / max(len(hist6), 1):.1f} evaluations each")
    except kpm.KpmError as e:
        out["illinois_spin_polarised"] = {"error": str(e)}
    # kernel durations: two more Illinois iterations, timed by the library
    n2, chi2, dlt2 = n.clone(), chi.clone(), dlt.clone()
    torch.cuda.synchronize()
    kpm.kpm_profile_begin(4)
    _, _, st = prob.rmft_iterate(n2, chi2, dlt2, mu_w, params(kpm.KPM_RMFT_ILLINOIS), 2)
    torch.cuda.synchronize()
    prof = kpm.kpm_profile_end()
    if st != kpm.KPM_OK:
        raise RuntimeError(f"rmft status {st}")
    R, N = prob.R, cfg.N
    adj_bytes = 6 * 16 * R * N + 36 * 8 * N
    _, _, adj_ms, n_adj = prof
    adj_s = adj_ms / max(n_adj, 1) * 1e-3
    achieved = adj_bytes / adj_s / 1e9
    pool = OraclePool(host_workers())
    try:
        tasks = _oracle_tasks(cfg, pool.workers)
        wall, _ = pool.wall(tasks)
    finally:
        pool.close()
    t_eval_cpu = wall * R / len(tasks)
    ill = out["illinois"]
    return {
        "workload": "48x96 torus, 2 vortices (plain-vortex seed, chi seeded 0), doping 0.16, M=1024, "
                    "128 colored Z4 probes (8x8, Nambu split), FP32 recurrence; mixing 0.1, mu search "
                    "to |mean n - 0.84| <= 1e-5",
        "iterations_timed": iters,
        "warmup_iterations": warmup,
        "s_per_iteration": ill["s_per_iteration"],
        "evaluations_per_iteration": ill["evaluations_per_iteration"],
        "ms_per_density_matrix_evaluation": ill["ms_per_density_matrix_evaluation"],
        "search": out,
        "speedup_illinois_over_bisection": out["bisection"]["s_per_iteration"] / ill["s_per_iteration"],
        "speedup_direct_estimate": ill["s_per_iteration"] / out["illinois_direct"]["s_per_iteration"],
        "roofline": {
            "kernel": "k_adj (fused adjoint step) at 48x96, R=128",
            "bound": "hbm",
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "algorithmic_bytes_per_launch": adj_bytes, "avg_launch_us": adj_s * 1e6,
            "launches_timed": n_adj,
            "launch": "timed on two further iterations of the same loop (every launch carries timing "
                      "events there, which would weigh on the timed iterations)",
        },
        "cpu_baseline": {
            "value": t_eval_cpu * ill["evaluations_per_iteration"], "unit": "s/iteration",
            "cores": len(tasks), "kind": "oracle",
            "sample": f"oracle forward + adjoint on {len(tasks)} of {R} probes at 48x96, M={cfg.M}, one "
                      f"single-threaded process per core: {wall:.2f} s wall, times {R}/{len(tasks)} and the "
                      f"measured {ill['evaluations_per_iteration']:.1f} evaluations per iteration",
        },
    }


def direct_form(steps: int, prob, th, dt_adjoint):
    """The same 100x100 step with rho from the direct probing estimate
    (forward recursion with the f' series accumulated per probe) instead of
    the adjoint; the two are different estimates of the same matrix."""
    import numpy as np
    import torch

    n, chi, dlt = th

    def step():
        h = prob.build_H(n, chi, dlt)
        ab = prob.bounds(h)
        C = prob.coefficients(ab)
        om, rho = prob.density_matrix_direct(h, ab, C)
        grads = prob.build_H_vjp(n, chi, dlt, rho)
        return om, rho, grads, (h, ab, C)

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        om, rho, grads, (h, ab, C) = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    if prob.status() != 0:
        raise RuntimeError(f"device status {prob.status()}")
    out = prob.density_matrix(h, ab, C)
    r_dir, r_adj = rho.cpu().numpy(), out["rho"].cpu().numpy()
    log(f"direct form: {dt * 1e3:.1f} ms/step")
    return {
        "ms_per_step": dt * 1e3,
        "speedup_over_adjoint_form": dt_adjoint / dt,
        "omega_rel_diff_vs_adjoint_form": abs(float(om.item()) - float(out["omega"].item()))
                                          / abs(float(out["omega"].item())),
        "rho_max_rel_diff_vs_adjoint_form": float(np.max(np.abs(r_dir - r_adj)) / np.max(np.abs(r_adj))),
        # even steps: the forward step plus read and write of the FP64 y records
        "accumulating_step_bytes_per_launch": 48 * prob.R * prob.N + 36 * 8 * prob.N + 64 * prob.R * prob.N,
    }


def doubling_form(steps: int, prob, th):
    """Omega alone on the 100x100 workload: the forward recursion of
    kpm_grand_potential (M - 1 steps) against moment doubling (M/2 steps)."""
    import torch

    n, chi, dlt = th
    h = prob.build_H(n, chi, dlt)
    ab = prob.bounds(h)
    C = prob.coefficients(ab)
    res = {}
    for name, fn in (("forward", lambda: prob.grand_potential(h, ab, C)),
                     ("doubling", lambda: prob.moments_doubling(h, ab, C)[0])):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            om = fn()
        torch.cuda.synchronize()
        res[name] = ((time.perf_counter() - t0) / steps, float(om.item()))
    if prob.status() != 0:
        raise RuntimeError(f"device status {prob.status()}")
    log(f"omega only: forward {res['forward'][0] * 1e3:.1f} ms, doubling {res['doubling'][0] * 1e3:.1f} ms")
    return {
        "ms_omega_forward": res["forward"][0] * 1e3,
        "ms_omega_doubling": res["doubling"][0] * 1e3,
        "speedup_doubling": res["forward"][0] / res["doubling"][0],
        "omega_rel_diff": abs(res["doubling"][1] - res["forward"][1]) / abs(res["forward"][1]),
    }


def ldos_form(steps: int, prob, th, cfg):
    """KPM local density of states along a 24-site line through a vortex core
    of the 100x100 workload (48 Nambu indices, M = 4096, 1001 energies)."""
    import torch
    import workloads as wl

    n, chi, dlt = th
    h = prob.build_H(n, chi, dlt)
    ab = prob.bounds(h)
    X, Y = wl.vortex_centres(cfg.Lx, cfg.Ly, cfg.n_v)[0]
    first = 2 * (int(Y) * cfg.Lx + int(X) - 12)
    a, b = (float(v) for v in ab.cpu())
    E = torch.linspace(b - 0.3 * a, b + 0.3 * a, 1001, dtype=torch.float64, device="cuda")
    prob.ldos(h, ab, first, 48, E)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = prob.ldos(h, ab, first, 48, E)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    log(f"ldos line: {dt * 1e3:.1f} ms")
    return {"workload": "48 Nambu indices (24 sites through a vortex core), M=4096, 1001 energies, FP32 "
                        "recursion, FP64 series", "ms_per_linecut": dt * 1e3,
            "finite": bool(torch.isfinite(out).all().item()), "min": float(out.min().item())}


def sdw_form(reps: int, cfg):
    """The spin-polarised builder against the singlet one on the 100x100
    lattice (staggered m = 0.03 seed); per-call time from HIP events."""
    import torch
    from paper_2212_05685_amd import kpm
    import workloads as wl

    lat = kpm.lattice(cfg.Lx, cfg.Ly, cfg.n_v)
    mdl = kpm.model(cfg.t, cfg.tp, cfg.J, cfg.mu)
    th = [torch.from_numpy(x).cuda() for x in wl.make_theta_sdw(cfg, 0.03)]
    n, chi, dlt = (torch.from_numpy(x).cuda() for x in wl.make_theta(cfg))
    h = torch.zeros(19, cfg.N, dtype=torch.complex128, device="cuda")
    rho = torch.from_numpy(wl.random_stencil(cfg.N, seed=3)).cuda()
    grads = [torch.empty_like(x) for x in th]
    out = {}
    for name, fn in (("singlet", lambda: kpm.kpm_build_H(lat, mdl, n, chi, dlt, h)),
                     ("sdw", lambda: kpm.kpm_build_H_sdw(lat, mdl, *th, h)),
                     ("sdw_vjp", lambda: kpm.kpm_build_H_sdw_vjp(lat, mdl, th, rho, grads))):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name] = e0.elapsed_time(e1) / reps * 1e3
    log(f"builders: singlet {out['singlet']:.1f} us, sdw {out['sdw']:.1f} us, sdw vjp {out['sdw_vjp']:.1f} us")
    return {"us_build_singlet": out["singlet"], "us_build_sdw": out["sdw"], "us_vjp_sdw": out["sdw_vjp"],
            "h_bytes_written": 19 * 16 * cfg.N}


def supercell_form(k_count: int = 8):
    """Magnetic super-cell ED + broadened LDOS on the paper's smallest cell,
    48 x 48 with two vortices, on an 8 x 8 k grid (8 x 48 = 384): k_count k
    points of the grid, all 2304 sites, 201 energies in [-0.25 t, 0.25 t]
    (+-100 meV at t = 400 meV), Gamma = 0.25 |omega| + 3e-4.  Wall clock of the
    synchronous call (one warm-up call with one k point first)."""
    import torch
    import workloads as wl

    cfg = wl.Config("sc48", 48, 48, 2, 0.16, 8, (wl.ProbeSpec("unit", 1),), vortex=True,
                    complex_noise=0.02, seed=4848)
    prob, th = make_problem(cfg, "fp64")
    h = prob.build_H(*th)
    om = torch.linspace(-0.25 * cfg.t, 0.25 * cfg.t, 201, dtype=torch.float64, device="cuda")
    sites = list(range(cfg.N))
    res = {"workload": "48x48 cell, 2 vortices, 8x8 k grid, all 2304 sites, 201 energies, FP64, "
                       "rocSOLVER zheevd (strided-batched over k)", "k_points_timed": k_count}
    outs = {}
    for kb in (1, 8):
        prob.supercell_ldos(h, 8, 8, sites, om, 0.25, 3e-4, k_first=0, k_count=kb, k_batch=kb)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out, _ = prob.supercell_ldos(h, 8, 8, sites, om, 0.25, 3e-4, k_first=8, k_count=k_count,
                                     k_batch=kb)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / k_count
        outs[kb] = out
        log(f"supercell ED, batch {kb}: {dt * 1e3:.0f} ms per k point (2N = {2 * cfg.N})")
        res[f"ms_per_k_batch{kb}"] = dt * 1e3
    res["s_full_grid_est"] = res["ms_per_k_batch8"] * 64 / 1e3
    res["batch8_vs_batch1_max_rel_diff"] = float(((outs[8] - outs[1]).abs().max() / outs[1].abs().max()).item())
    res["finite"] = bool(torch.isfinite(outs[8]).all().item())
    res["min"] = float(outs[8].min().item())
    del prob, outs
    torch.cuda.empty_cache()
    return res


def cpu_dense_ed():
    """The oracle's dense exact diagonalisation (O1: eigh of the 2N x 2N BdG
    matrix, then the Fermi sums for Omega and rho) on the 32x32 vortex lattice
    (D = 2048), timed on the host with threaded LAPACK.  Reported beside the
    KPM baseline; the build of h is not timed."""
    import os
    from threadpoolctl import threadpool_info

    from oracle import builder, dense
    import workloads as wl

    cfg = wl.C2("fp64")
    n, chi, dlt = wl.make_theta(cfg)
    st = builder.build_stencil(cfg.Lx, cfg.Ly, cfg.n_v, cfg.t, cfg.tp, cfg.J, cfg.mu, n, chi, dlt)
    H = builder.dense_from_stencil(st, cfg.Lx, cfg.Ly)
    t0 = time.perf_counter()
    dense.exact(H, cfg.T)
    dt = time.perf_counter() - t0
    threads = max((p.get("num_threads", 1) for p in threadpool_info() if p.get("user_api") == "blas"),
                  default=1)
    log(f"cpu dense ED (D = {2 * cfg.N}): {dt:.2f} s on {threads} threads")
    return {"seconds": dt, "D": 2 * cfg.N, "cores": threads, "host_cpus": os.cpu_count(),
            "kind": "oracle (dense ED, O1)",
            "sample": "32x32 torus, 2 vortices: eigh of the 2048 x 2048 BdG matrix + Fermi sums for Omega and rho"}


def _oracle_probe(task):
    """Pool worker: the oracle's plain FP64 forward recursion + beta adjoint
    (O2, every vector stored) on one probe, single-threaded; returns seconds,
    the probe's moments and its (weighted) grand-potential term."""
    from threadpoolctl import threadpool_limits

    from oracle import kpm_plain
    Hs, a, b, r, w, C, Lx, Ly = task
    with threadpool_limits(1):
        t0 = time.perf_counter()
        out = kpm_plain.plain_kpm(Hs, a, b, r, w, C, Lx, Ly, want_grad=True)
        return time.perf_counter() - t0, out["mu"][0], out["omega"]


def _oracle_tasks(cfg, nprobe):
    """The oracle's own inputs (stencil, Gershgorin bounds, coefficients: not
    timed) and its first `nprobe` probes of the config as pool tasks."""
    import workloads as wl
    from oracle import builder, chebyshev, probes

    kinds = {"unit": probes.UNIT, "dense_z4": probes.DENSE_Z4, "colored_z4": probes.COLORED_Z4}
    n, chi, dlt = wl.make_theta(cfg)
    st = builder.build_stencil(cfg.Lx, cfg.Ly, cfg.n_v, cfg.t, cfg.tp, cfg.J, cfg.mu, n, chi, dlt)
    Hs = builder.sparse_from_stencil(st, cfg.Lx, cfg.Ly)
    a, b = chebyshev.rescale(*chebyshev.gershgorin_sparse(Hs))
    C = chebyshev.kpm_coefficients(cfg.M, cfg.T, a, b)
    groups = [probes.ProbeGroup(kinds[p.kind], p.count, p.seed, p.px, p.py, p.split_nambu, p.first, p.weight)
              for p in cfg.probes]
    R, w = probes.probe_set(groups, cfg.Lx, cfg.Ly)
    return [(Hs, a, b, R[q:q + 1], w[q:q + 1], C, cfg.Lx, cfg.Ly) for q in range(min(nprobe, R.shape[0]))]


def host_workers():
    """Worker processes for the oracle baselines: the CPUs this process may run
    on, at most 16 (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


class OraclePool:
    """Single-threaded oracle processes, one per worker core (spawned, so that
    no GPU context is inherited)."""

    def __init__(self, workers):
        from multiprocessing import get_context
        self.workers = workers
        self.pool = get_context("spawn").Pool(workers)
        self.pool.map(_noop, range(workers))            # start-up outside the timed samples

    def wall(self, tasks, timeout=900):
        """Wall-clock seconds to run `tasks` (one probe each) on the pool, and
        the per-probe results in task order."""
        t0 = time.perf_counter()
        res = self.pool.map_async(_oracle_probe, tasks, chunksize=1).get(timeout)
        return time.perf_counter() - t0, res

    def close(self):
        self.pool.terminate()


def _noop(x):
    """Worker start-up: the oracle's imports happen here, outside the samples."""
    import threadpoolctl  # noqa: F401
    from oracle import kpm_plain  # noqa: F401
    return x


def cpu_baseline(pool):
    """The oracle (O2: plain FP64 forward + beta adjoint, every vector stored)
    on all worker cores, parallel over probes (one single-threaded process per
    core, one probe per process), for the five workloads.  Each workload runs a
    bounded sample of one probe per core; its energy + gradient time is the
    sample's wall time scaled by the workload's probe work (probes x sites, M
    fixed), i.e. the model is perfect probe parallelism at `cores` processes.
    The headline entry is the 100 x 100 workload.  Also returns the oracle's
    moments and grand-potential terms of the 100 x 100 sample's probes (the
    first P), for the error of the GPU path against the oracle."""
    import workloads as wl

    P = pool.workers
    out = {}
    c5_sample = []
    for name, cfgs in (("C1_8x8", [wl.C1()]), ("C2_32x32", [wl.C2("fp64")]), ("C3_64x64", [wl.C3()]),
                       ("C4_48_lattices", wl.C4_instances(48)), ("C5_100x100", [wl.C5("fp64")])):
        if len(cfgs) == 1:
            tasks = _oracle_tasks(cfgs[0], P)
            sample_work = len(tasks) * cfgs[0].N
        else:                              # one probe of each of the first P lattices
            tasks = [_oracle_tasks(c, 1)[0] for c in cfgs[:P]]
            sample_work = sum(c.N for c in cfgs[:P])
        total_work = sum(c.R * c.N for c in cfgs)
        M = cfgs[0].M
        wall, res = pool.wall(tasks)
        if name == "C5_100x100":
            c5_sample = [(mu, om) for _, mu, om in res]
        s_eg = wall * total_work / sample_work
        vsteps = sum(c.R for c in cfgs) * (3 * M - 5)
        out[name] = {"s_per_energy_grad": s_eg, "vector_steps_per_s": vsteps / s_eg,
                     "sample_probes": len(tasks), "sample_wall_s": wall, "M": M,
                     "probes_total": sum(c.R for c in cfgs)}
        log(f"cpu baseline {name}: {len(tasks)} probes on {P} processes in {wall:.1f} s -> "
            f"{s_eg:.1f} s per energy + gradient")
    c5 = out["C5_100x100"]
    return {"value": c5["vector_steps_per_s"], "unit": "vector-steps/s", "cores": P, "kind": "oracle",
            "host_cpus": os.cpu_count(),
            "s_per_energy_grad": c5["s_per_energy_grad"],
            "sample": f"oracle O2 (plain FP64 forward recursion + beta adjoint, every vector stored) on "
                      f"{c5['sample_probes']} of the 256 probes of the 100x100 workload (M=4096), one "
                      f"single-threaded process per core on {P} cores, {c5['sample_wall_s']:.1f} s wall; "
                      f"energy + gradient time = wall x 256 / {c5['sample_probes']} (perfect probe "
                      f"parallelism at {P} processes)",
            "per_config": out}, c5_sample


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-form", action="store_true")
    ap.add_argument("--no-batched-form", action="store_true")
    ap.add_argument("--no-rmft-form", action="store_true")
    ap.add_argument("--no-direct-form", action="store_true")
    ap.add_argument("--no-supercell-form", action="store_true")
    ap.add_argument("--only-supercell-form", action="store_true",
                    help="run only the magnetic super-cell ED form and print its JSON")
    ap.add_argument("--only-batched-form", action="store_true",
                    help="run only the 48-lattice batched form and print its record")
    ap.add_argument("--only-rmft-form", action="store_true",
                    help="run only the self-consistent iteration timing and print its JSON (profiling)")
    ap.add_argument("--no-kernel-timing", action="store_true",
                    help="time the steps without per-kernel events (roofline fields omitted)")
    ap.add_argument("--moments", type=int, default=0,
                    help="profiling runs only: override M (same launch shape, fewer steps)")
    ap.add_argument("--probe-block", type=int, default=0,
                    help="probes per wave of the recursion kernels (0 = library default)")
    ap.add_argument("--streams", type=int, default=0, choices=(0, 1, 2),
                    help="kpm_set_streams: 0 automatic (probe halves on two streams for this "
                         "workload), 1 one stream, 2 halves")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="run one plain device-to-device copy of BYTES (counter calibration) and exit")
    ap.add_argument("--traffic-summary", default="", metavar="DIR",
                    help="summarise rocprofv3 FETCH_SIZE/WRITE_SIZE runs under DIR (fetch/ write/ copyf/ "
                         "copyw/) into profiles/k_*_c5_fp32_traffic.json and exit (no GPU needed)")
    args = ap.parse_args()
    if args.traffic_summary:
        traffic_summary(args.traffic_summary, args.copy_calibration or (1 << 30))
        return
    if args.gpus != 1:
        print("bench.py measures one MI355X: multi-GPU runs are not supported (the path would shard "
              "over probes, with one all-reduce of the moments and of rho per step).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as wl

    if args.copy_calibration:
        n = args.copy_calibration // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": 4 * n, "copy_calibration_bytes_written": 4 * n}))
        return

    if args.probe_block:
        from paper_2212_05685_amd import kpm
        kpm.kpm_set_probe_block(args.probe_block)
    if args.streams:
        from paper_2212_05685_amd import kpm
        kpm.kpm_set_streams(args.streams)
    if args.only_batched_form:
        print(json.dumps({"batched_form": batched_form(args.steps)}), flush=True)
        return
    if args.only_rmft_form:
        print(json.dumps({"rmft_form": rmft_form(args.steps, args.warmup)}), flush=True)
        return
    if args.only_supercell_form:
        print(json.dumps({"supercell_form": supercell_form()}), flush=True)
        return
    cfg = wl.C5("fp32")
    if args.moments:
        cfg = wl.scaled(cfg, M=args.moments)
    prob, th = make_problem(cfg, "fp32")
    R, M, N = prob.R, cfg.M, cfg.N
    log(f"workload 100x100 M={M} R={R}; building and warming up")
    dt, per_step, wall_mean, out32, grads32, prof = timed(prob, th, args.steps, args.warmup,
                                                          profile=not args.no_kernel_timing)
    vsteps = R * (M - 1) + 2 * R * (M - 2)
    fwd_ms, n_fwd, adj_ms, n_adj = prof if prof else (float("nan"), 0, float("nan"), 0)
    rec = 16                                    # FP32 complex record of one site (2 components)
    coef_bytes = 36 * 8 * N                     # row-form H~ coefficients, FP32 complex
    adj_bytes = 6 * rec * R * N + coef_bytes     # read a_{m+1}, g_{m+1}, a_{m+2}, g_{m+2}; write a_m, g_m
    fwd_bytes = 3 * rec * R * N + coef_bytes     # read a_m, a_{m-1}; write a_{m+1}
    adj_avg_s = adj_ms / max(n_adj, 1) * 1e-3
    fwd_avg_s = fwd_ms / max(n_fwd, 1) * 1e-3
    achieved = adj_bytes / adj_avg_s / 1e9
    traffic = traffic_record("k_adj")
    if halves_used(R, N, args.streams):
        launch_note = (f"one recursion step of all {R} probes: the launches of the two probe halves "
                       f"({(R + 1) // 2} and {R // 2} probes) that run side by side on two streams; "
                       "timed as runs of 16 consecutive steps on the caller's stream while the other "
                       "half runs beside them, so the average is the time per step of both halves")
    else:
        launch_note = f"one launch over all {R} probes on one stream"

    result = {
        "metric": METRIC,
        "value": vsteps / dt,
        "unit": "vector-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "ms_per_step_timing": f"median of {args.steps} per-step HIP event pairs after {args.warmup} warm-up steps",
        "ms_per_step_wall_mean": wall_mean * 1e3,
        "ms_per_step_events": [round(x * 1e3, 3) for x in per_step],
        "s_per_energy_grad": dt,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "reductions_dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "100x100 torus, 2 vortices + period-8 PDW/CDW seed (0.02), doping 0.125, "
                        "M=4096 Jackson, 256 colored Z4 probes (8x8, Nambu split, 2 draws), "
                        "FP32 recurrence, checkpoints every 64; step = energy + gradient",
            "Lx": cfg.Lx, "Ly": cfg.Ly, "M": M, "R": R, "ckpt_k": cfg.ckpt_k,
            "vector_steps_per_step": vsteps,
        },
        "roofline": {
            "kernel": "k_adj (fused adjoint step)",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "algorithmic_bytes_per_launch": adj_bytes,
            "avg_launch_us": adj_avg_s * 1e6,
            "launches_timed": n_adj,
            "launch": launch_note,
        },
        "forward_kernel": {
            "kernel": "k_fwd (forward step)", "algorithmic_bytes_per_launch": fwd_bytes,
            "avg_launch_us": fwd_avg_s * 1e6, "achieved_GBs": fwd_bytes / fwd_avg_s / 1e9,
            "launches_timed": n_fwd, "launch": launch_note,
        },
        "hbm_GBs_algorithmic_whole_step": ((M - 1) * fwd_bytes + (M - 2) * adj_bytes) / dt / 1e9,
    }

    # per-probe moments of the FP32 path (and its coefficients), for the error
    # against the oracle on the probes the cpu_baseline leg runs
    mu32 = C32 = None
    if not args.no_cpu_baseline and not args.moments:
        n, chi, dlt = th
        h = prob.build_H(n, chi, dlt)
        ab = prob.bounds(h)
        C = prob.coefficients(ab)
        _, mu = prob.grand_potential(h, ab, C, want_mu=True)
        mu32, C32 = mu.cpu().numpy(), C.cpu().numpy()
        w32 = float(cfg.probes[0].weight)

    if not args.no_direct_form and not args.moments:
        result["direct_form"] = direct_form(args.steps, prob, th, dt)
        result["doubling_form"] = doubling_form(args.steps, prob, th)
        result["ldos_form"] = ldos_form(args.steps, prob, th, cfg)
        result["sdw_form"] = sdw_form(50, cfg)
    if not args.no_supercell_form and not args.moments:
        result["supercell_form"] = supercell_form()

    if not args.no_fp64_form:
        del prob
        torch.cuda.empty_cache()
        prob64, th64 = make_problem(wl.C5("fp64"), "fp64")
        dt64, _, _, out64, grads64, _ = timed(prob64, th64, 3, 1, profile=False)
        om32 = float(out32["omega"].item())
        om64 = float(out64["omega"].item())
        r32, r64 = out32["rho"].cpu().numpy(), out64["rho"].cpu().numpy()
        g32, g64 = grads32[1].cpu().numpy(), grads64[1].cpu().numpy()
        result["fp64_form"] = {
            "ms_per_step": dt64 * 1e3,
            "speedup_fp32_over_fp64": dt64 / dt,
            "fp32_vs_fp64_rel_err_omega": abs(om32 - om64) / abs(om64),
            "fp32_vs_fp64_rel_err_rho": float(np.max(np.abs(r32 - r64)) / np.max(np.abs(r64))),
            "fp32_vs_fp64_rel_err_dchi": float(np.max(np.abs(g32 - g64)) / np.max(np.abs(g64))),
        }
        del prob64
        torch.cuda.empty_cache()

    if not args.no_batched_form and not args.moments:
        result["batched_form"] = batched_form(3)
        torch.cuda.empty_cache()

    if not args.no_rmft_form and not args.moments:
        result["rmft_form"] = rmft_form(5, 2)
        torch.cuda.empty_cache()

    if not args.no_cpu_baseline:
        pool = OraclePool(host_workers())
        try:
            result["cpu_baseline"], c5_sample = cpu_baseline(pool)
        finally:
            pool.close()
        if mu32 is not None and c5_sample:
            e_mu = max(float(np.max(np.abs(mu32[q] - mu)) / np.max(np.abs(mu))) for q, (mu, _) in enumerate(c5_sample))
            e_om = max(abs(w32 * float(np.dot(C32, mu32[q])) - om) / abs(om) for q, (_, om) in enumerate(c5_sample))
            result["fp32_vs_oracle"] = {
                "probes": len(c5_sample),
                "moments_max_rel_err": e_mu,
                "omega_term_max_rel_err": e_om,
                "sample": f"the first {len(c5_sample)} of the 256 probes of the 100x100 workload, those the "
                          "cpu_baseline leg runs through the oracle (O2, FP64, its own stencil, bounds and "
                          "coefficients); per probe: max |mu_gpu - mu_oracle| / max |mu_oracle| over the 4096 "
                          "moments, and the probe's term w C.mu of Omega",
                "rho": "rho sums all probes on the GPU and is not compared here; against the oracle at this "
                       "size it is tested in tests/test_gpu_fullsize_oracle.py (FP32 1e-7 with 8 dense probes)",
            }
        result["cpu_dense_ed"] = cpu_dense_ed()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
