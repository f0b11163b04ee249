"""Shared test helpers: turn a ``workloads.Config`` into oracle inputs and
oracle results (CPU, FP64).  GPU-side conversions live in ``gpu_helpers``.
"""
from __future__ import annotations

import functools

import numpy as np

import workloads as wl
from oracle import builder, chebyshev, dense, kpm_plain, mapping, probes

KIND = {"unit": probes.UNIT, "dense_z4": probes.DENSE_Z4, "colored_z4": probes.COLORED_Z4}


def oracle_groups(cfg: wl.Config):
    return [probes.ProbeGroup(KIND[p.kind], p.count, p.seed, p.px, p.py, p.split_nambu, p.first, p.weight)
            for p in cfg.probes]


def theta(cfg: wl.Config):
    return wl.make_theta(cfg)


def stencil(cfg: wl.Config, th=None):
    n, chi, dlt = theta(cfg) if th is None else th
    return builder.build_stencil(cfg.Lx, cfg.Ly, cfg.n_v, cfg.t, cfg.tp, cfg.J, cfg.mu, n, chi, dlt)


def bounds(cfg: wl.Config, st):
    Hs = builder.sparse_from_stencil(st, cfg.Lx, cfg.Ly)
    return chebyshev.rescale(*chebyshev.gershgorin_sparse(Hs))


def coefficients(cfg: wl.Config, a, b, M=None):
    return chebyshev.kpm_coefficients(cfg.M if M is None else M, cfg.T, a, b)


def oracle_inputs(cfg: wl.Config, M=None):
    """Stencil, rescaling (a, b) and coefficients, all computed by the oracle."""
    st = stencil(cfg)
    a, b = bounds(cfg, st)
    return st, a, b, coefficients(cfg, a, b, M)


def probe_matrix(cfg: wl.Config):
    return probes.probe_set(oracle_groups(cfg), cfg.Lx, cfg.Ly)


def plain(cfg: wl.Config, st, a, b, C, want_grad=True, subset=None):
    """O2 on the config's probes (or a subset of probe indices)."""
    R, w = probe_matrix(cfg)
    if subset is not None:
        R, w = R[subset], w[subset]
    Hs = builder.sparse_from_stencil(st, cfg.Lx, cfg.Ly)
    return kpm_plain.plain_kpm(Hs, a, b, R, w, C, cfg.Lx, cfg.Ly, want_grad=want_grad)


def dense_truncated(cfg: wl.Config, st, a, b, C):
    H = builder.dense_from_stencil(st, cfg.Lx, cfg.Ly)
    om, rho = dense.truncated(H, C, a, b)
    return om, builder.stencil_from_dense(rho, cfg.Lx, cfg.Ly)


def rel_err(x, ref):
    x = np.asarray(x)
    ref = np.asarray(ref)
    return float(np.max(np.abs(x - ref)) / max(np.max(np.abs(ref)), 1e-300))


def _plain_part(args):
    """One worker's share of O2 (a contiguous group of probes), one thread."""
    from threadpoolctl import threadpool_limits
    Hs, a, b, R, w, C, Lx, Ly, want_grad = args
    with threadpool_limits(1):
        return kpm_plain.plain_kpm(Hs, a, b, R, w, C, Lx, Ly, want_grad=want_grad)


def plain_parallel(cfg: wl.Config, st, a, b, C, subset=None, want_grad=True, workers=None,
                   timeout=600):
    """O2 on the config's probes (or a subset), one probe per task in a pool of
    single-threaded processes (spawned: the parent may hold a GPU context); the
    per-probe results are summed in probe order.  For the full-size parity
    cases, where one probe of the 100 x 100 workload takes seconds.  Raises
    multiprocessing.TimeoutError after `timeout` seconds (the pool is then
    terminated)."""
    import os
    from multiprocessing import get_context

    R, w = probe_matrix(cfg)
    if subset is not None:
        R, w = R[subset], w[subset]
    Hs = builder.sparse_from_stencil(st, cfg.Lx, cfg.Ly)
    n = R.shape[0]
    workers = workers or max(1, min(16, os.cpu_count() or 1, n))
    tasks = [(Hs, a, b, R[q:q + 1], w[q:q + 1], C, cfg.Lx, cfg.Ly, want_grad) for q in range(n)]
    with get_context("spawn").Pool(workers) as pool:
        parts = pool.map_async(_plain_part, tasks, chunksize=1).get(timeout)
    out = {"mu": np.concatenate([p["mu"] for p in parts]),
           "mu_imag": np.concatenate([p["mu_imag"] for p in parts]),
           "omega": float(sum(p["omega"] for p in parts))}
    if want_grad:
        rho = np.zeros_like(parts[0]["rho"])
        for p in parts:
            rho += p["rho"]
        out["rho"] = rho
    return out
