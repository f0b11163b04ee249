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
