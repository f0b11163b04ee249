"""GPU-side helpers for the parity tests: config -> torch device tensors and a
``KPMProblem`` of the library binding."""
from __future__ import annotations

import numpy as np
import torch

import workloads as wl

KIND = {"unit": 0, "dense_z4": 1, "colored_z4": 2}


def problem(cfg: wl.Config, precision=None, M=None, ckpt_k=None, probes=None):
    from paper_2212_05685_amd import kpm
    from paper_2212_05685_amd.solver import KPMProblem

    prec = {"fp64": kpm.KPM_FP64, "fp32": kpm.KPM_FP32}[precision or cfg.precision]
    specs = [kpm.ProbeSpec(KIND[p.kind], p.count, p.seed, p.px, p.py, p.split_nambu, p.first, p.weight)
             for p in (probes or cfg.probes)]
    return KPMProblem(cfg.Lx, cfg.Ly, cfg.n_v, cfg.t, cfg.tp, cfg.J, cfg.mu, cfg.T,
                      M or cfg.M, specs, prec, ckpt_k or cfg.ckpt_k)


def dev(x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def theta_dev(cfg: wl.Config):
    n, chi, dlt = wl.make_theta(cfg)
    return dev(n, torch.float64), dev(chi, torch.complex128), dev(dlt, torch.complex128)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()
