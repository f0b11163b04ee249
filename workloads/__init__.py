"""Seeded synthetic inputs for the KPM path (shared by the oracle tests, the GPU
tests and the benchmark).

This module holds input construction only -- lattice sizes, order-parameter
maps, probe specifications and seeds -- and none of the method's arithmetic
(no Hamiltonian, no Chebyshev algebra, no probe phases).

The paper's self-consistent order-parameter maps are not available, so seeded
ansatz maps stand in for them, with the paper's shapes (Model and methods and
Results): square torus, t'/t = -0.3, J/t = 0.3, d-wave bond pairing,
two superconducting vortices half a lattice apart in y with a tanh core of
radius 3 lattice constants, hole doping 0.05-0.25, and an optional period-8
checkerboard pair/charge-density modulation.

Recipe (every config):
* chi = chi0 (default 0.2) on nearest-neighbour bonds, 0 on next-nearest-
  neighbour bonds.  A real chi does not carry the Peierls phases of a field,
  so with a field the self-consistent runs seed chi0 = 0 and let the first
  density matrix supply the bond phases;
* Delta = +0.1 on x bonds, -0.1 on y bonds, 0 on diagonal bonds;
* n_i = 1 - delta (m_i = 0);
* ``noise``: uniform(-noise, noise) real noise per nn bond on chi and Delta and
  per site on n; ``complex_noise``: complex noise on every direction instead;
* ``vortex``: Delta_ij *= prod_v tanh(|r_ij - R_v| / core) exp(i sum_v arg(r_ij - R_v))
  with r_ij the bond midpoint, minimum-image displacement, R_v as in
  ``vortex_centres`` and core = 3 unless a config sets it;
* ``pdw``: Delta_ij += pdw * eta_ij [cos(2 pi x_ij / 8) + cos(2 pi y_ij / 8)]
  (eta = +1 on x bonds, -1 on y bonds), and delta_i += pdw [cos(2 pi x_i/8) +
  cos(2 pi y_i/8)], applied before the vortex factor;
* mu: the chemical potential giving the target doping in the uniform
  zero-field state, read from ``mu_table.json`` (written by
  ``oracle/gen_mu_table.py``) and linearly interpolated.
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass, field, replace
from typing import List, Tuple

import numpy as np

DIRS = ((1, 0), (0, 1), (1, 1), (1, -1))   # +x, +y, +x+y, +x-y
T_HOP, TP_HOP, J_EX, TEMP = 1.0, -0.3, 0.3, 0.005
BASE_SEED = 20221205


@dataclass(frozen=True)
class ProbeSpec:
    kind: str                # "unit" | "dense_z4" | "colored_z4"
    count: int               # unit/dense: vectors; colored: draws
    seed: int = 0
    px: int = 1
    py: int = 1
    split_nambu: int = 0
    first: int = 0
    weight: float = 1.0

    def nprobes(self) -> int:
        if self.kind == "colored_z4":
            return self.count * self.px * self.py * (2 if self.split_nambu else 1)
        return self.count


@dataclass(frozen=True)
class Config:
    name: str
    Lx: int
    Ly: int
    n_v: int
    doping: float
    M: int
    probes: Tuple[ProbeSpec, ...]
    precision: str = "fp64"      # "fp64" | "fp32"
    ckpt_k: int = 64
    seed: int = BASE_SEED
    noise: float = 0.0
    complex_noise: float = 0.0
    vortex: bool = False
    pdw: float = 0.0
    T: float = TEMP
    t: float = T_HOP
    tp: float = TP_HOP
    J: float = J_EX
    chi0: float = 0.2            # seed chi on nearest-neighbour bonds
    core: float = 3.0            # tanh radius of the vortex seed (lattice constants)
    vortex_dx: float = 0.0       # shift of the seeded vortex centres along x (lattice constants)

    @property
    def N(self) -> int:
        return self.Lx * self.Ly

    @property
    def R(self) -> int:
        return sum(p.nprobes() for p in self.probes)

    @property
    def mu(self) -> float:
        return mu_for(self.doping)


_MU_TABLE = None


def mu_for(doping: float) -> float:
    global _MU_TABLE
    if _MU_TABLE is None:
        with open(os.path.join(os.path.dirname(__file__), "mu_table.json")) as fh:
            _MU_TABLE = json.load(fh)
    d = np.array(_MU_TABLE["doping"])
    m = np.array(_MU_TABLE["mu"])
    if not (d[0] - 1e-12 <= doping <= d[-1] + 1e-12):
        raise ValueError("doping outside the tabulated range")
    return float(np.interp(doping, d, m))


def vortex_centres(Lx: int, Ly: int, n_v: int) -> List[Tuple[float, float]]:
    if n_v == 0:
        return []
    if n_v == 2:   # one vortex per superconducting flux quantum, half a lattice apart in y
        return [(Lx / 2 - 1, Ly / 4 - 1), (Lx / 2 - 1, 3 * Ly / 4 - 1)]
    if n_v == 4:
        return [(Lx / 4 - 1, Ly / 4 - 1), (3 * Lx / 4 - 1, Ly / 4 - 1),
                (Lx / 4 - 1, 3 * Ly / 4 - 1), (3 * Lx / 4 - 1, 3 * Ly / 4 - 1)]
    raise ValueError("vortex seeds are defined for n_v in {0, 2, 4}")


def _min_image(d, L):
    return (d + L / 2) % L - L / 2


def make_theta(cfg: Config):
    """(n[N] float64, chi[4,N] complex128, delta[4,N] complex128)."""
    Lx, Ly, N = cfg.Lx, cfg.Ly, cfg.N
    rng = np.random.default_rng(cfg.seed)
    x = np.arange(N) % Lx
    y = np.arange(N) // Lx
    n = np.full(N, 1.0 - cfg.doping)
    chi = np.zeros((4, N), dtype=np.complex128)
    dlt = np.zeros((4, N), dtype=np.complex128)
    chi[0] = chi[1] = cfg.chi0
    dlt[0] = 0.1
    dlt[1] = -0.1
    if cfg.noise:
        chi[:2] += rng.uniform(-cfg.noise, cfg.noise, size=(2, N))
        dlt[:2] += rng.uniform(-cfg.noise, cfg.noise, size=(2, N))
        n += rng.uniform(-cfg.noise, cfg.noise, size=N)
    if cfg.complex_noise:
        a = cfg.complex_noise
        chi += rng.uniform(-a, a, size=(4, N)) + 1j * rng.uniform(-a, a, size=(4, N))
        dlt[:2] += rng.uniform(-a, a, size=(2, N)) + 1j * rng.uniform(-a, a, size=(2, N))
    if cfg.pdw:
        k = 2 * np.pi / 8
        for d in range(2):
            dx, dy = DIRS[d]
            xm, ym = x + 0.5 * dx, y + 0.5 * dy
            eta = 1.0 if d == 0 else -1.0
            dlt[d] += cfg.pdw * eta * (np.cos(k * xm) + np.cos(k * ym))
        n -= cfg.pdw * (np.cos(k * x) + np.cos(k * y))
    if cfg.vortex:
        for d in range(2):
            dx, dy = DIRS[d]
            xm, ym = x + 0.5 * dx, y + 0.5 * dy
            amp = np.ones(N)
            phase = np.zeros(N)
            for (X, Y) in vortex_centres(Lx, Ly, cfg.n_v):
                ux, uy = _min_image(xm - X - cfg.vortex_dx, Lx), _min_image(ym - Y, Ly)
                amp *= np.tanh(np.hypot(ux, uy) / cfg.core)
                phase += np.arctan2(uy, ux)
            dlt[d] *= amp * np.exp(1j * phase)
    return n, chi, dlt


def make_theta_sdw(cfg: Config, m_amp: float = 0.03, spin_noise: float = 0.01):
    """Per-spin inputs of a collinear SDW state: the seed of ``make_theta``
    with a staggered magnetisation m_i = m_amp (-1)^(x+y) (1 + 0.2 u_i), u_i
    uniform in [-1, 1], split as n_up/dn = n/2 +- m_i, and seeded complex
    spin-dependent noise of amplitude spin_noise on chi and Delta.
    Returns (n_up, n_dn, chi_up, chi_dn, delta_up, delta_dn)."""
    n, chi, dlt = make_theta(cfg)
    rng = np.random.default_rng(cfg.seed + 77)
    N = cfg.N
    x = np.arange(N) % cfg.Lx
    y = np.arange(N) // cfg.Lx
    m = m_amp * np.where((x + y) % 2 == 0, 1.0, -1.0) * (1.0 + 0.2 * rng.uniform(-1, 1, N))

    def noise():
        a = spin_noise
        return rng.uniform(-a, a, (4, N)) + 1j * rng.uniform(-a, a, (4, N))

    mask = np.array([1.0, 1.0, 0.0, 0.0])[:, None]
    return (n / 2 + m, n / 2 - m, chi + noise(), chi + noise(), dlt + mask * noise(), dlt + mask * noise())


def _seed(idx: int) -> int:
    return BASE_SEED + idx


def C1() -> Config:
    s = _seed(1)
    return Config("C1_8x8_fp64", 8, 8, 0, 0.125, 256,
                  (ProbeSpec("unit", 128, s),), "fp64", seed=s, noise=0.01)


def C2(precision="fp32") -> Config:
    s = _seed(2)
    return Config("C2_32x32_vortex", 32, 32, 2, 0.125, 1024,
                  (ProbeSpec("unit", 2048, s),), precision, seed=s, vortex=True)


def C3() -> Config:
    s = _seed(3)
    return Config("C3_64x64_vortex_fp64", 64, 64, 2, 0.15, 2048,
                  (ProbeSpec("colored_z4", 1, s, 8, 8, 0, 0, 0.5),
                   ProbeSpec("dense_z4", 128, s + 1000, weight=0.5 / 128)),
                  "fp64", seed=s, vortex=True)


def C4_instances(n_inst: int = 48) -> List[Config]:
    s = _seed(4)
    rng = np.random.default_rng(s)
    Ls = rng.choice([24, 32, 40, 48, 56, 64], size=n_inst)
    dop = rng.uniform(0.05, 0.25, size=n_inst)
    nvs = rng.choice([2, 4], size=n_inst)
    out = []
    for k in range(n_inst):
        sk = s * 1000 + k
        out.append(Config(f"C4_{k}_{Ls[k]}x{Ls[k]}", int(Ls[k]), int(Ls[k]), int(nvs[k]),
                          float(dop[k]), 1024, (ProbeSpec("colored_z4", 1, sk, 8, 8, 0, 0, 1.0),),
                          "fp32", seed=sk, vortex=True))
    return out


def C5(precision="fp32") -> Config:
    s = _seed(5)
    return Config("C5_100x100_vortex_pdw", 100, 100, 2, 0.125, 4096,
                  (ProbeSpec("colored_z4", 2, s, 8, 8, 1, 0, 0.5),),
                  precision, ckpt_k=64, seed=s, vortex=True, pdw=0.02)


def RMFT(precision="fp32") -> Config:
    """Plain-vortex self-consistency workload of the Results section: 48 x 96
    torus, two vortices half the lattice apart in y, mean hole density 0.16,
    M = 1024 (paper range 1000-2000), 128 colored probes (range 64-144)."""
    s = _seed(6)
    return Config("RMFT_48x96_plain_vortex", 48, 96, 2, 0.16, 1024,
                  (ProbeSpec("colored_z4", 1, s, 8, 8, 1, 0, 1.0),),
                  precision, ckpt_k=64, seed=s, vortex=True, chi0=0.0)


def random_stencil(N: int, seed: int, scale: float = 0.5):
    """Seeded complex [19, N] array of stencil entries, uniform in
    [-scale, scale] for both parts (a stand-in density matrix for tests of the
    order-parameter map)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-scale, scale, (19, N)) + 1j * rng.uniform(-scale, scale, (19, N))


def scaled(cfg: Config, **kw) -> Config:
    """A copy with some fields replaced (smaller test variants of a config)."""
    return replace(cfg, **kw)
