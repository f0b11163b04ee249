"""Pins of the direct probing estimate of rho (oracle/kpm_direct.py):

* the derivative coefficients reproduce F_M'(x) of the sine formula
  (oracle.chebyshev.series_derivative) at random points;
* with the complete set of unit vectors it equals the truncated density
  matrix of dense diagonalisation (O1), (1/a) F_M'(H~)^T;
* with colored or random Z4 probes it equals (1/a) [F_M'(H~) P]^T, P the
  weighted probe projector, built from the eigendecomposition (diagonal
  entries as their real part, the stencil layout's convention);
* Omega equals the plain recursion's (O2).
"""
import numpy as np
import pytest

import workloads as wl
from oracle import builder, chebyshev, dense, kpm_direct, kpm_plain
from tests import helpers as H


def _setup(cfg, M):
    st = H.stencil(cfg)
    a, b = H.bounds(cfg, st)
    C = H.coefficients(cfg, a, b, M)
    return st, a, b, C


def test_derivative_coefficients_match_sine_formula():
    rng = np.random.default_rng(3)
    x = rng.uniform(-0.99, 0.99, 50)
    for C in (rng.normal(size=40), chebyshev.kpm_coefficients(128, 0.005, 2.1, 0.3)):
        D = kpm_direct.derivative_coefficients(C)
        assert D[-1] == 0.0
        got = np.cos(np.multiply.outer(np.arccos(x), np.arange(len(D)))) @ D
        ref = chebyshev.series_derivative(C, x)
        assert np.max(np.abs(got - ref)) < 1e-9 * max(1.0, np.max(np.abs(ref)))


def test_unit_probes_equal_truncated_density_matrix():
    cfg = wl.Config("d", 5, 4, 2, 0.13, 64, (wl.ProbeSpec("unit", 40),), vortex=True, complex_noise=0.03)
    st, a, b, C = _setup(cfg, 64)
    R, w = H.probe_matrix(cfg)
    Hs = builder.sparse_from_stencil(st, cfg.Lx, cfg.Ly)
    out = kpm_direct.direct_rho(Hs, a, b, R, w, C, cfg.Lx, cfg.Ly)
    om, rho = H.dense_truncated(cfg, st, a, b, C)
    assert abs(out["omega"] - om) < 1e-11 * abs(om)
    assert H.rel_err(out["rho"], rho) < 1e-11


@pytest.mark.parametrize("probes", [
    (wl.ProbeSpec("colored_z4", 1, 11, 2, 2, 1, 0, 1.0),),
    (wl.ProbeSpec("dense_z4", 6, 12, weight=1 / 6),),
], ids=["colored", "dense"])
def test_probe_estimate_equals_projector_form(probes):
    cfg = wl.Config("d", 6, 4, 2, 0.13, 48, probes, vortex=True, complex_noise=0.03)
    st, a, b, C = _setup(cfg, 48)
    R, w = H.probe_matrix(cfg)
    Hs = builder.sparse_from_stencil(st, cfg.Lx, cfg.Ly)
    out = kpm_direct.direct_rho(Hs, a, b, R, w, C, cfg.Lx, cfg.Ly)
    Hd = builder.dense_from_stencil(st, cfg.Lx, cfg.Ly)
    E, U = dense.eig(Hd)
    dF = chebyshev.series_derivative(C, (E - b) / a)
    Fp = (U * dF[None, :]) @ U.conj().T                     # F_M'(H~)
    P = (R.T * w[None, :]) @ R.conj()                       # sum_l w_l r_l r_l^dag
    ref = builder.stencil_from_dense((Fp @ P).T, cfg.Lx, cfg.Ly) / a
    ref[16], ref[17] = ref[16].real, ref[17].real       # diagonal stored as real
    assert H.rel_err(out["rho"], ref) < 1e-11
    plain = kpm_plain.plain_kpm(Hs, a, b, R, w, C, cfg.Lx, cfg.Ly, want_grad=False)
    assert abs(out["omega"] - plain["omega"]) < 1e-12 * abs(plain["omega"])


def test_moment_doubling_identity():
    """The identities used by kpm_moments_doubling, checked on a random
    Hermitian matrix with spectrum in (-1, 1) through its eigendecomposition:
    r^dag T_{2j} r = 2 |T_j r|^2 - r^dag r and
    r^dag T_{2j+1} r = 2 Re((T_{j+1} r)^dag T_j r) - r^dag T_1 r."""
    rng = np.random.default_rng(9)
    n = 24
    A = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    Hm = (A + A.conj().T) / 2
    E, U = np.linalg.eigh(Hm)
    Hm = Hm / (1.05 * np.max(np.abs(E)))
    E, U = np.linalg.eigh(Hm)
    th = np.arccos(E)
    r = np.exp(0.5j * np.pi * rng.integers(0, 4, n))

    def T(j):
        return (U * np.cos(j * th)[None, :]) @ U.conj().T

    mu = [np.vdot(r, T(m) @ r).real for m in range(20)]
    for j in range(1, 10):
        a_j, a_j1 = T(j) @ r, T(j + 1) @ r
        assert abs(2 * np.vdot(a_j, a_j).real - mu[0] - mu[2 * j]) < 1e-12 * mu[0]
        assert abs(2 * np.vdot(a_j1, a_j).real - mu[1] - mu[2 * j + 1]) < 1e-12 * mu[0]
