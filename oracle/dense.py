"""O1: dense diagonalisation references (oracle; test infrastructure only).

Paper App. B: rho_IJ = <d^dag_I d_J> = dE/dh_IJ, with E the grand potential of
the quadratic TB-BdG Hamiltonian, E = int rho(e) f(e) de = sum_n f(E_n).

* exact(): the target the expansion approximates,
    Omega* = sum_n f(E_n),
    rho*_IJ = sum_n n_F(E_n) conj(U_In) U_Jn = [U n_F U^dag]_JI,  n_F = f'.
* truncated(): the same functional with f replaced by the damped Chebyshev
  series F_M(x) = sum_m C_m T_m(x) of f(a x + b) -- exactly what the
  recursion of App. B computes when the trace is exact:
    Omega_M = sum_n F_M(x_n),  rho_M = conj(U diag(F_M'(x_n)) U^dag) / a,
  x_n = (E_n - b)/a.
* probe_estimator_grad(): the derivative of the probe estimator
  Omega_P = sum_l w_l r_l^dag F_M(H~) r_l = Tr(P F_M(H~)), P = sum_l w_l r_l r_l^dag,
  by the Daleckii-Krein formula: with S = U^dag P U and divided differences
  Gamma_nk = (F_M(x_n) - F_M(x_k))/(x_n - x_k) (F_M'(x_n) on the diagonal),
    dOmega_P/dH~_IJ = [conj(U) (Gamma o S^T) U^T]_IJ.
These use LAPACK eigh only; they share nothing with the recursion of O2.
"""
from __future__ import annotations

import numpy as np

from .chebyshev import fermi_energy_density, fermi_occupation, series, series_derivative


def eig(H: np.ndarray):
    E, U = np.linalg.eigh(H)
    return E, U


def exact(H: np.ndarray, T: float, E=None, U=None):
    if E is None:
        E, U = eig(H)
    omega = float(np.sum(fermi_energy_density(E, T)))
    nf = fermi_occupation(E, T)
    rho = ((U * nf[None, :]) @ U.conj().T).T
    return omega, rho


def truncated(H: np.ndarray, C: np.ndarray, a: float, b: float, E=None, U=None):
    if E is None:
        E, U = eig(H)
    x = (E - b) / a
    omega = float(np.sum(series(C, x)))
    dF = series_derivative(C, x)
    rho = np.conj((U * dF[None, :]) @ U.conj().T) / a
    return omega, rho


def exact_trace_moments(H: np.ndarray, M: int, a: float, b: float, E=None):
    """mu_m = Tr T_m(H~) = sum_n cos(m arccos x_n)."""
    if E is None:
        E = np.linalg.eigvalsh(H)
    th = np.arccos(np.clip((E - b) / a, -1.0, 1.0))
    return np.cos(np.multiply.outer(np.arange(M), th)).sum(axis=1)


def probe_estimator(H, C, a, b, probes, weights, E=None, U=None):
    """(Omega_P, dOmega_P/dh dense) for the probe estimator, by Daleckii-Krein."""
    if E is None:
        E, U = eig(H)
    x = (E - b) / a
    F = series(C, x)
    dF = series_derivative(C, x)
    P = (probes.T * weights[None, :]) @ probes.conj()      # sum_l w r r^dag
    omega = float(np.real(np.trace(P @ ((U * F[None, :]) @ U.conj().T))))
    S = U.conj().T @ P @ U
    Gam = divided_differences(C, x)
    G = np.conj(U) @ (Gam * S.T) @ U.T
    return omega, G / a


def divided_differences(C: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Gamma_nk = (F_M(x_n) - F_M(x_k)) / (x_n - x_k), F_M' on the diagonal.

    Well-separated pairs use the quotient directly.  Close pairs (where the
    quotient cancels) use the exact identity, with x = cos(theta),
    s = (theta_n + theta_k)/2, t = (theta_n - theta_k)/2:
        (cos m theta_n - cos m theta_k)/(cos theta_n - cos theta_k)
            = [sin(m s)/sin s] [sin(m t)/sin t],
    which has no cancellation as t -> 0 (the second factor tends to m).
    """
    F = series(C, x)
    dx = np.subtract.outer(x, x)
    close = np.abs(dx) < 1e-4
    with np.errstate(divide="ignore", invalid="ignore"):
        Gam = np.where(close, 0.0, np.subtract.outer(F, F) / np.where(close, 1.0, dx))
    th = np.arccos(np.clip(x, -1.0, 1.0))
    n_idx, k_idx = np.nonzero(close)
    s = 0.5 * (th[n_idx] + th[k_idx])
    t = 0.5 * (th[n_idx] - th[k_idx])
    val = np.zeros(len(n_idx))
    for m in range(1, len(C)):
        st = np.sin(m * t)
        ratio_t = np.where(t == 0.0, float(m), st / np.where(t == 0.0, 1.0, np.sin(t)))
        val += C[m] * (np.sin(m * s) / np.sin(s)) * ratio_t
    Gam[n_idx, k_idx] = val
    return Gam
