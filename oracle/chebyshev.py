"""Spectral rescale, Jackson damping and Fermi-function Chebyshev coefficients.

Paper App. B: the Chebyshev expansion needs every eigenvalue inside [-1, 1],
reached by shifting and rescaling h; damping factors g_m suppress Gibbs
oscillations; the energy is E = sum_{m<M} C_m mu_m with
C_m = (2 - delta_{m0}) g_m int_{-1}^{1} T_m(e) f(e) / (pi sqrt(1 - e^2)) de,
evaluated by Chebyshev-Gauss quadrature, and f(e) = -T log(1 + e^{-(e - mu)/T}).

Readings (the paper fixes none of these):
* rescale: Gershgorin bounds Emin/Emax of h, a = (Emax - Emin)/(2 - 0.01),
  b = (Emax + Emin)/2, H~ = (h - b)/a; (a, b) are constants for derivatives.
* damping: the Jackson kernel of Weisse et al., Rev. Mod. Phys. 78, 275 (2006)
  (the paper's KPM reference), closed form
  g_m = [(M - m + 1) cos(pi m/(M+1)) + sin(pi m/(M+1)) cot(pi/(M+1))] / (M+1).
* the chemical potential already sits on the diagonal of h, so f uses mu = 0
  and is the grand-potential density, f(e) = min(e, 0) - T log1p(e^{-|e|/T}).
* quadrature: K = max(4M, 2^14) Chebyshev-Gauss nodes theta_k = pi (k + 1/2)/K,
  c_m = (1/K) sum_k cos(m theta_k) F(cos theta_k), F(x) = f(a x + b).
"""
from __future__ import annotations

import numpy as np


def gershgorin(H: np.ndarray):
    """(Emin, Emax) Gershgorin bounds of a dense Hermitian matrix."""
    d = np.real(np.diag(H))
    off = np.abs(H).sum(axis=1) - np.abs(np.diag(H))
    return float(np.min(d - off)), float(np.max(d + off))


def gershgorin_sparse(Hs):
    """Same bounds for a scipy sparse matrix."""
    d = np.real(Hs.diagonal())
    off = np.asarray(abs(Hs).sum(axis=1)).ravel() - np.abs(Hs.diagonal())
    return float(np.min(d - off)), float(np.max(d + off))


def rescale(Emin: float, Emax: float, pad: float = 0.01):
    a = (Emax - Emin) / (2.0 - pad)
    b = (Emax + Emin) / 2.0
    return a, b


def jackson(M: int) -> np.ndarray:
    m = np.arange(M, dtype=np.float64)
    q = np.pi / (M + 1)
    return ((M - m + 1) * np.cos(q * m) + np.sin(q * m) / np.tan(q)) / (M + 1)


def fermi_energy_density(e, T):
    """f(e) = -T log(1 + exp(-e/T)), written without overflow."""
    e = np.asarray(e, dtype=np.float64)
    return np.minimum(e, 0.0) - T * np.log1p(np.exp(-np.abs(e) / T))


def fermi_occupation(e, T):
    """n_F(e) = 1/(1 + exp(e/T)) = f'(e), written without overflow."""
    e = np.asarray(e, dtype=np.float64)
    z = np.exp(-np.abs(e) / T)
    return np.where(e > 0, z / (1.0 + z), 1.0 / (1.0 + z))


def quad_nodes(M: int, K: int | None = None) -> int:
    return max(4 * M, 1 << 14) if K is None else K


def cheb_moments_of(F, M: int, K: int) -> np.ndarray:
    """c_m = (1/K) sum_k cos(m theta_k) F(cos theta_k), m < M, by direct sums."""
    th = np.pi * (np.arange(K) + 0.5) / K
    Fk = F(np.cos(th))
    c = np.empty(M)
    step = max(1, (1 << 22) // K)
    for m0 in range(0, M, step):
        ms = np.arange(m0, min(M, m0 + step))
        c[ms] = np.cos(np.outer(ms, th)) @ Fk / K
    return c


def kpm_coefficients(M: int, T: float, a: float, b: float, K: int | None = None,
                     damping: bool = True) -> np.ndarray:
    """C_m = (2 - delta_m0) g_m c_m for the grand-potential density f(a x + b)."""
    K = quad_nodes(M, K)
    c = cheb_moments_of(lambda x: fermi_energy_density(a * x + b, T), M, K)
    g = jackson(M) if damping else np.ones(M)
    C = 2.0 * g * c
    C[0] = g[0] * c[0]
    return C


def series(C: np.ndarray, x):
    """F_M(x) = sum_m C_m T_m(x) for |x| <= 1 (T_m(cos t) = cos(m t))."""
    th = np.arccos(np.clip(np.asarray(x, dtype=np.float64), -1.0, 1.0))
    m = np.arange(len(C))
    return np.cos(np.multiply.outer(th, m)) @ C


def series_derivative(C: np.ndarray, x):
    """F_M'(x) = sum_m C_m m U_{m-1}(x), U_{m-1}(cos t) = sin(m t)/sin(t)."""
    th = np.arccos(np.clip(np.asarray(x, dtype=np.float64), -1.0, 1.0))
    m = np.arange(len(C))
    s = np.sin(th)
    return (np.sin(np.multiply.outer(th, m)) * m) @ C / s
