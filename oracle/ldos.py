"""O5: local density of states by KPM (oracle; test infrastructure only).

Results (LDOS N_i(omega) of the vortex states) computed with the expansion of
App. B: for a unit probe e_I the moments mu_{I,m} = e_I^dag T_m(H~) e_I give
the spectral density of Nambu index I,

    A_I(E) = [g_0 mu_{I,0} + 2 sum_{m>=1} g_m mu_{I,m} T_m(x)] / (pi a sqrt(1 - x^2)),

x = (E - b)/a, with the Jackson damping g_m (Weisse et al., RMP 78, 275).
A_{(i,0)} is the spin-up electron spectral density of site i; A_{(i,1)}(E)
is the spin-down hole density (the spin-down electron density at -E).

``ldos`` takes the steps in this order: plain recursion moments (O2's
recursion on unit vectors), then the damped series at each energy.
``ldos_from_eigen`` is the same functional from the eigendecomposition,
A_I(E) = sum_n |U_In|^2 delta_M(x, x_n), with the damped kernel
delta_M(x, y) = [g_0 + 2 sum_m g_m T_m(x) T_m(y)] / (pi a sqrt(1 - x^2)).
"""
from __future__ import annotations

import numpy as np

from .chebyshev import jackson
from .kpm_plain import plain_kpm


def series_at(mu, a, b, energies):
    """A(E) for moment rows mu [R, M] at the given energies -> [R, len(E)].
    The expansion lives on the open interval -1 < x < 1 of the rescaled
    spectrum; A is 0 at energies outside it."""
    mu = np.atleast_2d(np.asarray(mu, dtype=np.float64))
    M = mu.shape[1]
    g = jackson(M)
    x = (np.asarray(energies, dtype=np.float64) - b) / a
    inside = np.abs(x) < 1.0
    xi = x[inside]
    Tm = np.cos(np.multiply.outer(np.arange(M), np.arccos(xi)))   # [M, E inside]
    wts = 2.0 * g
    wts[0] = g[0]
    out = np.zeros((mu.shape[0], len(x)))
    out[:, inside] = (mu * wts[None, :]) @ Tm / (np.pi * a * np.sqrt(1.0 - xi ** 2))[None, :]
    return out


def ldos(Hs, a, b, first, count, M, energies, Lx, Ly):
    """A_I(E) for I = first .. first + count - 1 from the recursion moments."""
    D = Hs.shape[0]
    P = np.zeros((count, D), dtype=np.complex128)
    P[np.arange(count), first + np.arange(count)] = 1.0
    C = np.zeros(M)
    out = plain_kpm(Hs, a, b, P, np.ones(count), C, Lx, Ly, want_grad=False)
    return series_at(out["mu"], a, b, energies), out["mu"]


def ldos_from_eigen(H, a, b, first, count, M, energies):
    """The same A_I(E) from the eigendecomposition of the dense h."""
    E, U = np.linalg.eigh(H)
    g = jackson(M)
    xn = np.clip((E - b) / a, -1.0, 1.0)
    x = (np.asarray(energies, dtype=np.float64) - b) / a
    inside = np.abs(x) < 1.0                                   # A is 0 outside the interval
    xi = x[inside]
    m = np.arange(M)
    Tx = np.cos(np.multiply.outer(m, np.arccos(xi)))          # [M, E inside]
    Tn = np.cos(np.multiply.outer(m, np.arccos(xn)))          # [M, n]
    wts = 2.0 * g
    wts[0] = g[0]
    kern = (Tn.T * wts[None, :]) @ Tx                          # [n, E inside]
    w = np.abs(U[first:first + count, :]) ** 2                 # [I, n]
    out = np.zeros((count, len(x)))
    out[:, inside] = (w @ kern) / (np.pi * a * np.sqrt(1.0 - xi ** 2))[None, :]
    return out
