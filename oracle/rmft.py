"""Self-consistent RMFT iteration (oracle; test infrastructure only).

Model and methods: the site and bond parameters theta = (n_i, chi_ij, Delta_ij)
that define the effective TB-BdG matrix are themselves the local order
parameters (eqs. delta, chi, pairing) of that matrix's ground state, so they
are found by iterating theta -> h(theta) -> rho -> theta' until they stop
changing.  App. A: the electron number is held fixed by the Lagrange multiplier
mu of W.  The paper gives neither the update rule nor the way mu is found; the
readings used here, step by step:

1. map (spin-singlet theta): n' = n_up + n_dn, chi' = (chi_up + chi_dn)/2,
   Delta' = (Delta_up + Delta_dn)/2 with the per-spin order parameters of
   ``mapping.order_parameters``; for a singlet state the two spin estimates of
   chi and of Delta are the same quantity;
2. residual = largest |theta' - theta| over n and every chi, Delta entry
   (complex moduli), density nbar = (1/N) sum_i n'_i;
3. mu at fixed theta: e(mu) = nbar(mu) - (1 - doping).  Accept the first
   evaluation with |e| <= tol_n.  Otherwise walk away from the start on the
   side that e(mu_0) points to (up for e < 0, down for e > 0) with steps
   mu_step, 2 mu_step, 4 mu_step, ... until e changes sign, then halve the
   bracket; a midpoint is accepted when |e| <= tol_n or the half-width of the
   bracket it splits is <= tol_mu.  Alternatively (search = "illinois") the
   bracket [a, b], b the newest point, is narrowed by false position,
   m = b - e_b (b - a)/(e_b - e_a), with the Illinois modification (Dowell and
   Jarratt, BIT 11, 168 (1971)): if e(m) has the sign of e_b the kept end's
   value e_a is halved, otherwise a takes b's place; b <- m; accepted when
   |e| <= tol_n or |b - a| <= tol_mu;
4. theta <- theta + mix (theta' - theta) with the rho of the accepted mu; or,
   with anderson = m > 0, Anderson mixing (Anderson, J. ACM 12, 547 (1965);
   in the form of Walker and Ni, SIAM J. Numer. Anal. 49, 1715 (2011)) on the
   flat vector x = (n, Re/Im chi, Re/Im Delta) with residual f = x' - x: with
   the differences dF_j, dX_j of the last min(k, m) iterations,
   gamma = argmin |f - dF gamma| (normal equations, with a Tikhonov shift of
   1e-12 times the largest diagonal entry), x <- x + mix f - sum_j gamma_j
   (dX_j + mix dF_j); the first iteration of a call, and any iteration whose
   differences are all zero, is a linear step.

A spin-polarised theta (six arrays: n_up, n_dn, chi_up, chi_dn, Delta_up,
Delta_dn, for the builder of ``sdw``) takes the same steps with the per-spin map
of ``sdw.order_parameters_sdw`` in place of step 1 (no spin average), the
mean density from n_up + n_dn.

``rho_fn(theta, mu) -> (omega, rho)`` supplies the density matrix: the plain
KPM of ``kpm_plain`` (the path's own truncation and probes; the adjoint), the
direct probing estimate of ``kpm_direct``, or the exact dense Fermi-function
result of ``dense`` (no truncation).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import builder, chebyshev, dense, kpm_direct, kpm_plain, mapping, sdw


class NoConvergence(RuntimeError):
    """The mu search used its evaluation budget without accepting."""


class NonFinite(FloatingPointError):
    """An evaluation produced a non-finite density (e.g. a site density at or
    above one, where the Gutzwiller factors are undefined)."""


@dataclass(frozen=True)
class Params:
    doping: float
    mix: float = 0.5
    tol_n: float = 1e-6
    tol_mu: float = 1e-10
    mu_step: float = 0.02
    tol_residual: float = 0.0
    max_evals: int = 60
    coef_K: int | None = None
    search: str = "bisection"      # or "illinois"
    anderson: int = 0              # history depth of Anderson mixing (0: linear mixing)


def singlet_theta(rho):
    """Step 1: (n', chi', Delta') from the [19, N] density-matrix stencil."""
    op = mapping.order_parameters(rho)
    n = op["n_up"] + op["n_dn"]
    chi = 0.5 * (op["chi_up"] + op["chi_dn"])
    dlt = 0.5 * (op["delta_up"] + op["delta_dn"])
    return n, chi, dlt


def spin_theta(rho):
    """Step 1 for a spin-polarised theta: the per-spin order parameters."""
    op = sdw.order_parameters_sdw(rho)
    return (op["n_up"], op["n_dn"], op["chi_up"], op["chi_dn"], op["delta_up"], op["delta_dn"])


def mapped(rho, theta):
    return spin_theta(rho) if len(theta) == 6 else singlet_theta(rho)


def measure(rho, theta):
    """Step 2: (nbar, residual) of rho against the current theta."""
    new = mapped(rho, theta)
    res = max(np.max(np.abs(a - b)) for a, b in zip(new, theta))
    nbar = np.mean(new[0] + new[1]) if len(theta) == 6 else np.mean(new[0])
    return float(nbar), float(res)


def update(rho, theta, mix):
    """Step 4: theta + mix (theta' - theta), with (nbar, residual) of step 2."""
    new = mapped(rho, theta)
    nbar, res = measure(rho, theta)
    return tuple(a + mix * (b - a) for a, b in zip(theta, new)), nbar, res


def pack(theta):
    """Flat real vector of theta's arrays in order (real arrays as they are,
    complex ones as interleaved re/im): (n, chi, Delta) or (n_up, n_dn,
    chi_up, chi_dn, Delta_up, Delta_dn)."""
    parts = []
    for a in theta:
        a = np.asarray(a)
        parts.append(np.ascontiguousarray(a, dtype=np.complex128).ravel().view(np.float64)
                     if np.iscomplexobj(a) else np.asarray(a, dtype=np.float64).ravel())
    return np.concatenate(parts)


def unpack(x, N, spin=False):
    nreal = 2 if spin else 1
    out, o = [], 0
    for _ in range(nreal):
        out.append(x[o:o + N].copy())
        o += N
    for _ in range(4 if spin else 2):
        out.append(x[o:o + 8 * N].copy().view(np.complex128).reshape(4, N))
        o += 8 * N
    return tuple(out)


class Anderson:
    """Step 4 with history depth m (see the module docstring)."""

    def __init__(self, m, mix):
        self.m, self.mix = m, mix
        self.dF, self.dX = [], []
        self.f_prev = self.x_prev = None

    def step(self, x, f):
        if self.f_prev is not None:
            self.dF.append(f - self.f_prev)
            self.dX.append(x - self.x_prev)
            if len(self.dF) > self.m:
                self.dF.pop(0)
                self.dX.pop(0)
        self.f_prev, self.x_prev = f, x
        new = x + self.mix * f
        if self.dF:
            F = np.stack(self.dF, axis=1)
            G = F.T @ F
            if not np.max(np.diag(G)) > 0.0:      # an all-zero history: the linear step
                return new
            G = G + 1e-12 * np.max(np.diag(G)) * np.eye(len(self.dF))
            gamma = np.linalg.solve(G, F.T @ f)
            for j, g in enumerate(gamma):
                new = new - g * (self.dX[j] + self.mix * self.dF[j])
        return new


def solve_mu(e_fn, mu0, prm: Params):
    """Step 3.  e_fn(mu) -> (e, payload).  Returns (mu, payload, evaluations)."""
    def ev(m):
        e, pay = e_fn(m)
        if not np.isfinite(e):
            raise NonFinite(f"mean density not finite at mu = {m}")
        return e, pay

    evals = 1
    e0, pay = ev(mu0)
    if abs(e0) <= prm.tol_n:
        return mu0, pay, evals
    below = e0 < 0.0
    direction = 1.0 if below else -1.0
    a, ea, s = mu0, e0, prm.mu_step
    while True:                       # bracket: walk with doubling steps
        if evals >= prm.max_evals:
            raise NoConvergence(f"mu search: {evals} evaluations")
        m = a + direction * s
        e, pay = ev(m)
        evals += 1
        if abs(e) <= prm.tol_n:
            return m, pay, evals
        if (e < 0.0) == below:
            a, ea, s = m, e, 2.0 * s
        else:
            b, eb = m, e
            break
    if prm.search == "illinois":
        while True:
            if evals >= prm.max_evals:
                raise NoConvergence(f"mu search: {evals} evaluations")
            m = b - eb * (b - a) / (eb - ea)
            e, pay = ev(m)
            evals += 1
            if (e < 0.0) != (eb < 0.0):
                a, ea = b, eb
            else:
                ea = 0.5 * ea
            b, eb = m, e
            if abs(e) <= prm.tol_n or abs(b - a) <= prm.tol_mu:
                return m, pay, evals
    if prm.search != "bisection":
        raise ValueError(f"unknown search {prm.search!r}")
    while True:                       # bisection of [a, b]
        if evals >= prm.max_evals:
            raise NoConvergence(f"mu search: {evals} evaluations")
        m = 0.5 * (a + b)
        e, pay = ev(m)
        evals += 1
        if abs(e) <= prm.tol_n or 0.5 * abs(b - a) <= prm.tol_mu:
            return m, pay, evals
        if (e < 0.0) == below:
            a = m
        else:
            b = m


def iterate(rho_fn, theta, mu, prm: Params, n_iter: int):
    """Up to n_iter iterations from (theta, mu).  Returns (theta, mu, history);
    history rows are dicts with mu, nbar, residual, omega, evals."""
    target = 1.0 - prm.doping
    hist = []
    acc = Anderson(prm.anderson, prm.mix) if prm.anderson > 0 else None
    for _ in range(n_iter):
        def e_fn(m, th=theta):
            omega, rho = rho_fn(th, m)
            nbar, res = measure(rho, th)
            return nbar - target, (omega, rho, nbar, res)

        mu, (omega, rho, nbar, res), evals = solve_mu(e_fn, mu, prm)
        if acc is None:
            theta, _, _ = update(rho, theta, prm.mix)
        else:
            x = pack(theta)
            theta = unpack(acc.step(x, pack(mapped(rho, theta)) - x), len(theta[0]), len(theta) == 6)
        hist.append({"mu": mu, "nbar": nbar, "residual": res, "omega": omega, "evals": evals})
        if prm.tol_residual > 0.0 and res <= prm.tol_residual:
            break
    return theta, mu, hist


# ------------------------------------------------------------- rho suppliers
def kpm_rho_fn(Lx, Ly, n_v, t, tp, J, T, M, probes, weights, K=None):
    """Plain KPM (App. B) on the given probe matrix, with the rescale and
    coefficients recomputed for every h."""
    def fn(theta, mu):
        n, chi, dlt = theta
        st = builder.build_stencil(Lx, Ly, n_v, t, tp, J, mu, n, chi, dlt)
        Hs = builder.sparse_from_stencil(st, Lx, Ly)
        a, b = chebyshev.rescale(*chebyshev.gershgorin_sparse(Hs))
        C = chebyshev.kpm_coefficients(M, T, a, b, K)
        out = kpm_plain.plain_kpm(Hs, a, b, probes, weights, C, Lx, Ly, want_grad=True)
        return float(out["omega"]), out["rho"]
    return fn


def direct_rho_fn(Lx, Ly, n_v, t, tp, J, T, M, probes, weights, K=None):
    """Direct probing estimate (series of f' per probe) on the given probes."""
    def fn(theta, mu):
        n, chi, dlt = theta
        st = builder.build_stencil(Lx, Ly, n_v, t, tp, J, mu, n, chi, dlt)
        Hs = builder.sparse_from_stencil(st, Lx, Ly)
        a, b = chebyshev.rescale(*chebyshev.gershgorin_sparse(Hs))
        C = chebyshev.kpm_coefficients(M, T, a, b, K)
        out = kpm_direct.direct_rho(Hs, a, b, probes, weights, C, Lx, Ly)
        return float(out["omega"]), out["rho"]
    return fn


def sdw_kpm_rho_fn(Lx, Ly, n_v, t, tp, J, T, M, probes, weights, K=None):
    """Plain KPM on the spin-polarised builder's h (theta of six arrays)."""
    def fn(theta, mu):
        st = sdw.build_stencil_sdw(Lx, Ly, n_v, t, tp, J, mu, *theta)
        Hs = builder.sparse_from_stencil(st, Lx, Ly)
        a, b = chebyshev.rescale(*chebyshev.gershgorin_sparse(Hs))
        C = chebyshev.kpm_coefficients(M, T, a, b, K)
        out = kpm_plain.plain_kpm(Hs, a, b, probes, weights, C, Lx, Ly, want_grad=True)
        return float(out["omega"]), out["rho"]
    return fn


def sdw_direct_rho_fn(Lx, Ly, n_v, t, tp, J, T, M, probes, weights, K=None):
    """Direct probing estimate (series of f' per probe) on the spin-polarised
    builder's h."""
    def fn(theta, mu):
        st = sdw.build_stencil_sdw(Lx, Ly, n_v, t, tp, J, mu, *theta)
        Hs = builder.sparse_from_stencil(st, Lx, Ly)
        a, b = chebyshev.rescale(*chebyshev.gershgorin_sparse(Hs))
        C = chebyshev.kpm_coefficients(M, T, a, b, K)
        out = kpm_direct.direct_rho(Hs, a, b, probes, weights, C, Lx, Ly)
        return float(out["omega"]), out["rho"]
    return fn


def sdw_exact_rho_fn(Lx, Ly, n_v, t, tp, J, T):
    """Exact Fermi-function rho of the spin-polarised builder's h."""
    def fn(theta, mu):
        st = sdw.build_stencil_sdw(Lx, Ly, n_v, t, tp, J, mu, *theta)
        H = builder.dense_from_stencil(st, Lx, Ly)
        omega, rho = dense.exact(H, T)
        return omega, builder.stencil_from_dense(rho, Lx, Ly)
    return fn


def exact_rho_fn(Lx, Ly, n_v, t, tp, J, T):
    """Exact Fermi-function density matrix by dense diagonalisation."""
    def fn(theta, mu):
        n, chi, dlt = theta
        st = builder.build_stencil(Lx, Ly, n_v, t, tp, J, mu, n, chi, dlt)
        H = builder.dense_from_stencil(st, Lx, Ly)
        omega, rho = dense.exact(H, T)
        return omega, builder.stencil_from_dense(rho, Lx, Ly)
    return fn
