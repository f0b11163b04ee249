"""Convenience layer over the C ABI: allocates torch device buffers and calls
the library entry points in the order of the method (App. B): build h, rescale
bounds, expansion coefficients, forward recursion (Omega), adjoint (rho), and
the builder VJP.  No arithmetic of the method happens here.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Sequence

import torch

from . import kpm


@dataclass
class KPMProblem:
    Lx: int
    Ly: int
    n_vortex: int
    t: float
    tp: float
    J: float
    mu: float
    T: float
    M: int
    probes: Sequence[kpm.ProbeSpec]
    precision: int = kpm.KPM_FP64
    ckpt_k: int = 64
    device: str = "cuda"
    _ws: torch.Tensor = field(default=None, repr=False)
    _rmft_ws: torch.Tensor = field(default=None, repr=False)
    _sc_ws: torch.Tensor = field(default=None, repr=False)

    def __post_init__(self):
        self.lat = kpm.lattice(self.Lx, self.Ly, self.n_vortex)
        self.mdl = kpm.model(self.t, self.tp, self.J, self.mu)
        self.N = self.Lx * self.Ly
        self.R = kpm.kpm_probe_count(self.lat, self.probes)

    # -- buffers
    def workspace(self) -> torch.Tensor:
        if self._ws is None:
            self._ws = kpm.workspace(self.lat, self.R, self.M, self.ckpt_k, self.precision, self.device)
        return self._ws

    def zeros(self, *shape, dtype=torch.complex128):
        return torch.zeros(*shape, dtype=dtype, device=self.device)

    # -- steps
    def build_H(self, n, chi, delta):
        h = self.zeros(kpm.NENT, self.N)
        kpm.kpm_build_H(self.lat, self.mdl, n, chi, delta, h)
        return h

    def build_H_vjp(self, n, chi, delta, rho):
        dn = self.zeros(self.N, dtype=torch.float64)
        dchi = self.zeros(4, self.N)
        ddelta = self.zeros(4, self.N)
        kpm.kpm_build_H_vjp(self.lat, self.mdl, n, chi, delta, rho, dn, dchi, ddelta)
        return dn, dchi, ddelta

    def build_H_sdw(self, n_up, n_dn, chi_up, chi_dn, delta_up, delta_dn):
        h = self.zeros(kpm.NENT, self.N)
        kpm.kpm_build_H_sdw(self.lat, self.mdl, n_up, n_dn, chi_up, chi_dn, delta_up, delta_dn, h)
        return h

    def build_H_sdw_vjp(self, theta, rho):
        """theta: (n_up, n_dn, chi_up, chi_dn, delta_up, delta_dn).  Returns the
        six gradients in the same order."""
        grads = [self.zeros(self.N, dtype=torch.float64), self.zeros(self.N, dtype=torch.float64)]
        grads += [self.zeros(4, self.N) for _ in range(4)]
        kpm.kpm_build_H_sdw_vjp(self.lat, self.mdl, list(theta), rho, grads)
        return tuple(grads)

    def bounds(self, h):
        ab = self.zeros(2, dtype=torch.float64)
        kpm.kpm_bounds(self.lat, h, ab)
        return ab

    def coefficients(self, ab, K=0):
        C = self.zeros(self.M, dtype=torch.float64)
        kpm.kpm_coefficients(self.M, self.T, ab, C, K)
        return C

    def moments(self, h, ab):
        mu = self.zeros(self.R, self.M, dtype=torch.float64)
        kpm.kpm_moments(self.lat, h, ab, self.probes, self.M, self.precision, self.ckpt_k, mu,
                        self.workspace())
        return mu

    def grand_potential(self, h, ab, C, want_mu=False):
        omega = self.zeros(1, dtype=torch.float64)
        mu = self.zeros(self.R, self.M, dtype=torch.float64) if want_mu else None
        kpm.kpm_grand_potential(self.lat, h, ab, self.probes, self.M, C, self.precision, self.ckpt_k,
                                omega, mu, self.workspace())
        return (omega, mu) if want_mu else omega

    def grand_potential_grad(self, h, ab, C, omega_bar=None):
        rho = self.zeros(kpm.NENT, self.N)
        kpm.kpm_grand_potential_grad(self.lat, h, ab, self.probes, self.M, C, self.precision,
                                     self.ckpt_k, omega_bar, rho, self.workspace())
        return rho

    def density_matrix(self, h, ab, C):
        out = {"omega": self.zeros(1, dtype=torch.float64), "rho": self.zeros(kpm.NENT, self.N),
               "n_up": self.zeros(self.N, dtype=torch.float64),
               "n_dn": self.zeros(self.N, dtype=torch.float64),
               "chi_up": self.zeros(4, self.N), "chi_dn": self.zeros(4, self.N),
               "delta_up": self.zeros(4, self.N), "delta_dn": self.zeros(4, self.N)}
        kpm.kpm_density_matrix(self.lat, h, ab, self.probes, self.M, C, self.precision, self.ckpt_k,
                               out["omega"], out["rho"], out["n_up"], out["n_dn"], out["chi_up"],
                               out["chi_dn"], out["delta_up"], out["delta_dn"], self.workspace())
        return out

    def density_matrix_direct(self, h, ab, C):
        """(omega, rho) by the direct probing estimate (forward recursion only)."""
        omega = self.zeros(1, dtype=torch.float64)
        rho = self.zeros(kpm.NENT, self.N)
        kpm.kpm_density_matrix_direct(self.lat, h, ab, self.probes, self.M, C, self.precision, omega,
                                      rho, self.workspace())
        return omega, rho

    def moments_doubling(self, h, ab, C=None):
        """(omega or None, mu [R][M]) from half the recursion (moment doubling)."""
        mu = self.zeros(self.R, self.M, dtype=torch.float64)
        omega = self.zeros(1, dtype=torch.float64) if C is not None else None
        kpm.kpm_moments_doubling(self.lat, h, ab, self.probes, self.M, C, self.precision, omega, mu,
                                 self.workspace())
        return omega, mu

    def ldos(self, h, ab, first, count, energies):
        """A_I(E) [count][len(energies)] for Nambu indices first .. first+count-1,
        with its own workspace sized for count unit probes."""
        ws = kpm.workspace(self.lat, count, self.M, self.M, self.precision, self.device)
        out = self.zeros(count, energies.numel(), dtype=torch.float64)
        kpm.kpm_ldos(self.lat, h, ab, first, count, self.M, self.precision, energies, out, ws)
        return out

    def status(self) -> int:
        return kpm.kpm_status_read(self.workspace())

    # -- self-consistent iteration (kpm_rmft_iterate)
    def rmft_workspace(self) -> torch.Tensor:
        if self._rmft_ws is None:
            nb = kpm.kpm_rmft_workspace_size(self.lat, self.R, self.M, self.ckpt_k, self.precision)
            self._rmft_ws = torch.empty(nb, dtype=torch.uint8, device=self.device)
        return self._rmft_ws

    def rmft_iterate(self, n, chi, delta, mu, params, n_iter):
        """Up to n_iter iterations on (n, chi, delta) in place from chemical
        potential mu.  Returns (mu, history, status)."""
        return kpm.kpm_rmft_iterate(self.lat, self.mdl, self.probes, self.M, self.T, self.precision,
                                    self.ckpt_k, params, n_iter, n, chi, delta, mu,
                                    self.rmft_workspace())

    # -- magnetic super-cell ED and broadened LDOS (kpm_supercell_ldos)
    def supercell_ldos(self, h, Mx, My, sites, omega, alpha=0.25, gamma0=3e-4, w_up=None, w_dn=None,
                       k_first=0, k_count=None, want_evals=False, k_batch=1):
        """N_i(omega) for the listed sites over the Mx x My k grid (or the slice
        k_first .. k_first + k_count - 1 of it), k_batch k points per
        eigensolver call.  Returns (ldos [S, W], eigenvalues [k_count, 2N] or
        None)."""
        nb = kpm.kpm_supercell_workspace_size(self.lat, k_batch)
        if self._sc_ws is None or self._sc_ws.numel() < nb:
            self._sc_ws = None
            self._sc_ws = torch.empty(nb, dtype=torch.uint8, device=self.device)
        k_count = Mx * My - k_first if k_count is None else k_count
        N = self.lat.Lx * self.lat.Ly
        out = torch.empty(len(sites), omega.numel(), dtype=torch.float64, device=self.device)
        ev = torch.empty(k_count, 2 * N, dtype=torch.float64, device=self.device) if want_evals else None
        kpm.kpm_supercell_ldos(self.lat, h, Mx, My, k_first, k_count, sites, omega, alpha, gamma0, w_up,
                               w_dn, False, out, ev, self._sc_ws, k_batch)
        return out, ev

    def rmft_iterate_sdw(self, n_up, n_dn, chi_up, chi_dn, delta_up, delta_dn, mu, params, n_iter):
        """rmft_iterate on a spin-polarised theta (kpm_rmft_iterate_sdw)."""
        return kpm.kpm_rmft_iterate_sdw(self.lat, self.mdl, self.probes, self.M, self.T, self.precision,
                                        self.ckpt_k, params, n_iter, n_up, n_dn, chi_up, chi_dn,
                                        delta_up, delta_dn, mu, self.rmft_workspace())


def save_rmft_state(path, n, chi, delta, mu, history=()):
    """Writes theta, mu and the iteration history to an .npz file (a restart
    point of the self-consistent iteration)."""
    import numpy as np

    def host(t):
        return t.detach().cpu().numpy()

    rec = np.array([(h["mu"], h["nbar"], h["residual"], h["omega"], h["evals"]) for h in history],
                   dtype=np.float64).reshape(-1, 5)
    np.savez(path, n=host(n), chi=host(chi), delta=host(delta), mu=np.float64(mu), history=rec)


def load_rmft_state(path, device="cuda"):
    """(n, chi, delta, mu, history) from ``save_rmft_state``; tensors on device."""
    import numpy as np

    with np.load(path, allow_pickle=False) as z:
        n = torch.from_numpy(z["n"]).to(device)
        chi = torch.from_numpy(z["chi"]).to(device)
        delta = torch.from_numpy(z["delta"]).to(device)
        hist = [{"mu": r[0], "nbar": r[1], "residual": r[2], "omega": r[3], "evals": int(r[4])}
                for r in z["history"]]
        return n, chi, delta, float(z["mu"]), hist
