"""O3: Bloch (k-space) reference for translation-invariant, zero-field states.

Paper App. B (Nambu form of H_eff) and App. A (eqs. Tij / Dij / mu_i at m = 0).
For a stencil that is the same at every site, a Bloch vector
v_(j,b) = e^{i k.r_j} u_b turns h into the 2x2 matrix
    h(k) = O + sum_d [ B_d e^{i k.d} + B_d^dag e^{-i k.d} ],
with O the onsite block and B_d the bond blocks.  The spectrum of the 2N x 2N
matrix is the union over the N allowed k of the eigenvalues of h(k), and
rho_(i a),(j b) = (1/N) sum_k e^{i k.(r_j - r_i)} [n_F(h(k))]_{b a}.

``uniform_blocks`` writes the uniform-state blocks in closed form from the
printed coefficient formulas at m = 0 (eq. Tij: T = -g^t t - (3/4) J g^s chi*;
pairing amplitude (3/4) J g^s Delta; onsite eps = dW/dn worked out by hand
for a uniform state), independently of the autograd builder.
"""
from __future__ import annotations

import numpy as np

from .chebyshev import fermi_energy_density, fermi_occupation
from .lattice import DIRS


def kgrid(Lx: int, Ly: int):
    kx = 2 * np.pi * np.arange(Lx) / Lx
    ky = 2 * np.pi * np.arange(Ly) / Ly
    KX, KY = np.meshgrid(kx, ky, indexing="xy")
    return KX.ravel(), KY.ravel()


def bloch_matrices(onsite: np.ndarray, blocks: np.ndarray, Lx: int, Ly: int):
    """h(k) for every allowed k: onsite (2,2), blocks (4,2,2) -> (N,2,2)."""
    KX, KY = kgrid(Lx, Ly)
    hk = np.repeat(onsite[None, :, :].astype(np.complex128), len(KX), axis=0)
    for d, (dx, dy) in enumerate(DIRS):
        ph = np.exp(1j * (KX * dx + KY * dy))
        B = blocks[d]
        hk += ph[:, None, None] * B[None] + np.conj(ph)[:, None, None] * B.conj().T[None]
    return hk


def blocks_from_stencil_site(st_col: np.ndarray):
    """(onsite 2x2, blocks 4x2x2) from one site's 19 stencil entries."""
    blocks = np.array([[[st_col[4 * d + 0], st_col[4 * d + 1]],
                        [st_col[4 * d + 2], st_col[4 * d + 3]]] for d in range(4)])
    onsite = np.array([[st_col[16].real, st_col[18]], [np.conj(st_col[18]), st_col[17].real]])
    return onsite, blocks


def uniform_blocks(delta, chi, dlt, t, tp, J, mu):
    """Closed-form uniform-state blocks at m = 0.

    chi, dlt: length-4 complex per direction (+x, +y, +x+y, +x-y).
    g = 2 delta/(1 + delta) (hopping), gs = 4/(1 + delta)^2 (exchange).
    eps = -mu + 8 sum_d Re(t_d chi_d)/(1+delta)^2
              - 12 J sum_{d nn} (|chi_d|^2 + |Delta_d|^2)/(1+delta)^3,
    the derivative of W per site with respect to n = 1 - delta (each bond
    direction touches a site twice, as tail and as head).
    """
    g = 2 * delta / (1 + delta)
    gs = 4 / (1 + delta) ** 2
    tt = [t, t, tp, tp]
    blocks = np.zeros((4, 2, 2), dtype=np.complex128)
    kin = 0.0
    ex = 0.0
    for d in range(4):
        T = -g * tt[d] - (0.75 * J * gs * np.conj(chi[d]) if d < 2 else 0.0)
        P = 0.75 * J * gs * dlt[d] if d < 2 else 0.0
        blocks[d] = [[T, P], [np.conj(P), -np.conj(T)]]
        kin += np.real(tt[d] * chi[d])
        if d < 2:
            ex += abs(chi[d]) ** 2 + abs(dlt[d]) ** 2
    eps = -mu + 8 * kin / (1 + delta) ** 2 - 12 * J * ex / (1 + delta) ** 3
    onsite = np.array([[eps, 0.0], [0.0, -eps]], dtype=np.complex128)
    return onsite, blocks


def spectrum(onsite, blocks, Lx, Ly) -> np.ndarray:
    return np.sort(np.linalg.eigvalsh(bloch_matrices(onsite, blocks, Lx, Ly)).ravel())


def exact_omega_rho_site(onsite, blocks, Lx, Ly, T):
    """(Omega*, rho entries of one site's 19-entry stencil) in k-space."""
    hk = bloch_matrices(onsite, blocks, Lx, Ly)
    E, U = np.linalg.eigh(hk)
    omega = float(fermi_energy_density(E, T).sum())
    nf = fermi_occupation(E, T)
    nk = np.einsum("kan,kn,kbn->kab", U, nf, U.conj())   # n_F(h(k))
    KX, KY = kgrid(Lx, Ly)
    N = len(KX)
    out = np.zeros(19, dtype=np.complex128)
    for d, (dx, dy) in enumerate(DIRS):
        ph = np.exp(1j * (KX * dx + KY * dy))
        for a in range(2):
            for b in range(2):
                # rho_(i a),(j b) = [n_F(h)]_(j b),(i a), j = i + d
                out[4 * d + 2 * a + b] = np.sum(ph * nk[:, b, a]) / N
    out[16] = np.sum(nk[:, 0, 0]) / N
    out[17] = np.sum(nk[:, 1, 1]) / N
    out[18] = np.sum(nk[:, 1, 0]) / N
    return omega, out


def density(onsite, blocks, Lx, Ly, T) -> float:
    """n = n_up + n_dn = rho_{i1,i1} + 1 - rho_{i2,i2} for the uniform state."""
    _, r = exact_omega_rho_site(onsite, blocks, Lx, Ly, T)
    return float(r[16].real + 1.0 - r[17].real)


def mu_for_doping(delta, chi, dlt, t, tp, J, T, L=128, lo=-4.0, hi=4.0, tol=1e-12):
    """Bisection for the mu that gives n = 1 - delta in the uniform state."""
    target = 1.0 - delta
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        on, bl = uniform_blocks(delta, chi, dlt, t, tp, J, mid)
        if density(on, bl, L, L, T) < target:
            lo = mid
        else:
            hi = mid
        if hi - lo < tol:
            break
    return 0.5 * (lo + hi)
