"""O6: magnetic super-cell exact diagonalisation and the broadened LDOS
(oracle; test infrastructure only).

App. "Calculation of local density of states and magnetic super-cell
method".  The converged TB-BdG matrix of one N_x x N_y magnetic unit cell
(eq. diagbdg; here the [19, N] stencil h on the torus, whose wrap-around bonds
already carry the magnetic boundary phases of the field) is repeated over
M_x x M_y cells.  By the magnetic Bloch theorem (eq. matrixeqn) every
quasiparticle of the enlarged lattice has, from one cell to the next, the
same factor on both Nambu amplitudes, exp(-i k.R) (the +-xi/2 magnetic phases
are those of the cell's own wrap bonds), with k on the grid
k = 2 pi (m_x / (M_x N_x), m_y / (M_y N_y)).  So the enlarged problem splits
into M_x M_y cell-sized Bloch matrices H(k): the torus h with every matrix
element of a bond whose head lies in the neighbouring cell R = (s_x N_x,
s_y N_y) (s = +-1, 0) multiplied by exp(-i k.R) = exp(-i (s_x phi_x + s_y
phi_y)), phi = (k_x N_x, k_y N_y) = 2 pi (m_x / M_x, m_y / M_y); its
Hermitian partner carries the conjugate factor.

LDOS (eqs. N_i, Gij with the broadening of the same appendix): from the
eigenpairs (E_n, (u^n_i, v^n_i)) of every H(k), normalised over one cell,

    N_i(omega) = 1/(M_x M_y) sum_k sum_n [ w_up,i |u^n_i|^2 L(omega - E_n)
                                          + w_dn,i |v^n_i|^2 L(omega + E_n) ],
    L(x) = (Gamma / pi) / (x^2 + Gamma^2),  Gamma = alpha |omega| + gamma_0,

the spin-up electron weight at +E_n and the spin-down electron weight (the
hole amplitude) at -E_n.  w_up,i, w_dn,i stand for the g^t factors of eq. Gij
at i = j (the caller's choice; 1 gives the bare quasiparticle LDOS).  The
1/(M_x M_y) is the normalisation of an enlarged-lattice eigenvector over its
M_x M_y cells.

``tiled_dense`` builds the enlarged lattice itself (brute force: the cell's
matrix elements copied into every cell, bonds across a cell edge joining the
neighbouring cell) for the pins: its spectrum is the union of the H(k)
spectra, and its broadened LDOS at a site equals ``supercell_ldos``.
"""
from __future__ import annotations

import numpy as np

from . import lattice


def bloch_dense(st, Lx, Ly, phi_x, phi_y):
    """Dense 2N x 2N H(k) for the twist angles (phi_x, phi_y), written out
    bond by bond."""
    N = Lx * Ly
    H = np.zeros((2 * N, 2 * N), dtype=np.complex128)
    for i in range(N):
        x, y = i % Lx, i // Lx
        for d in range(4):
            dx, dy = lattice.DIRS[d]
            xh, yh = x + dx, y + dy
            sx = (xh >= Lx) - (xh < 0)             # cell of the head: -1, 0, +1
            sy = (yh >= Ly) - (yh < 0)
            j = (yh % Ly) * Lx + xh % Lx
            tw = np.exp(-1j * (sx * phi_x + sy * phi_y))
            for a in range(2):
                for b in range(2):
                    v = st[4 * d + 2 * a + b, i] * tw
                    H[2 * i + a, 2 * j + b] += v
                    H[2 * j + b, 2 * i + a] += np.conj(v)
        H[2 * i, 2 * i] += st[16, i].real
        H[2 * i + 1, 2 * i + 1] += st[17, i].real
        H[2 * i, 2 * i + 1] += st[18, i]
        H[2 * i + 1, 2 * i] += np.conj(st[18, i])
    return H


def kgrid(Mx, My):
    """Twist angles (phi_x, phi_y) of the M_x x M_y grid, k index
    q = m_y M_x + m_x."""
    return [(2 * np.pi * mx / Mx, 2 * np.pi * my / My) for my in range(My) for mx in range(Mx)]


def tiled_dense(st, Lx, Ly, Mx, My):
    """The enlarged (M_x L_x) x (M_y L_y) lattice with the cell's stencil in
    every cell, periodic over the enlarged torus."""
    LX, LY = Mx * Lx, My * Ly
    NN = LX * LY
    H = np.zeros((2 * NN, 2 * NN), dtype=np.complex128)
    for Y in range(LY):
        for X in range(LX):
            I = Y * LX + X
            i = (Y % Ly) * Lx + X % Lx                # the cell site it copies
            for d in range(4):
                dx, dy = lattice.DIRS[d]
                J = ((Y + dy) % LY) * LX + (X + dx) % LX
                for a in range(2):
                    for b in range(2):
                        v = st[4 * d + 2 * a + b, i]
                        H[2 * I + a, 2 * J + b] += v
                        H[2 * J + b, 2 * I + a] += np.conj(v)
            H[2 * I, 2 * I] += st[16, i].real
            H[2 * I + 1, 2 * I + 1] += st[17, i].real
            H[2 * I, 2 * I + 1] += st[18, i]
            H[2 * I + 1, 2 * I] += np.conj(st[18, i])
    return H


def lorentz(x, gamma):
    return (gamma / np.pi) / (x ** 2 + gamma ** 2)


def ldos_from_eigen(E, U, sites, omega, alpha, gamma0, w_up=None, w_dn=None):
    """sum_n [w_up |u_i^n|^2 L(omega - E_n) + w_dn |v_i^n|^2 L(omega + E_n)]
    for the given eigenpairs (columns of U), sites and energies -> [S, W]."""
    sites = np.asarray(sites)
    omega = np.asarray(omega, dtype=np.float64)
    gam = alpha * np.abs(omega) + gamma0
    wu = np.ones(len(sites)) if w_up is None else np.asarray(w_up)[sites]
    wd = np.ones(len(sites)) if w_dn is None else np.asarray(w_dn)[sites]
    out = np.zeros((len(sites), len(omega)))
    for s, i in enumerate(sites):
        pu = np.abs(U[2 * i, :]) ** 2
        pv = np.abs(U[2 * i + 1, :]) ** 2
        for e, (w, g) in enumerate(zip(omega, gam)):
            out[s, e] = wu[s] * np.sum(pu * lorentz(w - E, g)) + wd[s] * np.sum(pv * lorentz(w + E, g))
    return out


def supercell_ldos(st, Lx, Ly, Mx, My, sites, omega, alpha, gamma0, w_up=None, w_dn=None, ks=None):
    """N_i(omega) over the k grid (or the k indices ``ks`` of it, still with
    the 1/(M_x M_y) weight).  Returns (ldos [S, W], eigenvalues [K, 2N])."""
    grid = kgrid(Mx, My)
    ks = range(len(grid)) if ks is None else ks
    out = 0.0
    evals = []
    for q in ks:
        E, U = np.linalg.eigh(bloch_dense(st, Lx, Ly, *grid[q]))
        evals.append(E)
        out = out + ldos_from_eigen(E, U, sites, omega, alpha, gamma0, w_up, w_dn)
    return out / (Mx * My), np.array(evals)
