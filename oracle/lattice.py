"""Square-torus geometry and Peierls phases (oracle; test infrastructure only).

Paper: Model and methods (t-t'-J model with nearest- and next-nearest-neighbour
hopping; Peierls substitution t_ij -> t e^{i phi_ij}, phi_ij = -(pi/Phi0) times
the line integral of A from r_i to r_j, Landau gauge A = B(0, x)) and App. C
(field B = 2 Phi0 / (N_x N_y), i.e. two superconducting flux quanta through the
torus).

Conventions (readings where the paper is silent):

* site index i = y * Lx + x, 0 <= x < Lx, 0 <= y < Ly; both Lx, Ly >= 3 so the
  eight neighbours of a site are distinct sites.
* stencil directions d = 0..3: +x, +y, +x+y, +x-y.  Every undirected bond is
  stored once, at its tail site i, pointing to j = i + d (mod the torus).
* B = n_v Phi0 / (Lx Ly) with n_v the number of superconducting flux quanta
  (n_v = 2 in the paper).  The line integral is taken along the straight
  segment in unwrapped coordinates, so phi_ij = -pi n_v (x_i + dx/2) dy / (Lx Ly).
* A bond whose +x step crosses the x seam (x_i = Lx - 1) additionally carries
  the gauge twist +pi n_v y_j / Ly, y_j the row of its head site.  With it every
  elementary plaquette (seams included) encloses the same phase
  -pi n_v / (Lx Ly), every nn+nnn triangle half of it; this requires n_v even.
"""
from __future__ import annotations

import numpy as np

DIRS = ((1, 0), (0, 1), (1, 1), (1, -1))


def check_lattice(Lx: int, Ly: int, n_v: int) -> None:
    if Lx < 3 or Ly < 3:
        raise ValueError("torus sides must be >= 3")
    if n_v % 2 != 0:
        raise ValueError("flux count n_v must be even on a torus")


def coords(Lx: int, Ly: int):
    """(x, y) integer arrays of length N = Lx*Ly in site order."""
    i = np.arange(Lx * Ly)
    return i % Lx, i // Lx


def neighbour(Lx: int, Ly: int, d: int) -> np.ndarray:
    """j(i) = i + DIRS[d] on the torus, as an index array over all sites."""
    x, y = coords(Lx, Ly)
    dx, dy = DIRS[d]
    return ((y + dy) % Ly) * Lx + (x + dx) % Lx


def peierls_phase(Lx: int, Ly: int, n_v: int, d: int) -> np.ndarray:
    """phi_ij for the bond (i, i + DIRS[d]) for every tail site i.

    Written out bond by bond with a plain loop (the oracle favours loops over
    vectorised tricks for readability).
    """
    dx, dy = DIRS[d]
    out = np.zeros(Lx * Ly)
    for y in range(Ly):
        for x in range(Lx):
            xmid = x + 0.5 * dx
            phi = -np.pi * n_v * xmid * dy / (Lx * Ly)
            if x + dx == Lx:  # +x step across the seam
                yj = (y + dy) % Ly
                phi += np.pi * n_v * yj / Ly
            out[y * Lx + x] = phi
    return out


def hopping(Lx: int, Ly: int, n_v: int, t: float, tp: float) -> np.ndarray:
    """Complex bare hoppings t_ij = t e^{i phi_ij} as [4, N] (nn t, nnn t')."""
    out = np.zeros((4, Lx * Ly), dtype=np.complex128)
    for d in range(4):
        amp = t if d < 2 else tp
        out[d] = amp * np.exp(1j * peierls_phase(Lx, Ly, n_v, d))
    return out
