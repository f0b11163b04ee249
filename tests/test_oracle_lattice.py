"""Pins for oracle/lattice.py: Peierls phases and field normalisation.

* every plaquette encloses -pi n_v/(Lx Ly), every nn+nnn triangle half of it,
  seams included (uniform field on the torus, gauge invariant);
* the phase of single bonds equals a numerical quadrature of the Landau-gauge
  line integral -(pi/Phi0) int A.dl with A = B(0, x) (Model and methods);
* lattice sizes map to the fields printed in the paper (golden fixture).
"""
import os

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import lattice

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _phase_between(phi, Lx, Ly, a, b):
    """Phase for hopping site a -> b using the stored bonds (reverse = minus)."""
    ax, ay = a % Lx, a // Lx
    for d, (dx, dy) in enumerate(lattice.DIRS):
        if ((ay + dy) % Ly) * Lx + (ax + dx) % Lx == b:
            return phi[d][a]
    bx, by = b % Lx, b // Lx
    for d, (dx, dy) in enumerate(lattice.DIRS):
        if ((by + dy) % Ly) * Lx + (bx + dx) % Lx == a:
            return -phi[d][b]
    raise AssertionError("not a stencil bond")


def _wrap(p):
    return (p + np.pi) % (2 * np.pi) - np.pi


@pytest.mark.parametrize("Lx,Ly,nv", [(6, 10, 2), (5, 7, 2), (8, 8, 4), (4, 6, 6)])
def test_uniform_flux_every_plaquette_and_triangle(Lx, Ly, nv):
    phi = [lattice.peierls_phase(Lx, Ly, nv, d) for d in range(4)]
    s = lambda x, y: (y % Ly) * Lx + (x % Lx)
    want = -np.pi * nv / (Lx * Ly)
    for y in range(Ly):
        for x in range(Lx):
            loop = [s(x, y), s(x + 1, y), s(x + 1, y + 1), s(x, y + 1), s(x, y)]
            circ = sum(_phase_between(phi, Lx, Ly, loop[k], loop[k + 1]) for k in range(4))
            assert abs(_wrap(circ - want)) < 1e-12
            # counter-clockwise triangles: (x,y)->(x+1,y)->(x+1,y+1) and (x,y)->(x+1,y-1)->(x+1,y)
            for tri in ([s(x, y), s(x + 1, y), s(x + 1, y + 1), s(x, y)],
                        [s(x, y), s(x + 1, y - 1), s(x + 1, y), s(x, y)]):
                circ = sum(_phase_between(phi, Lx, Ly, tri[k], tri[k + 1]) for k in range(3))
                assert abs(_wrap(circ - want / 2)) < 1e-12


def test_bond_phase_equals_line_integral_in_the_bulk():
    Lx, Ly, nv = 9, 7, 2
    B_over_phi0 = nv / (Lx * Ly)          # B in units of Phi0 per unit cell area
    for d, (dx, dy) in enumerate(lattice.DIRS):
        phi = lattice.peierls_phase(Lx, Ly, nv, d)
        for (x, y) in [(0, 0), (3, 2), (Lx - 2, Ly - 1), (4, 0)]:
            # straight path r(s) = r_i + s (dx, dy), A = B (0, x) -> A.dl = B x(s) dy ds
            integral, _ = quad(lambda s: B_over_phi0 * (x + s * dx) * dy, 0.0, 1.0)
            assert abs(phi[y * Lx + x] - (-np.pi * integral)) < 1e-13


def test_paper_field_values():
    phi0 = 6.62607015e-34 / (2 * 1.602176634e-19)      # superconducting flux quantum hc/2e (SI h/2e)
    a = 3.88e-10
    for line in open(os.path.join(GOLDEN, "paper_fields.txt")):
        if line.startswith("#") or not line.strip():
            continue
        Nx, Ny, B = line.split()
        Nx, Ny, B = int(Nx), int(Ny), float(B)
        phi = [lattice.peierls_phase(Nx, Ny, 2, d) for d in range(2)]
        # circulation of the plaquette at the origin, converted to a field
        circ = phi[0][0] + phi[1][1] - phi[0][Nx] - phi[1][0]
        flux = abs(circ) / np.pi * phi0
        assert abs(flux / a ** 2 - B) < 0.01


def test_rejects_small_and_odd():
    with pytest.raises(ValueError):
        lattice.check_lattice(2, 5, 2)
    with pytest.raises(ValueError):
        lattice.check_lattice(4, 4, 1)
