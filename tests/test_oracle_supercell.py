"""Pins of the magnetic super-cell ED and its broadened LDOS (oracle/supercell.py):

* Bloch's theorem, by brute force: the union of the M_x M_y cell spectra
  equals the spectrum of the enlarged lattice built cell by cell
  (``tiled_dense``), in a field with pairing; a wrong twist sign or a twist
  missing on one Nambu block fails it;
* the super-cell LDOS at a site equals the broadened LDOS of the enlarged
  lattice at every copy of that site (normalisation 1/(M_x M_y) included);
* at the zero twist H(k) is the torus h (``builder.dense_from_stencil``);
* sum rule: with a constant width each site's LDOS integrates to
  w_up + w_dn (completeness of the eigenvectors), up to the Lorentzian tails
  outside the window;
* for the spin-singlet builder, the (u, v) -> (-conj v, conj u), E -> -E
  symmetry of the BdG matrix makes the spin-up part (|u|^2 at +E) equal the
  spin-down part (|v|^2 at -E); for the spin-polarised builder at m != 0 they
  differ.
"""
import numpy as np

import workloads as wl
from oracle import builder, sdw, supercell
from tests import helpers as H


def _cell(Lx=4, Ly=3, nv=2, seed=11):
    cfg = wl.Config("sc", Lx, Ly, nv, 0.15, 8, (wl.ProbeSpec("unit", 1),), vortex=nv > 0,
                    complex_noise=0.05, seed=seed)
    st, _, _, _ = H.oracle_inputs(cfg)
    return cfg, st


def test_union_of_bloch_spectra_is_tiled_spectrum():
    cfg, st = _cell()
    for Mx, My in ((3, 2), (2, 3), (1, 4)):
        ev = np.sort(np.concatenate([np.linalg.eigvalsh(supercell.bloch_dense(st, cfg.Lx, cfg.Ly, *k))
                                     for k in supercell.kgrid(Mx, My)]))
        big = np.linalg.eigvalsh(supercell.tiled_dense(st, cfg.Lx, cfg.Ly, Mx, My))
        assert np.max(np.abs(ev - big)) < 1e-12 * np.max(np.abs(big))
    # the twist matters: the cell spectrum alone repeated is not the tiled one
    E0 = np.linalg.eigvalsh(supercell.bloch_dense(st, cfg.Lx, cfg.Ly, 0.0, 0.0))
    assert np.max(np.abs(np.sort(np.tile(E0, Mx * My)) - big)) > 1e-3


def test_supercell_ldos_equals_tiled_ldos():
    cfg, st = _cell()
    Mx, My = 3, 2
    om = np.linspace(-3.0, 3.0, 13)
    rng = np.random.default_rng(2)
    wu, wd = rng.uniform(0.3, 1.0, cfg.N), rng.uniform(0.3, 1.0, cfg.N)
    sites = [0, 5, cfg.N - 1]
    got, _ = supercell.supercell_ldos(st, cfg.Lx, cfg.Ly, Mx, My, sites, om, 0.25, 0.05, wu, wd)
    E, U = np.linalg.eigh(supercell.tiled_dense(st, cfg.Lx, cfg.Ly, Mx, My))
    LX = Mx * cfg.Lx
    for s, i in enumerate(sites):
        x, y = i % cfg.Lx, i // cfg.Lx
        for cx, cy in ((0, 0), (2, 1), (1, 0)):
            I = (y + cy * cfg.Ly) * LX + x + cx * cfg.Lx
            wU = np.zeros(Mx * My * cfg.N)
            wD = np.zeros(Mx * My * cfg.N)
            wU[I], wD[I] = wu[i], wd[i]
            ref = supercell.ldos_from_eigen(E, U, [I], om, 0.25, 0.05, wU, wD)[0]
            assert np.max(np.abs(got[s] - ref)) < 1e-12 * np.max(np.abs(ref))


def test_zero_twist_is_torus_h():
    cfg, st = _cell(5, 4)
    assert np.array_equal(supercell.bloch_dense(st, cfg.Lx, cfg.Ly, 0.0, 0.0),
                          builder.dense_from_stencil(st, cfg.Lx, cfg.Ly))
    Hk = supercell.bloch_dense(st, cfg.Lx, cfg.Ly, 0.7, -1.9)
    assert np.max(np.abs(Hk - Hk.conj().T)) == 0.0


def test_sum_rule():
    cfg, st = _cell(4, 4)
    om = np.linspace(-60.0, 60.0, 12001)             # trapezoid error ~ exp(-2 pi Gamma / step)
    rng = np.random.default_rng(5)
    wu, wd = rng.uniform(0.3, 1.0, cfg.N), rng.uniform(0.3, 1.0, cfg.N)
    sites = [1, 9]
    got, _ = supercell.supercell_ldos(st, cfg.Lx, cfg.Ly, 2, 2, sites, om, 0.0, 0.05, wu, wd)
    integ = np.trapezoid(got, om, axis=1)
    tail = 2 * 0.05 / (np.pi * 55.0)               # Lorentzian weight beyond the window, bound
    for s, i in enumerate(sites):
        assert abs(integ[s] - (wu[i] + wd[i])) < 2 * tail * (wu[i] + wd[i])


def test_spin_parts_singlet_symmetric_sdw_not():
    cfg, st = _cell(4, 3)
    om = np.linspace(-2.5, 2.5, 21)
    one, zero = np.ones(cfg.N), np.zeros(cfg.N)
    sites = list(range(cfg.N))
    up, _ = supercell.supercell_ldos(st, cfg.Lx, cfg.Ly, 2, 2, sites, om, 0.25, 0.02, one, zero)
    dn, _ = supercell.supercell_ldos(st, cfg.Lx, cfg.Ly, 2, 2, sites, om, 0.25, 0.02, zero, one)
    assert np.max(np.abs(up - dn)) < 1e-12 * np.max(up)
    th = wl.make_theta_sdw(cfg, m_amp=0.05)
    st2 = sdw.build_stencil_sdw(cfg.Lx, cfg.Ly, cfg.n_v, cfg.t, cfg.tp, cfg.J, cfg.mu, *th)
    up2, _ = supercell.supercell_ldos(st2, cfg.Lx, cfg.Ly, 2, 2, sites, om, 0.25, 0.02, one, zero)
    dn2, _ = supercell.supercell_ldos(st2, cfg.Lx, cfg.Ly, 2, 2, sites, om, 0.25, 0.02, zero, one)
    assert np.max(np.abs(up2 - dn2)) > 1e-3 * np.max(up2)
