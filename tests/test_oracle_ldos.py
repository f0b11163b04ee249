"""Pins of the KPM local density of states (oracle/ldos.py):

* the recursion-moment form equals the same damped functional built from the
  eigendecomposition of the dense h (no recursion): sum_n |U_In|^2 delta_M;
* sum rule: with the Jackson kernel g_0 = 1, the integral of A_I over the
  band is mu_{I,0} = 1 (Chebyshev-Gauss quadrature in x);
* positivity of the Jackson-damped density (the kernel is non-negative).
"""
import numpy as np

import workloads as wl
from oracle import builder, chebyshev, ldos
from tests import helpers as H


def _setup(cfg):
    st = H.stencil(cfg)
    a, b = H.bounds(cfg, st)
    Hs = builder.sparse_from_stencil(st, cfg.Lx, cfg.Ly)
    return st, a, b, Hs


def test_recursion_form_equals_eigen_form():
    cfg = wl.Config("l", 6, 5, 2, 0.16, 96, (wl.ProbeSpec("unit", 1),), vortex=True, complex_noise=0.02)
    st, a, b, Hs = _setup(cfg)
    E = np.linspace(b - 0.9 * a, b + 0.9 * a, 37)
    A, _ = ldos.ldos(Hs, a, b, 8, 10, 96, E, cfg.Lx, cfg.Ly)
    Hd = builder.dense_from_stencil(st, cfg.Lx, cfg.Ly)
    ref = ldos.ldos_from_eigen(Hd, a, b, 8, 10, 96, E)
    assert np.max(np.abs(A - ref)) < 1e-11 * np.max(np.abs(ref))


def test_sum_rule_and_positivity():
    cfg = wl.Config("l", 8, 8, 2, 0.16, 128, (wl.ProbeSpec("unit", 1),), vortex=True)
    st, a, b, Hs = _setup(cfg)
    K = 4096
    x = np.cos(np.pi * (np.arange(K) + 0.5) / K)          # Chebyshev-Gauss nodes
    E = a * x + b
    A, mu = ldos.ldos(Hs, a, b, 0, 6, 128, E, cfg.Lx, cfg.Ly)
    # int A dE = a int A(x) dx = a (pi/K) sum_k A(x_k) sqrt(1 - x_k^2)
    integral = a * (np.pi / K) * (A * np.sqrt(1 - x ** 2)[None, :]).sum(axis=1)
    assert np.allclose(integral, 1.0, atol=1e-12)
    assert np.allclose(mu[:, 0], 1.0)
    assert A.min() > -1e-12


def test_jackson_kernel_is_positive():
    M = 64
    g = chebyshev.jackson(M)
    x = np.linspace(-0.999, 0.999, 301)
    w = 2.0 * g
    w[0] = g[0]
    for y in (-0.7, 0.0, 0.35):
        k = (w[:, None] * np.cos(np.multiply.outer(np.arange(M), np.arccos(x))) *
             np.cos(np.arange(M) * np.arccos(y))[:, None]).sum(axis=0)
        assert k.min() > -1e-12
