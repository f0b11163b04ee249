"""O2: plain KPM forward recursion and reverse-mode adjoint (oracle).

Paper App. B, taken in the paper's order and notation:

1. moments  mu_m = r^dag alpha_m  with  alpha_0 = r, alpha_1 = H~ r,
   alpha_m = 2 H~ alpha_{m-1} - alpha_{m-2}          (eq. alpha);
2. energy   E = sum_{m<M} C_m mu_m                    (eq. F_KPM), here with the
   probe average E = sum_l w_l sum_m C_m mu_{m,l};
3. adjoint  beta_m = dE/dalpha_{m+1} (row vectors), beta_{M-1} = beta_M = 0,
   beta_m = w C_{m+1} r^dag + 2 beta_{m+1} H~ - beta_{m+2}   (m < M-1);
4. gradient dE/dH~_IJ = beta_{0,I} alpha_{0,J} + 2 sum_{m=1}^{M-2} beta_{m,I} alpha_{m,J}
                                                      (eqs. dFdH, dalphadH).

Every alpha_m and beta_m is stored (no checkpointing, no reversal, no fusion);
the sparse matrix-vector product is scipy's.  The recursion runs on the
rescaled H~ = (h - b)/a, so rho = dE/dh = (dE/dH~)/a with (a, b) held fixed.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import lattice
from .builder import NENT


def stencil_pairs(Lx: int, Ly: int):
    """(I, J) Nambu index arrays of the 19 stencil entries for every site."""
    N = Lx * Ly
    i = np.arange(N)
    I = np.zeros((NENT, N), dtype=np.int64)
    J = np.zeros((NENT, N), dtype=np.int64)
    for d in range(4):
        j = lattice.neighbour(Lx, Ly, d)
        for a in range(2):
            for b in range(2):
                I[4 * d + 2 * a + b] = 2 * i + a
                J[4 * d + 2 * a + b] = 2 * j + b
    I[16], J[16] = 2 * i, 2 * i
    I[17], J[17] = 2 * i + 1, 2 * i + 1
    I[18], J[18] = 2 * i, 2 * i + 1
    return I, J


def rescaled(Hs, a: float, b: float):
    D = Hs.shape[0]
    return ((sp.csr_matrix(Hs) - b * sp.identity(D, dtype=np.complex128, format="csr")) / a).tocsr()


def plain_kpm(Hs, a, b, probes, weights, C, Lx, Ly, want_grad=True, full=False):
    """Run O2 on probes (R x D).  Returns dict with mu[R, M] (real parts),
    omega, and if want_grad: rho on the stencil [19, N] (and the dense
    dE/dh if full=True, small D only)."""
    Ht = rescaled(Hs, a, b)
    HtT = Ht.T.tocsr()
    M = len(C)
    R, D = probes.shape
    mu = np.zeros((R, M))
    mu_imag = np.zeros((R, M))
    I, J = stencil_pairs(Lx, Ly)
    G = np.zeros(I.shape, dtype=np.complex128)
    Gfull = np.zeros((D, D), dtype=np.complex128) if full else None
    cm = np.full(M, 2.0)
    cm[0] = 1.0
    cm[M - 1] = 0.0       # beta_{M-1} = 0: the top index never contributes
    for ell in range(R):
        r = probes[ell]
        w = weights[ell]
        alpha = np.zeros((M, D), dtype=np.complex128)
        alpha[0] = r
        if M > 1:
            alpha[1] = Ht @ r
        for m in range(2, M):
            alpha[m] = 2.0 * (Ht @ alpha[m - 1]) - alpha[m - 2]
        z = alpha @ r.conj()
        mu[ell] = z.real
        mu_imag[ell] = z.imag
        if not want_grad:
            continue
        beta = np.zeros((M + 1, D), dtype=np.complex128)
        for m in range(M - 2, -1, -1):
            # row vector times H~:  (beta H~)_J = sum_I beta_I H~_IJ = (H~^T beta)_J
            beta[m] = w * C[m + 1] * r.conj() + 2.0 * (HtT @ beta[m + 1]) - beta[m + 2]
        Iv, Jv = I.ravel(), J.ravel()
        acc = np.zeros(Iv.shape, dtype=np.complex128)
        for m0 in range(0, M, 64):
            m1 = min(M, m0 + 64)
            acc += np.einsum("m,mk,mk->k", cm[m0:m1], beta[m0:m1][:, Iv], alpha[m0:m1][:, Jv])
        G += acc.reshape(I.shape)
        if full:
            Gfull += np.einsum("m,mi,mj->ij", cm, beta[:M], alpha)
    omega = float(np.sum(C[None, :] * weights[:, None] * mu))
    out = {"mu": mu, "mu_imag": mu_imag, "omega": omega}
    if want_grad:
        out["rho"] = G / a
        if full:
            out["rho_full"] = Gfull / a
    return out
