"""TB-BdG builder h(theta) = dW/drho and its vector-Jacobian product (oracle).

Paper: Model and methods eq. H_eff and eq. model_param (T = dW/dchi,
D = dW/dDelta*, mu_i = dW/dn), App. A eqs. Tij / Dij / mu_i, App. B (Nambu
spinor d_i = (c_{i up}, c^dag_{i dn}) and the 2x2 block form of h).

Reading of the paper's sign/label conventions (the paper is inconsistent
between eq. H_eff, eq. model_param and the Nambu matrix): the single-particle
matrix is the Wirtinger derivative h_IJ = dW/drho_IJ of W written as a function
of rho_IJ = <d^dag_I d_J>, with

    n_{i up}  = rho_{i1,i1},       n_{i dn}  = 1 - rho_{i2,i2},
    chi_ij up = rho_{i1,j1},       chi_ij dn = -rho_{j2,i2},
    <c_{i up} c_{j dn}> = -conj rho_{i1,j2},  <c_{j up} c_{i dn}> = -conj rho_{j1,i2}.

For the singlet W of ``gutzwiller.energy_W`` this gives, for bond (i, j=i+d),

    h_{i1,j1} = T_ij = (1/2) dW/dchi_ij        (eq. Tij at m = 0:
                       = -g^t_ij t_ij - (3/4) J g^s_ij conj(chi_ij)),
    h_{i2,j2} = -conj(T_ij),
    h_{i1,j2} = h_{j1,i2} = P_ij = -(1/2) dW/dconj(Delta_ij)
                       = (3/4) J g^s_ij Delta_ij     (|P| as in eq. Dij),
    h_{i1,i1} = eps_i = dW/dn_i,   h_{i2,i2} = -eps_i,   h_{i1,i2} = 0,

and every reverse bond block is the Hermitian conjugate.  The derivatives are
taken here by torch autograd of W (no hand-derived formulas), so the oracle
is independent of the hand-written GPU builder.

Stencil layout shared with the C-ABI (complex, entry-major): entry 4d + 2a + b
is h_{(i,a),(i+d,b)} (a, b = 0 for Nambu component 1, 1 for component 2),
entry 16 = h_{i1,i1}, 17 = h_{i2,i2} (real), 18 = h_{i1,i2}.
"""
from __future__ import annotations

import numpy as np
import torch

from . import lattice
from .gutzwiller import energy_W

NENT = 19


def _torch_inputs(n, chi, dlt):
    n_t = torch.tensor(np.asarray(n, dtype=np.float64), requires_grad=True)
    c_t = torch.tensor(np.asarray(chi, dtype=np.complex128), requires_grad=True)
    d_t = torch.tensor(np.asarray(dlt, dtype=np.complex128), requires_grad=True)
    return n_t, c_t, d_t


def _geometry(Lx, Ly, n_v, t, tp):
    hop = torch.tensor(lattice.hopping(Lx, Ly, n_v, t, tp))
    nbr = torch.tensor(np.stack([lattice.neighbour(Lx, Ly, d) for d in range(4)]))
    return hop, nbr


def coefficients_torch(n_t, c_t, d_t, Lx, Ly, n_v, t, tp, J, mu, create_graph=False):
    """(eps[N], T[4,N], P[4,N]) as torch tensors from autograd of W.

    torch's gradient of a real W w.r.t. a complex z is dW/dRe z + i dW/dIm z
    = 2 dW/dconj(z), so dW/dz = conj(grad)/2 and dW/dconj(z) = grad/2.
    """
    hop, nbr = _geometry(Lx, Ly, n_v, t, tp)
    W = energy_W(n_t, c_t, d_t, hop, nbr, J, mu)
    gn, gc, gd = torch.autograd.grad(W, (n_t, c_t, d_t), create_graph=create_graph)
    eps = gn
    T = 0.5 * (gc.conj() / 2.0)
    P = -0.5 * (gd / 2.0)
    return eps, T, P


def stencil_from_blocks(eps, T, P):
    """Assemble the [19, N] complex stencil from eps, T, P (numpy or torch)."""
    lib = torch if isinstance(eps, torch.Tensor) else np
    N = eps.shape[0]
    ents = []
    for d in range(4):
        ents += [T[d], P[d], P[d].conj(), -T[d].conj()]
    zero = 0.0 * T[0]
    ents += [eps + zero, -eps + zero, zero]
    out = lib.stack(ents)
    assert out.shape[0] == NENT and out.shape[1] == N
    return out


def build_stencil(Lx, Ly, n_v, t, tp, J, mu, n, chi, dlt):
    """h on the stencil, [19, N] complex128 numpy (kpm_build_H)."""
    n_t, c_t, d_t = _torch_inputs(n, chi, dlt)
    eps, T, P = coefficients_torch(n_t, c_t, d_t, Lx, Ly, n_v, t, tp, J, mu)
    return stencil_from_blocks(eps, T, P).detach().numpy()


def dense_from_stencil(st, Lx, Ly):
    """Dense 2N x 2N Hermitian h from a [19, N] stencil (Nambu index I = 2i + a).

    Plain loops: block B_d(i) at (i, j) and its conjugate transpose at (j, i).
    """
    N = Lx * Ly
    H = np.zeros((2 * N, 2 * N), dtype=np.complex128)
    nbrs = [lattice.neighbour(Lx, Ly, d) for d in range(4)]
    for i in range(N):
        for d in range(4):
            j = nbrs[d][i]
            for a in range(2):
                for b in range(2):
                    v = st[4 * d + 2 * a + b, i]
                    H[2 * i + a, 2 * j + b] += v
                    H[2 * j + b, 2 * i + a] += np.conj(v)
        H[2 * i, 2 * i] += st[16, i].real
        H[2 * i + 1, 2 * i + 1] += st[17, i].real
        H[2 * i, 2 * i + 1] += st[18, i]
        H[2 * i + 1, 2 * i] += np.conj(st[18, i])
    return H


def sparse_from_stencil(st, Lx, Ly):
    """Same matrix as ``dense_from_stencil`` in scipy CSR form (for large N)."""
    import scipy.sparse as sp

    N = Lx * Ly
    rows, cols, vals = [], [], []
    i = np.arange(N)
    for d in range(4):
        j = lattice.neighbour(Lx, Ly, d)
        for a in range(2):
            for b in range(2):
                v = st[4 * d + 2 * a + b]
                rows += [2 * i + a, 2 * j + b]
                cols += [2 * j + b, 2 * i + a]
                vals += [v, np.conj(v)]
    rows += [2 * i, 2 * i + 1, 2 * i, 2 * i + 1]
    cols += [2 * i, 2 * i + 1, 2 * i + 1, 2 * i]
    vals += [st[16].real + 0j, st[17].real + 0j, st[18], np.conj(st[18])]
    return sp.csr_matrix(
        (np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
        shape=(2 * N, 2 * N),
    )


def stencil_from_dense(G, Lx, Ly):
    """Read the [19, N] stencil entries G_IJ (forward half + onsite) off a dense matrix."""
    N = Lx * Ly
    out = np.zeros((NENT, N), dtype=np.complex128)
    for d in range(4):
        j = lattice.neighbour(Lx, Ly, d)
        for a in range(2):
            for b in range(2):
                out[4 * d + 2 * a + b] = G[2 * np.arange(N) + a, 2 * j + b]
    i = np.arange(N)
    out[16] = G[2 * i, 2 * i]
    out[17] = G[2 * i + 1, 2 * i + 1]
    out[18] = G[2 * i, 2 * i + 1]
    return out


def build_vjp(Lx, Ly, n_v, t, tp, J, mu, n, chi, dlt, rho):
    """dOmega/dtheta = sum_IJ rho_IJ dh_IJ/dtheta (kpm_build_H_vjp).

    rho is the [19, N] stencil of dOmega/dh (forward half + onsite).  With both
    h and rho Hermitian, dOmega = sum_fwd 2 Re(rho_IJ dh_IJ) + sum_diag rho_II dh_II
    + 2 Re(rho_{i1,i2} dh_{i1,i2}); the linearisation below is differentiated by
    autograd (second derivatives of W).  Returned gradients follow torch's
    convention for complex parameters: dOmega/dRe z + i dOmega/dIm z.
    """
    n_t, c_t, d_t = _torch_inputs(n, chi, dlt)
    eps, T, P = coefficients_torch(n_t, c_t, d_t, Lx, Ly, n_v, t, tp, J, mu, create_graph=True)
    h = stencil_from_blocks(eps, T, P)
    r = torch.tensor(np.asarray(rho, dtype=np.complex128))
    lin = 2.0 * (r[:16] * h[:16]).real.sum()
    lin = lin + (r[16].real * h[16].real).sum() + (r[17].real * h[17].real).sum()
    lin = lin + 2.0 * (r[18] * h[18]).real.sum()
    gn, gc, gd = torch.autograd.grad(lin, (n_t, c_t, d_t), allow_unused=True)
    gd = torch.zeros_like(d_t) if gd is None else gd
    return gn.detach().numpy(), gc.detach().numpy(), gd.detach().numpy()
