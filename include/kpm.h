/*
 * kpm.h -- C ABI of the MI355X (gfx950) kernel-polynomial-method library for
 * the renormalized mean-field t-t'-J model with vortices (Liu, Tu, Chern, Lee,
 * "Intertwined Orders and Electronic Structure in Superconducting Vortex
 * Halos", arXiv:2212.05685).
 *
 * The library computes, for the 2N x 2N Nambu (BdG) single-particle matrix h
 * of an Lx x Ly torus, the Chebyshev moments mu_m, the grand potential
 * Omega = sum_m C_m mu_m and its adjoint dOmega/dh, which is the density
 * matrix rho_IJ = <d^dag_I d_J> restricted to the stencil (App. B).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Pointers are DEVICE pointers unless the argument says "host".  The caller
 *   owns every buffer; the library allocates device memory only inside batch
 *   plans (kpm_batch_create).
 * - `stream` is a hipStream_t passed as void* (NULL = default stream).  All
 *   device work is enqueued on it; calls return before it finishes.
 * - Argument errors are returned synchronously (nothing is enqueued then).
 *   Errors found by the device (spectrum outside the rescaled interval,
 *   non-finite values) are latched in the workspace status word; read it with
 *   kpm_status_read.
 * - Complex numbers are stored as interleaved (re, im) doubles.
 * - Sites are i = y*Lx + x.  Stencil directions d = 0..3 are +x, +y, +x+y,
 *   +x-y; every undirected bond is stored once, at its tail site i, pointing to
 *   j = i + d on the torus.  Nambu index I = 2i + a with a = 0 for c_{i up} and
 *   a = 1 for c^dag_{i dn}.
 * - STENCIL layout ([19][N] complex, entry-major): entry 4d + 2a + b holds the
 *   matrix element (i a, j b) of the bond block, j = i + d; entry 16 holds
 *   (i0, i0), 17 holds (i1, i1) (both real, imaginary part ignored on input and
 *   written as 0), 18 holds (i0, i1).  Every other element of the matrix
 *   follows by Hermiticity.  Both h and rho = dOmega/dh use this layout.
 * - Functions are re-entrant for distinct workspaces.  Calls that share one
 *   workspace must be ordered on one stream.
 * - Lx, Ly >= 3 (the eight neighbours of a site must be distinct sites);
 *   n_vortex even (whole electron flux quanta through the torus); M >= 2.
 */
#ifndef KPM_H
#define KPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  KPM_OK = 0,
  KPM_EINVAL = -1,     /* bad argument (size, pointer, option)                  */
  KPM_ENOMEM = -2,     /* plan allocation failed                                */
  KPM_EDEVICE = -3,    /* HIP runtime error                                     */
  KPM_EBOUNDS = -4,    /* device status: |mu_m| > mu_0 or non-finite value, i.e.
                          the spectrum is not inside the rescaled interval       */
  KPM_ENOTSUP = -5,    /* option not supported                                  */
  KPM_EWORKSPACE = -6, /* workspace too small or not prepared by the forward call */
  KPM_ENOCONV = -7,    /* chemical-potential search used its evaluation budget    */
  KPM_ETOOBIG = -8     /* problem does not fit the static scratch of a no-alloc call */
};

enum { KPM_FP64 = 0, KPM_FP32 = 1 };   /* recurrence vectors; reductions always FP64 */

enum { KPM_PROBE_UNIT = 0, KPM_PROBE_DENSE_Z4 = 1, KPM_PROBE_COLORED_Z4 = 2 };

typedef struct {
  int32_t Lx, Ly;      /* torus sides, >= 3                                     */
  int32_t n_vortex;    /* superconducting flux quanta through the torus (even); */
} kpm_lattice;         /* B = n_vortex Phi0 / (Lx Ly), App. C                    */

typedef struct {
  double t, tp;        /* nn and nnn bare hoppings (-t c^dag c convention)      */
  double J;            /* nn exchange                                           */
  double mu;           /* chemical potential (Lagrange multiplier of App. A)    */
} kpm_model;

/* One group of probe vectors for the stochastic trace (App. B).  The Z4 phase
 * of Nambu index I in draw s is i^k with k the top two bits of
 * SplitMix64(seed, s * 2^32 + I) (Steele, Lea & Flood 2014; Vigna's form:
 * z = seed + (counter + 1) * 0x9E3779B97F4A7C15, then the two xor-shift-
 * multiply rounds and a final xor-shift).
 *   UNIT        count vectors e_I, I = first .. first + count - 1.
 *   DENSE_Z4    count vectors, every entry a Z4 phase (draw s = probe index).
 *   COLORED_Z4  count draws; in each, one probe per colour (x mod px) +
 *               px (y mod py) (and per Nambu component if split_nambu), Z4
 *               phases on its colour class, zero elsewhere; probe q of the
 *               group is draw q / C, colour (q % C) [/ 2 if split], component
 *               (q % 2 if split), C = px py (2 if split).
 * `weight` multiplies every probe of the group in Omega and in rho. */
typedef struct {
  int32_t kind;
  int32_t count;
  int32_t px, py;
  int32_t split_nambu;
  int32_t first;
  uint64_t seed;
  double weight;
} kpm_probe_group;

#define KPM_MAX_PROBE_GROUPS 4

typedef struct {
  const kpm_probe_group* groups;   /* host array                               */
  int32_t ngroups;                 /* 1 .. KPM_MAX_PROBE_GROUPS                */
} kpm_probes;

/* Number of probe vectors R described by `probes` (host only), or < 0 on error. */
int32_t kpm_probe_count(const kpm_lattice* lat, const kpm_probes* probes);

/* Build h on the stencil from the order parameters at m_i = 0
 * (App. A eqs. Tij, Dij, mu_i; App. B Nambu matrix; Peierls phases of Model
 * and methods / App. C).  h_IJ = dW/drho_IJ for the spin-singlet energy
 *   W = -sum_bonds 4 g_i g_j Re(t_ij chi_ij) - (3/2) J sum_nn g^s_i g^s_j
 *       (|chi_ij|^2 + |Delta_ij|^2) - mu sum_i n_i,
 * g_i = sqrt(2 delta_i/(1+delta_i)), g^s_i = 2/(1+delta_i), delta_i = 1 - n_i:
 *   (i0,j0) = T = -g_i g_j t_ij - (3/4) J g^s_i g^s_j conj(chi_ij) [nn only for J],
 *   (i1,j1) = -conj(T), (i0,j1) = P = (3/4) J g^s_i g^s_j Delta_ij (nn only),
 *   (i1,j0) = conj(P), (i0,i0) = eps_i = dW/dn_i = -(i1,i1), (i0,i1) = 0.
 * n     [N] real, electron density per site (0 < 1 - n < 1).
 * chi   [4][N] complex, <c^dag_{i s} c_{j s}> per spin on bond (i, i+d).
 * delta [4][N] complex, singlet <c_{i up} c_{j dn}> on bond (i, i+d); the
 *       diagonal directions d = 2, 3 do not enter W (no nnn pairing).
 * h     [19][N] complex out (STENCIL layout). */
int kpm_build_H(const kpm_lattice* lat, const kpm_model* model, const double* n,
                const double* chi, const double* delta, double* h, void* stream);

/* Build h for a collinear spin-density-wave state (App. A at m_i != 0,
 * magnetisation along z): per spin s = up/down the densities n_s [N], bond
 * variables chi_s = <c^dag_{i s} c_{j s}> [4][N] and Delta_s = s <c_{i s} c_{j -s}>
 * [4][N] (complex; both pairing components are nearest-neighbour only in W).
 * h_IJ = dW/drho_IJ (Wirtinger) with rho_{i0,j0} = chi_up, rho_{i1,j1} =
 * -conj(chi_dn), rho_{i0,j1} = -conj(Delta_up), rho_{i1,j0} = -Delta_dn,
 * rho_{i0,i0} = n_up, rho_{i1,i1} = 1 - n_dn, for
 *   W = - sum_bonds sum_s g^t_{i s} g^t_{j s} 2 Re(t_ij chi_s)
 *       + J sum_nn [g^z_ij (m_i m_j - (1/4) sum_s (|chi_s|^2 + |Delta_s|^2))
 *                   - g^xy_ij Re(chi_up conj(chi_dn) + conj(Delta_up) Delta_dn)]
 *       - mu sum_i n_i,
 * the energy of the renormalised Hamiltonian of App. A in the BdG Slater
 * determinant (Wick's theorem), with the printed g^t_{i s}, g^xy_i, X_ij and
 * g^z_ij = g^xy_ij [2(|Dbar|^2 - |chibar|^2) - 4 m_i m_j X^2] / [2(|Dbar|^2 -
 * |chibar|^2) - 4 m_i m_j] (squares read as moduli; chibar, Dbar the spin
 * means).  Its derivatives are the printed eqs. Tij, Dij and mu_i.  At m = 0
 * with equal spins it is kpm_build_H.  The g^z ratio is singular where its
 * denominator vanishes; h is then non-finite (no check here; the recursion
 * reports it). */
int kpm_build_H_sdw(const kpm_lattice* lat, const kpm_model* model, const double* n_up,
                    const double* n_dn, const double* chi_up, const double* chi_dn,
                    const double* delta_up, const double* delta_dn, double* h, void* stream);

/* Vector-Jacobian product of kpm_build_H_sdw, as kpm_build_H_vjp: given rho
 * = dOmega/dh ([19][N] complex, Hermitian), writes dOmega/dtheta = sum_IJ
 * rho_IJ dh_IJ/dtheta over all matrix elements for the per-spin parameters
 * (second derivatives of the W of kpm_build_H_sdw, App. A).  Complex
 * gradients use dOmega/dRe z + i dOmega/dIm z.  dn_up, dn_dn [N] and dchi_up,
 * dchi_dn, ddelta_up, ddelta_dn [4][N] complex are overwritten (ddelta is 0 on
 * the diagonal directions).  rho_{i0,i1} (entry 18) does not enter: that
 * element of h is 0 for every theta. */
int kpm_build_H_sdw_vjp(const kpm_lattice* lat, const kpm_model* model, const double* n_up,
                        const double* n_dn, const double* chi_up, const double* chi_dn,
                        const double* delta_up, const double* delta_dn, const double* rho,
                        double* dn_up, double* dn_dn, double* dchi_up, double* dchi_dn,
                        double* ddelta_up, double* ddelta_dn, void* stream);

/* Vector-Jacobian product of kpm_build_H: given rho = dOmega/dh on the
 * stencil ([19][N] complex), writes dOmega/dtheta = sum_IJ rho_IJ dh_IJ/dtheta
 * over all matrix elements (both halves).  Complex gradients use the
 * convention dOmega/dRe z + i dOmega/dIm z.  dn [N], dchi [4][N], ddelta [4][N]
 * (complex) are overwritten; ddelta is 0 on the diagonal directions. */
int kpm_build_H_vjp(const kpm_lattice* lat, const kpm_model* model, const double* n,
                    const double* chi, const double* delta, const double* rho,
                    double* dn, double* dchi, double* ddelta, void* stream);

/* Spectral rescale (App. B: all eigenvalues must lie in [-1, 1]): Gershgorin
 * bounds Emin, Emax of h and ab[0] = a = (Emax - Emin)/1.99,
 * ab[1] = b = (Emax + Emin)/2, so H~ = (h - b)/a has spectrum in
 * [-0.995, 0.995].  ab: device double[2]. */
int kpm_bounds(const kpm_lattice* lat, const double* h, double* ab, void* stream);

/* Expansion coefficients C_m, m < M, of the grand-potential density
 * f(e) = -T log(1 + e^{-e/T}) (App. B eq. F_KPM):
 *   C_m = (2 - delta_m0) g_m (1/K) sum_k cos(m th_k) f(a cos th_k + b),
 * th_k = pi (k + 1/2)/K (Chebyshev-Gauss quadrature), g_m the Jackson kernel
 * of Weisse et al. (Rev. Mod. Phys. 78, 275), (a, b) read from ab on the
 * device.  K = 0 selects max(4M, 16384).  C: device double[M]. */
int kpm_coefficients(int32_t M, double T, const double* ab, int32_t K, double* C, void* stream);

/* Workspace bytes needed by kpm_moments / kpm_grand_potential(_grad) /
 * kpm_density_matrix for this lattice, R probes, M moments, checkpoint
 * interval ckpt_k (>= 2) and precision.  Returns 0 on invalid arguments. */
size_t kpm_workspace_size(const kpm_lattice* lat, int32_t R, int32_t M, int32_t ckpt_k,
                          int32_t precision);

/* Chebyshev moments mu_{l,m} = r_l^dag T_m(H~) r_l, H~ = (h - ab[1])/ab[0],
 * from the recursion alpha_0 = r, alpha_1 = H~ r, alpha_{m+1} = 2 H~ alpha_m -
 * alpha_{m-1} (App. B eq. alpha).  Vectors in `precision`, sums in FP64.
 * mu: [R][M] doubles (real parts; the imaginary parts vanish for Hermitian h).
 * ws: workspace of at least kpm_workspace_size(lat, R, M, ckpt_k, precision)
 * bytes, 256-byte aligned.  R * Lx * Ly must be below 2^30 (else KPM_EINVAL;
 * the same holds for every instance of a batch plan). */
int kpm_moments(const kpm_lattice* lat, const double* h, const double* ab,
                const kpm_probes* probes, int32_t M, int32_t precision, int32_t ckpt_k,
                double* mu, void* ws, size_t ws_bytes, void* stream);

/* Bytes of the library's static device scratch (one per GPU, held until the
 * process ends) used by kpm_moments_noalloc. */
#define KPM_NOALLOC_SCRATCH_BYTES (64u << 20)

/* kpm_moments for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid allocation): the
 * same moments, with no workspace argument.  Its buffers live in a file-scope
 * static device array of KPM_NOALLOC_SCRATCH_BYTES per GPU; the call makes no
 * hipMalloc, hipFree or other allocation.  It needs the forward-only
 * workspace: 2 vector sets of R * Lx * Ly records (16 B FP32, 32 B FP64), the
 * FP64 moment partials [M][tiles][R] (tiles = ceil(Lx/8) ceil(Ly/4)),
 * the rescaled coefficients (288 B FP32 / 576 B FP64 per tile site) and
 * per-probe tables; a problem beyond the scratch returns KPM_ETOOBIG with
 * nothing enqueued (e.g. 48 x 48 with 64 probes and M = 1024 fits in FP32).
 * The scratch is shared by every call on one GPU and keeps the last call's
 * contents: every part a call reads is written by it first.  Calls that
 * overlap on one GPU (different streams or threads) race on the scratch and
 * must be serialised by the caller.  The stream must belong to the current
 * device.  Arguments, mu layout and device errors as kpm_moments. */
int kpm_moments_noalloc(const kpm_lattice* lat, const double* h, const double* ab,
                        const kpm_probes* probes, int32_t M, int32_t precision, double* mu,
                        void* stream);

/* Grand potential Omega = sum_l w_l sum_m C_m mu_{l,m} (App. B eq. F_KPM with
 * the probe average).  Runs the forward recursion, keeps the checkpoint pairs
 * (alpha_{jk}, alpha_{jk+1}), j = 0,1,..., in ws for kpm_grand_potential_grad.
 * omega: device double[1].  mu: optional ([R][M] doubles) or NULL. */
int kpm_grand_potential(const kpm_lattice* lat, const double* h, const double* ab,
                        const kpm_probes* probes, int32_t M, const double* C,
                        int32_t precision, int32_t ckpt_k, double* omega, double* mu,
                        void* ws, size_t ws_bytes, void* stream);

/* Adjoint of kpm_grand_potential (App. B eqs. dFdH, dalphadH and the beta
 * recursion): with gamma_m = beta_m^dag,
 *   gamma_{M-1} = 0, gamma_{M-2} = w C_{M-1} r,
 *   gamma_m = w C_{m+1} r + 2 H~ gamma_{m+1} - gamma_{m+2},
 *   rho_IJ = omega_bar/a * sum_l [conj(gamma_{0,I}) alpha_{0,J}
 *            + 2 sum_{m=1}^{M-2} conj(gamma_{m,I}) alpha_{m,J}],
 * on the stencil.  alpha_m is recomputed backwards by the reversible
 * recursion alpha_m = 2 H~ alpha_{m+1} - alpha_{m+2}, reset at each stored
 * checkpoint pair.  Must follow kpm_grand_potential on the same ws with the
 * same arguments (else KPM_EWORKSPACE).  It may be called again after that one
 * forward call (e.g. a second backward pass): a repeated call first rebuilds
 * alpha_{M-2}, alpha_{M-1} from the last checkpoint pair (fewer than ckpt_k
 * forward steps) and returns the same rho.  omega_bar: device double[1] or
 * NULL (= 1).  rho: [19][N] complex out (STENCIL layout, FP64). */
int kpm_grand_potential_grad(const kpm_lattice* lat, const double* h, const double* ab,
                             const kpm_probes* probes, int32_t M, const double* C,
                             int32_t precision, int32_t ckpt_k, const double* omega_bar,
                             double* rho, void* ws, size_t ws_bytes, void* stream);

/* kpm_grand_potential followed by kpm_grand_potential_grad with omega_bar = 1,
 * then the order parameters (Model and methods eqs. delta, chi, pairing, via
 * App. B): n_up = rho_{i0,i0}, n_dn = 1 - rho_{i1,i1},
 * chi_up = rho_{i0,j0}, chi_dn = -conj(rho_{i1,j1}),
 * delta_up = <c_{i up} c_{j dn}> = -conj(rho_{i0,j1}),
 * delta_dn = <c_{j up} c_{i dn}> = -rho_{i1,j0}, for every bond (i, j = i+d).
 * omega [1], rho [19][N] complex, n_up/n_dn [N], chi_up/chi_dn/delta_up/
 * delta_dn [4][N] complex; any output except omega and rho may be NULL. */
int kpm_density_matrix(const kpm_lattice* lat, const double* h, const double* ab,
                       const kpm_probes* probes, int32_t M, const double* C,
                       int32_t precision, int32_t ckpt_k, double* omega, double* rho,
                       double* n_up, double* n_dn, double* chi_up, double* chi_dn,
                       double* delta_up, double* delta_dn, void* ws, size_t ws_bytes,
                       void* stream);

/* Direct probing estimate of the density matrix: the probe average of App. B
 * applied to the Chebyshev series of f' = n_F instead of differentiating the
 * probe-estimated Omega (Weisse et al., Rev. Mod. Phys. 78, 275, for KPM
 * correlation functions):
 *   rho_IJ ~= (1/a) sum_l w_l conj(r_{l,I}) [F_M'(H~) r_l]_J,
 * F_M(x) = sum_m C_m T_m(x) the damped series of kpm_coefficients and F_M' its
 * exact derivative, sum_k D_k T_k with D from e_{k-1} = e_{k+1} + 2k C_k.
 * One forward recursion (eq. alpha) with y_l = sum_m D_m alpha_m accumulated
 * in FP64 every second step; no checkpoints, no adjoint.  For the complete
 * unit-vector set it equals kpm_grand_potential_grad's rho; for other probes
 * the two are different estimates of the same matrix.  omega [1] receives
 * Omega as kpm_grand_potential; rho [19][N] complex (STENCIL layout).
 * ws: at least kpm_workspace_size(lat, R, M, M, precision) bytes (any ckpt_k
 * <= M gives a large enough size); the call invalidates the workspace for
 * kpm_grand_potential_grad.  Device errors are latched as for the recursion. */
int kpm_density_matrix_direct(const kpm_lattice* lat, const double* h, const double* ab,
                              const kpm_probes* probes, int32_t M, const double* C,
                              int32_t precision, double* omega, double* rho, void* ws,
                              size_t ws_bytes, void* stream);

/* Chebyshev moments by moment doubling (Weisse et al., Rev. Mod. Phys. 78,
 * 275): with T_{2j} = 2 T_j^2 - T_0 and T_{2j+1} = 2 T_{j+1} T_j - T_1 and
 * T_j(H~) Hermitian,
 *   mu_{2j}   = 2 alpha_j^dag alpha_j - mu_0,
 *   mu_{2j+1} = 2 Re(alpha_{j+1}^dag alpha_j) - mu_1,
 * so the recursion of App. B (eq. alpha) runs to alpha_{M/2} only: half the
 * steps of kpm_moments for the same M moments.  The two sums per step are
 * reduced inside the forward step in FP64.  mu: [R][M] doubles or NULL;
 * with C (kpm_coefficients) and omega both given, Omega as kpm_grand_potential;
 * at least one of mu, omega.  ws: as kpm_density_matrix_direct; the call
 * invalidates the workspace for kpm_grand_potential_grad.  In FP32 the
 * doubled moments carry the rounding of the squared norms (about twice the
 * relative error of the direct moments). */
int kpm_moments_doubling(const kpm_lattice* lat, const double* h, const double* ab,
                         const kpm_probes* probes, int32_t M, const double* C, int32_t precision,
                         double* omega, double* mu, void* ws, size_t ws_bytes, void* stream);

/* Local density of states by KPM (Results: LDOS of the vortex states; the
 * expansion of App. B applied to unit probes, with the Jackson kernel of
 * Weisse et al., Rev. Mod. Phys. 78, 275): for the Nambu indices
 * I = first .. first + count - 1 (I = 2i + a),
 *   A_I(E) = [g_0 mu_{I,0} + 2 sum_{m=1}^{M-1} g_m mu_{I,m} T_m(x)] / (pi a sqrt(1 - x^2)),
 * x = (E - ab[1])/ab[0], mu_{I,m} = e_I^dag T_m(H~) e_I, and A = 0 for |x| >= 1.
 * A_{(i,0)} is the spin-up electron spectral density of site i; A_{(i,1)}(E)
 * the spin-down hole density, i.e. the spin-down electron density at -E.
 * energies: device double[ne]; out: device double[count][ne]; 1 <= count <=
 * 65535 (one grid row per probe).  The series
 * is summed in FP64 whatever the recursion precision.  ws: as
 * kpm_density_matrix_direct with R = count; the call invalidates the
 * workspace for kpm_grand_potential_grad. */
int kpm_ldos(const kpm_lattice* lat, const double* h, const double* ab, int32_t first,
             int32_t count, int32_t M, int32_t precision, const double* energies, int32_t ne,
             double* out, void* ws, size_t ws_bytes, void* stream);

/* Device status word latched by the last recursion on ws: KPM_OK or
 * KPM_EBOUNDS.  Synchronises `stream`. *status is host memory. */
int kpm_status_read(const void* ws, int32_t* status, void* stream);

/* ---- batches of uneven lattices (many instances per launch) -------------- */

/* Create a plan for n_inst lattices of possibly different size, vortex count
 * and probes, all with the same M, precision and checkpoint interval.  The
 * plan owns its device memory.  It runs its instances in groups sized to the
 * Infinity Cache (kpm_batch_groups), each group, when large enough, as two
 * halves on two streams (kpm_batch_streams).  On first use it chooses the
 * probes-per-thread
 * blocking and the block schedule of the forward and of the adjoint kernel by
 * timing every pair (autotune), unless kpm_set_probe_block fixed the block.
 * Picks are remembered per shape (device, precision, every instance's N and
 * R; not M or the checkpoint interval, which do not change a step's cost) in
 * the process and in a text file: the path in the environment variable
 * KPM_TUNE_CACHE, else $XDG_CACHE_HOME/kpm_tune.txt, else
 * $HOME/.cache/kpm_tune.txt.  Each line of that file is
 * "<key> <Pf> <Sf> <Pa> <Sa>", with <key> =
 * "<arch>:<compute units>:<f|d>:<N_0>x<R_0>,<N_1>x<R_1>,...", followed by
 * "/2" for a shape that runs as two halves on two streams (the probe halves
 * of a single lattice, keyed by the whole lattice's N and R; the instance
 * halves of a plan, keyed by all its instances), whose candidates are timed
 * on both halves at once and whose pick serves both halves;
 * a shape tuned with M < 3 (no adjoint step to time) is not remembered;
 * the last valid line of a key is used, and a file that cannot be read or
 * written only disables the disk cache (so does KPM_TUNE_CACHE set to the
 * empty string).  lats/probes: host arrays [n_inst]. */
int kpm_batch_create(int32_t n_inst, const kpm_lattice* lats, const kpm_probes* probes,
                     int32_t M, int32_t precision, int32_t ckpt_k, void** plan);

/* Energy + gradient for every instance: for instance k, with h[k], ab[k],
 * C[k] (host arrays of device pointers), writes omega[k] (device double
 * [n_inst]) and rho[k] ([19][N_k] complex, device).  The forward and adjoint
 * recursions of all instances of a group run as one sequence of batched
 * kernels (the groups one after another on the caller's stream), captured
 * once into a hipGraph and replayed on later calls with the same pointers
 * (use_graph != 0).  A group of two instance halves (see
 * kpm_batch_streams) runs the halves side by side on the caller's stream and
 * on a second stream of the device that the library creates once (default
 * priority): with use_graph, as one graph per half; else with their step
 * launches interleaved.  The caller's stream waits for the second stream
 * before it returns to its own work. */
int kpm_batch_energy_grad(void* plan, const double* const* h, const double* const* ab,
                          const double* const* C, double* omega, double* const* rho,
                          int32_t use_graph, void* stream);

int kpm_batch_destroy(void* plan);

/* Streams a batch plan runs on: 2 when its instances (or those of any of its
 * groups, see kpm_batch_groups) form two halves of nearly equal R N (largest
 * first, each to the lighter half), each half with its own kernel tables,
 * both tuned together (one pick, timed on the pair); 1 otherwise;
 * KPM_EINVAL for a null plan.  Fixed when the plan is created, from
 * kpm_set_streams: 1, one stream; 2, halves (groups of two or more
 * instances); 0 (default), automatic: halves when the group's instances hold
 * sum R N >= 2^19 site-probes.  Each instance's
 * results are the same either way, bit for bit, for a fixed probe block and
 * schedule: an instance's kernels and sums do not depend on the other
 * instances. */
int32_t kpm_batch_streams(const void* plan);

/* Instance groups of a batch plan: the plan runs its instances as groups of
 * nearly equal R N (largest first, each to the lightest group), one group
 * after another, each group with its own kernel tables, tuning and (see
 * kpm_batch_streams) halves.  Automatic (kpm_set_batch_groups(0), the
 * default): as many groups as keep each group's adjoint step traffic, 6
 * passes of sum R N records (16 B FP32, 32 B FP64) over 4 distinct vector
 * sets, within 240 MB, so that those sets stay in the 256 MB Infinity Cache
 * of the MI355X from one step to the next instead of streaming from HBM
 * (the 48 uneven lattices of 24-64 sites a side with 64 probes each: 3
 * groups in FP32, 191 ms per energy + gradient against 259 ms as one
 * group).  Fixed when the plan is created.  Each instance's
 * results are the same either way, bit for bit, for a fixed probe block and
 * schedule.  Returns the group count (1: no groups), KPM_EINVAL for a null
 * plan.  kpm_batch_tuning reports the first group's configuration;
 * kpm_batch_streams is 2 when any group runs as halves. */
int32_t kpm_batch_groups(const void* plan);

/* Group count of the batch plans created from now on: 0 automatic (see
 * kpm_batch_groups), else that many groups (at most one per instance).
 * Process-wide; returns the previous value (negative values leave the
 * setting unchanged). */
int32_t kpm_set_batch_groups(int32_t groups);

/* The plan's kernel configuration (host int32_t out[5]): forward probe block,
 * forward schedule, adjoint probe block, adjoint schedule, and where they
 * came from: 0 timed by this plan, 1 this process's cache, 2 the disk cache,
 * -1 not tuned (fixed by kpm_set_probe_block / kpm_set_schedule, or the plan
 * has not run yet).  Schedules are KPM_SCHED_* values.  A plan of two
 * instance halves runs one configuration on both; a plan of instance groups
 * (kpm_batch_groups) reports its first group's. */
int kpm_batch_tuning(const void* plan, int32_t* out);

/* Probes-per-thread blocking used by the single-lattice calls (0 = automatic,
 * else one of 1, 2, 4, 8, 16, 32).  Process-wide; returns the previous value.
 * Batch plans created while it is nonzero use it too, and are not tuned.
 * Automatic: the configuration remembered for the call's shape (see
 * kpm_batch_create for the process and file caches); a shape not seen yet is
 * tuned by its first kpm_grand_potential (or kpm_density_matrix) call, on
 * that call's workspace, unless the stream is being captured; until then a
 * size heuristic picks the blocks.  A shape's entry in the file is read at
 * most once per process.  kpm_moments_noalloc always uses the heuristic.
 * The picks change results only through the order of floating-point sums
 * (the FP32 per-wave sums and the FP64 partial sums of the adjoint): within
 * 1e-7 relative in FP32, 1e-14 in FP64.  Fixing the block (and the schedules
 * with kpm_set_schedule), or a prepared cache file, makes runs repeatable
 * across processes. */
int32_t kpm_set_probe_block(int32_t probes_per_thread);

/* Streams of the single-lattice energy, gradient and moment calls
 * (kpm_moments, kpm_grand_potential, kpm_grand_potential_grad,
 * kpm_density_matrix), and of the batch plans created while it is set (see
 * kpm_batch_streams): 1, everything on the caller's stream; 2, the probes in
 * two halves (ceil(R/2) and floor(R/2) probes) whose recursions run side by
 * side on the caller's stream and on a second stream of the device that the
 * library creates once (default priority), with their step launches
 * interleaved, so that one half's blocks fill the slots another launch leaves
 * idle; Omega, the moments and rho are then reduced over both halves on the
 * caller's stream, which waits for the second stream before it returns to
 * its own work; 0 (default), automatic: halves when R >= 128 and
 * R N >= 2^19 (with fewer probes a half leaves the chip short of work).
 * A stream being captured into a graph always runs on one stream, and a
 * gradient follows the layout of the forward call it completes.  Halves
 * change results only through the order of floating-point sums (FP64 sums
 * of the moments and the partial sums, 1e-14 relative; the FP32 per-wave
 * sums of the adjoint, 1e-7).  The halves are tuned as a pair (see
 * kpm_batch_create for the cache key).
 * Process-wide; returns the previous value (values outside 0..2 leave the
 * setting unchanged). */
int32_t kpm_set_streams(int32_t n);

/* Block schedules of the recursion kernels (how (tile, probe range) work
 * items map to blocks, and so to the 8 XCDs that blocks are dealt to in
 * turn): KPM_SCHED_TILE_MAJOR, tiles in order with the probe range fastest;
 * KPM_SCHED_RANGES, each XCD one probe range on its share of contiguous tiles
 * (when the range count divides 8, else tile-major); KPM_SCHED_STRIPS, each
 * XCD one eighth of the tiles, range after range; KPM_SCHED_STRIP_TILES, each
 * XCD one eighth of the tiles, tile after tile with all probe ranges of a
 * tile in a row; KPM_SCHED_BALANCED (adjoint steps of a single lattice; the
 * forward steps run their default), the (tile, probe) work cut into one equal
 * share per block that the chip holds at once, so every compute unit gets the
 * same work in a single round (each XCD one eighth of the work, the probes in
 * two halves when R is even; the partial sums use up to ceil(R/4) FP64 slices,
 * and the schedule falls back to ranges when that is not enough or the
 * lattice is too small to fill the grid).  KPM_SCHED_DEFAULT is strips for
 * the forward steps and ranges for the adjoint. */
#define KPM_SCHED_DEFAULT (-1)
#define KPM_SCHED_TILE_MAJOR 0
#define KPM_SCHED_RANGES 1
#define KPM_SCHED_STRIPS 2
#define KPM_SCHED_STRIP_TILES 3
#define KPM_SCHED_BALANCED 4

/* Schedules used, while the probe block is fixed (kpm_set_probe_block
 * nonzero), by the single-lattice calls and the batch plans created then;
 * with the automatic block the tuned schedules apply.  Process-wide.
 * Returns KPM_EINVAL (nothing changed) for a value outside -1..4.  The
 * results do not depend on the schedule, up to the order of FP64 sums of the
 * adjoint partial sums. */
int kpm_set_schedule(int32_t fwd, int32_t adj);

/* ---- self-consistent iteration (RMFT outer loop) ---------------------------
 * Model and methods: the local order parameters that define h (eqs. delta,
 * chi, pairing) are fixed by self-consistency, theta -> h(theta) -> rho ->
 * theta', iterated until they stop changing; App. A: the electron number is
 * held by the Lagrange multiplier mu.  The paper states neither the update
 * rule nor how mu is found; this library uses linear mixing of the spin-
 * averaged map below and a bracketed bisection of mu at every iteration. */

/* Length, in doubles, of the `stats` buffer of kpm_rmft_update: [0] mean n',
 * [1] max residual, [2] Omega (written by kpm_rmft_iterate), [3..7] unused,
 * then per-block partial results. */
#define KPM_RMFT_STATS_LEN 520

/* Largest history depth of Anderson mixing in kpm_rmft_iterate. */
#define KPM_RMFT_MAX_ANDERSON 8

/* Spin-singlet map of the density matrix onto the builder's parameters
 * (eqs. delta, chi, pairing through App. B's Nambu spinor; the two spin
 * estimates of a singlet quantity are averaged), for every site i and bond
 * (i, j = i + d), d = 0..3:
 *   n'_i       = rho_{i0,i0} + 1 - rho_{i1,i1}
 *   chi'_d,i   = (rho_{i0,j0} - conj(rho_{i1,j1})) / 2
 *   delta'_d,i = (-conj(rho_{i0,j1}) - rho_{i1,j0}) / 2,
 * then theta <- theta + mix (theta' - theta) for theta = (n, chi, delta), in
 * place.  mix in [0, 1]; mix = 0 leaves theta unchanged (measurement only).
 * stats (device double[KPM_RMFT_STATS_LEN]) receives [0] = (1/N) sum_i n'_i
 * and [1] = max over i, d of |n' - n|, |chi' - chi|, |delta' - delta|
 * (complex moduli; theta before the update); NaN propagates to both.  The
 * reductions run in a fixed order (bitwise reproducible).
 * rho [19][N] complex (STENCIL layout), n [N], chi/delta [4][N] complex. */
int kpm_rmft_update(const kpm_lattice* lat, const double* rho, double mix, double* n,
                    double* chi, double* delta, double* stats, void* stream);

enum { KPM_RMFT_BISECTION = 0, KPM_RMFT_ILLINOIS = 1 };   /* mu search inside the bracket */
enum { KPM_RMFT_ADJOINT = 0, KPM_RMFT_DIRECT = 1 };       /* rho of an evaluation           */

typedef struct {
  double doping;      /* target hole density: (1/N) sum_i n_i = 1 - doping, 0 < doping < 1 */
  double mix;         /* linear mixing weight, 0 < mix <= 1                          */
  double tol_n;       /* accept mu when |mean n' - (1 - doping)| <= tol_n (>= 0)      */
  double tol_mu;      /* or when half the bisection bracket is <= tol_mu (>= 0)       */
  double mu_step;     /* first step of the bracket search (> 0)                       */
  double tol_residual;/* stop once an iteration's residual <= tol_residual (0: never) */
  int32_t max_evals;  /* density-matrix evaluations allowed per iteration (>= 1)      */
  int32_t coef_K;     /* quadrature points of kpm_coefficients (0 = default)          */
  int32_t search;     /* KPM_RMFT_BISECTION or KPM_RMFT_ILLINOIS                      */
  int32_t estimator;  /* KPM_RMFT_ADJOINT (kpm_grand_potential + _grad) or
                         KPM_RMFT_DIRECT (kpm_density_matrix_direct)                 */
  int32_t anderson;   /* 0: linear mixing; 1 .. KPM_RMFT_MAX_ANDERSON: Anderson mixing
                         with that history depth (see kpm_rmft_iterate)              */
  int32_t pad;
} kpm_rmft_params;

typedef struct {      /* one completed iteration (host memory)                        */
  double mu;          /* accepted chemical potential                                  */
  double nbar;        /* mean n' at mu                                                */
  double residual;    /* max |theta' - theta| at mu, before mixing                    */
  double omega;       /* grand potential Omega of h(theta, mu)                        */
  int32_t evals;      /* density-matrix evaluations spent                             */
  int32_t pad;
} kpm_rmft_record;

/* Workspace bytes of kpm_rmft_iterate and kpm_rmft_iterate_sdw (the
 * kpm_workspace_size region first, then h, rho, ab, C, stats and the Anderson
 * vectors, sized for the 34 N doubles of a spin-polarised theta).  0 on
 * invalid arguments. */
size_t kpm_rmft_workspace_size(const kpm_lattice* lat, int32_t R, int32_t M, int32_t ckpt_k,
                               int32_t precision);

/* Up to n_iter self-consistency iterations.  One iteration, with theta fixed:
 * an evaluation at mu builds h(theta, mu) (kpm_build_H with model->mu
 * replaced), rescales it (kpm_bounds), expands f (kpm_coefficients with T and
 * coef_K) and runs kpm_grand_potential + kpm_grand_potential_grad for rho
 * (or kpm_density_matrix_direct when estimator is KPM_RMFT_DIRECT),
 * then measures e(mu) = mean n' - (1 - doping) (kpm_rmft_update, mix = 0).
 * mu search, starting at *mu: accept an evaluation with |e| <= tol_n;
 * otherwise step from the last point on the side of e(*mu) by s = mu_step,
 * 2 mu_step, 4 mu_step, ... (up if e < 0, down if e > 0) until e changes
 * sign, then narrow the bracket [a, b] (b the newest point):
 *   BISECTION: m = (a + b)/2; accept m when |e(m)| <= tol_n or
 *              |b - a|/2 <= tol_mu, else keep the half that brackets the root;
 *   ILLINOIS:  m = b - e_b (b - a)/(e_b - e_a) (false position); if e(m) and
 *              e_b differ in sign a <- b, else e_a <- e_a/2; then b <- m;
 *              accept m when |e(m)| <= tol_n or |b - a| <= tol_mu
 *              (Dowell & Jarratt, BIT 11, 168 (1971)).
 * The accepted rho then updates theta with `mix` (kpm_rmft_update), or, with
 * anderson = m > 0, by Anderson mixing (Anderson, J. ACM 12, 547 (1965); the
 * form of Walker & Ni, SIAM J. Numer. Anal. 49, 1715 (2011)) on the flat
 * vector x = (n, chi, delta as interleaved re/im), 17 N doubles, with
 * residual f = x' - x (x' the map of kpm_rmft_update): keeping the
 * differences dX_j, dF_j of the last min(k, m) iterations of this call,
 *   gamma = solve(G + 1e-12 max_i G_ii I, dF^T f), G = dF^T dF,
 *   x <- x + mix f - sum_j gamma_j (dX_j + mix dF_j)   (oldest j first);
 * the history starts empty at each call (its first iteration is linear).
 * *mu becomes the accepted mu.
 * n, chi, delta: device, updated in place (layouts of kpm_build_H).
 * mu: host double in/out.  history: host [n_iter] or NULL.  n_done: host,
 * iterations completed.  ws: kpm_rmft_workspace_size bytes, 256-byte aligned.
 * Synchronises `stream` after every evaluation (the host decides the next mu).
 * Returns KPM_ENOCONV when an iteration spends max_evals evaluations without
 * accepting (theta, *mu and history hold the last completed iteration), the
 * recursion's KPM_EBOUNDS when h leaves the rescaled interval or a value is
 * non-finite, KPM_EINVAL for bad arguments (nothing enqueued). */
int kpm_rmft_iterate(const kpm_lattice* lat, const kpm_model* model, const kpm_probes* probes,
                     int32_t M, double T, int32_t precision, int32_t ckpt_k,
                     const kpm_rmft_params* params, int32_t n_iter, double* n, double* chi,
                     double* delta, double* mu, kpm_rmft_record* history, int32_t* n_done,
                     void* ws, size_t ws_bytes, void* stream);

/* Per-spin map for a collinear spin-polarised theta (App. A at m_i != 0, the
 * inverse of the rho entries of kpm_build_H_sdw; no spin average), for every
 * site i and bond (i, j = i + d), d = 0..3:
 *   n'_up = rho_{i0,i0},           n'_dn = 1 - rho_{i1,i1},
 *   chi'_up = rho_{i0,j0},         chi'_dn = -conj(rho_{i1,j1}),
 *   delta'_up = -conj(rho_{i0,j1}), delta'_dn = -rho_{i1,j0},
 * then theta <- theta + mix (theta' - theta) in place, as kpm_rmft_update:
 * stats [0] = (1/N) sum_i (n'_up + n'_dn), [1] = max over all components of
 * |theta' - theta| (theta before the update).  For equal spins the spin
 * means of theta' are the singlet map of kpm_rmft_update.  Layouts of
 * kpm_build_H_sdw. */
int kpm_rmft_update_sdw(const kpm_lattice* lat, const double* rho, double mix, double* n_up,
                        double* n_dn, double* chi_up, double* chi_dn, double* delta_up,
                        double* delta_dn, double* stats, void* stream);

/* kpm_rmft_iterate for a spin-polarised theta: each evaluation builds h with
 * kpm_build_H_sdw and measures with kpm_rmft_update_sdw (mix = 0); the update
 * is kpm_rmft_update_sdw with `mix`, or Anderson mixing on the flat vector
 * x = (n_up, n_dn, chi_up, chi_dn, delta_up, delta_dn as interleaved re/im),
 * 34 N doubles.  The mu search, arguments, workspace and returns are those
 * of kpm_rmft_iterate. */
int kpm_rmft_iterate_sdw(const kpm_lattice* lat, const kpm_model* model, const kpm_probes* probes,
                         int32_t M, double T, int32_t precision, int32_t ckpt_k,
                         const kpm_rmft_params* params, int32_t n_iter, double* n_up,
                         double* n_dn, double* chi_up, double* chi_dn, double* delta_up,
                         double* delta_dn, double* mu, kpm_rmft_record* history, int32_t* n_done,
                         void* ws, size_t ws_bytes, void* stream);

/* ---- magnetic super-cell exact diagonalisation and LDOS -------------------
 * App. on the local density of states and the magnetic super-cell method.
 * The converged h of one magnetic unit cell (the [19][N] stencil on the
 * torus; its wrap-around bonds carry the field's magnetic boundary phases)
 * is repeated over Mx x My cells.  By the magnetic Bloch theorem (eq.
 * matrixeqn) both Nambu amplitudes of a quasiparticle pick up the same factor
 * exp(-i k.R) from cell to cell, with k = 2 pi (m_x/(Mx Lx), m_y/(My Ly)), so
 * the enlarged lattice splits into Mx My cell-sized Bloch matrices H(k). */

#define KPM_SUPERCELL_MAX_N 16384   /* sites per cell (dense matrices of (2N)^2) */
#define KPM_SUPERCELL_MAX_K 4096    /* Mx * My                                   */
#define KPM_SUPERCELL_MAX_BATCH 16  /* k points per batched eigensolver call      */

/* Dense Bloch matrix H(k) for twist angles phi = (k_x Lx, k_y Ly): the torus h
 * with every element of a bond whose head lies in the neighbouring cell
 * (s_x, s_y) (s = -1, 0, +1) multiplied by exp(-i (s_x phi_x + s_y phi_y)),
 * its Hermitian partner by the conjugate.  Hk: device complex, column-major,
 * 2N columns of leading dimension ld >= 2N (Nambu index I = 2i + a); rows
 * 0..2N-1 of every column are overwritten.  Lx, Ly >= 3. */
int kpm_bloch_H(const kpm_lattice* lat, const double* h, double phi_x, double phi_y, double* Hk,
                int64_t ld, void* stream);

/* The site weights of eq. Gij at i = j for kpm_supercell_ldos: w_s =
 * (g^t_{i s})^2 with the per-spin Gutzwiller factor of App. A,
 *   (g^t_s)^2 = 2 delta (1 - delta)/(1 - delta^2 + 4 m^2)
 *               * (1 + delta + 2 s m)/(1 + delta - 2 s m),
 * delta = 1 - n_up - n_dn, m = (n_up - n_dn)/2 (2 delta/(1 + delta) at m = 0;
 * reading g^t_ij = g^t_i g^t_j at i = j).  n_up, n_dn, w_up, w_dn: device [N]
 * (a singlet state passes n_up = n_dn = n/2). */
int kpm_gutzwiller_weights(const kpm_lattice* lat, const double* n_up, const double* n_dn,
                           double* w_up, double* w_dn, void* stream);

/* Workspace bytes of kpm_supercell_ldos with k_batch (1..KPM_SUPERCELL_MAX_BATCH)
 * k points per eigensolver call: k_batch dense matrices of (2N)^2 complex
 * values, their eigenvalues, the site list and per-k solver flags.  0 on
 * invalid arguments. */
size_t kpm_supercell_workspace_size(const kpm_lattice* lat, int32_t k_batch);

/* Broadened LDOS of eqs. N_i and Gij over the k grid, for the k indices
 * q = k_first .. k_first + k_count - 1 (q = m_y Mx + m_x; phi = 2 pi (m_x/Mx,
 * m_y/My)).  For each k: H(k) (kpm_bloch_H), its eigenpairs (E_q, (u, v)) by
 * rocSOLVER zheevd (k_batch k points per strided-batched call; the workspace
 * must be sized for that k_batch), then for every listed site i and energy omega
 *   ldos[s][e] += 1/(Mx My) sum_q [w_up_i |u_i^q|^2 L(omega - E_q)
 *                                + w_dn_i |v_i^q|^2 L(omega + E_q)],
 *   L(x) = (Gamma/pi) / (x^2 + Gamma^2),  Gamma = alpha |omega| + gamma0,
 * the spin-up electron weight at +E and the spin-down one (hole amplitude) at
 * -E.  Splitting the k grid over calls (accumulate = 1) sums the same result.
 * h: device [19][N] stencil.  sites: HOST int32 [n_sites] site indices in
 * [0, N) (validated here).  omega: device [n_omega].  alpha >= 0, gamma0 > 0.
 * w_up, w_dn: device [N] weights (the g^t factors at i = j of eq. Gij) or
 * NULL for 1.  accumulate: 0 overwrites ldos, 1 adds to it.  ldos: device
 * [n_sites][n_omega].  evals: device [k_count][2N] ascending eigenvalues, or
 * NULL.  ws: kpm_supercell_workspace_size bytes, 256-byte aligned.  Returns
 * after the stream has drained (it reads the solver flags); KPM_EDEVICE when
 * the eigensolver fails or does not converge for some k. */
int kpm_supercell_ldos(const kpm_lattice* lat, const double* h, int32_t Mx, int32_t My,
                       int32_t k_first, int32_t k_count, int32_t k_batch, const int32_t* sites,
                       int32_t n_sites,
                       const double* omega, int32_t n_omega, double alpha, double gamma0,
                       const double* w_up, const double* w_dn, int32_t accumulate, double* ldos,
                       double* evals, void* ws, size_t ws_bytes, void* stream);

/* ---- measurement ----------------------------------------------------------
 * Between kpm_profile_begin and kpm_profile_end, runs of min(16, sample_every)
 * consecutive forward-step (or adjoint-step) kernel launches of this library,
 * one run starting every `sample_every` launches of that kind, are timed by
 * start/stop events recorded by the first and last dispatch of the run on its
 * own stream (not inside a graph capture; a run interrupted by any other
 * launch of the library is dropped).  kpm_profile_end synchronises those
 * events and returns, for both kinds, the summed run durations (milliseconds,
 * host memory) and the number of launches they cover, so that the ratio is the
 * average launch duration, inter-kernel gaps included. */
int kpm_profile_begin(int32_t sample_every);
int kpm_profile_end(double* fwd_ms, int32_t* n_fwd, double* adj_ms, int32_t* n_adj);

const char* kpm_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif /* KPM_H */
