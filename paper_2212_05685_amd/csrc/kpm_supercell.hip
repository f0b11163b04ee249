// Magnetic super-cell exact diagonalisation and the broadened LDOS (App. on
// the local density of states and the magnetic super-cell method): the
// twisted Bloch matrices H(k) of one magnetic unit cell (eq. matrixeqn),
// their eigenpairs (rocSOLVER zheevd, the one dense library step), and
// N_i(omega) of eqs. N_i and Gij with an energy-dependent Lorentzian width.
//
// Data layout in HBM (N sites, n = 2N):
//   H(k)  [n][ld] double2, column-major (the eigensolver's layout); after the
//         eigensolver column q holds eigenvector q (u at row 2i, v at 2i + 1)
//   E     [n] ascending eigenvalues of one k
//   ldos  [S][W] double (site-major), accumulated over k
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/kpm.h"

namespace {

constexpr int kZB = 256;                  // fill / scatter threads per block
constexpr int kLS = 64;                   // LDOS: sites per block (one per lane)
constexpr int kQL = 8;                    // LDOS: waves per block, splitting the eigenvectors
constexpr int kEC = 16;                   // LDOS: energies per block (registers per thread)
constexpr int kNT = 64;                   // LDOS: eigenvectors per LDS tile

__constant__ int kDx[4] = {1, 0, 1, 1};
__constant__ int kDy[4] = {0, 1, 1, -1};

// Zero rows 0..n-1 of columns 0..n-1.
__global__ __launch_bounds__(kZB) void k_bloch_zero(long long n, long long ld, double2* __restrict__ H) {
  const long long total = n * n;
  for (long long e = (long long)blockIdx.x * kZB + threadIdx.x; e < total; e += (long long)gridDim.x * kZB) {
    const long long col = e / n, row = e - col * n;
    H[col * ld + row] = make_double2(0.0, 0.0);
  }
}

// One thread per site: its four tail bonds (both Nambu rows and columns, and
// the Hermitian partner entries) and its on-site block.  A bond whose head
// lies in the neighbouring cell (sx, sy) carries exp(-i (sx phi_x + sy phi_y)).
// With Lx, Ly >= 3 the eight neighbours of a site are distinct and differ from
// it, so every entry has at most one writer.
__global__ __launch_bounds__(kZB) void k_bloch_scatter(int Lx, int Ly, const double2* __restrict__ st,
                                                       double phx, double phy, long long ld,
                                                       double2* __restrict__ H) {
  const int N = Lx * Ly;
  const int i = blockIdx.x * kZB + threadIdx.x;
  if (i >= N) return;
  const int x = i % Lx, y = i / Lx;
  for (int d = 0; d < 4; ++d) {
    const int xh = x + kDx[d], yh = y + kDy[d];
    const int sx = (xh >= Lx) - (xh < 0), sy = (yh >= Ly) - (yh < 0);
    const int j = (yh - sy * Ly) * Lx + (xh - sx * Lx);
    double sn = 0.0, cs = 1.0;
    if (sx != 0 || sy != 0) sincos(-(sx * phx + sy * phy), &sn, &cs);
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        const double2 h = st[(size_t)(4 * d + 2 * a + b) * N + i];
        const double2 v = make_double2(h.x * cs - h.y * sn, h.x * sn + h.y * cs);
        const long long I = 2LL * i + a, J = 2LL * j + b;
        H[J * ld + I] = v;                                 // H[I][J]
        H[I * ld + J] = make_double2(v.x, -v.y);           // H[J][I] = conj
      }
  }
  const long long I0 = 2LL * i, I1 = I0 + 1;
  const double2 od = st[(size_t)18 * N + i];
  H[I0 * ld + I0] = make_double2(st[(size_t)16 * N + i].x, 0.0);
  H[I1 * ld + I1] = make_double2(st[(size_t)17 * N + i].x, 0.0);
  H[I1 * ld + I0] = od;                                    // H[i0][i1]
  H[I0 * ld + I1] = make_double2(od.x, -od.y);             // H[i1][i0]
}

// N_i(omega_e) += wk * sum_q [wu_i |U_{2i,q}|^2 L(omega_e - E_q) + wd_i |U_{2i+1,q}|^2 L(omega_e + E_q)],
// L(x) = (G/pi)/(x^2 + G^2), G = alpha |omega_e| + gamma0.  A block owns kLS
// sites of the list and kEC energies (block.y); its kQL waves split the
// eigenvector index q (wave w takes q = w mod kQL), each lane one site, so a
// wave's loads of one column are coalesced.  The Lorentzians of kNT
// eigenvalues x kEC energies are staged in LDS per tile; the kQL partial sums
// are added in a fixed order at the end (bitwise reproducible).
__global__ __launch_bounds__(kLS * kQL) void k_sc_ldos(int n, long long ld, const double2* __restrict__ U,
                                                       const double* __restrict__ E,
                                                       const int* __restrict__ sites, int S,
                                                       const double* __restrict__ omega, int W,
                                                       double alpha, double gamma0,
                                                       const double* __restrict__ wu,
                                                       const double* __restrict__ wd, double wk,
                                                       double* __restrict__ out) {
  __shared__ double Lm[kNT][kEC], Lp[kNT][kEC];
  __shared__ double red[kQL][kEC][kLS];
  const int sl = threadIdx.x % kLS, ql = threadIdx.x / kLS;
  const int s = blockIdx.x * kLS + sl;
  const int site = sites[min(s, S - 1)];
  const int e0 = blockIdx.y * kEC;
  const double pu = wu ? wu[site] : 1.0, pd = wd ? wd[site] : 1.0;
  double acc[kEC];
#pragma unroll
  for (int e = 0; e < kEC; ++e) acc[e] = 0.0;
  const double2* urow = U + 2LL * site;
  for (int q0 = 0; q0 < n; q0 += kNT) {
    __syncthreads();
    for (int t = threadIdx.x; t < kNT * kEC; t += kLS * kQL) {
      const int q = t / kEC, e = t % kEC;
      double lm = 0.0, lp = 0.0;
      if (q0 + q < n && e0 + e < W) {
        const double w = omega[e0 + e], Eq = E[q0 + q];
        const double g = alpha * fabs(w) + gamma0;
        const double c = g / M_PI;
        lm = c / ((w - Eq) * (w - Eq) + g * g);
        lp = c / ((w + Eq) * (w + Eq) + g * g);
      }
      Lm[q][e] = lm;
      Lp[q][e] = lp;
    }
    __syncthreads();
    const int qn = min(kNT, n - q0);
    for (int q = ql; q < qn; q += kQL) {
      const double2* col = urow + (long long)(q0 + q) * ld;
      const double2 u = col[0], v = col[1];
      const double au = pu * (u.x * u.x + u.y * u.y), av = pd * (v.x * v.x + v.y * v.y);
#pragma unroll
      for (int e = 0; e < kEC; ++e) acc[e] = fma(au, Lm[q][e], fma(av, Lp[q][e], acc[e]));
    }
  }
#pragma unroll
  for (int e = 0; e < kEC; ++e) red[ql][e][sl] = acc[e];
  __syncthreads();
  for (int t = threadIdx.x; t < kEC * kLS; t += kLS * kQL) {
    const int e = t / kLS, l = t % kLS;
    const int so = blockIdx.x * kLS + l;
    if (so >= S || e0 + e >= W) continue;
    double sum = 0.0;
    for (int w = 0; w < kQL; ++w) sum += red[w][e][l];
    out[(size_t)so * W + e0 + e] += wk * sum;
  }
}

// w_s = (g^t_{i s})^2, the Gutzwiller factor of eq. Gij at i = j, with the
// per-spin g^t of App. A: (g^t_s)^2 = 2 delta (1 - delta)/(1 - delta^2 + 4 m^2)
// * (1 + delta + 2 s m)/(1 + delta - 2 s m), delta = 1 - n_up - n_dn,
// m = (n_up - n_dn)/2 (2 delta/(1 + delta) at m = 0).
__global__ __launch_bounds__(kZB) void k_gt_weights(int N, const double* __restrict__ nu,
                                                    const double* __restrict__ nd,
                                                    double* __restrict__ wu, double* __restrict__ wd) {
  const int i = blockIdx.x * kZB + threadIdx.x;
  if (i >= N) return;
  const double dl = 1.0 - nu[i] - nd[i], m = 0.5 * (nu[i] - nd[i]);
  const double base = 2.0 * dl * (1.0 - dl) / (1.0 - dl * dl + 4.0 * m * m);
  wu[i] = base * (1.0 + dl + 2.0 * m) / (1.0 + dl - 2.0 * m);
  wd[i] = base * (1.0 + dl - 2.0 * m) / (1.0 + dl + 2.0 * m);
}

__global__ __launch_bounds__(kZB) void k_fill0(long long len, double* __restrict__ p) {
  for (long long e = (long long)blockIdx.x * kZB + threadIdx.x; e < len; e += (long long)gridDim.x * kZB)
    p[e] = 0.0;
}

bool valid_cell(const kpm_lattice* L) {
  return L && L->Lx >= 3 && L->Ly >= 3 && (L->n_vortex % 2) == 0 &&
         (long long)L->Lx * L->Ly <= KPM_SUPERCELL_MAX_N;
}

size_t align_up(size_t b) { return (b + 255) & ~(size_t)255; }

struct ScLayout {
  size_t H, E, sites, info, total;
};

ScLayout sc_layout(long long N, int kb) {
  const long long n = 2 * N;
  ScLayout z{};
  size_t off = 0;
  z.H = off;     off += align_up((size_t)kb * n * n * sizeof(double2));
  z.E = off;     off += align_up((size_t)kb * n * sizeof(double) * 2);   // eigenvalues + tridiagonal scratch
  z.sites = off; off += align_up((size_t)N * sizeof(int));
  z.info = off;  off += align_up((size_t)KPM_SUPERCELL_MAX_K * sizeof(int));
  z.total = off;
  return z;
}

int launch_bloch(const kpm_lattice* lat, const double* h, double phx, double phy, double2* H,
                 long long ld, hipStream_t s) {
  const long long N = (long long)lat->Lx * lat->Ly, n = 2 * N;
  const long long zb = std::min<long long>((n * n + kZB - 1) / kZB, 1 << 16);
  hipLaunchKernelGGL(k_bloch_zero, dim3((unsigned)zb), dim3(kZB), 0, s, n, ld, H);
  if (hipGetLastError() != hipSuccess) return KPM_EDEVICE;
  hipLaunchKernelGGL(k_bloch_scatter, dim3((unsigned)((N + kZB - 1) / kZB)), dim3(kZB), 0, s, lat->Lx,
                     lat->Ly, reinterpret_cast<const double2*>(h), phx, phy, ld, H);
  if (hipGetLastError() != hipSuccess) return KPM_EDEVICE;
  return KPM_OK;
}

}  // namespace

extern "C" {

int kpm_bloch_H(const kpm_lattice* lat, const double* h, double phi_x, double phi_y, double* Hk,
                int64_t ld, void* stream) {
  if (!valid_cell(lat) || !h || !Hk || !std::isfinite(phi_x) || !std::isfinite(phi_y)) return KPM_EINVAL;
  const long long n = 2LL * lat->Lx * lat->Ly;
  if (ld < n) return KPM_EINVAL;
  return launch_bloch(lat, h, phi_x, phi_y, reinterpret_cast<double2*>(Hk), ld,
                      static_cast<hipStream_t>(stream));
}

int kpm_gutzwiller_weights(const kpm_lattice* lat, const double* n_up, const double* n_dn,
                           double* w_up, double* w_dn, void* stream) {
  if (!lat || lat->Lx < 1 || lat->Ly < 1 || !n_up || !n_dn || !w_up || !w_dn) return KPM_EINVAL;
  const long long N = (long long)lat->Lx * lat->Ly;
  if (N >= (1LL << 31)) return KPM_EINVAL;
  hipLaunchKernelGGL(k_gt_weights, dim3((unsigned)((N + kZB - 1) / kZB)), dim3(kZB), 0,
                     static_cast<hipStream_t>(stream), (int)N, n_up, n_dn, w_up, w_dn);
  return hipGetLastError() == hipSuccess ? KPM_OK : KPM_EDEVICE;
}

size_t kpm_supercell_workspace_size(const kpm_lattice* lat, int32_t k_batch) {
  if (!valid_cell(lat) || k_batch < 1 || k_batch > KPM_SUPERCELL_MAX_BATCH) return 0;
  return sc_layout((long long)lat->Lx * lat->Ly, k_batch).total;
}

int kpm_supercell_ldos(const kpm_lattice* lat, const double* h, int32_t Mx, int32_t My,
                       int32_t k_first, int32_t k_count, int32_t k_batch, const int32_t* sites,
                       int32_t n_sites,
                       const double* omega, int32_t n_omega, double alpha, double gamma0,
                       const double* w_up, const double* w_dn, int32_t accumulate, double* ldos,
                       double* evals, void* ws, size_t ws_bytes, void* stream) {
  if (!valid_cell(lat) || !h || !sites || !omega || !ldos || !ws) return KPM_EINVAL;
  if (Mx < 1 || My < 1 || (long long)Mx * My > KPM_SUPERCELL_MAX_K) return KPM_EINVAL;
  if (k_first < 0 || k_count < 1 || (long long)k_first + k_count > (long long)Mx * My) return KPM_EINVAL;
  if (k_batch < 1 || k_batch > KPM_SUPERCELL_MAX_BATCH) return KPM_EINVAL;
  if (n_sites < 1 || n_omega < 1 || !(alpha >= 0.0) || !(gamma0 > 0.0) || !std::isfinite(alpha) ||
      !std::isfinite(gamma0) || (accumulate != 0 && accumulate != 1))
    return KPM_EINVAL;
  const long long N = (long long)lat->Lx * lat->Ly, n = 2 * N;
  if (n_sites > N || (long long)n_sites * n_omega >= (1LL << 31) || (n_omega + kEC - 1) / kEC > 65535)
    return KPM_EINVAL;
  for (int s = 0; s < n_sites; ++s)
    if (sites[s] < 0 || sites[s] >= N) return KPM_EINVAL;
  const ScLayout z = sc_layout(N, k_batch);
  if (ws_bytes < z.total || (reinterpret_cast<uintptr_t>(ws) & 255) != 0) return KPM_EWORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  double2* H = reinterpret_cast<double2*>(base + z.H);
  double* Ebuf = reinterpret_cast<double*>(base + z.E);
  double* Etri = Ebuf + (size_t)k_batch * n;
  int* dsites = reinterpret_cast<int*>(base + z.sites);
  int* dinfo = reinterpret_cast<int*>(base + z.info);

  if (hipMemcpyAsync(dsites, sites, (size_t)n_sites * sizeof(int), hipMemcpyHostToDevice, s) != hipSuccess)
    return KPM_EDEVICE;
  const long long outlen = (long long)n_sites * n_omega;
  if (!accumulate) {
    hipLaunchKernelGGL(k_fill0, dim3((unsigned)std::min<long long>((outlen + kZB - 1) / kZB, 4096)),
                       dim3(kZB), 0, s, outlen, ldos);
    if (hipGetLastError() != hipSuccess) return KPM_EDEVICE;
  }
  rocblas_handle hb = nullptr;
  if (rocblas_create_handle(&hb) != rocblas_status_success) return KPM_EDEVICE;
  int st = KPM_OK;
  if (rocblas_set_stream(hb, s) != rocblas_status_success) st = KPM_EDEVICE;
  const double wk = 1.0 / ((double)Mx * My);
  const dim3 lgrid((unsigned)((n_sites + kLS - 1) / kLS), (unsigned)((n_omega + kEC - 1) / kEC));
  // k points in groups of up to k_batch: one batched eigensolver call per group
  // (its many small panel kernels then serve the whole group), then the LDOS
  // of each member in k order.
  for (int q0 = k_first; st == KPM_OK && q0 < k_first + k_count; q0 += k_batch) {
    const int kb = std::min(k_batch, k_first + k_count - q0);
    for (int j = 0; j < kb && st == KPM_OK; ++j) {
      const int q = q0 + j, mx = q % Mx, my = q / Mx;
      st = launch_bloch(lat, h, 2.0 * M_PI * mx / Mx, 2.0 * M_PI * my / My, H + (size_t)j * n * n, n, s);
    }
    if (st != KPM_OK) break;
    double* D = evals ? evals + (size_t)(q0 - k_first) * n : Ebuf;
    if (rocsolver_zheevd_strided_batched(hb, rocblas_evect_original, rocblas_fill_lower, (rocblas_int)n,
                                         reinterpret_cast<rocblas_double_complex*>(H), (rocblas_int)n,
                                         (rocblas_stride)n * n, D, (rocblas_stride)n, Etri,
                                         (rocblas_stride)n, dinfo + (q0 - k_first),
                                         kb) != rocblas_status_success) {
      st = KPM_EDEVICE;
      break;
    }
    for (int j = 0; j < kb; ++j) {
      hipLaunchKernelGGL(k_sc_ldos, lgrid, dim3(kLS * kQL), 0, s, (int)n, n, H + (size_t)j * n * n,
                         D + (size_t)j * n, dsites, n_sites, omega, n_omega, alpha, gamma0, w_up, w_dn,
                         wk, ldos);
      if (hipGetLastError() != hipSuccess) {
        st = KPM_EDEVICE;
        break;
      }
    }
  }
  std::vector<int> info(k_count, 0);
  if (hipMemcpyAsync(info.data(), dinfo, (size_t)k_count * sizeof(int), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    st = KPM_EDEVICE;
  rocblas_destroy_handle(hb);
  if (st != KPM_OK) return st;
  for (int v : info)
    if (v != 0) return KPM_EDEVICE;
  return KPM_OK;
}

}  // extern "C"
