// Self-consistent RMFT iteration (Model and methods: theta -> h -> rho -> theta';
// App. A: mu keeps the electron number): the spin-singlet map with linear
// mixing as one bandwidth-bound kernel plus two fixed-order reductions, and
// the outer loop with its chemical-potential search on the host, driving the
// library's own entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "../../include/kpm.h"

namespace {

constexpr int kRB = 256;                       // threads per block
constexpr int kMaxBlocks = 256;                // partial results per reduction
constexpr int kHead = 8;                       // stats[0..7]: results, then partials
static_assert(kHead + 2 * kMaxBlocks <= KPM_RMFT_STATS_LEN, "stats buffer too small");
constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// max that keeps a NaN from either side
__device__ __forceinline__ double nan_max(double a, double b) { return (a > b || a != a) ? a : b; }

__device__ __forceinline__ double cabs(double2 z) { return hypot(z.x, z.y); }

// One site per thread (grid-stride over sites).  The bond (i, i + d) is stored
// at its tail i, so every read and write is coalesced along i:
//   rho entries 4d + {0,1,2,3} and 16, 17; n[i]; chi, delta [d][i].
// Per block: sum of n'_i and max residual -> part[b], part[kMaxBlocks + b].
__global__ __launch_bounds__(kRB) void k_rmft_map(int N, const double2* __restrict__ rho, double mix,
                                                  double* __restrict__ n, double2* __restrict__ chi,
                                                  double2* __restrict__ dlt, double* __restrict__ part) {
  double nsum = 0.0, res = 0.0;
  const bool write = mix != 0.0;
  for (int i = blockIdx.x * kRB + threadIdx.x; i < N; i += gridDim.x * kRB) {
    const double n1 = rho[(size_t)16 * N + i].x + 1.0 - rho[(size_t)17 * N + i].x;
    const double n0 = n[i];
    nsum += n1;
    res = nan_max(res, fabs(n1 - n0));
    if (write) n[i] = n0 + mix * (n1 - n0);
    for (int d = 0; d < 4; ++d) {
      const double2 r0 = rho[(size_t)(4 * d + 0) * N + i], r1 = rho[(size_t)(4 * d + 1) * N + i];
      const double2 r2 = rho[(size_t)(4 * d + 2) * N + i], r3 = rho[(size_t)(4 * d + 3) * N + i];
      // chi' = (rho_{i0,j0} - conj rho_{i1,j1}) / 2, delta' = (-conj rho_{i0,j1} - rho_{i1,j0}) / 2
      const double2 c1 = make_double2(0.5 * (r0.x - r3.x), 0.5 * (r0.y + r3.y));
      const double2 d1 = make_double2(0.5 * (-r1.x - r2.x), 0.5 * (r1.y - r2.y));
      const size_t k = (size_t)d * N + i;
      const double2 c0 = chi[k], d0 = dlt[k];
      const double2 dc = make_double2(c1.x - c0.x, c1.y - c0.y);
      const double2 dd = make_double2(d1.x - d0.x, d1.y - d0.y);
      res = nan_max(res, nan_max(cabs(dc), cabs(dd)));
      if (write) {
        chi[k] = make_double2(c0.x + mix * dc.x, c0.y + mix * dc.y);
        dlt[k] = make_double2(d0.x + mix * dd.x, d0.y + mix * dd.y);
      }
    }
  }
  __shared__ double s_sum[kRB], s_max[kRB];
  s_sum[threadIdx.x] = nsum;
  s_max[threadIdx.x] = res;
  __syncthreads();
  for (unsigned s = kRB / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      s_sum[threadIdx.x] += s_sum[threadIdx.x + s];
      s_max[threadIdx.x] = nan_max(s_max[threadIdx.x], s_max[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s_sum[0];
    part[kMaxBlocks + blockIdx.x] = s_max[0];
  }
}

// One block: the per-block partials in block order -> stats[0] = mean n',
// stats[1] = max residual.
__global__ __launch_bounds__(kRB) void k_rmft_finish(int N, int nblocks, double* __restrict__ stats) {
  const double* part = stats + kHead;
  __shared__ double s_sum[kRB], s_max[kRB];
  const int t = threadIdx.x;
  s_sum[t] = t < nblocks ? part[t] : 0.0;
  s_max[t] = t < nblocks ? part[kMaxBlocks + t] : 0.0;
  __syncthreads();
  for (unsigned s = kRB / 2; s > 0; s >>= 1) {
    if (t < (int)s) {
      s_sum[t] += s_sum[t + s];
      s_max[t] = nan_max(s_max[t], s_max[t + s]);
    }
    __syncthreads();
  }
  if (t == 0) {
    stats[0] = s_sum[0] / (double)N;
    stats[1] = s_max[0];
  }
}

// ------------------------------------------------------- Anderson mixing
// Flat parameter vector x of L = 17 N doubles: n [N], chi [4][N] and delta
// [4][N] as interleaved (re, im) -- the byte layout of the three user arrays
// one after the other.  The residual f = x' - x uses the map above.
constexpr int kMaxAnd = KPM_RMFT_MAX_ANDERSON;
constexpr int kDotChunk = 8 * kRB;                 // elements per block in the dot products

__global__ __launch_bounds__(kRB) void k_and_resid(int N, const double2* __restrict__ rho,
                                                   const double* __restrict__ x,
                                                   double* __restrict__ f) {
  const int i = blockIdx.x * kRB + threadIdx.x;
  if (i >= N) return;
  f[i] = rho[(size_t)16 * N + i].x + 1.0 - rho[(size_t)17 * N + i].x - x[i];
  for (int d = 0; d < 4; ++d) {
    const double2 r0 = rho[(size_t)(4 * d + 0) * N + i], r1 = rho[(size_t)(4 * d + 1) * N + i];
    const double2 r2 = rho[(size_t)(4 * d + 2) * N + i], r3 = rho[(size_t)(4 * d + 3) * N + i];
    const size_t c = (size_t)N + 2 * ((size_t)d * N + i), e = c + 8 * (size_t)N;
    f[c] = 0.5 * (r0.x - r3.x) - x[c];
    f[c + 1] = 0.5 * (r0.y + r3.y) - x[c + 1];
    f[e] = 0.5 * (-r1.x - r2.x) - x[e];
    f[e + 1] = 0.5 * (r1.y - r2.y) - x[e + 1];
  }
}

// Spin-polarised theta: the per-spin map (no spin average),
//   n'_up = rho_{i0,i0}, n'_dn = 1 - rho_{i1,i1}, chi'_up = rho_{i0,j0},
//   chi'_dn = -conj rho_{i1,j1}, Delta'_up = -conj rho_{i0,j1}, Delta'_dn = -rho_{i1,j0},
// with the mixing, mean density and residual of k_rmft_map.
__global__ __launch_bounds__(kRB) void k_rmft_map_sdw(int N, const double2* __restrict__ rho, double mix,
                                                      double* __restrict__ nu, double* __restrict__ nd,
                                                      double2* __restrict__ cu, double2* __restrict__ cd,
                                                      double2* __restrict__ du, double2* __restrict__ dd,
                                                      double* __restrict__ part) {
  double nsum = 0.0, res = 0.0;
  const bool write = mix != 0.0;
  for (int i = blockIdx.x * kRB + threadIdx.x; i < N; i += gridDim.x * kRB) {
    const double u1 = rho[(size_t)16 * N + i].x, d1 = 1.0 - rho[(size_t)17 * N + i].x;
    const double u0 = nu[i], d0 = nd[i];
    nsum += u1 + d1;
    res = nan_max(res, nan_max(fabs(u1 - u0), fabs(d1 - d0)));
    if (write) {
      nu[i] = u0 + mix * (u1 - u0);
      nd[i] = d0 + mix * (d1 - d0);
    }
    for (int d = 0; d < 4; ++d) {
      const double2 r0 = rho[(size_t)(4 * d + 0) * N + i], r1 = rho[(size_t)(4 * d + 1) * N + i];
      const double2 r2 = rho[(size_t)(4 * d + 2) * N + i], r3 = rho[(size_t)(4 * d + 3) * N + i];
      const double2 nw[4] = {r0, make_double2(-r3.x, r3.y), make_double2(-r1.x, r1.y),
                             make_double2(-r2.x, -r2.y)};
      double2* dst[4] = {cu, cd, du, dd};
      const size_t k = (size_t)d * N + i;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double2 o = dst[q][k];
        const double2 df = make_double2(nw[q].x - o.x, nw[q].y - o.y);
        res = nan_max(res, cabs(df));
        if (write) dst[q][k] = make_double2(o.x + mix * df.x, o.y + mix * df.y);
      }
    }
  }
  __shared__ double s_sum[kRB], s_max[kRB];
  s_sum[threadIdx.x] = nsum;
  s_max[threadIdx.x] = res;
  __syncthreads();
  for (unsigned s = kRB / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      s_sum[threadIdx.x] += s_sum[threadIdx.x + s];
      s_max[threadIdx.x] = nan_max(s_max[threadIdx.x], s_max[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s_sum[0];
    part[kMaxBlocks + blockIdx.x] = s_max[0];
  }
}

// Residual of the per-spin flat vector: n_up [N], n_dn [N], then chi_up,
// chi_dn, Delta_up, Delta_dn as [4][N] interleaved (re, im), 34 N doubles.
__global__ __launch_bounds__(kRB) void k_and_resid_sdw(int N, const double2* __restrict__ rho,
                                                       const double* __restrict__ x,
                                                       double* __restrict__ f) {
  const int i = blockIdx.x * kRB + threadIdx.x;
  if (i >= N) return;
  f[i] = rho[(size_t)16 * N + i].x - x[i];
  f[N + i] = 1.0 - rho[(size_t)17 * N + i].x - x[N + i];
  for (int d = 0; d < 4; ++d) {
    const double2 r0 = rho[(size_t)(4 * d + 0) * N + i], r1 = rho[(size_t)(4 * d + 1) * N + i];
    const double2 r2 = rho[(size_t)(4 * d + 2) * N + i], r3 = rho[(size_t)(4 * d + 3) * N + i];
    const double2 nw[4] = {r0, make_double2(-r3.x, r3.y), make_double2(-r1.x, r1.y),
                           make_double2(-r2.x, -r2.y)};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const size_t c = 2 * (size_t)N + (size_t)q * 8 * N + 2 * ((size_t)d * N + i);
      f[c] = nw[q].x - x[c];
      f[c + 1] = nw[q].y - x[c + 1];
    }
  }
}

// dX = x - x_prev, dF = f - f_prev (when have_prev), then x_prev = x, f_prev = f.
__global__ __launch_bounds__(kRB) void k_and_hist(long long L, const double* __restrict__ x,
                                                  const double* __restrict__ f,
                                                  double* __restrict__ xp, double* __restrict__ fp,
                                                  double* __restrict__ dX, double* __restrict__ dF,
                                                  int have_prev) {
  for (long long k = (long long)blockIdx.x * kRB + threadIdx.x; k < L; k += (long long)gridDim.x * kRB) {
    const double xv = x[k], fv = f[k];
    if (have_prev) {
      dX[k] = xv - xp[k];
      dF[k] = fv - fp[k];
    }
    xp[k] = xv;
    fp[k] = fv;
  }
}

struct Slots {
  int s[kMaxAnd];
};

// Partial dot products, block (chunk c, pair q): pairs q < T = mk (mk + 1)/2
// are <dF_i, dF_j>, i <= j (row-major upper triangle), pairs T + i are
// <dF_i, f>; i, j index the chronological slot list.
__global__ __launch_bounds__(kRB) void k_and_dots(long long L, const double* __restrict__ dFbase,
                                                  const double* __restrict__ f, Slots sl, int mk,
                                                  double* __restrict__ part, int nchunk) {
  const int q = blockIdx.y, T = mk * (mk + 1) / 2;
  int i, j = -1;
  if (q < T) {
    int r = q;
    i = 0;
    while (r >= mk - i) { r -= mk - i; ++i; }
    j = i + r;
  } else {
    i = q - T;
  }
  const double* u = dFbase + (size_t)sl.s[i] * L;
  const double* v = j >= 0 ? dFbase + (size_t)sl.s[j] * L : f;
  const long long k0 = (long long)blockIdx.x * kDotChunk;
  double acc = 0.0;
  for (int t = threadIdx.x; t < kDotChunk; t += kRB) {
    const long long k = k0 + t;
    if (k < L) acc = fma(u[k], v[k], acc);
  }
  __shared__ double sh[kRB];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (unsigned s = kRB / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(size_t)q * nchunk + blockIdx.x] = sh[0];
}

// One block per pair: the chunk partials in chunk order.
__global__ __launch_bounds__(kRB) void k_and_dots_finish(const double* __restrict__ part, int nchunk,
                                                         double* __restrict__ out) {
  const int q = blockIdx.x;
  __shared__ double sh[kRB];
  double acc = 0.0;
  for (int c = threadIdx.x; c < nchunk; c += kRB) acc += part[(size_t)q * nchunk + c];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (unsigned s = kRB / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[q] = sh[0];
}

struct Gammas {
  double g[kMaxAnd];
};

// x <- x + beta f - sum_j gamma_j (dX_j + beta dF_j), j in chronological order.
__global__ __launch_bounds__(kRB) void k_and_update(long long L, double* __restrict__ x,
                                                    const double* __restrict__ f,
                                                    const double* __restrict__ dXbase,
                                                    const double* __restrict__ dFbase, Slots sl,
                                                    Gammas gm, int mk, double beta) {
  for (long long k = (long long)blockIdx.x * kRB + threadIdx.x; k < L; k += (long long)gridDim.x * kRB) {
    double v = x[k] + beta * f[k];
    for (int j = 0; j < mk; ++j) {
      const size_t o = (size_t)sl.s[j] * L + k;
      v -= gm.g[j] * (dXbase[o] + beta * dFbase[o]);
    }
    x[k] = v;
  }
}

bool valid_lattice(const kpm_lattice* L) {
  return L && L->Lx >= 3 && L->Ly >= 3 && (L->n_vortex % 2) == 0 &&
         (long long)L->Lx * L->Ly <= (1LL << 26);
}

// Workspace of kpm_rmft_iterate: the recursion workspace first (so that
// kpm_status_read works on the same pointer), then h, rho, ab, C, stats.
struct RmftLayout {
  size_t kws, h, rho, ab, C, stats, and_vec, and_part, and_dots, total;
};

RmftLayout rmft_layout(const kpm_lattice* L, int R, int M, int ckpt_k, int precision) {
  RmftLayout z{};
  const size_t kws = kpm_workspace_size(L, R, M, ckpt_k, precision);
  if (kws == 0) return z;
  const size_t N = (size_t)L->Lx * L->Ly;
  z.kws = kws;
  size_t off = align_up(kws);
  z.h = off;     off += align_up(19 * N * 16);
  z.rho = off;   off += align_up(19 * N * 16);
  z.ab = off;    off += align_up(2 * sizeof(double));
  z.C = off;     off += align_up((size_t)M * sizeof(double));
  z.stats = off; off += align_up(KPM_RMFT_STATS_LEN * sizeof(double));
  // Anderson: x, f, x_prev, f_prev, then kMaxAnd dX and kMaxAnd dF vectors
  const size_t Lv = 34 * N;                       // sized for a spin-polarised theta
  const size_t nchunk = (Lv + kDotChunk - 1) / kDotChunk;
  const size_t npair = (size_t)kMaxAnd * (kMaxAnd + 1) / 2 + kMaxAnd;
  z.and_vec = off;  off += align_up((4 + 2 * (size_t)kMaxAnd) * Lv * sizeof(double));
  z.and_part = off; off += align_up(npair * nchunk * sizeof(double));
  z.and_dots = off; off += align_up(npair * sizeof(double));
  z.total = off;
  return z;
}

// Gaussian elimination with partial pivoting on the mk x mk system (in place).
bool solve_small(std::vector<double>& A, std::vector<double>& b, int n) {
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[p * n + c])) p = r;
    if (!(std::fabs(A[p * n + c]) > 0.0)) return false;
    if (p != c) {
      for (int k = 0; k < n; ++k) std::swap(A[c * n + k], A[p * n + k]);
      std::swap(b[c], b[p]);
    }
    for (int r = c + 1; r < n; ++r) {
      const double l = A[r * n + c] / A[c * n + c];
      for (int k = c; k < n; ++k) A[r * n + k] -= l * A[c * n + k];
      b[r] -= l * b[c];
    }
  }
  for (int r = n - 1; r >= 0; --r) {
    double v = b[r];
    for (int k = r + 1; k < n; ++k) v -= A[r * n + k] * b[k];
    b[r] = v / A[r * n + r];
  }
  return true;
}

// The parameter arrays of the iteration: singlet (n, chi, delta) or
// spin-polarised (n_up, n_dn, chi_up, chi_dn, delta_up, delta_dn); each array
// is one segment of the flat Anderson vector, in this order.
struct ThetaSet {
  bool spin;
  int nseg;
  double* p[6];
  size_t len[6];                 // doubles per segment
  long long total() const {
    long long t = 0;
    for (int k = 0; k < nseg; ++k) t += (long long)len[k];
    return t;
  }
};

int copy_segments(const ThetaSet& th, double* flat, bool to_flat, hipStream_t s) {
  size_t o = 0;
  for (int k = 0; k < th.nseg; ++k) {
    const size_t b = th.len[k] * sizeof(double);
    const hipError_t e = to_flat ? hipMemcpyAsync(flat + o, th.p[k], b, hipMemcpyDeviceToDevice, s)
                                 : hipMemcpyAsync(th.p[k], flat + o, b, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return KPM_EDEVICE;
    o += th.len[k];
  }
  return KPM_OK;
}

// The map with mixing (mix = 0: measurement only) and its two reductions.
int map_update(const kpm_lattice* lat, const double* rho, double mix, const ThetaSet& th,
               double* stats, hipStream_t s) {
  const int N = lat->Lx * lat->Ly;
  const int nb = std::min((N + kRB - 1) / kRB, kMaxBlocks);
  const double2* r = reinterpret_cast<const double2*>(rho);
  if (th.spin)
    hipLaunchKernelGGL(k_rmft_map_sdw, dim3(nb), dim3(kRB), 0, s, N, r, mix, th.p[0], th.p[1],
                       reinterpret_cast<double2*>(th.p[2]), reinterpret_cast<double2*>(th.p[3]),
                       reinterpret_cast<double2*>(th.p[4]), reinterpret_cast<double2*>(th.p[5]),
                       stats + kHead);
  else
    hipLaunchKernelGGL(k_rmft_map, dim3(nb), dim3(kRB), 0, s, N, r, mix, th.p[0],
                       reinterpret_cast<double2*>(th.p[1]), reinterpret_cast<double2*>(th.p[2]),
                       stats + kHead);
  if (hipGetLastError() != hipSuccess) return KPM_EDEVICE;
  hipLaunchKernelGGL(k_rmft_finish, dim3(1), dim3(kRB), 0, s, N, nb, stats);
  if (hipGetLastError() != hipSuccess) return KPM_EDEVICE;
  return KPM_OK;
}

// One Anderson update of theta from the accepted rho (see kpm_rmft_params).
int anderson_step(const kpm_rmft_params* prm, int N, long long Lv, const double* rho,
                  const ThetaSet& th, double* ax, double* af, double* axp, double* afp,
                  double* adX, double* adF, double* apart, double* adots, int nchunk, int vgrid,
                  std::vector<int>& order, bool& have_prev, hipStream_t s) {
  if (copy_segments(th, ax, true, s) != KPM_OK) return KPM_EDEVICE;
  if (th.spin)
    hipLaunchKernelGGL(k_and_resid_sdw, dim3((N + kRB - 1) / kRB), dim3(kRB), 0, s, N,
                       reinterpret_cast<const double2*>(rho), ax, af);
  else
    hipLaunchKernelGGL(k_and_resid, dim3((N + kRB - 1) / kRB), dim3(kRB), 0, s, N,
                       reinterpret_cast<const double2*>(rho), ax, af);
  int slot = -1;
  if (have_prev) {
    if ((int)order.size() < prm->anderson) {
      slot = (int)order.size();
    } else {
      slot = order.front();
      order.erase(order.begin());
    }
    order.push_back(slot);
  }
  hipLaunchKernelGGL(k_and_hist, dim3(vgrid), dim3(kRB), 0, s, Lv, ax, af, axp, afp,
                     adX + (size_t)std::max(slot, 0) * Lv, adF + (size_t)std::max(slot, 0) * Lv,
                     have_prev ? 1 : 0);
  have_prev = true;
  const int mk = (int)order.size();
  Slots sl{};
  for (int j = 0; j < mk; ++j) sl.s[j] = order[j];
  Gammas gm{};
  if (mk > 0) {
    const int T = mk * (mk + 1) / 2;
    hipLaunchKernelGGL(k_and_dots, dim3(nchunk, T + mk), dim3(kRB), 0, s, Lv, adF, af, sl, mk,
                       apart, nchunk);
    hipLaunchKernelGGL(k_and_dots_finish, dim3(T + mk), dim3(kRB), 0, s, apart, nchunk, adots);
    std::vector<double> d(T + mk);
    if (hipMemcpyAsync(d.data(), adots, d.size() * sizeof(double), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return KPM_EDEVICE;
    std::vector<double> A(mk * mk), b(mk);
    int q = 0;
    for (int i = 0; i < mk; ++i)
      for (int j = i; j < mk; ++j) A[i * mk + j] = A[j * mk + i] = d[q++];
    double dmax = 0.0;
    for (int i = 0; i < mk; ++i) dmax = std::max(dmax, A[i * mk + i]);
    if (!std::isfinite(dmax)) return KPM_EBOUNDS;
    if (dmax > 0.0) {                    // an all-zero history leaves the linear step
      for (int i = 0; i < mk; ++i) A[i * mk + i] += 1e-12 * dmax;
      for (int i = 0; i < mk; ++i) b[i] = d[T + i];
      if (!solve_small(A, b, mk)) return KPM_EBOUNDS;
      for (int j = 0; j < mk; ++j) {
        if (!std::isfinite(b[j])) return KPM_EBOUNDS;
        gm.g[j] = b[j];
      }
    }
  }
  hipLaunchKernelGGL(k_and_update, dim3(vgrid), dim3(kRB), 0, s, Lv, ax, af, adX, adF, sl, gm, mk,
                     prm->mix);
  if (hipGetLastError() != hipSuccess) return KPM_EDEVICE;
  return copy_segments(th, ax, false, s);
}

ThetaSet singlet_set(const kpm_lattice* lat, double* n, double* chi, double* delta) {
  const size_t N = (size_t)lat->Lx * lat->Ly;
  ThetaSet t{};
  t.spin = false;
  t.nseg = 3;
  t.p[0] = n;   t.len[0] = N;
  t.p[1] = chi; t.len[1] = 8 * N;
  t.p[2] = delta; t.len[2] = 8 * N;
  return t;
}

ThetaSet spin_set(const kpm_lattice* lat, double* nu, double* nd, double* cu, double* cd,
                  double* du, double* dd) {
  const size_t N = (size_t)lat->Lx * lat->Ly;
  ThetaSet t{};
  t.spin = true;
  t.nseg = 6;
  double* p[6] = {nu, nd, cu, cd, du, dd};
  for (int k = 0; k < 6; ++k) {
    t.p[k] = p[k];
    t.len[k] = k < 2 ? N : 8 * N;
  }
  return t;
}

int rmft_loop(const kpm_lattice* lat, const kpm_model* model, const kpm_probes* probes, int32_t M,
              double T, int32_t precision, int32_t ckpt_k, const kpm_rmft_params* prm,
              int32_t n_iter, const ThetaSet& th, double* mu, kpm_rmft_record* history,
              int32_t* n_done, void* ws, size_t ws_bytes, void* stream);

}  // namespace

extern "C" {

int kpm_rmft_update(const kpm_lattice* lat, const double* rho, double mix, double* n, double* chi,
                    double* delta, double* stats, void* stream) {
  if (!valid_lattice(lat) || !rho || !n || !chi || !delta || !stats) return KPM_EINVAL;
  if (!(mix >= 0.0 && mix <= 1.0)) return KPM_EINVAL;
  return map_update(lat, rho, mix, singlet_set(lat, n, chi, delta), stats,
                    static_cast<hipStream_t>(stream));
}

int kpm_rmft_update_sdw(const kpm_lattice* lat, const double* rho, double mix, double* n_up,
                        double* n_dn, double* chi_up, double* chi_dn, double* delta_up,
                        double* delta_dn, double* stats, void* stream) {
  if (!valid_lattice(lat) || !rho || !n_up || !n_dn || !chi_up || !chi_dn || !delta_up ||
      !delta_dn || !stats)
    return KPM_EINVAL;
  if (!(mix >= 0.0 && mix <= 1.0)) return KPM_EINVAL;
  return map_update(lat, rho, mix, spin_set(lat, n_up, n_dn, chi_up, chi_dn, delta_up, delta_dn),
                    stats, static_cast<hipStream_t>(stream));
}

size_t kpm_rmft_workspace_size(const kpm_lattice* lat, int32_t R, int32_t M, int32_t ckpt_k,
                               int32_t precision) {
  if (!valid_lattice(lat)) return 0;
  return rmft_layout(lat, R, M, ckpt_k, precision).total;
}

int kpm_rmft_iterate(const kpm_lattice* lat, const kpm_model* model, const kpm_probes* probes,
                     int32_t M, double T, int32_t precision, int32_t ckpt_k,
                     const kpm_rmft_params* prm, int32_t n_iter, double* n, double* chi,
                     double* delta, double* mu, kpm_rmft_record* history, int32_t* n_done,
                     void* ws, size_t ws_bytes, void* stream) {
  if (!valid_lattice(lat)) return KPM_EINVAL;
  return rmft_loop(lat, model, probes, M, T, precision, ckpt_k, prm, n_iter,
                   singlet_set(lat, n, chi, delta), mu, history, n_done, ws, ws_bytes, stream);
}

int kpm_rmft_iterate_sdw(const kpm_lattice* lat, const kpm_model* model, const kpm_probes* probes,
                         int32_t M, double T, int32_t precision, int32_t ckpt_k,
                         const kpm_rmft_params* prm, int32_t n_iter, double* n_up, double* n_dn,
                         double* chi_up, double* chi_dn, double* delta_up, double* delta_dn,
                         double* mu, kpm_rmft_record* history, int32_t* n_done, void* ws,
                         size_t ws_bytes, void* stream) {
  if (!valid_lattice(lat)) return KPM_EINVAL;
  return rmft_loop(lat, model, probes, M, T, precision, ckpt_k, prm, n_iter,
                   spin_set(lat, n_up, n_dn, chi_up, chi_dn, delta_up, delta_dn), mu, history, n_done,
                   ws, ws_bytes, stream);
}

}  // extern "C"

namespace {

int rmft_loop(const kpm_lattice* lat, const kpm_model* model, const kpm_probes* probes, int32_t M,
              double T, int32_t precision, int32_t ckpt_k, const kpm_rmft_params* prm,
              int32_t n_iter, const ThetaSet& th, double* mu, kpm_rmft_record* history,
              int32_t* n_done, void* ws, size_t ws_bytes, void* stream) {
  if (!valid_lattice(lat) || !model || !probes || !prm || !mu || !n_done || !ws || n_iter < 0)
    return KPM_EINVAL;
  for (int k = 0; k < th.nseg; ++k)
    if (!th.p[k]) return KPM_EINVAL;
  if (!(prm->doping > 0.0 && prm->doping < 1.0) || !(prm->mix > 0.0 && prm->mix <= 1.0) ||
      !(prm->tol_n >= 0.0) || !(prm->tol_mu >= 0.0) || !(prm->mu_step > 0.0) ||
      !std::isfinite(prm->mu_step) || !(prm->tol_residual >= 0.0) || prm->max_evals < 1 ||
      prm->coef_K < 0 || !std::isfinite(*mu) || !(T > 0.0) ||
      (prm->search != KPM_RMFT_BISECTION && prm->search != KPM_RMFT_ILLINOIS) ||
      (prm->estimator != KPM_RMFT_ADJOINT && prm->estimator != KPM_RMFT_DIRECT) ||
      prm->anderson < 0 || prm->anderson > KPM_RMFT_MAX_ANDERSON)
    return KPM_EINVAL;
  const int32_t R = kpm_probe_count(lat, probes);
  if (R < 1) return KPM_EINVAL;
  const RmftLayout z = rmft_layout(lat, R, M, ckpt_k, precision);
  if (z.total == 0) return KPM_EINVAL;
  if (ws_bytes < z.total || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0) return KPM_EWORKSPACE;
  *n_done = 0;

  char* base = static_cast<char*>(ws);
  double* h = reinterpret_cast<double*>(base + z.h);
  double* rho = reinterpret_cast<double*>(base + z.rho);
  double* ab = reinterpret_cast<double*>(base + z.ab);
  double* C = reinterpret_cast<double*>(base + z.C);
  double* stats = reinterpret_cast<double*>(base + z.stats);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const double target = 1.0 - prm->doping;
  const int N = lat->Lx * lat->Ly;
  const long long Lv = th.total();
  double* ax = reinterpret_cast<double*>(base + z.and_vec);
  double* af = ax + Lv;
  double* axp = af + Lv;
  double* afp = axp + Lv;
  double* adX = afp + Lv;
  double* adF = adX + (size_t)kMaxAnd * Lv;
  double* apart = reinterpret_cast<double*>(base + z.and_part);
  double* adots = reinterpret_cast<double*>(base + z.and_dots);
  const int nchunk = (int)((Lv + kDotChunk - 1) / kDotChunk);
  const int vgrid = (int)std::min<long long>((Lv + kRB - 1) / kRB, 4096);
  std::vector<int> order;            // Anderson slots, oldest first
  bool have_prev = false;

  // One density-matrix evaluation at chemical potential m with theta fixed:
  // out[0] = mean n', out[1] = residual, out[2] = Omega.
  auto evaluate = [&](double m, double out[3]) -> int {
    kpm_model md = *model;
    md.mu = m;
    int st;
    st = th.spin ? kpm_build_H_sdw(lat, &md, th.p[0], th.p[1], th.p[2], th.p[3], th.p[4], th.p[5], h,
                                   stream)
                 : kpm_build_H(lat, &md, th.p[0], th.p[1], th.p[2], h, stream);
    if (st != KPM_OK) return st;
    if ((st = kpm_bounds(lat, h, ab, stream)) != KPM_OK) return st;
    if ((st = kpm_coefficients(M, T, ab, prm->coef_K, C, stream)) != KPM_OK) return st;
    if (prm->estimator == KPM_RMFT_DIRECT) {
      if ((st = kpm_density_matrix_direct(lat, h, ab, probes, M, C, precision, stats + 2, rho, ws,
                                          z.kws, stream)) != KPM_OK)
        return st;
    } else {
      if ((st = kpm_grand_potential(lat, h, ab, probes, M, C, precision, ckpt_k, stats + 2,
                                    nullptr, ws, z.kws, stream)) != KPM_OK)
        return st;
      if ((st = kpm_grand_potential_grad(lat, h, ab, probes, M, C, precision, ckpt_k, nullptr, rho,
                                         ws, z.kws, stream)) != KPM_OK)
        return st;
    }
    if ((st = map_update(lat, rho, 0.0, th, stats, s)) != KPM_OK) return st;
    int32_t dev = KPM_OK;
    if ((st = kpm_status_read(ws, &dev, stream)) != KPM_OK) return st;
    if (dev != KPM_OK) return dev;
    if (hipMemcpyAsync(out, stats, 3 * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return KPM_EDEVICE;
    if (!std::isfinite(out[0]) || !std::isfinite(out[1])) return KPM_EBOUNDS;
    return KPM_OK;
  };

  double cur = *mu;
  for (int it = 0; it < n_iter; ++it) {
    double v[3];
    int evals = 0, st;
    // accepted evaluation: its rho is in the workspace, its figures in v
    double acc = cur;
    if ((st = evaluate(cur, v)) != KPM_OK) return st;
    ++evals;
    const double e0 = v[0] - target;
    if (!(std::fabs(e0) <= prm->tol_n)) {
      const bool below = e0 < 0.0;
      const double dir = below ? 1.0 : -1.0;
      double a = cur, b = cur, fa = e0, fb = e0, step = prm->mu_step;
      bool done = false;
      for (;;) {                                   // walk with doubling steps
        if (evals >= prm->max_evals) return KPM_ENOCONV;
        const double m = a + dir * step;
        if ((st = evaluate(m, v)) != KPM_OK) return st;
        ++evals;
        const double e = v[0] - target;
        if (std::fabs(e) <= prm->tol_n) { acc = m; done = true; break; }
        if ((e < 0.0) == below) { a = m; fa = e; step *= 2.0; }
        else { b = m; fb = e; break; }
      }
      while (!done && prm->search == KPM_RMFT_BISECTION) {   // bisection of [a, b]
        if (evals >= prm->max_evals) return KPM_ENOCONV;
        const double m = 0.5 * (a + b);
        if ((st = evaluate(m, v)) != KPM_OK) return st;
        ++evals;
        const double e = v[0] - target;
        if (std::fabs(e) <= prm->tol_n || 0.5 * std::fabs(b - a) <= prm->tol_mu) { acc = m; break; }
        if ((e < 0.0) == below) a = m;
        else b = m;
      }
      // Illinois false position on [a, b], b the newest point: the secant
      // root of (a, fa), (b, fb); the retained end's value is halved when it
      // is kept twice in a row (Dowell & Jarratt, BIT 11, 168 (1971)).
      while (!done && prm->search == KPM_RMFT_ILLINOIS) {
        if (evals >= prm->max_evals) return KPM_ENOCONV;
        const double m = b - fb * (b - a) / (fb - fa);
        if ((st = evaluate(m, v)) != KPM_OK) return st;
        ++evals;
        const double e = v[0] - target;
        if ((e < 0.0) != (fb < 0.0)) { a = b; fa = fb; }
        else fa = 0.5 * fa;
        b = m;
        fb = e;
        if (std::fabs(e) <= prm->tol_n || std::fabs(b - a) <= prm->tol_mu) { acc = m; break; }
      }
    }
    if (prm->anderson == 0) {
      if ((st = map_update(lat, rho, prm->mix, th, stats, s)) != KPM_OK) return st;
    } else if ((st = anderson_step(prm, N, Lv, rho, th, ax, af, axp, afp, adX, adF, apart,
                                   adots, nchunk, vgrid, order, have_prev, s)) != KPM_OK) {
      return st;
    }
    cur = acc;
    *mu = acc;
    if (history) {
      kpm_rmft_record& r = history[it];
      r.mu = acc;
      r.nbar = v[0];
      r.residual = v[1];
      r.omega = v[2];
      r.evals = evals;
      r.pad = 0;
    }
    *n_done = it + 1;
    if (prm->tol_residual > 0.0 && v[1] <= prm->tol_residual) break;
  }
  if (hipStreamSynchronize(s) != hipSuccess) return KPM_EDEVICE;
  return KPM_OK;
}

}  // namespace
