// Internal device-side definitions of the KPM library (not part of the ABI).
//
// Data layout in HBM (per lattice instance, N = Lx*Ly sites, R probes):
//   h      [19][N] double2   stencil of h (ABI layout)
//   coef   [tile][9][64] 4-vectors  rescaled rows of H~ = (h - b)/a in lane
//                            order: pair k of lane l (site l >> 1 of the tile,
//                            row a = l & 1) holds H~_{(i,a),(nb_k(i),0)} and
//                            H~_{(i,a),(nb_k(i),1)}, nb_0 = i, nb_{1+d} = i + d,
//                            nb_{5+d} = i - d
//   A[2], G[2]  [R][N] rec   alpha_j lives in A[j & 1], gamma_j in G[j & 1];
//                            rec = two complex values (Nambu 0, 1) of one site
//                            (float4 = 16 B in FP32, 2 x double2 = 32 B in FP64)
//   ckpt   [S][R][N] rec     checkpoint alpha_j for j % k in {0, 1}, slot 2(j/k)+j%k
//   mom    [M][ntile][R]     per-(step, 8x4 tile, probe) moment partials
//   gpart  [nrange][19][N] double2  per-probe-range partial dOmega/dH~ (FP64)
//   pcode  [R][N] bytes      probe entries (written once per call by the alpha_0 kernel)
//   sink   4 KB              target of the stores of lanes outside the lattice (never read)
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kpm {

constexpr int kBlock = 256;          // threads per block = sites per chunk
constexpr int kNent = 19;            // stencil entries per site
constexpr int kNcoef = 36;           // row-form coefficients per site
constexpr int kMaxGroups = 4;

enum : int { kUnit = 0, kDenseZ4 = 1, kColoredZ4 = 2 };

struct GroupDev {
  int kind, count, px, py, split, first, nprobes, base;
  unsigned long long seed;
  double weight;
};

struct ModelDev {
  int Lx, Ly, nv, N;
  double t, tp, J, mu;
};

struct InstDev {
  // poff: global index of the instance's first probe (a probe half of a
  // single lattice; 0 otherwise), for the probe hash of k_init
  int Lx, Ly, N, R, nchunk, npb, ngroups, poff;
  GroupDev g[kMaxGroups];
  const double2* h;
  const double* ab;
  const double* C;
  void* coef;
  void* A[2];
  void* G[2];
  void* ckpt;
  double* mom;        // [M][nchunk][R] moment partials (nchunk = recursion tiles)
  double* musum;      // [R][M] reduced moments
  double2* gpart;     // [npb][19][N] partial dOmega/dH~ per probe range
  double* opart;      // [ceil(M/256)] partial sums of Omega
  unsigned char* pcode;  // [R][N] probe entries: nibble a (bits 4a..4a+3) of site i is
                         // 8 | k for entry i^k of Nambu component a, 0 for a zero entry
  double* pw;            // [R] probe weights
  void* sink;            // 4 KB that stores of lanes outside the lattice go to (never read)
  double2* rho;       // [19][N] output
  const double* omega_bar;
  double* omega;
  int* status;
};

// Four values of one precision moved as one vector (a site record of both
// Nambu components, or a coefficient pair).
typedef float KF4 __attribute__((ext_vector_type(4)));
typedef double KD4 __attribute__((ext_vector_type(4)));
template <typename V> struct RecT4;
template <> struct RecT4<float> { using T = KF4; };
template <> struct RecT4<double> { using T = KD4; };

// ---------------------------------------------------------------- complex
template <typename V> struct Cx { V x, y; };

template <typename V>
__device__ __forceinline__ void cfma(Cx<V>& acc, const Cx<V>& a, const Cx<V>& b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}

// acc += conj(a) * b
template <typename V>
__device__ __forceinline__ void cfma_conj(Cx<V>& acc, const Cx<V>& a, const Cx<V>& b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
}

// One site's record: Nambu components 0 and 1.
template <typename V> struct Rec { Cx<V> c[2]; };

template <typename V> __device__ __forceinline__ Rec<V> ld_rec(const void* base, long long idx);
template <> __device__ __forceinline__ Rec<float> ld_rec<float>(const void* base, long long idx) {
  float4 v = reinterpret_cast<const float4*>(base)[idx];
  Rec<float> r;
  r.c[0] = {v.x, v.y};
  r.c[1] = {v.z, v.w};
  return r;
}
template <> __device__ __forceinline__ Rec<double> ld_rec<double>(const void* base, long long idx) {
  const double2* p = reinterpret_cast<const double2*>(base) + 2 * idx;
  double2 a = p[0], b = p[1];
  Rec<double> r;
  r.c[0] = {a.x, a.y};
  r.c[1] = {b.x, b.y};
  return r;
}
template <typename V> __device__ __forceinline__ void st_rec(void* base, long long idx, const Rec<V>& r);
template <> __device__ __forceinline__ void st_rec<float>(void* base, long long idx, const Rec<float>& r) {
  reinterpret_cast<float4*>(base)[idx] = make_float4(r.c[0].x, r.c[0].y, r.c[1].x, r.c[1].y);
}
template <> __device__ __forceinline__ void st_rec<double>(void* base, long long idx, const Rec<double>& r) {
  double2* p = reinterpret_cast<double2*>(base) + 2 * idx;
  p[0] = make_double2(r.c[0].x, r.c[0].y);
  p[1] = make_double2(r.c[1].x, r.c[1].y);
}

template <typename V> __device__ __forceinline__ Cx<V> ld_cx(const void* base, long long idx) {
  const V* p = reinterpret_cast<const V*>(base) + 2 * idx;
  return Cx<V>{p[0], p[1]};
}

// ---------------------------------------------------------------- probes
// SplitMix64 output for (seed, counter): Steele, Lea & Flood (2014), in the
// form of Vigna's splitmix64.c (state advanced by the golden gamma).
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long seed,
                                                         unsigned long long counter) {
  unsigned long long z = seed + (counter + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ int z4(unsigned long long seed, int draw, int index) {
  return (int)(splitmix64(seed, ((unsigned long long)draw << 32) + (unsigned)index) >> 62);
}

// Probe p's entry at site i (x, y) for both Nambu components: code k means
// i^k, -1 means zero.  Returns the group weight through w.
__device__ __forceinline__ void probe_codes(const InstDev& I, int p, int i, int x, int y,
                                            int& k0, int& k1, double& w) {
  k0 = -1;
  k1 = -1;
  w = 0.0;
#pragma unroll
  for (int gi = 0; gi < kMaxGroups; ++gi) {
    if (gi >= I.ngroups) break;
    const GroupDev& g = I.g[gi];
    int q = p - g.base;
    if (q < 0 || q >= g.nprobes) continue;
    w = g.weight;
    if (g.kind == kUnit) {
      int J = g.first + q;
      if (J == 2 * i) k0 = 0;
      if (J == 2 * i + 1) k1 = 0;
    } else if (g.kind == kDenseZ4) {
      k0 = z4(g.seed, q, 2 * i);
      k1 = z4(g.seed, q, 2 * i + 1);
    } else {
      int per = g.px * g.py * (g.split ? 2 : 1);
      int draw = q / per;
      int c = q - draw * per;
      int comp = -1;
      if (g.split) {
        comp = c & 1;
        c >>= 1;
      }
      int col = (x % g.px) + g.px * (y % g.py);
      if (col == c) {
        if (comp != 1) k0 = z4(g.seed, draw, 2 * i);
        if (comp != 0) k1 = z4(g.seed, draw, 2 * i + 1);
      }
    }
    break;
  }
}

// Re(conj(i^k) z)
template <typename V>
__device__ __forceinline__ double re_conjphase(int k, const Cx<V>& z) {
  double r = 0.0;
  if (k == 0) r = (double)z.x;
  else if (k == 1) r = (double)z.y;
  else if (k == 2) r = -(double)z.x;
  else if (k == 3) r = -(double)z.y;
  return r;
}

// s * i^k as a complex value (0 if k < 0)
template <typename V>
__device__ __forceinline__ Cx<V> phase_scaled(int k, V s) {
  Cx<V> r{V(0), V(0)};
  if (k == 0) r.x = s;
  else if (k == 1) r.y = s;
  else if (k == 2) r.x = -s;
  else if (k == 3) r.y = -s;
  return r;
}

// ---------------------------------------------------------------- neighbours
struct Nbr { int i[9]; };

__device__ __forceinline__ Nbr neighbours(int i, int Lx, int Ly) {
  int y = i / Lx, x = i - y * Lx;
  int xp = (x + 1 == Lx) ? 0 : x + 1;
  int xm = (x == 0) ? Lx - 1 : x - 1;
  int yp = (y + 1 == Ly) ? 0 : y + 1;
  int ym = (y == 0) ? Ly - 1 : y - 1;
  Nbr n;
  n.i[0] = i;
  n.i[1] = y * Lx + xp;     // +x
  n.i[2] = yp * Lx + x;     // +y
  n.i[3] = yp * Lx + xp;    // +x+y
  n.i[4] = ym * Lx + xp;    // +x-y
  n.i[5] = y * Lx + xm;     // -x
  n.i[6] = ym * Lx + x;     // -y
  n.i[7] = ym * Lx + xm;    // -x-y
  n.i[8] = yp * Lx + xm;    // -x+y
  return n;
}

}  // namespace kpm
