// Element-wise kernels around the recursion: the TB-BdG builder and its VJP,
// Gershgorin bounds, the rescaled row-form coefficients and the Chebyshev
// expansion coefficients of the grand-potential density.
#include "kpm_internal.h"

namespace kpm {

// ---------------------------------------------------------------- geometry
__device__ __forceinline__ void dir_step(int d, int& dx, int& dy) {
  dx = (d == 1) ? 0 : 1;
  dy = (d == 0) ? 0 : ((d == 3) ? -1 : 1);
}

// Peierls phase of bond (x, y) -> (x + dx, y + dy): the Landau-gauge line
// integral -(pi/Phi0) int A.dl with A = B(0, x), B = nv Phi0/(Lx Ly), along the
// straight segment, plus the gauge twist pi nv y_head/Ly on +x steps that
// cross the x seam (makes the flux uniform on the torus, nv even).
__device__ __forceinline__ double peierls(int x, int y, int d, int Lx, int Ly, int nv) {
  int dx, dy;
  dir_step(d, dx, dy);
  double xm = (double)x + 0.5 * (double)dx;
  double phi = -M_PI * (double)nv * xm * (double)dy / ((double)Lx * (double)Ly);
  if (x + dx == Lx) {
    int yh = y + dy;
    yh = (yh < 0) ? yh + Ly : (yh >= Ly ? yh - Ly : yh);
    phi += M_PI * (double)nv * (double)yh / (double)Ly;
  }
  return phi;
}

__device__ __forceinline__ int nbr_of(int i, int d, int sign, int Lx, int Ly) {
  int y = i / Lx, x = i - y * Lx;
  int dx, dy;
  dir_step(d, dx, dy);
  x += sign * dx;
  y += sign * dy;
  x = (x < 0) ? x + Lx : (x >= Lx ? x - Lx : x);
  y = (y < 0) ? y + Ly : (y >= Ly ? y - Ly : y);
  return y * Lx + x;
}

// Gutzwiller factors at m = 0 (App. A) and their derivatives in delta.
struct GF {
  double g, g1, g2;      // g = sqrt(2 d/(1+d)), g', g''
  double s, s1, s2;      // g^s = 2/(1+d), g^s', g^s''
};

__device__ __forceinline__ GF gfac(double n) {
  double d = 1.0 - n;
  double q = 1.0 + d;
  GF f;
  double u = 2.0 * d / q, u1 = 2.0 / (q * q), u2 = -4.0 / (q * q * q);
  f.g = sqrt(u);
  f.g1 = u1 / (2.0 * f.g);
  f.g2 = u2 / (2.0 * f.g) - u1 * u1 / (4.0 * f.g * f.g * f.g);
  f.s = 2.0 / q;
  f.s1 = -2.0 / (q * q);
  f.s2 = 4.0 / (q * q * q);
  return f;
}

__device__ __forceinline__ double2 hop(const ModelDev& md, int i, int d) {
  int y = i / md.Lx, x = i - y * md.Lx;
  double phi = peierls(x, y, d, md.Lx, md.Ly, md.nv);
  double s, c;
  sincos(phi, &s, &c);
  double amp = (d < 2) ? md.t : md.tp;
  return make_double2(amp * c, amp * s);
}

__device__ __forceinline__ double2 ld2(const double* p, long long idx) {
  return reinterpret_cast<const double2*>(p)[idx];
}

// h = dW/drho on the stencil (see kpm_build_H in kpm.h).
__global__ __launch_bounds__(kBlock) void k_build_h(ModelDev md, const double* __restrict__ n,
                                                    const double* __restrict__ chi,
                                                    const double* __restrict__ dlt,
                                                    double2* __restrict__ h) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= md.N) return;
  const int N = md.N;
  GF fi = gfac(n[i]);
  double eps = -md.mu;
  for (int d = 0; d < 4; ++d) {
    // forward bond (i, j = i + d), stored here
    int j = nbr_of(i, d, +1, md.Lx, md.Ly);
    GF fj = gfac(n[j]);
    double2 t = hop(md, i, d);
    double2 c = ld2(chi, (long long)d * N + i);
    double2 D = ld2(dlt, (long long)d * N + i);
    double gt = fi.g * fj.g;
    double2 T = make_double2(-gt * t.x, -gt * t.y);
    double2 P = make_double2(0.0, 0.0);
    double R = t.x * c.x - t.y * c.y;                 // Re(t chi)
    eps += 4.0 * fi.g1 * fj.g * R;
    if (d < 2) {
      double cb = 0.75 * md.J * fi.s * fj.s;
      T.x -= cb * c.x;                                // - c conj(chi)
      T.y += cb * c.y;
      P = make_double2(cb * D.x, cb * D.y);
      double Q = c.x * c.x + c.y * c.y + D.x * D.x + D.y * D.y;
      eps += 1.5 * md.J * fi.s1 * fj.s * Q;
    }
    h[(long long)(4 * d + 0) * N + i] = T;
    h[(long long)(4 * d + 1) * N + i] = P;
    h[(long long)(4 * d + 2) * N + i] = make_double2(P.x, -P.y);
    h[(long long)(4 * d + 3) * N + i] = make_double2(-T.x, T.y);
    // backward bond (k = i - d, i), stored at k: its energy terms touch i too
    int k = nbr_of(i, d, -1, md.Lx, md.Ly);
    GF fk = gfac(n[k]);
    double2 tb = hop(md, k, d);
    double2 cbk = ld2(chi, (long long)d * N + k);
    double2 Dbk = ld2(dlt, (long long)d * N + k);
    eps += 4.0 * fi.g1 * fk.g * (tb.x * cbk.x - tb.y * cbk.y);
    if (d < 2) {
      double Q = cbk.x * cbk.x + cbk.y * cbk.y + Dbk.x * Dbk.x + Dbk.y * Dbk.y;
      eps += 1.5 * md.J * fi.s1 * fk.s * Q;
    }
  }
  h[(long long)16 * N + i] = make_double2(eps, 0.0);
  h[(long long)17 * N + i] = make_double2(-eps, 0.0);
  h[(long long)18 * N + i] = make_double2(0.0, 0.0);
}

// ------------------------------------------------ spin-polarised builder
// Collinear magnetisation (App. A at m_i != 0).  Per spin s = +1 (up), -1
// (down): n_s, chi_s, Delta_s = s <c_s c_-s>.  With delta = 1 - n,
// m = (n_up - n_dn)/2, A = 1 - delta^2 + 4 m^2, the energy of one bond is
//   W_b = - sum_s g^t_{i s} g^t_{j s} 2 Re(t chi_s)
//         + J [g^z Szz + g^xy_ij Sxy]                 (nearest neighbours only),
//   Szz = m_i m_j - (1/4) sum_s (|chi_s|^2 + |Delta_s|^2),
//   Sxy = - Re(chi_up conj(chi_dn) + conj(Delta_up) Delta_dn),
//   g^z = g^xy_ij R,  R = (b - 4 mm X^2)/(b - 4 mm),  mm = m_i m_j,
//   b = 2 (|Dbar|^2 - |chibar|^2),  X = 1 + 12 n_i n_j / sqrt(A_i A_j),
// plus -mu sum_i n_i.  h_IJ = dW/drho_IJ as for kpm_build_H, written out by
// the chain rule through (delta, m) of each site.
// Scalar with one tangent (forward-mode derivative): the VJP of this builder
// runs the same code on (value, tangent) pairs.
struct Dual {
  double v, d;
};
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ Dual operator-(Dual a) { return {-a.v, -a.d}; }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ __forceinline__ Dual operator/(Dual a, Dual b) {
  return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)};
}
__device__ __forceinline__ Dual operator+(Dual a, double b) { return {a.v + b, a.d}; }
__device__ __forceinline__ Dual operator+(double a, Dual b) { return {a + b.v, b.d}; }
__device__ __forceinline__ Dual operator-(Dual a, double b) { return {a.v - b, a.d}; }
__device__ __forceinline__ Dual operator-(double a, Dual b) { return {a - b.v, -b.d}; }
__device__ __forceinline__ Dual operator*(Dual a, double b) { return {a.v * b, a.d * b}; }
__device__ __forceinline__ Dual operator*(double a, Dual b) { return {a * b.v, a * b.d}; }
__device__ __forceinline__ Dual operator/(Dual a, double b) { return {a.v / b, a.d / b}; }
__device__ __forceinline__ Dual operator/(double a, Dual b) { return {a / b.v, -a * b.d / (b.v * b.v)}; }
__device__ __forceinline__ Dual sqrt_t(Dual a) {
  const double r = ::sqrt(a.v);
  return {r, a.d / (2.0 * r)};
}
__device__ __forceinline__ double sqrt_t(double a) { return ::sqrt(a); }

template <typename T> struct CxT {
  T x, y;
};

template <typename T> struct SiteS {
  T n, m, A, gxy, gt[2];        // gt[0] spin up, gt[1] spin down
  T dA[2], dgxy[2], dgt[2][2];  // d/dn_up (index 0), d/dn_dn (index 1)
};

template <typename T>
__device__ __forceinline__ SiteS<T> site_s(T nu, T nd) {
  SiteS<T> f;
  f.n = nu + nd;
  const T dl = 1.0 - f.n;
  f.m = 0.5 * (nu - nd);
  f.A = 1.0 - dl * dl + 4.0 * f.m * f.m;
  f.gxy = 2.0 * f.n / f.A;
  const T B = 2.0 * dl * (1.0 - dl) / f.A;
  for (int q = 0; q < 2; ++q) {                         // derivative w.r.t. n_up (q = 0) or n_dn
    const double sq = q == 0 ? 1.0 : -1.0;
    f.dA[q] = 2.0 * dl + 4.0 * sq * f.m;
    f.dgxy[q] = (2.0 * f.A - 2.0 * f.n * f.dA[q]) / (f.A * f.A);
  }
  for (int s = 0; s < 2; ++s) {
    const double ss = s == 0 ? 1.0 : -1.0;
    const T p = 1.0 + dl + 2.0 * ss * f.m, qd = 1.0 + dl - 2.0 * ss * f.m;
    const T Q = p / qd;
    f.gt[s] = sqrt_t(B * Q);
    for (int q = 0; q < 2; ++q) {
      const double sq = q == 0 ? 1.0 : -1.0;
      const T dB = (2.0 * (2.0 * dl - 1.0) * f.A - 2.0 * dl * (1.0 - dl) * f.dA[q]) / (f.A * f.A);
      const double dp = -1.0 + ss * sq, dq = -1.0 - ss * sq;
      const T dQ = (dp * qd - p * dq) / (qd * qd);
      f.dgt[s][q] = (dB * Q + B * dQ) / (2.0 * f.gt[s]);
    }
  }
  return f;
}

template <typename T> struct BondIn {
  double2 t;                     // bare Peierls hopping (no tangent)
  CxT<T> cu, cd, du, dd;
};

// dW_b/dn_{a q} for the end a of a bond whose other end is b (W_b is
// symmetric in its two ends).
template <typename T>
__device__ __forceinline__ void bond_dn(const SiteS<T>& a, const SiteS<T>& b, const BondIn<T>& v, bool nn,
                                        double J, T out[2]) {
  const T Ru = v.t.x * v.cu.x - v.t.y * v.cu.y, Rd = v.t.x * v.cd.x - v.t.y * v.cd.y;
  for (int q = 0; q < 2; ++q)
    out[q] = -2.0 * (Ru * b.gt[0] * a.dgt[0][q] + Rd * b.gt[1] * a.dgt[1][q]);
  if (!nn) return;
  const T cbx = 0.5 * (v.cu.x + v.cd.x), cby = 0.5 * (v.cu.y + v.cd.y);
  const T dbx = 0.5 * (v.du.x + v.dd.x), dby = 0.5 * (v.du.y + v.dd.y);
  const T bb = 2.0 * (dbx * dbx + dby * dby - cbx * cbx - cby * cby);
  const T mm = a.m * b.m;
  const T sAB = sqrt_t(a.A * b.A);
  const T X = 1.0 + 12.0 * a.n * b.n / sAB;
  const T den = bb - 4.0 * mm;
  const T R = (bb - 4.0 * mm * X * X) / den;
  const T dRdmm = 4.0 * bb * (1.0 - X * X) / (den * den);
  const T dRdX = -8.0 * mm * X / den;
  const T gxy = a.gxy * b.gxy, gz = gxy * R;
  const T q2 = v.cu.x * v.cu.x + v.cu.y * v.cu.y + v.cd.x * v.cd.x + v.cd.y * v.cd.y +
               v.du.x * v.du.x + v.du.y * v.du.y + v.dd.x * v.dd.x + v.dd.y * v.dd.y;
  const T Szz = mm - 0.25 * q2;
  const T Sxy = -((v.cu.x * v.cd.x + v.cu.y * v.cd.y) + (v.du.x * v.dd.x + v.du.y * v.dd.y));
  for (int q = 0; q < 2; ++q) {
    const double sq = q == 0 ? 1.0 : -1.0;
    const T dmm = 0.5 * sq * b.m;
    const T dX = 12.0 * b.n * (1.0 / sAB - a.n * a.dA[q] / (2.0 * a.A * sAB));
    const T dgxy = b.gxy * a.dgxy[q];
    const T dgz = dgxy * R + gxy * (dRdmm * dmm + dRdX * dX);
    out[q] = out[q] + J * (dgz * Szz + gz * dmm + dgxy * Sxy);
  }
}

// Wirtinger derivatives dW_b/dz of the bond variables z = chi_up, chi_dn,
// Delta_up, Delta_dn (order of `g`).
template <typename T>
__device__ __forceinline__ void bond_dz(const SiteS<T>& a, const SiteS<T>& b, const BondIn<T>& v, bool nn,
                                        double J, CxT<T> g[4]) {
  const T tt = a.gt[0] * b.gt[0], td = a.gt[1] * b.gt[1];
  g[0] = CxT<T>{-tt * v.t.x, -tt * v.t.y};
  g[1] = CxT<T>{-td * v.t.x, -td * v.t.y};
  g[2] = CxT<T>{T{}, T{}};
  g[3] = CxT<T>{T{}, T{}};
  if (!nn) return;
  const T cbx = 0.5 * (v.cu.x + v.cd.x), cby = 0.5 * (v.cu.y + v.cd.y);
  const T dbx = 0.5 * (v.du.x + v.dd.x), dby = 0.5 * (v.du.y + v.dd.y);
  const T bb = 2.0 * (dbx * dbx + dby * dby - cbx * cbx - cby * cby);
  const T mm = a.m * b.m;
  const T X = 1.0 + 12.0 * a.n * b.n / sqrt_t(a.A * b.A);
  const T den = bb - 4.0 * mm;
  const T R = (bb - 4.0 * mm * X * X) / den;
  const T dRdb = 4.0 * mm * (X * X - 1.0) / (den * den);
  const T gxy = a.gxy * b.gxy, gz = gxy * R;
  const T q2 = v.cu.x * v.cu.x + v.cu.y * v.cu.y + v.cd.x * v.cd.x + v.cd.y * v.cd.y +
               v.du.x * v.du.x + v.du.y * v.du.y + v.dd.x * v.dd.x + v.dd.y * v.dd.y;
  const T Szz = mm - 0.25 * q2;
  // d b/d chi_s = -conj(chibar), d b/d Delta_s = conj(Dbar)
  const T k = J * gxy * dRdb * Szz;
  g[0].x = g[0].x + k * (-cbx) + J * (-0.25 * gz * v.cu.x - 0.5 * gxy * v.cd.x);
  g[0].y = g[0].y + k * (cby) + J * (0.25 * gz * v.cu.y + 0.5 * gxy * v.cd.y);
  g[1].x = g[1].x + k * (-cbx) + J * (-0.25 * gz * v.cd.x - 0.5 * gxy * v.cu.x);
  g[1].y = g[1].y + k * (cby) + J * (0.25 * gz * v.cd.y + 0.5 * gxy * v.cu.y);
  g[2].x = g[2].x + k * (dbx) + J * (-0.25 * gz * v.du.x - 0.5 * gxy * v.dd.x);
  g[2].y = g[2].y + k * (-dby) + J * (0.25 * gz * v.du.y + 0.5 * gxy * v.dd.y);
  g[3].x = g[3].x + k * (dbx) + J * (-0.25 * gz * v.dd.x - 0.5 * gxy * v.du.x);
  g[3].y = g[3].y + k * (-dby) + J * (0.25 * gz * v.dd.y + 0.5 * gxy * v.du.y);
}

__device__ __forceinline__ CxT<double> cx_in(const double* p, long long idx) {
  const double2 v = ld2(p, idx);
  return CxT<double>{v.x, v.y};
}

__global__ __launch_bounds__(kBlock) void k_build_sdw(ModelDev md, const double* __restrict__ nu,
                                                      const double* __restrict__ nd,
                                                      const double* __restrict__ cu,
                                                      const double* __restrict__ cd,
                                                      const double* __restrict__ du,
                                                      const double* __restrict__ dd,
                                                      double2* __restrict__ h) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= md.N) return;
  const int N = md.N;
  const SiteS<double> fi = site_s(nu[i], nd[i]);
  double eu = -md.mu, ed = -md.mu;
  for (int d = 0; d < 4; ++d) {
    const bool nn = d < 2;
    // forward bond (i, j = i + d), stored here
    {
      const int j = nbr_of(i, d, +1, md.Lx, md.Ly);
      const SiteS<double> fj = site_s(nu[j], nd[j]);
      const long long e = (long long)d * N + i;
      const BondIn<double> v{hop(md, i, d), cx_in(cu, e), cx_in(cd, e), cx_in(du, e), cx_in(dd, e)};
      CxT<double> g[4];
      bond_dz(fi, fj, v, nn, md.J, g);
      h[(long long)(4 * d + 0) * N + i] = make_double2(g[0].x, g[0].y);       // dW/dchi_up
      h[(long long)(4 * d + 1) * N + i] = make_double2(-g[2].x, g[2].y);      // -conj dW/dDelta_up
      h[(long long)(4 * d + 2) * N + i] = make_double2(-g[3].x, -g[3].y);     // -dW/dDelta_dn
      h[(long long)(4 * d + 3) * N + i] = make_double2(-g[1].x, g[1].y);      // -conj dW/dchi_dn
      double o[2];
      bond_dn(fi, fj, v, nn, md.J, o);
      eu += o[0];
      ed += o[1];
    }
    // backward bond (k = i - d, i), stored at k
    {
      const int k = nbr_of(i, d, -1, md.Lx, md.Ly);
      const SiteS<double> fk = site_s(nu[k], nd[k]);
      const long long e = (long long)d * N + k;
      const BondIn<double> v{hop(md, k, d), cx_in(cu, e), cx_in(cd, e), cx_in(du, e), cx_in(dd, e)};
      double o[2];
      bond_dn(fi, fk, v, nn, md.J, o);
      eu += o[0];
      ed += o[1];
    }
  }
  h[(long long)16 * N + i] = make_double2(eu, 0.0);
  h[(long long)17 * N + i] = make_double2(-ed, 0.0);
  h[(long long)18 * N + i] = make_double2(0.0, 0.0);
}

// VJP of k_build_sdw: dOmega/dtheta = sum_IJ rho_IJ dh_IJ/dtheta.  Since
// h_IJ = dW/drho_IJ, this is the derivative of the theta-gradient of W along
// the theta-direction v that moves the rho-coordinates by rho (symmetry of
// second derivatives): v = (Re rho_16, -Re rho_17, rho_e0, -conj rho_e3,
// -conj rho_e1, -rho_e2).  k_build_sdw's own chain rule runs on Dual values
// with those tangents; a complex parameter's output is 2 conj(tangent of
// dW/dz) = d/dRe z + i d/dIm z.
__device__ __forceinline__ Dual site_tan(const double* n, const double2* rho, int N, int j, int e,
                                         double sgn) {
  return Dual{n[j], sgn * rho[(long long)e * N + j].x};
}

__device__ __forceinline__ BondIn<Dual> bond_tan(const ModelDev& md, const double* cu, const double* cd,
                                                 const double* du, const double* dd,
                                                 const double2* rho, int k, int d) {
  const int N = md.N;
  const long long e = (long long)d * N + k;
  const double2 r0 = rho[(long long)(4 * d + 0) * N + k], r1 = rho[(long long)(4 * d + 1) * N + k];
  const double2 r2 = rho[(long long)(4 * d + 2) * N + k], r3 = rho[(long long)(4 * d + 3) * N + k];
  const double2 a = ld2(cu, e), b = ld2(cd, e), c = ld2(du, e), f = ld2(dd, e);
  BondIn<Dual> v;
  v.t = hop(md, k, d);
  v.cu = CxT<Dual>{Dual{a.x, r0.x}, Dual{a.y, r0.y}};      // + rho_e0
  v.cd = CxT<Dual>{Dual{b.x, -r3.x}, Dual{b.y, r3.y}};     // - conj rho_e3
  v.du = CxT<Dual>{Dual{c.x, -r1.x}, Dual{c.y, r1.y}};     // - conj rho_e1
  v.dd = CxT<Dual>{Dual{f.x, -r2.x}, Dual{f.y, -r2.y}};    // - rho_e2
  return v;
}

__global__ __launch_bounds__(kBlock) void k_build_sdw_vjp(ModelDev md, const double* __restrict__ nu,
                                                          const double* __restrict__ nd,
                                                          const double* __restrict__ cu,
                                                          const double* __restrict__ cd,
                                                          const double* __restrict__ du,
                                                          const double* __restrict__ dd,
                                                          const double2* __restrict__ rho,
                                                          double* __restrict__ gnu,
                                                          double* __restrict__ gnd,
                                                          double2* __restrict__ gcu,
                                                          double2* __restrict__ gcd,
                                                          double2* __restrict__ gdu,
                                                          double2* __restrict__ gdd) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= md.N) return;
  const int N = md.N;
  const SiteS<Dual> fi = site_s(site_tan(nu, rho, N, i, 16, 1.0), site_tan(nd, rho, N, i, 17, -1.0));
  double tu = 0.0, td = 0.0;
  for (int d = 0; d < 4; ++d) {
    const bool nn = d < 2;
    {
      const int j = nbr_of(i, d, +1, md.Lx, md.Ly);
      const SiteS<Dual> fj = site_s(site_tan(nu, rho, N, j, 16, 1.0), site_tan(nd, rho, N, j, 17, -1.0));
      const BondIn<Dual> v = bond_tan(md, cu, cd, du, dd, rho, i, d);
      CxT<Dual> g[4];
      bond_dz(fi, fj, v, nn, md.J, g);
      const long long e = (long long)d * N + i;
      gcu[e] = make_double2(2.0 * g[0].x.d, -2.0 * g[0].y.d);
      gcd[e] = make_double2(2.0 * g[1].x.d, -2.0 * g[1].y.d);
      gdu[e] = make_double2(2.0 * g[2].x.d, -2.0 * g[2].y.d);
      gdd[e] = make_double2(2.0 * g[3].x.d, -2.0 * g[3].y.d);
      Dual o[2];
      bond_dn(fi, fj, v, nn, md.J, o);
      tu += o[0].d;
      td += o[1].d;
    }
    {
      const int k = nbr_of(i, d, -1, md.Lx, md.Ly);
      const SiteS<Dual> fk = site_s(site_tan(nu, rho, N, k, 16, 1.0), site_tan(nd, rho, N, k, 17, -1.0));
      const BondIn<Dual> v = bond_tan(md, cu, cd, du, dd, rho, k, d);
      Dual o[2];
      bond_dn(fi, fk, v, nn, md.J, o);
      tu += o[0].d;
      td += o[1].d;
    }
  }
  gnu[i] = tu;
  gnd[i] = td;
}

// Per-site pieces of the VJP that every neighbour needs: w_i = Re rho16 -
// Re rho17 (weight of eps_i in the linearised energy).
__device__ __forceinline__ double onsite_w(const double2* rho, int N, int i) {
  return rho[(long long)16 * N + i].x - rho[(long long)17 * N + i].x;
}

// dOmega/dtheta = sum_IJ rho_IJ dh_IJ/dtheta.  With the linearisation
//   L = sum_b [2 Re(T_b U_b) + 2 Re(P_b V_b)] + sum_i w_i eps_i,
//   U_b = rho_{e0} - conj(rho_{e3}),  V_b = rho_{e1} + conj(rho_{e2}),
// the bond and site gradients are gathered per site from its 8 bonds.
__global__ __launch_bounds__(kBlock) void k_build_vjp(ModelDev md, const double* __restrict__ n,
                                                      const double* __restrict__ chi,
                                                      const double* __restrict__ dlt,
                                                      const double2* __restrict__ rho,
                                                      double* __restrict__ dn,
                                                      double2* __restrict__ dchi,
                                                      double2* __restrict__ ddlt) {
  int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= md.N) return;
  const int N = md.N;
  const double J = md.J;
  GF fi = gfac(n[i]);
  double wi = onsite_w(rho, N, i);
  double dLdd = 0.0;          // dL/d delta_i
  double deps_self = 0.0;     // d eps_i / d delta_i
  for (int d = 0; d < 4; ++d) {
    for (int side = 0; side < 2; ++side) {
      // side 0: bond (i, o = i + d) stored at i;  side 1: bond (o = i - d, i) stored at o
      int o = nbr_of(i, d, side == 0 ? +1 : -1, md.Lx, md.Ly);
      int tail = (side == 0) ? i : o;
      GF fo = gfac(n[o]);
      double wo = onsite_w(rho, N, o);
      double2 t = hop(md, tail, d);
      double2 c = ld2(chi, (long long)d * N + tail);
      double2 D = ld2(dlt, (long long)d * N + tail);
      double2 r0 = rho[(long long)(4 * d + 0) * N + tail];
      double2 r1 = rho[(long long)(4 * d + 1) * N + tail];
      double2 r2 = rho[(long long)(4 * d + 2) * N + tail];
      double2 r3 = rho[(long long)(4 * d + 3) * N + tail];
      double2 U = make_double2(r0.x - r3.x, r0.y + r3.y);
      double2 V = make_double2(r1.x + r2.x, r1.y - r2.y);
      double R = t.x * c.x - t.y * c.y;
      double Q = c.x * c.x + c.y * c.y + D.x * D.x + D.y * D.y;
      bool nn = d < 2;
      // dT/d delta_i = -g_i' g_o t - [nn] (3/4) J s_i' s_o conj(chi);  dP/d delta_i = [nn] (3/4) J s_i' s_o Delta
      double2 dT = make_double2(-fi.g1 * fo.g * t.x, -fi.g1 * fo.g * t.y);
      double2 dP = make_double2(0.0, 0.0);
      if (nn) {
        double k3 = 0.75 * J * fi.s1 * fo.s;
        dT.x -= k3 * c.x;
        dT.y += k3 * c.y;
        dP = make_double2(k3 * D.x, k3 * D.y);
      }
      dLdd += 2.0 * (dT.x * U.x - dT.y * U.y) + 2.0 * (dP.x * V.x - dP.y * V.y);
      deps_self += 4.0 * fi.g2 * fo.g * R + (nn ? 1.5 * J * fi.s2 * fo.s * Q : 0.0);
      // eps_o depends on delta_i through this bond
      dLdd += wo * (4.0 * fo.g1 * fi.g1 * R + (nn ? 1.5 * J * fo.s1 * fi.s1 * Q : 0.0));
      if (side == 0) {
        // gradients of the bond variables stored at i
        double cb = nn ? 0.75 * J * fi.s * fo.s : 0.0;
        double kt = 4.0 * (wi * fi.g1 * fo.g + wo * fo.g1 * fi.g);     // * conj(t)
        double kq = nn ? 3.0 * J * (wi * fi.s1 * fo.s + wo * fo.s1 * fi.s) : 0.0;
        double2 gc = make_double2(-2.0 * cb * U.x + kt * t.x + kq * c.x,
                                  -2.0 * cb * U.y - kt * t.y + kq * c.y);
        double2 gd = nn ? make_double2(2.0 * cb * V.x + kq * D.x, -2.0 * cb * V.y + kq * D.y)
                        : make_double2(0.0, 0.0);
        dchi[(long long)d * N + i] = gc;
        ddlt[(long long)d * N + i] = gd;
      }
    }
  }
  dLdd += wi * deps_self;
  dn[i] = -dLdd;
}

// Gershgorin bounds -> ab = (a, b); one block of kBoundsBlock threads (the
// max / min are order-independent, so the result is deterministic).  On a
// non-finite or empty interval a is set to NaN (the recursion then reports
// KPM_EBOUNDS).
constexpr int kBoundsBlock = 1024;

__global__ __launch_bounds__(kBoundsBlock) void k_bounds(int Lx, int Ly, const double2* __restrict__ h,
                                                   double* __restrict__ ab) {
  const int N = Lx * Ly;
  double emax = -1e300, emin = 1e300;
  int finite = 1;
  for (int i = threadIdx.x; i < N; i += kBoundsBlock) {
    double r0 = 0.0, r1 = 0.0;
    double2 p = h[(long long)18 * N + i];
    double ap = hypot(p.x, p.y);
    r0 += ap;
    r1 += ap;
    for (int d = 0; d < 4; ++d) {
      int j = nbr_of(i, d, -1, Lx, Ly);
      double2 f0 = h[(long long)(4 * d + 0) * N + i], f1 = h[(long long)(4 * d + 1) * N + i];
      double2 f2 = h[(long long)(4 * d + 2) * N + i], f3 = h[(long long)(4 * d + 3) * N + i];
      double2 b0 = h[(long long)(4 * d + 0) * N + j], b1 = h[(long long)(4 * d + 1) * N + j];
      double2 b2 = h[(long long)(4 * d + 2) * N + j], b3 = h[(long long)(4 * d + 3) * N + j];
      // row (i,0): (i0,j'b) forward entries 00, 01 and backward conj(B_{b0}(j)): 00, 10
      r0 += hypot(f0.x, f0.y) + hypot(f1.x, f1.y) + hypot(b0.x, b0.y) + hypot(b2.x, b2.y);
      // row (i,1): forward 11, 10 and backward conj(B_{b1}(j)): 11, 01 -- summed in the
      // order that mirrors row (i,0), so a particle-hole symmetric h gets Emin = -Emax exactly
      r1 += hypot(f3.x, f3.y) + hypot(f2.x, f2.y) + hypot(b3.x, b3.y) + hypot(b1.x, b1.y);
    }
    double c0 = h[(long long)16 * N + i].x, c1 = h[(long long)17 * N + i].x;
    emax = fmax(emax, fmax(c0 + r0, c1 + r1));
    emin = fmin(emin, fmin(c0 - r0, c1 - r1));
    if (!(isfinite(c0 + r0) && isfinite(c1 + r1) && isfinite(c0 - r0) && isfinite(c1 - r1))) finite = 0;
  }
  __shared__ double smax[kBoundsBlock], smin[kBoundsBlock];
  __shared__ int sfin[kBoundsBlock];
  smax[threadIdx.x] = emax;
  smin[threadIdx.x] = emin;
  sfin[threadIdx.x] = finite;
  __syncthreads();
  for (unsigned s = kBoundsBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
      sfin[threadIdx.x] = sfin[threadIdx.x] & sfin[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double a = (smax[0] - smin[0]) / (2.0 - 0.01);
    double b = (smax[0] + smin[0]) / 2.0;
    if (!sfin[0] || !(a > 0.0) || !isfinite(a)) a = __builtin_nan("");
    ab[0] = a;
    ab[1] = b;
  }
}

// Row-form rescaled coefficients H~ = (h - b)/a for the recursion kernels,
// laid out in the order the recursion waves read them: for tile t of an
// instance, pair k (record k = 0 site, 1..4 forward, 5..8 backward
// neighbours) and lane l (site l >> 1 of the 8 x 4 tile, Nambu row a = l & 1),
// the 4-vector (re, im) of H~_{(i,a),(nb_k(i),0)} followed by (re, im) of
// H~_{(i,a),(nb_k(i),1)} sits at [(t * 9 + k) * 64 + l].  A wave thus loads
// its whole row block with 9 contiguous 64-lane loads.  Lanes outside the
// lattice get zeros.  One 64-thread block per tile.
template <typename V>
__global__ __launch_bounds__(64) void k_rescale(const InstDev* __restrict__ insts,
                                                const int4* __restrict__ tmap) {
  using R4 = typename RecT4<V>::T;
  const int4 tm = tmap[blockIdx.x];
  const InstDev& I = insts[tm.x];
  const int l = threadIdx.x, al = l & 1, s = l >> 1;
  const int x = tm.y + (s & 7), y = tm.z + (s >> 3);
  R4* out = reinterpret_cast<R4*>(I.coef) + (size_t)tm.w * 9 * 64 + l;
  double c[18][2];
#pragma unroll
  for (int q = 0; q < 18; ++q) c[q][0] = c[q][1] = 0.0;
  if (x < I.Lx && y < I.Ly) {
    const int N = I.N, i = y * I.Lx + x;
    const double2* h = I.h;
    const double ia = 1.0 / I.ab[0], b = I.ab[1];
    const double2 p = h[(long long)18 * N + i];
    if (al == 0) {
      c[0][0] = (h[(long long)16 * N + i].x - b) * ia;
      c[1][0] = p.x * ia;
      c[1][1] = p.y * ia;
    } else {
      c[0][0] = p.x * ia;
      c[0][1] = -p.y * ia;
      c[1][0] = (h[(long long)17 * N + i].x - b) * ia;
    }
    for (int d = 0; d < 4; ++d) {
      const int j = nbr_of(i, d, -1, I.Lx, I.Ly);
      for (int be = 0; be < 2; ++be) {
        const double2 f = h[(long long)(4 * d + 2 * al + be) * N + i];
        c[2 * (1 + d) + be][0] = f.x * ia;
        c[2 * (1 + d) + be][1] = f.y * ia;
        const double2 r = h[(long long)(4 * d + 2 * be + al) * N + j];   // conj(B_{be al}(j))/a
        c[2 * (5 + d) + be][0] = r.x * ia;
        c[2 * (5 + d) + be][1] = -r.y * ia;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    R4 v;
    v.x = (V)c[2 * k][0];
    v.y = (V)c[2 * k][1];
    v.z = (V)c[2 * k + 1][0];
    v.w = (V)c[2 * k + 1][1];
    out[k * 64] = v;
  }
}

template __global__ void k_rescale<float>(const InstDev*, const int4*);
template __global__ void k_rescale<double>(const InstDev*, const int4*);

// C_m = (2 - delta_m0) g_m (1/K) sum_k cos(m th_k) f(a cos th_k + b).
// cos(m th_k) = cospi(j/(2K)) with the exact integer j = m(2k+1) mod 4K.
// A block handles kBlock / L consecutive m: L lanes per m run over k (lane l
// takes k = l, l + L, ...), f(x_k) is evaluated once per block in LDS, and
// the L lane sums of each m are added in a fixed butterfly order.  L is
// chosen per M (coeff_lanes) so that the grid of M L / kBlock blocks covers
// the chip (about 256 blocks) without more blocks, each of which evaluates
// f at all K nodes again.
template <int L>
__global__ __launch_bounds__(kBlock) void k_coeffs(int M, int K, double T,
                                                   const double* __restrict__ ab,
                                                   double* __restrict__ C) {
  __shared__ double F[kBlock];
  const int lane = threadIdx.x & (L - 1);
  const int m = blockIdx.x * (kBlock / L) + threadIdx.x / L;
  const double a = ab[0], b = ab[1];
  const long long fourK = 4LL * K;
  const double inv2K = 1.0 / (2.0 * (double)K);
  const long long mm = m < M ? m : 0;
  long long j = (mm * (2LL * lane + 1)) % fourK;           // k = lane
  const long long step = (2LL * L * mm) % fourK;           // k -> k + L
  double acc = 0.0;
  for (int k0 = 0; k0 < K; k0 += kBlock) {
    const int k = k0 + threadIdx.x;
    if (k < K) {
      const double x = cospi((2.0 * k + 1.0) * inv2K);
      const double e = a * x + b;
      F[threadIdx.x] = fmin(e, 0.0) - T * log1p(exp(-fabs(e) / T));
    }
    __syncthreads();
    const int kmax = min(kBlock, K - k0);
    for (int kk = lane; kk < kmax; kk += L) {
      acc += F[kk] * cospi((double)j * inv2K);
      j += step;
      if (j >= fourK) j -= fourK;
    }
    __syncthreads();
  }
#pragma unroll
  for (int o = L / 2; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, L);
  if (m < M && lane == 0) {
    const double c = acc / (double)K;
    const double q = 1.0 / (double)(M + 1);
    const double g = ((double)(M - m + 1) * cospi(m * q) + sinpi(m * q) * cospi(q) / sinpi(q)) * q;
    C[m] = (m == 0 ? 1.0 : 2.0) * g * c;
  }
}

}  // namespace kpm

// ------------------------------------------------------------------ launchers
namespace kpm {

hipError_t launch_build_h(const ModelDev& md, const double* n, const double* chi,
                          const double* dlt, double* h, hipStream_t s) {
  dim3 grid((md.N + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_build_h, grid, dim3(kBlock), 0, s, md, n, chi, dlt,
                     reinterpret_cast<double2*>(h));
  return hipGetLastError();
}

hipError_t launch_build_sdw(const ModelDev& md, const double* nu, const double* nd, const double* cu,
                            const double* cd, const double* du, const double* dd, double* h,
                            hipStream_t s) {
  dim3 grid((md.N + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_build_sdw, grid, dim3(kBlock), 0, s, md, nu, nd, cu, cd, du, dd,
                     reinterpret_cast<double2*>(h));
  return hipGetLastError();
}

hipError_t launch_build_sdw_vjp(const ModelDev& md, const double* nu, const double* nd,
                                const double* cu, const double* cd, const double* du,
                                const double* dd, const double* rho, double* gnu, double* gnd,
                                double* gcu, double* gcd, double* gdu, double* gdd, hipStream_t s) {
  dim3 grid((md.N + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_build_sdw_vjp, grid, dim3(kBlock), 0, s, md, nu, nd, cu, cd, du, dd,
                     reinterpret_cast<const double2*>(rho), gnu, gnd, reinterpret_cast<double2*>(gcu),
                     reinterpret_cast<double2*>(gcd), reinterpret_cast<double2*>(gdu),
                     reinterpret_cast<double2*>(gdd));
  return hipGetLastError();
}

hipError_t launch_build_vjp(const ModelDev& md, const double* n, const double* chi,
                            const double* dlt, const double* rho, double* dn, double* dchi,
                            double* ddlt, hipStream_t s) {
  dim3 grid((md.N + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_build_vjp, grid, dim3(kBlock), 0, s, md, n, chi, dlt,
                     reinterpret_cast<const double2*>(rho), dn, reinterpret_cast<double2*>(dchi),
                     reinterpret_cast<double2*>(ddlt));
  return hipGetLastError();
}

hipError_t launch_bounds(int Lx, int Ly, const double* h, double* ab, hipStream_t s) {
  hipLaunchKernelGGL(k_bounds, dim3(1), dim3(kBoundsBlock), 0, s, Lx, Ly,
                     reinterpret_cast<const double2*>(h), ab);
  return hipGetLastError();
}

hipError_t launch_rescale(const InstDev* insts, const int4* tmap, int ntiles, bool fp32,
                          hipStream_t s) {
  if (fp32)
    hipLaunchKernelGGL(k_rescale<float>, dim3(ntiles), dim3(64), 0, s, insts, tmap);
  else
    hipLaunchKernelGGL(k_rescale<double>, dim3(ntiles), dim3(64), 0, s, insts, tmap);
  return hipGetLastError();
}

// Lanes per coefficient of k_coeffs: measured at K = 16384, 200 us with 16
// lanes and 93 us with 64 at M = 1024; 228 us with 16 and 274 us with 64 at
// M = 4096 (where 64 lanes give 1024 blocks, each evaluating f again).
int coeff_lanes(int M) { return M <= 1024 ? 64 : M <= 2048 ? 32 : 16; }

hipError_t launch_coeffs(int M, int K, double T, const double* ab, double* C, hipStream_t s) {
  const int L = coeff_lanes(M);
  dim3 grid((M * L + kBlock - 1) / kBlock);
  if (L == 64) hipLaunchKernelGGL(k_coeffs<64>, grid, dim3(kBlock), 0, s, M, K, T, ab, C);
  else if (L == 32) hipLaunchKernelGGL(k_coeffs<32>, grid, dim3(kBlock), 0, s, M, K, T, ab, C);
  else hipLaunchKernelGGL(k_coeffs<16>, grid, dim3(kBlock), 0, s, M, K, T, ab, C);
  return hipGetLastError();
}

}  // namespace kpm
