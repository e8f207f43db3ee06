// Geometry setup (per geometry, not per apply): nodes, normals and weights
// (Section 2.1 Table 1, Section 2.2 Table 2, Section 4 density
// representation), the real surface-harmonic transform matrices, the spectra
// of Theorems 1 and 2, and the exact-distance near/far split of Section 4.1.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "legendre_dev.h"
#include "sbie_internal.h"

namespace sbie {

namespace {

constexpr int kCfMaxIter = 10000;

// ---------------------------------------------------------------- nodes

// One thread per node g = i*T + j*Nphi + k.
__global__ void k_nodes(const Particle* __restrict__ part, const double* __restrict__ gl, int p,
                        int64_t N, double* x, double* y, double* z, double* nx, double* ny,
                        double* nz, double* w, float* off32) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  const int Nphi = 2 * p + 2, T = (p + 1) * Nphi;
  const int i = (int)(g / T);
  const int r = (int)(g - (int64_t)i * T);
  const int j = r / Nphi, k = r - j * Nphi;
  const Particle P = part[i];
  const double v = gl[j], gw = gl[p + 1 + j];
  double sphi, cphi;
  sincospi(2.0 * k / Nphi, &sphi, &cphi);
  const double sv = sqrt((1.0 - v) * (1.0 + v));
  // body point on u = u0: (A sv cos, A sv sin, C v); gradient of the implicit equation
  const double b[3] = {P.A * sv * cphi, P.A * sv * sphi, P.C * v};
  const double gb[3] = {b[0] / (P.A * P.A), b[1] / (P.A * P.A), b[2] / (P.C * P.C)};
  const double gn = sqrt(gb[0] * gb[0] + gb[1] * gb[1] + gb[2] * gb[2]);
  double X[3], Nn[3];
  for (int a = 0; a < 3; ++a) {
    X[a] = P.c[a] + P.R[3 * a] * b[0] + P.R[3 * a + 1] * b[1] + P.R[3 * a + 2] * b[2];
    Nn[a] = (P.R[3 * a] * gb[0] + P.R[3 * a + 1] * gb[1] + P.R[3 * a + 2] * gb[2]) / gn;
  }
  x[g] = X[0];
  y[g] = X[1];
  z[g] = X[2];
  nx[g] = Nn[0];
  ny[g] = Nn[1];
  nz[g] = Nn[2];
  // area element a^2 sqrt(u0^2 -+ v^2) sqrt(u0^2 -+ 1), GL weight, trapezoid weight
  const double s = P.oblate ? 1.0 : -1.0;
  const double J = P.a * P.a * sqrt(fma(s * v, v, P.u0 * P.u0)) * sqrt(P.w0);
  w[g] = gw * (2.0 * kPi / Nphi) * J;
  // node offset from the particle centre in body-rotated lab axes (float)
  off32[4 * g + 0] = (float)(X[0] - P.c[0]);
  off32[4 * g + 1] = (float)(X[1] - P.c[1]);
  off32[4 * g + 2] = (float)(X[2] - P.c[2]);
  off32[4 * g + 3] = 0.0f;
}

// S weight sqrt(u0^2 -+ v_j^2) per (particle, v index) (Section 3.2 modified basis).
__global__ void k_ws(const Particle* __restrict__ part, const double* __restrict__ gl, int M, int p,
                     double* wS) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= M * (p + 1)) return;
  const int i = t / (p + 1), j = t - i * (p + 1);
  const Particle P = part[i];
  const double v = gl[j];
  wS[t] = sqrt(fma(P.oblate ? v : -v, v, P.u0 * P.u0));
}

// ---------------------------------------------------------------- transform matrices

// One thread per node of the reference grid: all real orthonormal harmonics
// Y_l(v_j, phi_k) (Definition 1 in real form) from the normalised Ferrers
// recurrence Pb_n^m = a_nm (v Pb_{n-1}^m - b_nm Pb_{n-2}^m), and their v and
// phi derivatives.  dPb_n^m/dv follows from the derivative identity of
// Section 2.3 on the cut, normalised:
//   (1 - v^2) dPb_n^m/dv = (n+1) v Pb_n^m - sqrt((2n+1)(n+m+1)(n-m+1)/(2n+3)) Pb_{n+1}^m.
__global__ void k_basis(const double* __restrict__ gl, const double* __restrict__ ab, int p,
                        double* An, double* Sy, float* An32, float* Sy32, double* Sv, double* Sp,
                        float* Sv32, float* Sp32) {
  const int Nphi = 2 * p + 2, T = (p + 1) * Nphi, K = (p + 1) * (p + 1);
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  const int j = t / Nphi, k = t - j * Nphi;
  const double v = gl[j];
  const double qw = gl[p + 1 + j] * (2.0 * kPi / Nphi);
  const double omv2 = (1.0 - v) * (1.0 + v);
  const double sv = sqrt(omv2);
  double pmm = 0.28209479177387814347;  // 1/sqrt(4 pi)
  for (int m = 0; m <= p; ++m) {
    if (m > 0) pmm *= sqrt((2.0 * m + 1.0) / (2.0 * m)) * sv;
    double sm, cm;
    sincospi(2.0 * m * k / Nphi, &sm, &cm);
    const double sq2 = m == 0 ? 1.0 : 1.41421356237309504880;
    double p2 = 0.0, p1 = pmm, prev = 0.0;
    for (int n = m; n <= p + 1; ++n) {
      double pn;
      if (n == m) {
        pn = pmm;
      } else if (n == m + 1) {
        pn = sqrt(2.0 * m + 3.0) * v * pmm;
      } else {
        const int h = n * (n + 1) / 2 + m;
        pn = ab[2 * h] * (v * p1 - ab[2 * h + 1] * p2);
      }
      if (n > m) {
        p2 = p1;
        p1 = pn;
        // derivative of degree n-1 from Pb_{n-1} (prev) and Pb_n (pn)
        const int d = n - 1;
        const double c = sqrt((2.0 * d + 1.0) * (d + m + 1.0) * (d - m + 1.0) / (2.0 * d + 3.0));
        const double dp = ((d + 1.0) * v * prev - c * pn) / omv2;
        if (m == 0) {
          const int l = d * d + d;
          Sv[(size_t)l * T + t] = dp;
          Sp[(size_t)l * T + t] = 0.0;
        } else {
          const int lc = d * d + d + m, ls = d * d + d - m;
          Sv[(size_t)lc * T + t] = sq2 * dp * cm;
          Sv[(size_t)ls * T + t] = sq2 * dp * sm;
          Sp[(size_t)lc * T + t] = -m * sq2 * prev * sm;
          Sp[(size_t)ls * T + t] = m * sq2 * prev * cm;
        }
      }
      prev = pn;
      if (n > p) break;
      if (m == 0) {
        const int l = n * n + n;
        An[(size_t)t * K + l] = qw * pn;
        Sy[(size_t)l * T + t] = pn;
      } else {
        const double yc = sq2 * pn * cm;
        const double ys = sq2 * pn * sm;
        const int lc = n * n + n + m, ls = n * n + n - m;
        An[(size_t)t * K + lc] = qw * yc;
        An[(size_t)t * K + ls] = qw * ys;
        Sy[(size_t)lc * T + t] = yc;
        Sy[(size_t)ls * T + t] = ys;
      }
    }
  }
  for (int l = 0; l < K; ++l) {
    An32[(size_t)t * K + l] = (float)An[(size_t)t * K + l];
    Sy32[(size_t)l * T + t] = (float)Sy[(size_t)l * T + t];
    Sv32[(size_t)l * T + t] = (float)Sv[(size_t)l * T + t];
    Sp32[(size_t)l * T + t] = (float)Sp[(size_t)l * T + t];
  }
}

// ---------------------------------------------------------------- spectra

// One thread per (particle, m).  lam[i][h][0..3] with h = n(n+1)/2 + m:
//  0: D principal value (average of the exterior and interior limits, Theorem 1)
//  1: D exterior limit b P'(z0) Q(z0), used for the near-field expansion
//  2: S on the surface in the modified basis, b~ P(z0) Q(z0) (Theorem 2)
//  3: 1 / Q_n^m(z0) (real form for oblates), the normaliser of the exterior ratio
//  dlr[i][h] = d/du [Q_n^m(u)/Q_n^m(u0)] at u = u0 (real form for oblates): the
//  exterior-limit normal-coordinate derivative used by gradients on the surface
__global__ void k_spectra(const Particle* __restrict__ part, int M, int p, double* lam, double* dlr,
                          unsigned* status) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= M * (p + 1)) return;
  const int i = t / (p + 1), m = t - i * (p + 1);
  const Particle P = part[i];
  const int N = p + 1;
  double Pv[kMaxP + 3], Qv[kMaxP + 3], wdP[kMaxP + 3], wdQ[kMaxP + 3];
  if (!legendre_column(P.oblate != 0, P.u0, m, N, kCfMaxIter, Pv, Qv, wdP, wdQ)) {
    atomicOr(status, kStatNumeric);
    return;
  }
  const int Kh = (p + 1) * (p + 2) / 2;
  const double sw0 = sqrt(P.w0);
  for (int n = m; n <= p; ++n) {
    // r = (n-m)!/(n+m)! (-1)^m
    double r = 1.0;
    for (int q = n - m + 1; q <= n + m; ++q) r /= (double)q;
    if (m & 1) r = -r;
    const double lp = r * wdP[n] * Qv[n];
    const double lm = r * wdQ[n] * Pv[n];
    const double ls = P.a * r * sw0 * Pv[n] * Qv[n];
    double* o = lam + ((size_t)i * Kh + n * (n + 1) / 2 + m) * 4;
    o[0] = 0.5 * (lp + lm);
    o[1] = lp;
    o[2] = ls;
    o[3] = 1.0 / Qv[n];
    dlr[(size_t)i * Kh + n * (n + 1) / 2 + m] = wdQ[n] / (P.w0 * Qv[n]);
  }
}

// ---------------------------------------------------------------- distances

struct Body {
  double c[3], R[9], A, C;
};

__device__ inline void to_body(const Body& B, const double x[3], double b[3]) {
  const double d0 = x[0] - B.c[0], d1 = x[1] - B.c[1], d2 = x[2] - B.c[2];
  for (int a = 0; a < 3; ++a) b[a] = B.R[a] * d0 + B.R[3 + a] * d1 + B.R[6 + a] * d2;
}

__device__ inline bool body_inside(const Body& B, const double x[3]) {
  double b[3];
  to_body(B, x, b);
  return (b[0] * b[0] + b[1] * b[1]) / (B.A * B.A) + b[2] * b[2] / (B.C * B.C) <= 1.0;
}

// nearest point of the spheroid to an exterior point: x_b scaled componentwise by
// a^2/(a^2 + t) with t >= 0 the root of the Lagrange condition (safeguarded Newton)
__device__ inline void body_project(const Body& B, const double x[3], double out[3]) {
  double b[3];
  to_body(B, x, b);
  const double A2 = B.A * B.A, C2 = B.C * B.C;
  const double r2 = b[0] * b[0] + b[1] * b[1], z2 = b[2] * b[2];
  double lo = 0.0, hi = fmax(B.A, B.C) * sqrt(r2 + z2) + 1e-300, t = 0.0;
  for (int it = 0; it < 200; ++it) {
    const double ea = A2 + t, ec = C2 + t;
    const double f = r2 * A2 / (ea * ea) + z2 * C2 / (ec * ec) - 1.0;
    if (f == 0.0) break;
    if (f > 0.0) lo = t; else hi = t;
    const double df = -2.0 * r2 * A2 / (ea * ea * ea) - 2.0 * z2 * C2 / (ec * ec * ec);
    double tn = t - f / df;
    if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
    const bool done = fabs(tn - t) <= 2e-16 * fmax(1.0, tn);
    t = tn;
    if (done) break;
  }
  const double fa = A2 / (A2 + t), fc = C2 / (C2 + t);
  const double y[3] = {b[0] * fa, b[1] * fa, b[2] * fc};
  for (int a = 0; a < 3; ++a)
    out[a] = B.c[a] + B.R[3 * a] * y[0] + B.R[3 * a + 1] * y[1] + B.R[3 * a + 2] * y[2];
}

__device__ inline double body_support(const Body& B, const double n[3]) {
  double nb[3];
  for (int a = 0; a < 3; ++a) nb[a] = B.R[a] * n[0] + B.R[3 + a] * n[1] + B.R[6 + a] * n[2];
  return B.c[0] * n[0] + B.c[1] * n[1] + B.c[2] * n[2] +
         sqrt(B.A * B.A * (nb[0] * nb[0] + nb[1] * nb[1]) + B.C * B.C * nb[2] * nb[2]);
}

// One thread per unordered pair (i < j).  Circumsphere prefilter, then
// alternating projections between the two surfaces (upper bounds) with the
// separation of the supporting planes normal to the current chord (lower
// bounds) until both directed decisions d < eta*diam are certain or the bounds
// meet to 1e-12.  near[i*M + j] = 1 iff j is in the near field of source i.
__global__ void k_classify(const Particle* __restrict__ part, int M, double eta, uint8_t* near,
                           unsigned* status) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t npairs = (int64_t)M * (M - 1) / 2;
  if (t >= npairs) return;
  // unrank t -> (i, j), i < j
  int i = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((int64_t)(i + 1) * (i + 2) / 2 <= t) ++i;
  while ((int64_t)i * (i + 1) / 2 > t) --i;
  const int jj = (int)(t - (int64_t)i * (i + 1) / 2);  // 0..i
  const int a = jj, bidx = i + 1;                       // pair (a, bidx) with a < bidx
  const Particle& Pa = part[a];
  const Particle& Pb = part[bidx];
  const double dc = sqrt((Pa.c[0] - Pb.c[0]) * (Pa.c[0] - Pb.c[0]) +
                         (Pa.c[1] - Pb.c[1]) * (Pa.c[1] - Pb.c[1]) +
                         (Pa.c[2] - Pb.c[2]) * (Pa.c[2] - Pb.c[2]));
  const double thr_a = eta * Pa.diam, thr_b = eta * Pb.diam;
  const double lb0 = dc - 0.5 * Pa.diam - 0.5 * Pb.diam;
  if (lb0 >= thr_a && lb0 >= thr_b) return;  // far both ways
  Body A, B;
  for (int q = 0; q < 3; ++q) { A.c[q] = Pa.c[q]; B.c[q] = Pb.c[q]; }
  for (int q = 0; q < 9; ++q) { A.R[q] = Pa.R[q]; B.R[q] = Pb.R[q]; }
  A.A = Pa.A; A.C = Pa.C; B.A = Pb.A; B.C = Pb.C;
  if (body_inside(A, B.c) || body_inside(B, A.c)) {
    atomicOr(status, kStatOverlap);
    return;
  }
  double xa[3], yb[3];
  body_project(A, B.c, xa);
  if (body_inside(B, xa)) {
    atomicOr(status, kStatOverlap);
    return;
  }
  double up = 1e300, lo = -1e300;
  for (int it = 0; it < 100000; ++it) {
    body_project(B, xa, yb);
    if (body_inside(A, yb)) {
      atomicOr(status, kStatOverlap);
      return;
    }
    body_project(A, yb, xa);
    const double d[3] = {yb[0] - xa[0], yb[1] - xa[1], yb[2] - xa[2]};
    const double dn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    up = fmin(up, dn);
    if (dn > 0.0) {
      const double n[3] = {d[0] / dn, d[1] / dn, d[2] / dn};
      const double mn[3] = {-n[0], -n[1], -n[2]};
      lo = fmax(lo, -body_support(B, mn) - body_support(A, n));
    }
    const bool dec_a = up < thr_a || lo >= thr_a;
    const bool dec_b = up < thr_b || lo >= thr_b;
    if ((dec_a && dec_b) || up - lo <= 1e-12) break;
  }
  if (lo <= 0.0 && up <= 1e-12) {
    atomicOr(status, kStatOverlap);
    return;
  }
  const double d = (up - lo <= 1e-12) ? 0.5 * (up + lo) : 0.5 * (up + lo);
  const bool near_a = (up < thr_a) ? true : (lo >= thr_a ? false : d < thr_a);
  const bool near_b = (up < thr_b) ? true : (lo >= thr_b ? false : d < thr_b);
  if (near_a) near[(size_t)a * M + bidx] = 1;   // target bidx near source a
  if (near_b) near[(size_t)bidx * M + a] = 1;   // target a near source bidx
}

void gauss_legendre_host(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double t = std::cos(kPi * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = t;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2 * k - 1) * t * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (t * p1 - p0) / (t * t - 1.0);
      const double dt = p1 / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    double p0 = 1.0, p1 = t;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2 * k - 1) * t * p1 - (k - 1) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (t * p1 - p0) / (t * t - 1.0);
    x[n - 1 - i] = t;
    w[n - 1 - i] = 2.0 / ((1.0 - t * t) * dp * dp);
  }
}

}  // namespace

#define SBIE_TRY(expr)                      \
  do {                                      \
    sbie_status _s = (expr);                \
    if (_s != SBIE_OK) return _s;           \
  } while (0)

sbie_status carve_geometry(sbie_geom* g, Carver& c) {
  const int M = g->M, p = g->p, T = g->T, K = g->K, Kh = g->Kh;
  const int64_t N = g->N;
  const int Kh2 = (p + 2) * (p + 3) / 2;
  const size_t n16 = (size_t)M * (16 * ((T + 15) / 16));
  const int words = (M + 31) / 32;
  SBIE_TRY(c.take(&g->d_part, M));
  SBIE_TRY(c.take(&g->d_x, N));
  SBIE_TRY(c.take(&g->d_y, N));
  SBIE_TRY(c.take(&g->d_z, N));
  SBIE_TRY(c.take(&g->d_nx, N));
  SBIE_TRY(c.take(&g->d_ny, N));
  SBIE_TRY(c.take(&g->d_nz, N));
  SBIE_TRY(c.take(&g->d_w, N));
  SBIE_TRY(c.take(&g->d_off32, 4 * N));
  SBIE_TRY(c.take(&g->d_gl, 2 * (p + 1)));
  SBIE_TRY(c.take(&g->d_An, (size_t)T * K));
  SBIE_TRY(c.take(&g->d_Sy, (size_t)K * T));
  SBIE_TRY(c.take(&g->d_An32, (size_t)T * K));
  SBIE_TRY(c.take(&g->d_Sy32, (size_t)K * T));
  SBIE_TRY(c.take(&g->d_wS, (size_t)M * (p + 1)));
  SBIE_TRY(c.take(&g->d_Sv, (size_t)K * T));
  SBIE_TRY(c.take(&g->d_Sp, (size_t)K * T));
  SBIE_TRY(c.take(&g->d_Sv32, (size_t)K * T));
  SBIE_TRY(c.take(&g->d_Sp32, (size_t)K * T));
  SBIE_TRY(c.take(&g->d_lam, (size_t)M * Kh * 4));
  SBIE_TRY(c.take(&g->d_dlr, (size_t)M * Kh));
  // Ferrers recurrence coefficients through degree p+1 (derivatives need Pb_{p+1})
  SBIE_TRY(c.take(&g->d_ab, (size_t)Kh2 * 2));
  SBIE_TRY(c.take(&g->d_cd, (size_t)Kh));
  SBIE_TRY(c.take(&g->d_status, 2));
  SBIE_TRY(c.take(&g->d_near_scratch, (size_t)M * M));
  SBIE_TRY(c.take(&g->d_near_ptr, M + 1));
  // near sources: at most M(M-1) directed pairs
  SBIE_TRY(c.take(&g->d_near_src, std::max<size_t>(1, (size_t)M * (M - 1))));
  SBIE_TRY(c.take(&g->d_excl, (size_t)M * words));
  SBIE_TRY(c.take(&g->d_f, (size_t)M * T));
  SBIE_TRY(c.take(&g->d_coef, (size_t)M * K));
  SBIE_TRY(c.take(&g->d_cself, (size_t)M * K));
  SBIE_TRY(c.take(&g->d_E, (size_t)M * K));
  SBIE_TRY(c.take(&g->d_uself, N));
  SBIE_TRY(c.take(&g->d_unear, (size_t)kNearSplit * N));
  SBIE_TRY(c.take(&g->d_src, 8 * N));
  SBIE_TRY(c.take(&g->d_partial, (size_t)g->nsplit * N));
  SBIE_TRY(c.take(&g->d_dens, N));
  SBIE_TRY(c.take(&g->d_out, N));
  SBIE_TRY(c.take(&g->d_srec64, 5 * n16));
  SBIE_TRY(c.take(&g->d_srec32, 5 * n16));
  // per-apply far strengths: up to 8 values per padded source (S')
  SBIE_TRY(c.take(&g->d_fstr64, 8 * n16));
  SBIE_TRY(c.take(&g->d_fstr32, 8 * n16));
  SBIE_TRY(c.take(&g->d_rcp, (size_t)kRcpN));
  // reverse sums of one launch of the pair-symmetric far field (matrix-core
  // path, T >= 32) and their running FP64 totals
  g->rev_slots = far_rev_slots(M, T);
  const size_t nrev = T >= 32 ? (size_t)M * g->rev_slots * far_row_groups(g, true) * T : 1;
  SBIE_TRY(c.take(&g->d_rev, nrev));
  SBIE_TRY(c.take(&g->d_racc, T >= 32 ? (size_t)N : 1));
  SBIE_TRY(c.take(&g->d_eta, (size_t)M));
  SBIE_TRY(c.take(&g->d_qint, (size_t)M));
  return SBIE_OK;
}

uint64_t plan_bytes(int M, int p, bool stokes) {
  sbie_geom g;
  g.M = M;
  g.p = p;
  g.Nphi = 2 * p + 2;
  g.T = (p + 1) * g.Nphi;
  g.K = (p + 1) * (p + 1);
  g.Kh = (p + 1) * (p + 2) / 2;
  g.N = (int64_t)M * g.T;
  Carver c;
  (void)carve_geometry(&g, c);
  if (stokes) (void)carve_stokes(&g, c);
  return (c.used + 255) & ~uint64_t(255);
}

namespace {

// Host buffers that asynchronous copies read.  HIP may read a pageable source
// when the copy executes rather than when it is queued, so every such buffer
// lives here and the destructor synchronises the stream before any of them is
// released, on every return path.  (The 128 KiB reciprocal table sits exactly
// at glibc's default mmap threshold: freed early in a fresh process, its pages
// were unmapped while the copy could still read them.)
struct SetupStaging {
  hipStream_t s;
  std::vector<double> cd, gl, ab, rcp;
  std::vector<uint8_t> near;
  std::vector<uint32_t> excl;
  unsigned status = 0;
  explicit SetupStaging(hipStream_t st) : s(st) {}
  ~SetupStaging() { (void)hipStreamSynchronize(s); }
  SetupStaging(const SetupStaging&) = delete;
  SetupStaging& operator=(const SetupStaging&) = delete;
};

}  // namespace

sbie_status setup_geometry(sbie_geom* g, hipStream_t s) {
  const int M = g->M, p = g->p, T = g->T, K = g->K, Kh = g->Kh;
  const int64_t N = g->N;
  (void)K;
  // one block for every buffer: lent by the caller (g->blk set), else owned
  if (!g->blk) {
    Carver measure;
    SBIE_TRY(carve_geometry(g, measure));
    const size_t bytes = (measure.used + 255) & ~size_t(255);
    hipError_t e = hipMalloc((void**)&g->blk, bytes);
    if (e != hipSuccess) {
      g->blk = nullptr;
      (void)hipGetLastError();
      set_error("device allocation of " + std::to_string(bytes) + " bytes failed");
      return SBIE_E_NOMEM;
    }
    g->blk_bytes = bytes;
    g->blk_owned = true;
  }
  {
    Carver c;
    c.base = g->blk;
    c.size = g->blk_bytes;
    SBIE_TRY(carve_geometry(g, c));
    g->blk_used = c.used;
  }
  g->footprint = g->blk_bytes;
  if (g->fork_near) {
    SBIE_HIP(hipStreamCreateWithFlags(&g->side, hipStreamNonBlocking));
    SBIE_HIP(hipEventCreateWithFlags(&g->ev_fork, hipEventDisableTiming));
    SBIE_HIP(hipEventCreateWithFlags(&g->ev_join, hipEventDisableTiming));
  }
  const int Kh2 = (p + 2) * (p + 3) / 2;
  SetupStaging h(s);  // host sources and destinations of the copies below
  {
    std::vector<double>& cd = h.cd;
    cd.assign(Kh, 0.0);
    for (int n = 0; n <= p; ++n)
      for (int m = 0; m <= n; ++m)
        cd[n * (n + 1) / 2 + m] = std::sqrt((2.0 * n + 1.0) * (n + m + 1.0) * (n - m + 1.0) / (2.0 * n + 3.0));
    SBIE_HIP(hipMemcpyAsync(g->d_cd, cd.data(), sizeof(double) * Kh, hipMemcpyHostToDevice, s));
  }

  std::vector<double>& gl = h.gl;
  gl.assign(2 * (p + 1), 0.0);
  gauss_legendre_host(p + 1, gl.data(), gl.data() + p + 1);
  // normalised Ferrers recurrence coefficients a_nm, b_nm for n >= m+2; in
  // the first slot of the otherwise unused rows n = m and n = m+1 the seeds
  // Pb_m^m = sqrt((2m+1)/(2m)) sqrt(1-v^2) Pb_{m-1}^{m-1} (m >= 1) and
  // Pb_{m+1}^m = sqrt(2m+3) v Pb_m^m
  std::vector<double>& ab = h.ab;
  ab.assign(2 * Kh2, 0.0);
  for (int n = 0; n <= p + 1; ++n)
    for (int m = 0; m <= n; ++m) {
      const size_t hh = (size_t)n * (n + 1) / 2 + m;
      if (n == m && m > 0) ab[2 * hh] = std::sqrt((2.0 * m + 1.0) / (2.0 * m));
      if (n == m + 1) ab[2 * hh] = std::sqrt(2.0 * m + 3.0);
      if (n < m + 2) continue;
      const double h = n * (n + 1) / 2 + m;
      ab[2 * (size_t)h] = std::sqrt((4.0 * n * n - 1.0) / ((double)n * n - (double)m * m));
      ab[2 * (size_t)h + 1] =
          std::sqrt(((n - 1.0) * (n - 1.0) - (double)m * m) / (4.0 * (n - 1.0) * (n - 1.0) - 1.0));
    }
  SBIE_HIP(hipMemcpyAsync(g->d_part, g->h_part.data(), sizeof(Particle) * M, hipMemcpyHostToDevice, s));
  SBIE_HIP(hipMemcpyAsync(g->d_gl, gl.data(), sizeof(double) * gl.size(), hipMemcpyHostToDevice, s));
  SBIE_HIP(hipMemcpyAsync(g->d_ab, ab.data(), sizeof(double) * ab.size(), hipMemcpyHostToDevice, s));
  SBIE_HIP(hipMemsetAsync(g->d_status, 0, sizeof(unsigned), s));
  SBIE_HIP(hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(g->d_status + 1), kMaxNearDepth, 1, s));

  const int B = 256;
  hipLaunchKernelGGL(k_nodes, dim3((unsigned)((N + B - 1) / B)), dim3(B), 0, s, g->d_part, g->d_gl, p, N,
                     g->d_x, g->d_y, g->d_z, g->d_nx, g->d_ny, g->d_nz, g->d_w, g->d_off32);
  SBIE_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_ws, dim3((M * (p + 1) + B - 1) / B), dim3(B), 0, s, g->d_part, g->d_gl, M, p, g->d_wS);
  SBIE_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_basis, dim3((T + 63) / 64), dim3(64), 0, s, g->d_gl, g->d_ab, p, g->d_An, g->d_Sy,
                     g->d_An32, g->d_Sy32, g->d_Sv, g->d_Sp, g->d_Sv32, g->d_Sp32);
  SBIE_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_spectra, dim3((M * (p + 1) + 63) / 64), dim3(64), 0, s, g->d_part, M, p, g->d_lam,
                     g->d_dlr, g->d_status);
  SBIE_HIP(hipGetLastError());

  // near/far split
  uint8_t* d_near = g->d_near_scratch;
  SBIE_HIP(hipMemsetAsync(d_near, 0, (size_t)M * M, s));
  const int64_t npairs = (int64_t)M * (M - 1) / 2;
  if (npairs > 0) {
    hipLaunchKernelGGL(k_classify, dim3((unsigned)((npairs + 63) / 64)), dim3(64), 0, s, g->d_part, M, g->eta,
                       d_near, g->d_status);
    SBIE_HIP(hipGetLastError());
  }
  std::vector<uint8_t>& near = h.near;
  near.assign((size_t)M * M, 0);
  unsigned& status = h.status;
  SBIE_HIP(hipMemcpyAsync(near.data(), d_near, near.size(), hipMemcpyDeviceToHost, s));
  SBIE_HIP(hipMemcpyAsync(&status, g->d_status, sizeof(unsigned), hipMemcpyDeviceToHost, s));
  SBIE_HIP(hipStreamSynchronize(s));
  if (status & kStatOverlap) {
    set_error("two particles touch or overlap");
    return SBIE_E_OVERLAP;
  }
  if (status & kStatNumeric) {
    set_error("continued fraction for Q_N/Q_{N-1} did not converge at a particle surface");
    return SBIE_E_NUMERIC;
  }

  // CSR of near sources by target particle (ascending source index) and the
  // far-field exclusion mask (self and near sources of each target particle)
  g->h_near_ptr.assign(M + 1, 0);
  g->h_near_src.clear();
  const int words = (M + 31) / 32;
  g->excl_words = words;
  std::vector<uint32_t>& excl = h.excl;
  excl.assign((size_t)M * words, 0u);
  int64_t excluded_pairs = 0;
  for (int j = 0; j < M; ++j) {
    excl[(size_t)j * words + j / 32] |= 1u << (j % 32);
    ++excluded_pairs;
    for (int i = 0; i < M; ++i) {
      if (near[(size_t)i * M + j]) {
        g->h_near_src.push_back(i);
        excl[(size_t)j * words + i / 32] |= 1u << (i % 32);
        ++excluded_pairs;
      }
    }
    g->h_near_ptr[j + 1] = (int32_t)g->h_near_src.size();
  }
  g->n_near = (int64_t)g->h_near_src.size();
  g->far_pairs = ((int64_t)M * M - excluded_pairs) * (int64_t)T * T;
  SBIE_HIP(hipMemcpyAsync(g->d_near_ptr, g->h_near_ptr.data(), sizeof(int32_t) * (M + 1), hipMemcpyHostToDevice, s));
  if (g->n_near)
    SBIE_HIP(hipMemcpyAsync(g->d_near_src, g->h_near_src.data(), sizeof(int32_t) * g->n_near,
                            hipMemcpyHostToDevice, s));
  SBIE_HIP(hipMemcpyAsync(g->d_excl, excl.data(), sizeof(uint32_t) * excl.size(), hipMemcpyHostToDevice, s));

  g->T16 = 16 * ((T + 15) / 16);
  SBIE_TRY(far_records(g, s));
  {
    std::vector<double>& rcp = h.rcp;
    rcp.assign(kRcpN, 0.0);
    for (int k = 1; k < kRcpN; ++k) rcp[k] = 1.0 / (double)k;
    SBIE_HIP(hipMemcpyAsync(g->d_rcp, rcp.data(), sizeof(double) * kRcpN, hipMemcpyHostToDevice, s));
  }

  // status after the spectra kernel
  SBIE_HIP(hipMemcpyAsync(&status, g->d_status, sizeof(unsigned), hipMemcpyDeviceToHost, s));
  SBIE_HIP(hipStreamSynchronize(s));
  if (status & kStatNumeric) {
    set_error("continued fraction for Q_N/Q_{N-1} did not converge at a particle surface");
    return SBIE_E_NUMERIC;
  }
  return SBIE_OK;
}

}  // namespace sbie
