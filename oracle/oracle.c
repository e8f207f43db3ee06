/*
 * FP64 CPU oracle for the spheroidal Laplace layer-potential apply of
 * Crowder, Li, Corona and Veerapaneni, "Boundary integral equation analysis for
 * spheroidal suspensions" (arXiv 2506.20809).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file; only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant with the HIP
 * library.
 *
 * It is deliberately plain: every step follows the paper's definitions or
 * Algorithm 1 in the paper's order, in double precision, with no blocking,
 * fusion or reordering beyond what those steps state.  Oblate Legendre
 * functions are evaluated with complex arithmetic at z = i*u exactly as the
 * paper writes them (Section 2.3, "Legendre function evaluation").
 *
 * Readings where the paper is silent or garbled (each also listed in the design
 * notes of the repository):
 *  - azimuthal grid has 2p+2 points (the paper's 2p aliases the m = +-p modes);
 *    phi_k = 2*pi*k/(2p+2), Gauss-Legendre nodes in ascending v;
 *  - real orthonormal surface basis (Definition 1 with cos/sin in place of
 *    exp(i m phi)); Ferrers functions without the Condon-Shortley phase;
 *  - the Wronskian seed uses the index N of the continued fraction,
 *    (N+m-1)!/(N-m)!, consistent with the Casoratian it comes from;
 *  - continued fraction order N = p+1, stop when |delta-1| < 1e-16;
 *  - oblate branch: (z^2-1)^(1/2) = i*sqrt(u^2+1) at z = i*u, derivatives d/dz;
 *  - on-surface D is the principal value (average of the one-sided spectra);
 *  - the near-field expansion of D uses the exterior-limit coefficients;
 *  - near/far split uses the exact minimum surface distance, diam = twice the
 *    largest semi-axis, "near" iff d < eta*diam(source) (strict);
 *  - S' and D' (Section 3.3, Theorem 3): derivative along the target's outward
 *    normal; on the surface S' is the principal value (average of the
 *    one-sided spectra) and D' has no jump; the self values are expansions in
 *    the modified basis Y/sqrt(u0^2 -+ v^2); near field from the gradient of
 *    the source's exterior expansion dotted with the target normal;
 *  - Stokes single layer (Section 4.3, Eq. (stokes)): viscosity 1, origin of
 *    the identity at each source particle's centre, self values from the
 *    exterior limit of the gradients (the jump cancels in the combination),
 *    far field from the Stokeslet with the raw nodal density.
 *
 * Every function here is pinned by the CPU tests against values fixed from
 * outside this file: mpmath Legendre values, closed forms (conductor, sphere,
 * translating-spheroid mobilities), identities (Gauss, Green, Casoratian,
 * null layer of the normal), brute-force quadrature and invariances.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_E_INVALID (-1)
#define ORC_E_DEGENERATE (-2)
#define ORC_E_OVERLAP (-3)
#define ORC_E_NUMERIC (-8)

#define OP_S 0
#define OP_D 1
#define OP_SP 3 /* normal derivative of the single layer at the target, S' */
#define OP_DP 4 /* normal derivative of the double layer at the target, D' */

static const double PI = 3.14159265358979323846264338327950288;

/* ------------------------------------------------------------------------ */
/* Small helpers                                                             */
/* ------------------------------------------------------------------------ */

static double factorial(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= (double)i;
  return f;
}

static double double_factorial(int n) { /* n!! with (-1)!! = 1 */
  double f = 1.0;
  for (int i = n; i > 1; i -= 2) f *= (double)i;
  return f;
}

/* Rotation matrix (row-major, body -> lab) of a unit quaternion (w,x,y,z). */
static void quat_to_rot(const double q_in[4], double R[9]) {
  double n = sqrt(q_in[0] * q_in[0] + q_in[1] * q_in[1] + q_in[2] * q_in[2] +
                  q_in[3] * q_in[3]);
  double w = q_in[0] / n, x = q_in[1] / n, y = q_in[2] / n, z = q_in[3] / n;
  R[0] = 1 - 2 * (y * y + z * z);
  R[1] = 2 * (x * y - w * z);
  R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);
  R[4] = 1 - 2 * (x * x + z * z);
  R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);
  R[7] = 2 * (y * z + w * x);
  R[8] = 1 - 2 * (x * x + y * y);
}

/* ------------------------------------------------------------------------ */
/* Particle parameters: Section 2.1, Table 1.  Surface u = u0 has semi-axes   */
/* A = a*sqrt(u0^2 -+ 1) (equatorial) and C = a*u0 (polar).                   */
/* ------------------------------------------------------------------------ */

typedef struct {
  int oblate;       /* 0 prolate (C > A), 1 oblate (C < A) */
  double a, u0;     /* focal parameter and coordinate of the surface */
  double A, C;      /* semi-axes */
  double c[3];      /* centre */
  double R[9];      /* body -> lab rotation */
  double diam;      /* twice the largest semi-axis */
} particle;

static int make_particle(const double* centre, const double* quat, double A,
                         double C, particle* out) {
  if (!(A > 0) || !(C > 0) || !isfinite(A) || !isfinite(C))
    return ORC_E_DEGENERATE;
  double mx = A > C ? A : C;
  if (fabs(A - C) <= 1e-6 * mx) return ORC_E_DEGENERATE;
  out->A = A;
  out->C = C;
  out->oblate = C < A;
  if (!out->oblate)
    out->a = sqrt((C - A) * (C + A));
  else
    out->a = sqrt((A - C) * (A + C));
  out->u0 = C / out->a;
  for (int k = 0; k < 3; ++k) out->c[k] = centre[k];
  quat_to_rot(quat, out->R);
  out->diam = 2.0 * mx;
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Gauss-Legendre rule on [-1,1]: Newton on the Legendre polynomial.          */
/* ------------------------------------------------------------------------ */

void orc_gauss_legendre(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    /* i-th root counted from the right end, then stored ascending */
    double t = cos(PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = t;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2 * k - 1) * t * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = t; p0 = 1.0; }
      dp = n * (t * p1 - p0) / (t * t - 1.0);
      double dt = p1 / dp;
      t -= dt;
      if (fabs(dt) < 1e-16) break;
    }
    {
      double p0 = 1.0, p1 = t;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2 * k - 1) * t * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = t; p0 = 1.0; }
      dp = n * (t * p1 - p0) / (t * t - 1.0);
    }
    x[n - 1 - i] = t;
    w[n - 1 - i] = 2.0 / ((1.0 - t * t) * dp * dp);
  }
}

/* ------------------------------------------------------------------------ */
/* Associated Legendre functions off the cut, Section 2.3 steps 1-4 and the   */
/* derivative identity.  z = u (prolate, u > 1) or z = i*u (oblate, u > 0).   */
/* Arrays are indexed by degree n = 0..N+1; entries with n < m are zero.       */
/* P, Q are filled for n = m..N; dP, dQ for n = m..N-1 (needs F_{n+1}).        */
/* ------------------------------------------------------------------------ */

static int cf_max_iter = 10000; /* continued-fraction cap (settable for tests) */

void orc_set_cf_max_iter(int it) { cf_max_iter = it; }

static int legendre_offcut(int oblate, double u, int m, int N,
                           double complex* P, double complex* Q,
                           double complex* dP, double complex* dQ) {
  double complex z = oblate ? I * u : u + 0.0 * I;
  /* branch of (z^2-1)^(1/2): sqrt(u^2-1) for real z > 1, i*sqrt(u^2+1) at z = iu */
  double complex s = oblate ? I * sqrt(u * u + 1.0) : sqrt(u * u - 1.0) + 0.0 * I;
  for (int n = 0; n <= N + 1; ++n) P[n] = Q[n] = dP[n] = dQ[n] = 0;

  /* step 1: forward recurrence for P_n^m, seeds P_m^m and P_{m+1}^m */
  double complex spow = 1.0;
  for (int k = 0; k < m; ++k) spow *= s;
  P[m] = double_factorial(2 * m - 1) * spow;
  if (m + 1 <= N + 1) P[m + 1] = z * (2 * m + 1) * P[m];
  for (int n = m + 1; n <= N; ++n)
    P[n + 1] = ((2 * n + 1) * z * P[n] - (n + m) * P[n - 1]) / (double)(n - m + 1);

  /* step 2: H_N = Q_N/Q_{N-1} by the modified Lentz method on the continued
     fraction H_n = a_n / (b_n + H_{n+1}),
     a_n = -(n+m)/(n-m+1), b_n = -(2n+1) z/(n-m+1). */
  const double tiny = 1e-300;
  double complex f = tiny, Cl = f, Dl = 0.0;
  int converged = 0;
  for (int k = N, it = 0; it < cf_max_iter; ++k, ++it) {
    double complex ak = -(double)(k + m) / (double)(k - m + 1);
    double complex bk = -(2.0 * k + 1.0) * z / (double)(k - m + 1);
    Dl = bk + ak * Dl;
    if (cabs(Dl) == 0.0) Dl = tiny;
    Dl = 1.0 / Dl;
    Cl = bk + ak / Cl;
    if (cabs(Cl) == 0.0) Cl = tiny;
    double complex delta = Cl * Dl;
    f *= delta;
    if (cabs(delta - 1.0) < 1e-16) { converged = 1; break; }
  }
  if (!converged) return ORC_E_NUMERIC;
  double complex H = f;

  /* step 3: Casoratian seed, Q_{N-1} and Q_N */
  double cas = factorial(N + m - 1) / factorial(N - m) * ((m & 1) ? -1.0 : 1.0);
  Q[N - 1] = cas / (P[N] - H * P[N - 1]);
  Q[N] = H * Q[N - 1];

  /* step 4: backward recurrence down to Q_m^m */
  for (int n = N - 1; n >= m + 1; --n)
    Q[n - 1] = ((2 * n + 1) * z * Q[n] - (n - m + 1) * Q[n + 1]) / (double)(n + m);

  /* derivative identity (1 - z^2) F_n' = (m-n-1) F_{n+1} + (n+1) z F_n */
  for (int n = m; n <= N - 1; ++n) {
    dP[n] = ((m - n - 1) * P[n + 1] + (n + 1) * z * P[n]) / (1.0 - z * z);
    dQ[n] = ((m - n - 1) * Q[n + 1] + (n + 1) * z * Q[n]) / (1.0 - z * z);
  }
  return ORC_OK;
}

/* Exported for the pins: values for one order m, degrees 0..N (P, Q) and
   0..N-1 (derivatives); real and imaginary parts separately. */
int orc_legendre(int oblate, double u, int m, int N, double* Pre, double* Pim,
                 double* Qre, double* Qim, double* dPre, double* dPim,
                 double* dQre, double* dQim) {
  if (m < 0 || N < m + 1) return ORC_E_INVALID;
  double complex* buf = (double complex*)malloc(sizeof(double complex) * 4 * (N + 2));
  double complex *P = buf, *Q = buf + (N + 2), *dP = buf + 2 * (N + 2),
                 *dQ = buf + 3 * (N + 2);
  int rc = legendre_offcut(oblate, u, m, N, P, Q, dP, dQ);
  for (int n = 0; n <= N; ++n) {
    Pre[n] = creal(P[n]); Pim[n] = cimag(P[n]);
    Qre[n] = creal(Q[n]); Qim[n] = cimag(Q[n]);
    dPre[n] = creal(dP[n]); dPim[n] = cimag(dP[n]);
    dQre[n] = creal(dQ[n]); dQim[n] = cimag(dQ[n]);
  }
  free(buf);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Spectra, Theorems 1 and 2, for n <= p and m >= 0 (index n(n+1)/2 + m).     */
/*  lamDp = D+ (exterior limit), lamDm = D- (interior limit),                 */
/*  lamD = principal value = (D+ + D-)/2, lamS = surface S in the modified    */
/*  basis.  Qu0 holds Q_n^m(z0) (complex, for the near-field ratio).          */
/* ------------------------------------------------------------------------ */

static int spectra(const particle* pt, int p, double* lamD, double* lamDp,
                   double* lamDm, double* lamS, double complex* Qu0) {
  int N = p + 1;
  double complex* buf = (double complex*)malloc(sizeof(double complex) * 4 * (N + 2));
  double complex *P = buf, *Q = buf + (N + 2), *dP = buf + 2 * (N + 2),
                 *dQ = buf + 3 * (N + 2);
  double u0 = pt->u0, a = pt->a;
  for (int m = 0; m <= p; ++m) {
    int rc = legendre_offcut(pt->oblate, u0, m, N, P, Q, dP, dQ);
    if (rc) { free(buf); return rc; }
    for (int n = m; n <= p; ++n) {
      double ratio = factorial(n - m) / factorial(n + m);
      double sgn = (m & 1) ? -1.0 : 1.0;
      double complex b, bt;
      if (!pt->oblate) {
        b = ratio * sgn * (u0 * u0 - 1.0);               /* b_n^m */
        bt = a * ratio * sgn * sqrt(u0 * u0 - 1.0);      /* b~_n^m */
      } else {
        b = ratio * (-sgn) * (u0 * u0 + 1.0);            /* c_n^m */
        bt = I * a * ratio * sgn * sqrt(u0 * u0 + 1.0);  /* c~_n^m */
      }
      double complex lp = b * dP[n] * Q[n];
      double complex lm = b * dQ[n] * P[n];
      double complex ls = bt * P[n] * Q[n];
      int idx = n * (n + 1) / 2 + m;
      if (lamDp) lamDp[idx] = creal(lp);
      if (lamDm) lamDm[idx] = creal(lm);
      if (lamD) lamD[idx] = 0.5 * (creal(lp) + creal(lm));
      if (lamS) lamS[idx] = creal(ls);
      if (Qu0) Qu0[idx] = Q[n];
    }
  }
  free(buf);
  return ORC_OK;
}

int orc_spectra(int oblate, double a, double u0, int p, double* lamD,
                double* lamDp, double* lamDm, double* lamS) {
  particle pt;
  memset(&pt, 0, sizeof pt);
  pt.oblate = oblate;
  pt.a = a;
  pt.u0 = u0;
  return spectra(&pt, p, lamD, lamDp, lamDm, lamS, NULL);
}

/* Spectra of the normal derivatives on the surface (Theorem 3, and the same
   construction for D).  With h = sqrt(u0^2 -+ 1)/a and dz/du = 1 (prolate) or
   i (oblate), in the modified basis Y_l / sqrt(u0^2 -+ v^2):
     S'+ = h dz/du b~ P(z0) Q'(z0),  S'- = h dz/du b~ Q(z0) P'(z0),
     lamSp = principal value (S'+ + S'-)/2, applied to the modified-basis
     coefficients of sigma (as for S);
     lamDd = h dz/du b P'(z0) Q'(z0), applied to the standard coefficients of
     mu; the normal derivative of the exterior expansion b P'(z0) Q(z) Y and
     of the interior one b Q'(z0) P(z) Y agree, so D' has no jump. */
static int derivative_spectra(const particle* pt, int p, double* lamSp, double* lamDd) {
  int N = p + 1;
  double complex* buf = (double complex*)malloc(sizeof(double complex) * 4 * (N + 2));
  double complex *P = buf, *Q = buf + (N + 2), *dP = buf + 2 * (N + 2),
                 *dQ = buf + 3 * (N + 2);
  double u0 = pt->u0, a = pt->a;
  double su = pt->oblate ? sqrt(u0 * u0 + 1.0) : sqrt(u0 * u0 - 1.0);
  double complex dzdu = pt->oblate ? I : 1.0 + 0.0 * I;
  for (int m = 0; m <= p; ++m) {
    int rc = legendre_offcut(pt->oblate, u0, m, N, P, Q, dP, dQ);
    if (rc) { free(buf); return rc; }
    for (int n = m; n <= p; ++n) {
      double ratio = factorial(n - m) / factorial(n + m);
      double sgn = (m & 1) ? -1.0 : 1.0;
      double complex b, bt;
      if (!pt->oblate) {
        b = ratio * sgn * (u0 * u0 - 1.0);
        bt = a * ratio * sgn * sqrt(u0 * u0 - 1.0);
      } else {
        b = ratio * (-sgn) * (u0 * u0 + 1.0);
        bt = I * a * ratio * sgn * sqrt(u0 * u0 + 1.0);
      }
      double complex h = su / a * dzdu;
      double complex spp = h * bt * P[n] * dQ[n];
      double complex spm = h * bt * Q[n] * dP[n];
      int idx = n * (n + 1) / 2 + m;
      if (lamSp) lamSp[idx] = 0.5 * (creal(spp) + creal(spm));
      if (lamDd) lamDd[idx] = creal(h * b * dP[n] * dQ[n]);
    }
  }
  free(buf);
  return ORC_OK;
}

int orc_derivative_spectra(int oblate, double a, double u0, int p, double* lamSp, double* lamDd) {
  particle pt;
  memset(&pt, 0, sizeof pt);
  pt.oblate = oblate;
  pt.a = a;
  pt.u0 = u0;
  return derivative_spectra(&pt, p, lamSp, lamDd);
}

/* ------------------------------------------------------------------------ */
/* Real orthonormal surface harmonics (Definition 1, real form).              */
/* Y_{n,0} = N_n^0 P_n(v); Y_{n,m} = sqrt2 N_n^m P_n^m(v) cos(m phi);          */
/* Y_{n,-m} = sqrt2 N_n^m P_n^m(v) sin(m phi).  Index l = n^2 + n + m.         */
/* Ferrers P_n^m(v) = (1-v^2)^(m/2) d^m P_n/dv^m, no Condon-Shortley phase,   */
/* computed by the same three-term recurrence in n with seed (2m-1)!!(1-v^2)^(m/2). */
/* ------------------------------------------------------------------------ */

static void ferrers_all(double v, int p, double* Pf /* [(p+1)(p+2)/2] */) {
  double sv = sqrt(fmax(0.0, 1.0 - v * v));
  for (int m = 0; m <= p; ++m) {
    double pmm = double_factorial(2 * m - 1) * pow(sv, m);
    Pf[m * (m + 1) / 2 + m] = pmm;
    if (m + 1 <= p) Pf[(m + 1) * (m + 2) / 2 + m] = v * (2 * m + 1) * pmm;
    for (int n = m + 1; n < p; ++n) {
      double pn = Pf[n * (n + 1) / 2 + m];
      double pn1 = (n - 1 >= m) ? Pf[(n - 1) * n / 2 + m] : 0.0;
      Pf[(n + 1) * (n + 2) / 2 + m] =
          ((2 * n + 1) * v * pn - (n + m) * pn1) / (double)(n - m + 1);
    }
  }
}

static void real_harmonics(double v, double phi, int p, double* Y /* [(p+1)^2] */) {
  int nh = (p + 1) * (p + 2) / 2;
  double* Pf = (double*)malloc(sizeof(double) * nh);
  ferrers_all(v, p, Pf);
  for (int n = 0; n <= p; ++n) {
    for (int m = 0; m <= n; ++m) {
      double Nnm = sqrt((2.0 * n + 1.0) / (4.0 * PI) * factorial(n - m) / factorial(n + m));
      double base = Nnm * Pf[n * (n + 1) / 2 + m];
      if (m == 0) {
        Y[n * n + n] = base;
      } else {
        Y[n * n + n + m] = sqrt(2.0) * base * cos(m * phi);
        Y[n * n + n - m] = sqrt(2.0) * base * sin(m * phi);
      }
    }
  }
  free(Pf);
}

void orc_real_harmonics(double v, double phi, int p, double* Y) {
  real_harmonics(v, phi, p, Y);
}

/* ------------------------------------------------------------------------ */
/* Grid, Section 4 "Integral density representation" and Tables 1-2:        */
/* node g = i*T + j*Nphi + k, T = (p+1)*Nphi, Nphi = 2p+2.                    */
/* Weight W = g_j * (2 pi / Nphi) * a^2 sqrt(u0^2 -+ v^2) sqrt(u0^2 -+ 1).     */
/* ------------------------------------------------------------------------ */

static void particle_grid(const particle* pt, int p, const double* gx,
                          const double* gw, double* xyz, double* nrm,
                          double* W) {
  int Nphi = 2 * p + 2;
  double a = pt->a, u0 = pt->u0;
  double sgn = pt->oblate ? 1.0 : -1.0;
  double s = sqrt(u0 * u0 + sgn);          /* sqrt(u0^2 -+ 1) */
  for (int j = 0; j <= p; ++j) {
    double v = gx[j];
    double sv = sqrt(1.0 - v * v);
    for (int k = 0; k < Nphi; ++k) {
      double phi = 2.0 * PI * k / Nphi;
      double xb[3] = {a * s * sv * cos(phi), a * s * sv * sin(phi), a * u0 * v};
      double gb[3] = {xb[0] / (pt->A * pt->A), xb[1] / (pt->A * pt->A),
                      xb[2] / (pt->C * pt->C)};
      double gn = sqrt(gb[0] * gb[0] + gb[1] * gb[1] + gb[2] * gb[2]);
      int g = j * Nphi + k;
      for (int r = 0; r < 3; ++r) {
        double xr = pt->c[r], nr = 0.0;
        for (int c2 = 0; c2 < 3; ++c2) {
          xr += pt->R[3 * r + c2] * xb[c2];
          nr += pt->R[3 * r + c2] * gb[c2] / gn;
        }
        if (xyz) xyz[3 * g + r] = xr;
        if (nrm) nrm[3 * g + r] = nr;
      }
      double J = a * a * sqrt(u0 * u0 + sgn * v * v) * s;
      if (W) W[g] = gw[j] * (2.0 * PI / Nphi) * J;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Discrete transform (Section 2.3; density representation in Section 4):     */
/* c_l = sum_{j,k} g_j (2 pi / Nphi) f_jk Y_l(v_j, phi_k).                    */
/* ------------------------------------------------------------------------ */

static void forward_transform(int p, const double* gx, const double* gw,
                              const double* f, double* coef) {
  int Nphi = 2 * p + 2, K = (p + 1) * (p + 1);
  double* Y = (double*)malloc(sizeof(double) * K);
  for (int l = 0; l < K; ++l) coef[l] = 0.0;
  for (int j = 0; j <= p; ++j)
    for (int k = 0; k < Nphi; ++k) {
      real_harmonics(gx[j], 2.0 * PI * k / Nphi, p, Y);
      double wf = gw[j] * (2.0 * PI / Nphi) * f[j * Nphi + k];
      for (int l = 0; l < K; ++l) coef[l] += wf * Y[l];
    }
  free(Y);
}

static void inverse_transform(int p, const double* gx, const double* coef,
                              double* f) {
  int Nphi = 2 * p + 2, K = (p + 1) * (p + 1);
  double* Y = (double*)malloc(sizeof(double) * K);
  for (int j = 0; j <= p; ++j)
    for (int k = 0; k < Nphi; ++k) {
      real_harmonics(gx[j], 2.0 * PI * k / Nphi, p, Y);
      double acc = 0.0;
      for (int l = 0; l < K; ++l) acc += coef[l] * Y[l];
      f[j * Nphi + k] = acc;
    }
  free(Y);
}

int orc_transform(int p, const double* f, double* coef) {
  double* gx = (double*)malloc(sizeof(double) * 2 * (p + 1));
  orc_gauss_legendre(p + 1, gx, gx + p + 1);
  forward_transform(p, gx, gx + p + 1, f, coef);
  free(gx);
  return ORC_OK;
}

int orc_inverse_transform(int p, const double* coef, double* f) {
  double* gx = (double*)malloc(sizeof(double) * 2 * (p + 1));
  orc_gauss_legendre(p + 1, gx, gx + p + 1);
  inverse_transform(p, gx, coef, f);
  free(gx);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Spheroidal coordinates of a body-frame point (inverse of Table 1).         */
/* Prolate: s = u^2-1 solves a^2 s^2 + (a^2 - r^2) s - rho^2 = 0.              */
/* Oblate:  t = u^2   solves a^2 t^2 + (a^2 - r^2) t - x3^2  = 0.              */
/* ------------------------------------------------------------------------ */

static void body_to_spheroidal(const particle* pt, const double xb[3], double* u,
                               double* v, double* phi) {
  double a = pt->a, a2 = a * a;
  double rho2 = xb[0] * xb[0] + xb[1] * xb[1];
  double r2 = rho2 + xb[2] * xb[2];
  double cst = pt->oblate ? xb[2] * xb[2] : rho2;     /* minus the constant term */
  double disc = sqrt((a2 - r2) * (a2 - r2) + 4.0 * a2 * cst);
  double root;
  if (r2 >= a2)
    root = ((r2 - a2) + disc) / (2.0 * a2);
  else
    root = 2.0 * cst / ((a2 - r2) + disc);
  double uu = pt->oblate ? sqrt(root) : sqrt(1.0 + root);
  *u = uu;
  *v = xb[2] / (a * uu);
  *phi = atan2(xb[1], xb[0]);
}

static void lab_to_body(const particle* pt, const double x[3], double xb[3]) {
  double d[3] = {x[0] - pt->c[0], x[1] - pt->c[1], x[2] - pt->c[2]};
  for (int c = 0; c < 3; ++c)
    xb[c] = pt->R[0 + c] * d[0] + pt->R[3 + c] * d[1] + pt->R[6 + c] * d[2];
}

/* Exterior solid-harmonic expansion of one particle at one exterior point:  */
/* sum_l E_l * Q_n^|m|(z) / Q_n^|m|(z0) * Y_l(v, phi)  (Theorems 1-2,         */
/* exterior rows, with E_l the on-surface exterior-limit coefficient).        */
static int eval_exterior(const particle* pt, int p, const double* E,
                         const double complex* Qu0, const double x[3],
                         double* out) {
  double xb[3], u, v, phi;
  lab_to_body(pt, x, xb);
  body_to_spheroidal(pt, xb, &u, &v, &phi);
  if (!(u > pt->u0)) return ORC_E_OVERLAP;
  int K = (p + 1) * (p + 1), N = p + 1;
  double* Y = (double*)malloc(sizeof(double) * K);
  double complex* buf = (double complex*)malloc(sizeof(double complex) * 4 * (N + 2));
  double complex *P = buf, *Q = buf + (N + 2), *dP = buf + 2 * (N + 2),
                 *dQ = buf + 3 * (N + 2);
  real_harmonics(v, phi, p, Y);
  double acc = 0.0;
  for (int m = 0; m <= p; ++m) {
    int rc = legendre_offcut(pt->oblate, u, m, N, P, Q, dP, dQ);
    if (rc) { free(Y); free(buf); return rc; }
    for (int n = m; n <= p; ++n) {
      double ratio = creal(Q[n] / Qu0[n * (n + 1) / 2 + m]);
      if (m == 0)
        acc += E[n * n + n] * ratio * Y[n * n + n];
      else
        acc += (E[n * n + n + m] * Y[n * n + n + m] + E[n * n + n - m] * Y[n * n + n - m]) * ratio;
    }
  }
  free(Y);
  free(buf);
  *out = acc;
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Exact minimum distance between two disjoint spheroids.  Alternating       */
/* projections give upper bounds |x - y|; the separation of the two support  */
/* planes orthogonal to (x - y) gives lower bounds.  Iterate until the gap   */
/* between the bounds is below tol.  Returns a negative number on overlap.   */
/* ------------------------------------------------------------------------ */

/* closest point of the body-frame spheroid (A,A,C) to body-frame point q outside */
static void project_body(double A, double C, const double q[3], double out[3]) {
  double rho = sqrt(q[0] * q[0] + q[1] * q[1]), z = fabs(q[2]);
  double A2 = A * A, C2 = C * C;
  /* f(t) = rho^2 A^2/(A^2+t)^2 + z^2 C^2/(C^2+t)^2 - 1, decreasing for t >= 0 */
  double lo = 0.0, hi = fmax(A, C) * sqrt(rho * rho + z * z) + 1e-300;
  double t = 0.0;
  double f0 = rho * rho / A2 + z * z / C2 - 1.0;
  if (f0 <= 0.0) { t = 0.0; }
  else {
    for (int it = 0; it < 200; ++it) {
      double ea = A2 + t, ec = C2 + t;
      double f = rho * rho * A2 / (ea * ea) + z * z * C2 / (ec * ec) - 1.0;
      double df = -2.0 * rho * rho * A2 / (ea * ea * ea) - 2.0 * z * z * C2 / (ec * ec * ec);
      if (f == 0.0) break;
      if (f > 0) lo = t; else hi = t;
      double tn = t - f / df;
      if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
      if (fabs(tn - t) <= 1e-16 * fmax(1.0, tn)) { t = tn; break; }
      t = tn;
    }
  }
  double fr = A2 / (A2 + t), fz = C2 / (C2 + t);
  out[0] = q[0] * fr;
  out[1] = q[1] * fr;
  out[2] = q[2] * fz;
}

static void project_lab(const particle* pt, const double x[3], double out[3]) {
  double xb[3], yb[3];
  lab_to_body(pt, x, xb);
  project_body(pt->A, pt->C, xb, yb);
  for (int r = 0; r < 3; ++r)
    out[r] = pt->c[r] + pt->R[3 * r] * yb[0] + pt->R[3 * r + 1] * yb[1] + pt->R[3 * r + 2] * yb[2];
}

/* support function h(n) = max_{x in spheroid} n.x */
static double support(const particle* pt, const double n[3]) {
  double nb[3];
  for (int c = 0; c < 3; ++c)
    nb[c] = pt->R[0 + c] * n[0] + pt->R[3 + c] * n[1] + pt->R[6 + c] * n[2];
  double q = pt->A * pt->A * (nb[0] * nb[0] + nb[1] * nb[1]) + pt->C * pt->C * nb[2] * nb[2];
  return pt->c[0] * n[0] + pt->c[1] * n[1] + pt->c[2] * n[2] + sqrt(q);
}

static int inside(const particle* pt, const double x[3]) {
  double xb[3];
  lab_to_body(pt, x, xb);
  return (xb[0] * xb[0] + xb[1] * xb[1]) / (pt->A * pt->A) + xb[2] * xb[2] / (pt->C * pt->C) <= 1.0;
}

static double spheroid_distance(const particle* P1, const particle* P2, double tol) {
  double x[3], y[3];
  if (inside(P1, P2->c) || inside(P2, P1->c)) return -1.0;
  project_lab(P1, P2->c, x);
  if (inside(P2, x)) return -1.0;
  double upper = INFINITY, lower = -INFINITY;
  for (int it = 0; it < 200000; ++it) {
    project_lab(P2, x, y);
    if (inside(P1, y)) return -1.0;
    project_lab(P1, y, x);
    double d[3] = {y[0] - x[0], y[1] - x[1], y[2] - x[2]};
    double dn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (dn < upper) upper = dn;
    if (dn > 0) {
      double n[3] = {d[0] / dn, d[1] / dn, d[2] / dn};
      double mn[3] = {-n[0], -n[1], -n[2]};
      /* P1 lies in n.z <= h1(n); P2 in n.z >= -h2(-n) */
      double lb = -support(P2, mn) - support(P1, n);
      if (lb > lower) lower = lb;
    }
    if (upper - lower <= tol) break;
  }
  if (lower <= 0.0 && upper <= tol) return -1.0;
  return 0.5 * (upper + lower);
}

int orc_distance(const double* c1, const double* q1, double A1, double C1,
                 const double* c2, const double* q2, double A2, double C2,
                 double* dist) {
  particle P1, P2;
  int rc = make_particle(c1, q1, A1, C1, &P1);
  if (rc) return rc;
  rc = make_particle(c2, q2, A2, C2, &P2);
  if (rc) return rc;
  *dist = spheroid_distance(&P1, &P2, 1e-12);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Setup shared by the apply entry points                                    */
/* ------------------------------------------------------------------------ */

typedef struct {
  int M, p, T, K, Kh, N;
  particle* pt;
  double *gx, *gw;
  double *xyz, *nrm, *W;
  uint8_t* near;  /* near[i*M + j] = 1 iff j in J_i^near (j != i) */
} geometry;

static void free_geometry(geometry* g) {
  free(g->pt); free(g->gx); free(g->xyz); free(g->nrm); free(g->W); free(g->near);
}

static int build_geometry(const double* centres, const double* quats,
                          const double* A, const double* C, int M, int p,
                          double eta, geometry* g) {
  memset(g, 0, sizeof *g);
  if (M < 1 || p < 1 || p > 32 || !(eta >= 0)) return ORC_E_INVALID;
  g->M = M; g->p = p; g->T = (p + 1) * (2 * p + 2); g->K = (p + 1) * (p + 1);
  g->Kh = (p + 1) * (p + 2) / 2; g->N = M * g->T;
  g->pt = (particle*)calloc(M, sizeof(particle));
  for (int i = 0; i < M; ++i) {
    int rc = make_particle(centres + 3 * i, quats + 4 * i, A[i], C[i], &g->pt[i]);
    if (rc) { free_geometry(g); return rc; }
  }
  g->gx = (double*)malloc(sizeof(double) * 2 * (p + 1));
  g->gw = g->gx + p + 1;
  orc_gauss_legendre(p + 1, g->gx, g->gw);
  g->xyz = (double*)malloc(sizeof(double) * 3 * g->N);
  g->nrm = (double*)malloc(sizeof(double) * 3 * g->N);
  g->W = (double*)malloc(sizeof(double) * g->N);
  for (int i = 0; i < M; ++i)
    particle_grid(&g->pt[i], p, g->gx, g->gw, g->xyz + 3 * (size_t)i * g->T,
                  g->nrm + 3 * (size_t)i * g->T, g->W + (size_t)i * g->T);
  /* Algorithm 1, near/far split: normalised distances */
  g->near = (uint8_t*)calloc((size_t)M * M, 1);
  int bad = 0;
#pragma omp parallel for schedule(dynamic)
  for (int i = 0; i < M; ++i) {
    for (int j = 0; j < M; ++j) {
      if (j == i) continue;
      const particle *Pi = &g->pt[i], *Pj = &g->pt[j];
      double dc = sqrt((Pi->c[0] - Pj->c[0]) * (Pi->c[0] - Pj->c[0]) +
                       (Pi->c[1] - Pj->c[1]) * (Pi->c[1] - Pj->c[1]) +
                       (Pi->c[2] - Pj->c[2]) * (Pi->c[2] - Pj->c[2]));
      double lb = dc - 0.5 * Pi->diam - 0.5 * Pj->diam;  /* circumsphere bound */
      if (lb >= eta * Pi->diam) continue;
      double d = spheroid_distance(Pi, Pj, 1e-12);
      if (d <= 0.0) {
#pragma omp atomic write
        bad = 1;
      }
      if (d < eta * Pi->diam) g->near[(size_t)i * M + j] = 1;
    }
  }
  if (bad) { free_geometry(g); return ORC_E_OVERLAP; }
  return ORC_OK;
}

int orc_grid(const double* centres, const double* quats, const double* A,
             const double* C, int M, int p, double* xyz, double* nrm, double* W) {
  if (M < 1 || p < 1 || p > 32) return ORC_E_INVALID;
  double* gx = (double*)malloc(sizeof(double) * 2 * (p + 1));
  orc_gauss_legendre(p + 1, gx, gx + p + 1);
  int T = (p + 1) * (2 * p + 2);
  for (int i = 0; i < M; ++i) {
    particle pt;
    int rc = make_particle(centres + 3 * i, quats + 4 * i, A[i], C[i], &pt);
    if (rc) { free(gx); return rc; }
    particle_grid(&pt, p, gx, gx + p + 1, xyz + 3 * (size_t)i * T,
                  nrm + 3 * (size_t)i * T, W + (size_t)i * T);
  }
  free(gx);
  return ORC_OK;
}

int orc_classify(const double* centres, const double* quats, const double* A,
                 const double* C, int M, double eta, uint8_t* near) {
  geometry g;
  int rc = build_geometry(centres, quats, A, C, M, 1, eta, &g);
  if (rc) return rc;
  memcpy(near, g.near, (size_t)M * M);
  free_geometry(&g);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1 (and its single-layer variant): u = u_self + u_near + u_far   */
/* at every node.  op = 0 (S) or 1 (D).  density[N] at the nodes.            */
/* Outputs may be NULL except u.                                              */
/* ------------------------------------------------------------------------ */

/* per-particle coefficients and exterior coefficients (Algorithm 1: forward transform, self and near-field steps) */
static int particle_coefficients(const geometry* g, int op, int i,
                                 const double* dens, double* coef_self,
                                 double* E, double complex* Qu0) {
  const particle* pt = &g->pt[i];
  int p = g->p, Nphi = 2 * p + 2, K = g->K, Kh = g->Kh;
  double* f = (double*)malloc(sizeof(double) * g->T);
  double* c = (double*)malloc(sizeof(double) * K);
  double* lamD = (double*)malloc(sizeof(double) * 5 * Kh);
  double *lamDp = lamD + Kh, *lamS = lamD + 2 * Kh, *lamSp = lamD + 3 * Kh, *lamDd = lamD + 4 * Kh;
  int rc = spectra(pt, p, lamD, lamDp, NULL, lamS, Qu0);
  if (!rc && (op == OP_SP || op == OP_DP)) rc = derivative_spectra(pt, p, lamSp, lamDd);
  if (rc) { free(f); free(c); free(lamD); return rc; }
  /* S and S' take the modified-basis coefficients of sigma (Section 3.2) */
  int modified = (op == OP_S || op == OP_SP);
  double sgn = pt->oblate ? 1.0 : -1.0;
  for (int j = 0; j <= p; ++j)
    for (int k = 0; k < Nphi; ++k) {
      double w = modified ? sqrt(pt->u0 * pt->u0 + sgn * g->gx[j] * g->gx[j]) : 1.0;
      f[j * Nphi + k] = w * dens[(size_t)i * g->T + j * Nphi + k];
    }
  forward_transform(p, g->gx, g->gw, f, c);
  for (int n = 0; n <= p; ++n)
    for (int m = -n; m <= n; ++m) {
      int l = n * n + n + m, h = n * (n + 1) / 2 + abs(m);
      double lself = op == OP_S ? lamS[h] : op == OP_D ? lamD[h] : op == OP_SP ? lamSp[h] : lamDd[h];
      double lext = modified ? lamS[h] : lamDp[h];
      coef_self[l] = lself * c[l];
      E[l] = lext * c[l];
    }
  free(f); free(c); free(lamD);
  return ORC_OK;
}

static int expansion_grad(const particle* pt, int p, int nset, const double* E, double u,
                          double v, double phi, int interior, double* val, double* grad);

static int valid_op(int op) { return op == OP_S || op == OP_D || op == OP_SP || op == OP_DP; }

/* S' and D' self values are expansions in the modified basis: the inverse
   transform's value at GL node j is divided by sqrt(u0^2 -+ v_j^2). */
static double self_node_factor(const geometry* g, int op, int i, int j) {
  if (op != OP_SP && op != OP_DP) return 1.0;
  const particle* pt = &g->pt[i];
  double sgn = pt->oblate ? 1.0 : -1.0;
  return 1.0 / sqrt(pt->u0 * pt->u0 + sgn * g->gx[j] * g->gx[j]);
}

/* Near-field value of source particle i at target node gt: the exterior
   expansion (S, D), or its gradient along the target's normal (S', D'). */
static int near_term(const geometry* g, int op, int i, const double* E, const double complex* Qu0,
                     size_t gt, double* out) {
  if (op == OP_S || op == OP_D) return eval_exterior(&g->pt[i], g->p, E, Qu0, g->xyz + 3 * gt, out);
  const particle* pt = &g->pt[i];
  double xb[3], u, v, phi, val, grad[3];
  lab_to_body(pt, g->xyz + 3 * gt, xb);
  body_to_spheroidal(pt, xb, &u, &v, &phi);
  if (!(u > pt->u0)) return ORC_E_OVERLAP;
  int rc = expansion_grad(pt, g->p, 1, E, u, v, phi, 0, &val, grad);
  if (rc) return rc;
  const double* nu = g->nrm + 3 * gt;
  *out = grad[0] * nu[0] + grad[1] * nu[1] + grad[2] * nu[2];
  return ORC_OK;
}

/* Smooth-quadrature term of source node gs at target node gt, d = x - y:
   S  W s / (4 pi r);  D  W m nu_y.d / (4 pi r^3);
   S' -W s nu_x.d / (4 pi r^3);
   D' W m (nu_x.nu_y / r^3 - 3 (nu_y.d)(nu_x.d) / r^5) / (4 pi). */
static double far_term(const geometry* g, int op, const double* density, size_t gt, size_t gs) {
  const double *x = g->xyz + 3 * gt, *y = g->xyz + 3 * gs;
  double d0 = x[0] - y[0], d1 = x[1] - y[1], d2 = x[2] - y[2];
  double r2 = d0 * d0 + d1 * d1 + d2 * d2;
  double r = sqrt(r2);
  double q = g->W[gs] * density[gs];
  const double *nx = g->nrm + 3 * gt, *ny = g->nrm + 3 * gs;
  switch (op) {
    case OP_S:
      return q / (4.0 * PI * r);
    case OP_D:
      return q * (ny[0] * d0 + ny[1] * d1 + ny[2] * d2) / (4.0 * PI * r2 * r);
    case OP_SP:
      return -q * (nx[0] * d0 + nx[1] * d1 + nx[2] * d2) / (4.0 * PI * r2 * r);
    default: {
      double nn = nx[0] * ny[0] + nx[1] * ny[1] + nx[2] * ny[2];
      double nyd = ny[0] * d0 + ny[1] * d1 + ny[2] * d2;
      double nxd = nx[0] * d0 + nx[1] * d1 + nx[2] * d2;
      return q * (nn / (r2 * r) - 3.0 * nyd * nxd / (r2 * r2 * r)) / (4.0 * PI);
    }
  }
}

int orc_apply(const double* centres, const double* quats, const double* A,
              const double* C, int M, int p, double eta, int op,
              const double* density, double* u_self, double* u_near,
              double* u_far, double* u) {
  if (!valid_op(op)) return ORC_E_INVALID;
  geometry g;
  int rc = build_geometry(centres, quats, A, C, M, p, eta, &g);
  if (rc) return rc;
  int T = g.T, K = g.K, Kh = g.Kh;
  size_t N = (size_t)g.N;
  double* us = (double*)calloc(N, sizeof(double));
  double* un = (double*)calloc(N, sizeof(double));
  double* uf = (double*)calloc(N, sizeof(double));
  double* cself = (double*)malloc(sizeof(double) * (size_t)M * K);
  double* E = (double*)malloc(sizeof(double) * (size_t)M * K);
  double complex* Qu0 = (double complex*)malloc(sizeof(double complex) * (size_t)M * Kh);

  /* Algorithm 1, forward transform and self step: transform, diagonal spectra, inverse transform */
  int err = 0;
#pragma omp parallel for schedule(dynamic)
  for (int i = 0; i < M; ++i) {
    int r = particle_coefficients(&g, op, i, density, cself + (size_t)i * K,
                                  E + (size_t)i * K, Qu0 + (size_t)i * Kh);
    if (r) {
#pragma omp atomic write
      err = r;
      continue;
    }
    inverse_transform(p, g.gx, cself + (size_t)i * K, us + (size_t)i * T);
    for (int t = 0; t < T; ++t) us[(size_t)i * T + t] *= self_node_factor(&g, op, i, t / (2 * p + 2));
  }
  if (err) rc = err;

  /* Algorithm 1, near-field step: neighbours' exterior expansions at the target nodes */
  if (!rc) {
#pragma omp parallel for schedule(dynamic)
    for (int j = 0; j < M; ++j) {
      for (int i = 0; i < M; ++i) {
        if (!g.near[(size_t)i * M + j]) continue;
        for (int t = 0; t < T; ++t) {
          size_t gt = (size_t)j * T + t;
          double val;
          int r = near_term(&g, op, i, E + (size_t)i * K, Qu0 + (size_t)i * Kh, gt, &val);
          if (r) {
#pragma omp atomic write
            err = r;
            continue;
          }
          un[gt] += val;
        }
      }
    }
    if (err) rc = err;
  }

  /* Algorithm 1, far-field step: smooth quadrature from far particles, Neumaier-compensated */
  if (!rc) {
#pragma omp parallel for schedule(dynamic)
    for (int j = 0; j < M; ++j) {
      for (int t = 0; t < T; ++t) {
        size_t gt = (size_t)j * T + t;
        double sum = 0.0, comp = 0.0;
        for (int i = 0; i < M; ++i) {
          if (i == j || g.near[(size_t)i * M + j]) continue;
          for (int q = 0; q < T; ++q) {
            double term = far_term(&g, op, density, gt, (size_t)i * T + q);
            double tsum = sum + term;
            if (fabs(sum) >= fabs(term)) comp += (sum - tsum) + term;
            else comp += (term - tsum) + sum;
            sum = tsum;
          }
        }
        uf[gt] = sum + comp;
      }
    }
  }

  /* Algorithm 1, assembly step: sum of the three pieces */
  if (!rc) {
    for (size_t gi = 0; gi < N; ++gi) {
      if (u_self) u_self[gi] = us[gi];
      if (u_near) u_near[gi] = un[gi];
      if (u_far) u_far[gi] = uf[gi];
      u[gi] = us[gi] + un[gi] + uf[gi];
    }
  }
  free(us); free(un); free(uf); free(cself); free(E); free(Qu0);
  free_geometry(&g);
  return rc;
}

/* Algorithm 1 evaluated at a subset of nodes only (for checks at full size):
   out_self/out_near/out_far/out[t] for node index targets[t].  The per-particle
   transforms are computed only for the particles that the targets need. */
int orc_apply_at(const double* centres, const double* quats, const double* A,
                 const double* C, int M, int p, double eta, int op,
                 const double* density, const int64_t* targets, int ntg,
                 double* out_self, double* out_near, double* out_far, double* out) {
  if (!valid_op(op)) return ORC_E_INVALID;
  geometry g;
  int rc = build_geometry(centres, quats, A, C, M, p, eta, &g);
  if (rc) return rc;
  int T = g.T, K = g.K, Kh = g.Kh;
  uint8_t* need = (uint8_t*)calloc(M, 1);
  for (int t = 0; t < ntg; ++t) {
    if (targets[t] < 0 || targets[t] >= (int64_t)g.N) { free(need); free_geometry(&g); return ORC_E_INVALID; }
    int j = (int)(targets[t] / T);
    need[j] = 1;
    for (int i = 0; i < M; ++i) if (g.near[(size_t)i * M + j]) need[i] = 1;
  }
  double* cself = (double*)calloc((size_t)M * K, sizeof(double));
  double* E = (double*)calloc((size_t)M * K, sizeof(double));
  double complex* Qu0 = (double complex*)calloc((size_t)M * Kh, sizeof(double complex));
  int err = 0;
#pragma omp parallel for schedule(dynamic)
  for (int i = 0; i < M; ++i) {
    if (!need[i]) continue;
    int r = particle_coefficients(&g, op, i, density, cself + (size_t)i * K,
                                  E + (size_t)i * K, Qu0 + (size_t)i * Kh);
    if (r) {
#pragma omp atomic write
      err = r;
    }
  }
  if (err) rc = err;
  double* Y = (double*)malloc(sizeof(double) * K);
#pragma omp parallel for schedule(dynamic)
  for (int t = 0; t < ntg; ++t) {
    if (rc) continue;
    int64_t gt = targets[t];
    int j = (int)(gt / T), loc = (int)(gt - (int64_t)j * T);
    int Nphi = 2 * p + 2;
    int jv = loc / Nphi, kp = loc - jv * Nphi;
    /* self: inverse transform of the diagonal coefficients at this node */
    double* Yl = (double*)malloc(sizeof(double) * K);
    real_harmonics(g.gx[jv], 2.0 * PI * kp / Nphi, p, Yl);
    double us = 0.0;
    for (int l = 0; l < K; ++l) us += cself[(size_t)j * K + l] * Yl[l];
    us *= self_node_factor(&g, op, j, jv);
    free(Yl);
    /* near */
    double un = 0.0;
    for (int i = 0; i < M; ++i) {
      if (!g.near[(size_t)i * M + j]) continue;
      double val;
      int r = near_term(&g, op, i, E + (size_t)i * K, Qu0 + (size_t)i * Kh, (size_t)gt, &val);
      if (r) {
#pragma omp atomic write
        err = r;
      }
      un += val;
    }
    /* far, Neumaier-compensated */
    double sum = 0.0, comp = 0.0;
    for (int i = 0; i < M; ++i) {
      if (i == j || g.near[(size_t)i * M + j]) continue;
      for (int q = 0; q < T; ++q) {
        double term = far_term(&g, op, density, (size_t)gt, (size_t)i * T + q);
        double ts = sum + term;
        if (fabs(sum) >= fabs(term)) comp += (sum - ts) + term;
        else comp += (term - ts) + sum;
        sum = ts;
      }
    }
    double uf = sum + comp;
    if (out_self) out_self[t] = us;
    if (out_near) out_near[t] = un;
    if (out_far) out_far[t] = uf;
    out[t] = us + un + uf;
  }
  if (err) rc = err;
  free(Y); free(need); free(cself); free(E); free(Qu0);
  free_geometry(&g);
  return rc;
}

/* Exterior evaluation of one particle's layer potential at arbitrary exterior
   points from its nodal density (the analytic near-field formula), for the
   pins: S or D exterior values of a single spheroid. */
int orc_eval_exterior(const double* centre, const double* quat, double A,
                      double C, int p, int op, const double* density,
                      const double* pts, int npts, double* out) {
  geometry g;
  int rc = build_geometry(centre, quat, &A, &C, 1, p, 1.0, &g);
  if (rc) return rc;
  double* cself = (double*)malloc(sizeof(double) * g.K);
  double* E = (double*)malloc(sizeof(double) * g.K);
  double complex* Qu0 = (double complex*)malloc(sizeof(double complex) * g.Kh);
  rc = particle_coefficients(&g, op, 0, density, cself, E, Qu0);
  for (int t = 0; t < npts && !rc; ++t)
    rc = eval_exterior(&g.pt[0], p, E, Qu0, pts + 3 * t, out + t);
  free(cself); free(E); free(Qu0);
  free_geometry(&g);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Gradients of single-layer expansions and the Stokes single layer through  */
/* Laplace single layers (Section 4.3, Eq. (stokes)).                        */
/* ------------------------------------------------------------------------ */

/* Values and lab-frame gradients of nset single-particle expansions
   Phi_s = sum_l E[s][l] R_n^|m|(u) Y_l(v, phi) at the point (u, v, phi) of
   particle pt, with R = Q_n^m(z)/Q_n^m(z0) (exterior) or P_n^m(z)/P_n^m(z0)
   (interior).  The gradient is the chain rule for the orthogonal coordinates
   of Table 1: grad = sum_q (dx/dq) |dx/dq|^-2 dPhi/dq in the body frame,
   then rotated to the lab frame.  dY/dv uses the derivative identity of
   Section 2.3 on the cut, (1-v^2) P_n^m' = (m-n-1) P_{n+1}^m + (n+1) v P_n^m. */
static int expansion_grad(const particle* pt, int p, int nset, const double* E, double u,
                          double v, double phi, int interior, double* val, double* grad) {
  int K = (p + 1) * (p + 1), N = p + 1;
  int nh = (p + 2) * (p + 3) / 2;
  double* Pf = (double*)malloc(sizeof(double) * nh);
  double complex* buf = (double complex*)malloc(sizeof(double complex) * 8 * (N + 2));
  double complex *P = buf, *Q = buf + (N + 2), *dP = buf + 2 * (N + 2), *dQ = buf + 3 * (N + 2);
  double complex *P0 = buf + 4 * (N + 2), *Q0 = buf + 5 * (N + 2), *dP0 = buf + 6 * (N + 2),
                 *dQ0 = buf + 7 * (N + 2);
  ferrers_all(v, p + 1, Pf);
  double dzdu_re = 1.0, dzdu_im = 0.0;
  if (pt->oblate) { dzdu_re = 0.0; dzdu_im = 1.0; }
  double complex dzdu = dzdu_re + dzdu_im * I;
  double Fu[16], Fv[16], Fp[16];
  if (nset < 1 || nset > 16) { free(Pf); free(buf); return ORC_E_INVALID; }
  for (int s = 0; s < nset; ++s) { val[s] = 0.0; Fu[s] = Fv[s] = Fp[s] = 0.0; }
  int rc = 0;
  for (int m = 0; m <= p && !rc; ++m) {
    rc = legendre_offcut(pt->oblate, u, m, N, P, Q, dP, dQ);
    if (!rc) rc = legendre_offcut(pt->oblate, pt->u0, m, N, P0, Q0, dP0, dQ0);
    if (rc) break;
    for (int n = m; n <= p; ++n) {
      double complex F = interior ? P[n] : Q[n], F0 = interior ? P0[n] : Q0[n];
      double complex dF = interior ? dP[n] : dQ[n];
      double R = creal(F / F0), dR = creal(dzdu * dF / F0);
      double Nnm = sqrt((2.0 * n + 1.0) / (4.0 * PI) * factorial(n - m) / factorial(n + m));
      if (m > 0) Nnm *= sqrt(2.0);
      double Pn = Pf[n * (n + 1) / 2 + m], Pn1 = Pf[(n + 1) * (n + 2) / 2 + m];
      double dPn = ((m - n - 1) * Pn1 + (n + 1) * v * Pn) / (1.0 - v * v);
      double cphi = cos(m * phi), sphi = sin(m * phi);
      for (int s = 0; s < nset; ++s) {
        const double* Es = E + (size_t)s * K;
        double ec = Es[n * n + n + m], es = (m > 0) ? Es[n * n + n - m] : 0.0;
        double ang = ec * cphi + es * sphi;          /* angular part of +m and -m terms */
        double dang = m * (es * cphi - ec * sphi);   /* its phi derivative */
        val[s] += Nnm * Pn * R * ang;
        Fu[s] += Nnm * Pn * dR * ang;
        Fv[s] += Nnm * dPn * R * ang;
        Fp[s] += Nnm * Pn * R * dang;
      }
    }
  }
  free(Pf);
  free(buf);
  if (rc) return rc;
  double a = pt->a;
  double su = pt->oblate ? sqrt(u * u + 1.0) : sqrt(u * u - 1.0);
  double sv = sqrt(1.0 - v * v), cph = cos(phi), sph = sin(phi);
  double xu[3] = {a * u / su * sv * cph, a * u / su * sv * sph, a * v};
  double xv[3] = {-a * su * v / sv * cph, -a * su * v / sv * sph, a * u};
  double xp[3] = {-a * su * sv * sph, a * su * sv * cph, 0.0};
  double hu2 = xu[0] * xu[0] + xu[1] * xu[1] + xu[2] * xu[2];
  double hv2 = xv[0] * xv[0] + xv[1] * xv[1] + xv[2] * xv[2];
  double hp2 = xp[0] * xp[0] + xp[1] * xp[1] + xp[2] * xp[2];
  for (int s = 0; s < nset; ++s) {
    double gb[3];
    for (int c = 0; c < 3; ++c) gb[c] = xu[c] * Fu[s] / hu2 + xv[c] * Fv[s] / hv2 + xp[c] * Fp[s] / hp2;
    for (int r = 0; r < 3; ++r)
      grad[3 * s + r] = pt->R[3 * r] * gb[0] + pt->R[3 * r + 1] * gb[1] + pt->R[3 * r + 2] * gb[2];
  }
  return ORC_OK;
}

/* Single-layer exterior coefficients E = lamS * T[w f] of one particle for a
   nodal density f (modified basis of Section 3.2). */
static int single_layer_coefficients(const geometry* g, int i, const double* f, double* E) {
  const particle* pt = &g->pt[i];
  int p = g->p, Nphi = 2 * p + 2, K = g->K, Kh = g->Kh;
  double* wf = (double*)malloc(sizeof(double) * g->T);
  double* lam = (double*)malloc(sizeof(double) * Kh);
  int rc = spectra(pt, p, NULL, NULL, NULL, lam, NULL);
  if (rc) { free(wf); free(lam); return rc; }
  double sgn = pt->oblate ? 1.0 : -1.0;
  for (int j = 0; j <= p; ++j)
    for (int k = 0; k < Nphi; ++k)
      wf[j * Nphi + k] = sqrt(pt->u0 * pt->u0 + sgn * g->gx[j] * g->gx[j]) * f[j * Nphi + k];
  forward_transform(p, g->gx, g->gw, wf, E);
  for (int n = 0; n <= p; ++n)
    for (int m = -n; m <= n; ++m) E[n * n + n + m] *= lam[n * (n + 1) / 2 + abs(m)];
  free(wf); free(lam);
  return ORC_OK;
}

/* The four single-layer expansions of particle i used by Eq. (stokes): the
   three density components and rho_i = (y - c_i).sigma (origin at the source
   centre).  density is [3][N]; E4 is [4][K]. */
static int stokes_coefficients(const geometry* g, int i, const double* density, double* E4) {
  int T = g->T, K = g->K;
  size_t N = (size_t)g->N;
  double* f = (double*)malloc(sizeof(double) * T);
  int rc = 0;
  for (int s = 0; s < 4 && !rc; ++s) {
    for (int t = 0; t < T; ++t) {
      size_t gi = (size_t)i * T + t;
      if (s < 3) {
        f[t] = density[s * N + gi];
      } else {
        double r = 0.0;
        for (int c = 0; c < 3; ++c) r += (g->xyz[3 * gi + c] - g->pt[i].c[c]) * density[c * N + gi];
        f[t] = r;
      }
    }
    rc = single_layer_coefficients(g, i, f, E4 + (size_t)s * K);
  }
  free(f);
  return rc;
}

/* Eq. (stokes) with viscosity 1 and origin c_i:
   u_k = 1/2 { S[sigma_k] - sum_j (x - c_i)_j d_k S[sigma_j] + d_k S[rho_i] } */
static void stokes_combine(const particle* pt, const double x[3], const double* val,
                           const double* grad, double out[4]) {
  for (int k = 0; k < 3; ++k) {
    double s = val[k] + grad[3 * 3 + k];
    for (int j = 0; j < 3; ++j) s -= (x[j] - pt->c[j]) * grad[3 * j + k];
    out[k] = 0.5 * s;
  }
  /* pressure with the kernel (1/4pi) r/|r|^3, r = x - y: p = -sum_j d_j S[sigma_j]
     (the printed identity sum_j e_j . grad S[sigma_j] has the opposite sign) */
  out[3] = -(grad[0] + grad[4] + grad[8]);
}

/* Self, near and far parts of Eq. (stokes) at node gt, and of the pressure
   (component 3): the exterior-limit expansions of the target's own particle
   at its node, the neighbours' exterior expansions (ascending source index),
   and the Stokeslet (1/8pi)(I/r + r r^T/r^3) with its pressure (1/4pi) r/r^3
   over the far sources by smooth quadrature, Neumaier-compensated. */
static int stokes_node(const geometry* g, const double* E4, const double* density, size_t gt,
                       double us[4], double un[4], double uf[4]) {
  int M = g->M, T = g->T, K = g->K, p = g->p, Nphi = 2 * p + 2;
  size_t N = (size_t)g->N;
  int j = (int)(gt / T), loc = (int)(gt - (size_t)j * T);
  int jv = loc / Nphi, kp = loc - jv * Nphi;
  const double* x = g->xyz + 3 * gt;
  double val[4], grad[12];
  int rc = expansion_grad(&g->pt[j], p, 4, E4 + (size_t)j * 4 * K, g->pt[j].u0, g->gx[jv],
                          2.0 * PI * kp / Nphi, 0, val, grad);
  if (rc) return rc;
  stokes_combine(&g->pt[j], x, val, grad, us);
  for (int k = 0; k < 4; ++k) un[k] = 0.0;
  for (int i = 0; i < M; ++i) {
    if (!g->near[(size_t)i * M + j]) continue;
    double xb[3], uu, vv, ph, o[4];
    lab_to_body(&g->pt[i], x, xb);
    body_to_spheroidal(&g->pt[i], xb, &uu, &vv, &ph);
    rc = expansion_grad(&g->pt[i], p, 4, E4 + (size_t)i * 4 * K, uu, vv, ph, 0, val, grad);
    if (rc) return rc;
    stokes_combine(&g->pt[i], x, val, grad, o);
    for (int k = 0; k < 4; ++k) un[k] += o[k];
  }
  double sum[4] = {0, 0, 0, 0}, comp[4] = {0, 0, 0, 0};
  for (int i = 0; i < M; ++i) {
    if (i == j || g->near[(size_t)i * M + j]) continue;
    for (int q = 0; q < T; ++q) {
      size_t gs = (size_t)i * T + q;
      const double* y = g->xyz + 3 * gs;
      double d[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
      double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2], r = sqrt(r2);
      double sg[3] = {density[gs], density[N + gs], density[2 * N + gs]};
      double dots = d[0] * sg[0] + d[1] * sg[1] + d[2] * sg[2];
      for (int k = 0; k < 4; ++k) {
        double term = k < 3 ? g->W[gs] * (sg[k] / r + d[k] * dots / (r2 * r)) / (8.0 * PI)
                            : g->W[gs] * dots / (r2 * r) / (4.0 * PI);
        double ts = sum[k] + term;
        if (fabs(sum[k]) >= fabs(term)) comp[k] += (sum[k] - ts) + term;
        else comp[k] += (term - ts) + sum[k];
        sum[k] = ts;
      }
    }
  }
  for (int k = 0; k < 4; ++k) uf[k] = sum[k] + comp[k];
  return ORC_OK;
}

/* The four expansions of every particle flagged in need (all when need is NULL). */
static int stokes_all_coefficients(const geometry* g, const double* density, const uint8_t* need,
                                   double* E4) {
  int err = 0;
#pragma omp parallel for schedule(dynamic)
  for (int i = 0; i < g->M; ++i) {
    if (need && !need[i]) continue;
    int r = stokes_coefficients(g, i, density, E4 + (size_t)i * 4 * g->K);
    if (r) {
#pragma omp atomic write
      err = r;
    }
  }
  return err;
}

/* ncomp = 3: velocity [3][N]; ncomp = 4: velocity and pressure [4][N]
   (the pressure on the surface is its exterior limit). */
int orc_stokes_apply(const double* centres, const double* quats, const double* A,
                     const double* C, int M, int p, double eta, const double* density, int ncomp,
                     double* u_self, double* u_near, double* u_far, double* u) {
  if (ncomp != 3 && ncomp != 4) return ORC_E_INVALID;
  geometry g;
  int rc = build_geometry(centres, quats, A, C, M, p, eta, &g);
  if (rc) return rc;
  size_t N = (size_t)g.N;
  double* E4 = (double*)malloc(sizeof(double) * 4 * g.K * (size_t)M);
  rc = stokes_all_coefficients(&g, density, NULL, E4);
  int err = 0;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t gt = 0; gt < (int64_t)N; ++gt) {
    if (rc || err) continue;
    double us[4], un[4], uf[4];
    int r = stokes_node(&g, E4, density, (size_t)gt, us, un, uf);
    if (r) {
#pragma omp atomic write
      err = r;
      continue;
    }
    for (int k = 0; k < ncomp; ++k) {
      size_t q = k * N + (size_t)gt;
      if (u_self) u_self[q] = us[k];
      if (u_near) u_near[q] = un[k];
      if (u_far) u_far[q] = uf[k];
      u[q] = us[k] + un[k] + uf[k];
    }
  }
  if (!rc) rc = err;
  free(E4);
  free_geometry(&g);
  return rc;
}

/* Eq. (stokes) at selected node indices only (full-size checks); outputs
   [3][ntg].  Only the target particles and their near neighbours are expanded. */
int orc_stokes_apply_at(const double* centres, const double* quats, const double* A,
                        const double* C, int M, int p, double eta, const double* density,
                        const int64_t* targets, int ntg, int ncomp, double* out_self, double* out_near,
                        double* out_far, double* out) {
  if (ncomp != 3 && ncomp != 4) return ORC_E_INVALID;
  geometry g;
  int rc = build_geometry(centres, quats, A, C, M, p, eta, &g);
  if (rc) return rc;
  int T = g.T;
  uint8_t* need = (uint8_t*)calloc(M, 1);
  for (int t = 0; t < ntg; ++t) {
    if (targets[t] < 0 || targets[t] >= (int64_t)g.N) { free(need); free_geometry(&g); return ORC_E_INVALID; }
    int j = (int)(targets[t] / T);
    need[j] = 1;
    for (int i = 0; i < M; ++i) if (g.near[(size_t)i * M + j]) need[i] = 1;
  }
  double* E4 = (double*)calloc((size_t)4 * g.K * M, sizeof(double));
  rc = stokes_all_coefficients(&g, density, need, E4);
  int err = 0;
#pragma omp parallel for schedule(dynamic)
  for (int t = 0; t < ntg; ++t) {
    if (rc || err) continue;
    double us[4], un[4], uf[4];
    int r = stokes_node(&g, E4, density, (size_t)targets[t], us, un, uf);
    if (r) {
#pragma omp atomic write
      err = r;
      continue;
    }
    for (int k = 0; k < ncomp; ++k) {
      size_t q = (size_t)k * ntg + t;
      if (out_self) out_self[q] = us[k];
      if (out_near) out_near[q] = un[k];
      if (out_far) out_far[q] = uf[k];
      out[q] = us[k] + un[k] + uf[k];
    }
  }
  if (!rc) rc = err;
  free(need);
  free(E4);
  free_geometry(&g);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Stokes double layer, the stresslet with the outward normal (viscosity 1):  */
/*   D_stk[mu]_i(x) = 3/(4 pi) int (r.mu)(r.nu) r_i / |r|^5 dS_y, r = x - y,  */
/* normalised so that a constant mu gives -mu inside, 0 outside and -mu/2 on  */
/* the surface (principal value), as the Laplace D of a constant.  Section    */
/* 4.3 only cites a decomposition into Laplace potentials; the one used here  */
/* (derived for this oracle) is, with origin c at each source centre,         */
/*   D_stk[mu]_i = -sum_j (x-c)_j d_i D[mu_j] + d_i D[(y-c).mu]               */
/*                 - sum_j d_j S[mu_j nu_i],                                  */
/* which follows from d_i (nu.r/r^3) and d_j (1/r) = -r_j/r^3.  Self values:  */
/* the exterior limits of the gradients give D_stk+, and the principal value  */
/* is D_stk+ - mu/2 (the jump of the double layer is mu).                     */
/* ------------------------------------------------------------------------ */

/* Double-layer exterior coefficients E = lamD+ * T[f] of one particle. */
static int double_layer_coefficients(const geometry* g, int i, const double* f, double* E) {
  const particle* pt = &g->pt[i];
  int p = g->p, Kh = g->Kh;
  double* lam = (double*)malloc(sizeof(double) * Kh);
  int rc = spectra(pt, p, NULL, lam, NULL, NULL, NULL);
  if (rc) { free(lam); return rc; }
  forward_transform(p, g->gx, g->gw, f, E);
  for (int n = 0; n <= p; ++n)
    for (int m = -n; m <= n; ++m) E[n * n + n + m] *= lam[n * (n + 1) / 2 + abs(m)];
  free(lam);
  return ORC_OK;
}

/* The thirteen expansions of particle i: double layers of mu_1, mu_2, mu_3 and
   (y - c_i).mu (sets 0-3), single layers of mu_j nu_k (set 4 + 3k + j). */
static int stokes_dl_coefficients(const geometry* g, int i, const double* density, double* E13) {
  int T = g->T, K = g->K;
  size_t N = (size_t)g->N;
  double* f = (double*)malloc(sizeof(double) * T);
  int rc = 0;
  for (int s = 0; s < 13 && !rc; ++s) {
    for (int t = 0; t < T; ++t) {
      size_t gi = (size_t)i * T + t;
      if (s < 3) {
        f[t] = density[s * N + gi];
      } else if (s == 3) {
        double r = 0.0;
        for (int c = 0; c < 3; ++c) r += (g->xyz[3 * gi + c] - g->pt[i].c[c]) * density[c * N + gi];
        f[t] = r;
      } else {
        int k = (s - 4) / 3, j = (s - 4) % 3;
        f[t] = density[j * N + gi] * g->nrm[3 * gi + k];
      }
    }
    rc = s < 4 ? double_layer_coefficients(g, i, f, E13 + (size_t)s * K)
               : single_layer_coefficients(g, i, f, E13 + (size_t)s * K);
  }
  free(f);
  return rc;
}

/* The decomposition from the lab gradients gD [4][3] of the double layers and
   gS [9][3] of the single layers (origin c). */
static void stokes_dl_combine(const particle* pt, const double x[3], const double* gD, const double* gS,
                              double out[3]) {
  for (int i = 0; i < 3; ++i) {
    double s = gD[3 * 3 + i];
    for (int j = 0; j < 3; ++j) s -= (x[j] - pt->c[j]) * gD[3 * j + i];
    for (int j = 0; j < 3; ++j) s -= gS[3 * (3 * i + j) + j];
    out[i] = s;
  }
}

/* Values (unused) and gradients of the thirteen expansions of particle pt at
   (u, v, phi), exterior side. */
static int stokes_dl_grads(const particle* pt, int p, const double* E13, double u, double v, double phi,
                           double* gD, double* gS) {
  int K = (p + 1) * (p + 1);
  double val[9];
  int rc = expansion_grad(pt, p, 4, E13, u, v, phi, 0, val, gD);
  if (!rc) rc = expansion_grad(pt, p, 9, E13 + (size_t)4 * K, u, v, phi, 0, val, gS);
  return rc;
}

/* Self (principal value), near and far parts of the Stokes double layer at node gt. */
static int stokes_dl_node(const geometry* g, const double* E13, const double* density, size_t gt, double us[3],
                          double un[3], double uf[3]) {
  int M = g->M, T = g->T, K = g->K, p = g->p, Nphi = 2 * p + 2;
  size_t N = (size_t)g->N;
  int j = (int)(gt / T), loc = (int)(gt - (size_t)j * T);
  int jv = loc / Nphi, kp = loc - jv * Nphi;
  const double* x = g->xyz + 3 * gt;
  double gD[12], gS[27], o[3];
  int rc = stokes_dl_grads(&g->pt[j], p, E13 + (size_t)j * 13 * K, g->pt[j].u0, g->gx[jv], 2.0 * PI * kp / Nphi,
                           gD, gS);
  if (rc) return rc;
  stokes_dl_combine(&g->pt[j], x, gD, gS, us);
  for (int k = 0; k < 3; ++k) us[k] -= 0.5 * density[k * N + gt];
  for (int k = 0; k < 3; ++k) un[k] = 0.0;
  for (int i = 0; i < M; ++i) {
    if (!g->near[(size_t)i * M + j]) continue;
    double xb[3], uu, vv, ph;
    lab_to_body(&g->pt[i], x, xb);
    body_to_spheroidal(&g->pt[i], xb, &uu, &vv, &ph);
    rc = stokes_dl_grads(&g->pt[i], p, E13 + (size_t)i * 13 * K, uu, vv, ph, gD, gS);
    if (rc) return rc;
    stokes_dl_combine(&g->pt[i], x, gD, gS, o);
    for (int k = 0; k < 3; ++k) un[k] += o[k];
  }
  double sum[3] = {0, 0, 0}, comp[3] = {0, 0, 0};
  for (int i = 0; i < M; ++i) {
    if (i == j || g->near[(size_t)i * M + j]) continue;
    for (int q = 0; q < T; ++q) {
      size_t gs = (size_t)i * T + q;
      const double *y = g->xyz + 3 * gs, *nu = g->nrm + 3 * gs;
      double d[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
      double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2], r = sqrt(r2);
      double dm = d[0] * density[gs] + d[1] * density[N + gs] + d[2] * density[2 * N + gs];
      double dn = d[0] * nu[0] + d[1] * nu[1] + d[2] * nu[2];
      double w = 3.0 / (4.0 * PI) * g->W[gs] * dm * dn / (r2 * r2 * r);
      for (int k = 0; k < 3; ++k) {
        double term = w * d[k];
        double ts = sum[k] + term;
        if (fabs(sum[k]) >= fabs(term)) comp[k] += (sum[k] - ts) + term;
        else comp[k] += (term - ts) + sum[k];
        sum[k] = ts;
      }
    }
  }
  for (int k = 0; k < 3; ++k) uf[k] = sum[k] + comp[k];
  return ORC_OK;
}

/* Stokes double layer at every node (targets NULL) or at ntg selected nodes;
   density [3][N], outputs [3][N] resp. [3][ntg]. */
int orc_stokes_dl_apply(const double* centres, const double* quats, const double* A, const double* C, int M,
                        int p, double eta, const double* density, const int64_t* targets, int ntg,
                        double* u_self, double* u_near, double* u_far, double* u) {
  geometry g;
  int rc = build_geometry(centres, quats, A, C, M, p, eta, &g);
  if (rc) return rc;
  int T = g.T, K = g.K;
  int64_t n = targets ? ntg : (int64_t)g.N;
  uint8_t* need = (uint8_t*)calloc(M, 1);
  for (int64_t t = 0; t < n; ++t) {
    int64_t gt = targets ? targets[t] : t;
    if (gt < 0 || gt >= (int64_t)g.N) { free(need); free_geometry(&g); return ORC_E_INVALID; }
    int j = (int)(gt / T);
    need[j] = 1;
    for (int i = 0; i < M; ++i) if (g.near[(size_t)i * M + j]) need[i] = 1;
  }
  double* E13 = (double*)calloc((size_t)13 * K * M, sizeof(double));
  int err = 0;
#pragma omp parallel for schedule(dynamic)
  for (int i = 0; i < M; ++i) {
    if (!need[i]) continue;
    int r = stokes_dl_coefficients(&g, i, density, E13 + (size_t)i * 13 * K);
    if (r) {
#pragma omp atomic write
      err = r;
    }
  }
  if (err) rc = err;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t t = 0; t < n; ++t) {
    if (rc || err) continue;
    double us[3], un[3], uf[3];
    int r = stokes_dl_node(&g, E13, density, (size_t)(targets ? targets[t] : t), us, un, uf);
    if (r) {
#pragma omp atomic write
      err = r;
      continue;
    }
    for (int k = 0; k < 3; ++k) {
      size_t q = (size_t)k * n + (size_t)t;
      if (u_self) u_self[q] = us[k];
      if (u_near) u_near[q] = un[k];
      if (u_far) u_far[q] = uf[k];
      u[q] = us[k] + un[k] + uf[k];
    }
  }
  if (!rc) rc = err;
  free(need);
  free(E13);
  free_geometry(&g);
  return rc;
}

/* One particle's Stokes single layer (near-field formula) at exterior points,
   or its self values at its own nodes with the exterior (interior = 0) or
   interior (interior = 1) limit of the gradients, for the pins.
   density [3][T]; out [npts][3] (pts == NULL: the T nodes). */
int orc_stokes_single(const double* centre, const double* quat, double A, double C, int p,
                      const double* density, const double* pts, int npts, int interior,
                      double* out) {
  geometry g;
  int rc = build_geometry(centre, quat, &A, &C, 1, p, 1.0, &g);
  if (rc) return rc;
  int K = g.K, Nphi = 2 * p + 2;
  double* E4 = (double*)malloc(sizeof(double) * 4 * K);
  rc = stokes_coefficients(&g, 0, density, E4);
  int n = pts ? npts : g.T;
  for (int t = 0; t < n && !rc; ++t) {
    double x[3], uu, vv, ph, val[4], grad[12];
    if (pts) {
      double xb[3];
      for (int c = 0; c < 3; ++c) x[c] = pts[3 * t + c];
      lab_to_body(&g.pt[0], x, xb);
      body_to_spheroidal(&g.pt[0], xb, &uu, &vv, &ph);
    } else {
      int jv = t / Nphi, kp = t - jv * Nphi;
      for (int c = 0; c < 3; ++c) x[c] = g.xyz[3 * t + c];
      uu = g.pt[0].u0;
      vv = g.gx[jv];
      ph = 2.0 * PI * kp / Nphi;
    }
    rc = expansion_grad(&g.pt[0], p, 4, E4, uu, vv, ph, interior, val, grad);
    if (!rc) {
      double o[4];
      stokes_combine(&g.pt[0], x, val, grad, o);
      for (int k = 0; k < 3; ++k) out[3 * t + k] = o[k];
    }
  }
  free(E4);
  free_geometry(&g);
  return rc;
}

/* Value and lab gradient of one particle's single-layer expansion of a nodal
   density at exterior points (pins of the chain rule): out [npts][4]. */
int orc_single_layer_grad(const double* centre, const double* quat, double A, double C, int p,
                          const double* density, const double* pts, int npts, double* out) {
  geometry g;
  int rc = build_geometry(centre, quat, &A, &C, 1, p, 1.0, &g);
  if (rc) return rc;
  double* E = (double*)malloc(sizeof(double) * g.K);
  rc = single_layer_coefficients(&g, 0, density, E);
  for (int t = 0; t < npts && !rc; ++t) {
    double xb[3], uu, vv, ph, val, grad[3];
    lab_to_body(&g.pt[0], pts + 3 * t, xb);
    body_to_spheroidal(&g.pt[0], xb, &uu, &vv, &ph);
    rc = expansion_grad(&g.pt[0], p, 1, E, uu, vv, ph, 0, &val, grad);
    out[4 * t] = val;
    for (int c = 0; c < 3; ++c) out[4 * t + 1 + c] = grad[c];
  }
  free(E);
  free_geometry(&g);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Particle-to-target evaluation (Section 4, "Particle-to-target algorithm"): */
/* S or D of the nodal density, and its lab gradient (Eq. (dSLevalformula)   */
/* and the same construction for D), at arbitrary points outside every       */
/* particle.  Each (target, source particle) pair is classified on its own:   */
/* near iff the exact distance from the point to the surface is below        */
/* eta * diam(source), then the source's exterior expansion is used, else the */
/* smooth quadrature.  grad ([npts][3]) and near_out ([npts][M]) may be NULL. */
/* ------------------------------------------------------------------------ */
int orc_eval_targets(const double* centres, const double* quats, const double* A, const double* C, int M,
                     int p, double eta, int op, const double* density, const double* pts, int npts,
                     double* val, double* grad, uint8_t* near_out) {
  if (op != OP_S && op != OP_D) return ORC_E_INVALID;
  geometry g;
  int rc = build_geometry(centres, quats, A, C, M, p, eta, &g);
  if (rc) return rc;
  int T = g.T, K = g.K, Kh = g.Kh;
  double* cself = (double*)malloc(sizeof(double) * (size_t)M * K);
  double* E = (double*)malloc(sizeof(double) * (size_t)M * K);
  double complex* Qu0 = (double complex*)malloc(sizeof(double complex) * (size_t)M * Kh);
  int err = 0;
#pragma omp parallel for schedule(dynamic)
  for (int i = 0; i < M; ++i) {
    int r = particle_coefficients(&g, op, i, density, cself + (size_t)i * K, E + (size_t)i * K,
                                  Qu0 + (size_t)i * Kh);
    if (r) {
#pragma omp atomic write
      err = r;
    }
  }
  if (err) rc = err;
#pragma omp parallel for schedule(dynamic)
  for (int t = 0; t < npts; ++t) {
    if (rc || err) continue;
    const double* x = pts + 3 * t;
    double v = 0.0, gr[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < M; ++i) {
      const particle* pt = &g.pt[i];
      if (inside(pt, x)) {
#pragma omp atomic write
        err = ORC_E_OVERLAP;
        break;
      }
      double y[3];
      project_lab(pt, x, y);
      double dist = sqrt((x[0] - y[0]) * (x[0] - y[0]) + (x[1] - y[1]) * (x[1] - y[1]) +
                         (x[2] - y[2]) * (x[2] - y[2]));
      int near = dist < eta * pt->diam;
      if (near_out) near_out[(size_t)t * M + i] = (uint8_t)near;
      if (near) {
        double xb[3], u, vv, ph, ev, eg[3];
        lab_to_body(pt, x, xb);
        body_to_spheroidal(pt, xb, &u, &vv, &ph);
        int r = expansion_grad(pt, p, 1, E + (size_t)i * K, u, vv, ph, 0, &ev, eg);
        if (r) {
#pragma omp atomic write
          err = r;
          break;
        }
        v += ev;
        for (int c = 0; c < 3; ++c) gr[c] += eg[c];
      } else {
        for (int q = 0; q < T; ++q) {
          size_t gs = (size_t)i * T + q;
          const double* ys = g.xyz + 3 * gs;
          const double* ny = g.nrm + 3 * gs;
          double d[3] = {x[0] - ys[0], x[1] - ys[1], x[2] - ys[2]};
          double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
          double r = sqrt(r2);
          double w = g.W[gs] * density[gs] / (4.0 * PI);
          if (op == OP_S) {
            v += w / r;
            for (int c = 0; c < 3; ++c) gr[c] -= w * d[c] / (r2 * r);
          } else {
            double nd = ny[0] * d[0] + ny[1] * d[1] + ny[2] * d[2];
            v += w * nd / (r2 * r);
            for (int c = 0; c < 3; ++c) gr[c] += w * (ny[c] / (r2 * r) - 3.0 * nd * d[c] / (r2 * r2 * r));
          }
        }
      }
    }
    val[t] = v;
    if (grad)
      for (int c = 0; c < 3; ++c) grad[3 * t + c] = gr[c];
  }
  if (err) rc = err;
  free(cself); free(E); free(Qu0);
  free_geometry(&g);
  return rc;
}

int orc_num_threads(void) {
#ifdef _OPENMP
  extern int omp_get_max_threads(void);
  return omp_get_max_threads();
#else
  return 1;
#endif
}
