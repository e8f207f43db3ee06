// Legendre functions of the second kind for the near-field exterior
// expansions (Section 2.3, "Legendre function evaluation"; Theorems 1 and 2,
// exterior rows), shared by the Laplace and Stokes near-field kernels.  Real
// forms: prolate Q_n^m(u), oblate q_n^m(u) = i^(n+1) Q_n^m(iu); w = u^2 -+ 1,
// sgn = -1 (prolate) or +1 (oblate), N = p + 1.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "sbie_internal.h"

namespace sbie {

// f(std::integral_constant<int, B>{}), ..., f(std::integral_constant<int, E>{}).
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B <= E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// The orders m = 0 .. p in ascending order.  With UNROLL (the order fixed at
// PMAX at compile time) every call sees m as a constant, so each degree test
// n >= m and every recurrence coefficient folds and the order's code is
// straight-line; otherwise a plain loop with m at run time.
template <int PMAX, bool UNROLL, typename F>
__device__ __forceinline__ void for_orders(int p, F&& f) {
  if constexpr (UNROLL) {
    static_for<0, PMAX>(f);
  } else {
#pragma unroll 1
    for (int m = 0; m <= p; ++m) f(m);
  }
}

// Unrolling the orders pays while the kernel's code stays in the instruction
// cache: (p+1)(p+2)/2 straight-line (n, m) steps for p up to 16.
template <int PMAX, bool EXACT>
constexpr bool kUnrollOrders = EXACT && PMAX <= 16;

// Depth L of the backward recurrence: the ratio of the minimal to the
// dominant solution shrinks by (u + sqrt(w))^-2 per degree; 2^-58 plus a
// margin, the largest over the wave (wave-uniform), in whole chunks of eight
// steps; past cap steps (at most kMaxNearDepth) the depth is capped and
// numeric_flag is set in *bad.
// With own, *own receives the lane's own depth (capped and rounded the same
// way), for q_top_orders01's lane-exact start.
__device__ inline int near_depth(double u, double sw, int N, int cap, unsigned numeric_flag, unsigned* bad,
                                 int* own = nullptr) {
  // clamped in floating point: a point on the focal set (u + sw = 1, only
  // reachable from inside the spheroid) or a NaN gives the capped depth
  const double sd = ceil(20.1 / log(u + sw)) + 8.0;
  const int mine = sd < 200000.0 ? (int)sd : 200000;
  int steps = mine;
  for (int off = 32; off >= 1; off >>= 1) steps = max(steps, __shfl_xor(steps, off, 64));
  steps = __builtin_amdgcn_readfirstlane(steps);
  cap = min(cap, kMaxNearDepth);
  if (steps > cap) {
    steps = cap;
    *bad |= numeric_flag;
  }
  steps = (steps + 7) & ~7;
  if (own) *own = N + ((min(mine, cap) + 7) & ~7);
  return N + steps;
}

// Q_N^m and Q_{N+1}^m for m = 0 and 1.  With own > 0 the lane starts its
// recurrence at degree own (<= L, on the same chunks of eight) instead of L:
// its result then depends on its own point only, not on the wave's deepest.  The minimal solution of the
// recurrence in n comes from backward recurrence from degree L (the continued
// fraction for Q_N/Q_{N-1} evaluated bottom-up), free of divisions with
// Q_n = s_n R_n and s_{n-1} = s_n/(n+m):
//   R_{n-1} = (2n+1) u R_n -+ ((n+1)^2 - m^2) R_{n+1},
// rescaled by 2^-600 whenever it grows past 2^600; the Casoratian at degree N
// against the forward P (division-free as Pt_n = (n-m)! P_n^m),
//   Pt_N Q_{N-1} -+ (N-m) Pt_{N-1} Q_N = (-1)^m (N+m-1)!,
// fixes the scale.  rcp[k] = 1/k.
__device__ inline void q_top_orders01(double u, double sw, double sgn, int N, int L, const double* __restrict__ rcp,
                                      double qN[2], double qN1[2], int own = 0) {
  double qh[2] = {0.0, 0.0}, qc[2] = {1.0, 1.0};
  const double smsq[2] = {0.0, sgn};
  double c2n1 = (double)(2 * L + 1), snp = sgn * (double)(L + 1) * (double)(L + 1), sc = sgn * c2n1;
  const double dsc = -2.0 * sgn;
  for (int n = L; n > N; n -= 8) {
    if (own > 0 && n >= own) {
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        qh[k] = 0.0;
        qc[k] = 1.0;
      }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const double cu = c2n1 * u;
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const double qn = fma(cu, qc[k], (snp - smsq[k]) * qh[k]);
        qh[k] = qc[k];
        qc[k] = qn;
      }
      snp -= sc;
      sc += dsc;
      c2n1 -= 2.0;
    }
#pragma unroll
    for (int k = 0; k < 2; ++k)
      if (fabs(qc[k]) > 0x1p600) {
        qc[k] *= 0x1p-600;
        qh[k] *= 0x1p-600;
      }
  }
  double cas2 = 1.0;  // (-1)^m (N+m-1)!
  for (int k = 2; k < N; ++k) cas2 *= (double)k;
  double pmm = 1.0;  // P_m^m(u), real form: (2m-1)!! w^(m/2)
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    if (m == 1) {
      pmm = sw;
      cas2 = -cas2 * (double)N;
    }
    //   Pt_{n+1} = (2n+1) u Pt_n -+ (n+m)(n-m) Pt_{n-1}
    double pa = pmm, pb = (double)(2 * m + 1) * u * pmm;  // Pt_m, Pt_{m+1}
    double c2 = (double)(2 * m + 3), cnm = (double)(2 * m + 1), cdn = 1.0;
    for (int n = m + 1; n < N; ++n) {
      const double pc = fma(c2 * u, pb, sgn * (cnm * cdn) * pa);
      pa = pb;
      pb = pc;
      c2 += 2.0;
      cnm += 1.0;
      cdn += 1.0;
    }
    // pa = Pt_{N-1}, pb = Pt_N; Q~_N = R_N/(N+m+1), Q~_{N+1} = R_{N+1}, Q~_{N-1} one step down
    const double q0 = qc[m] * rcp[N + m + 1], q1 = qh[m];
    const double qm1 = fma((double)(2 * N + 1) * u, q0, sgn * (double)(N - m + 1) * q1) * rcp[N + m];
    const double scale = cas2 / fma(sgn * (double)(N - m) * pa, q0, pb * qm1);
    qN[m] = scale * q0;
    qN1[m] = scale * q1;
  }
}

// Order step at fixed degree n (m >= 2), in which Q grows faster than P so it
// is run upward:  F^m = -2(m-1) u w^(-1/2) F^(m-1) + (n-m+2)(n+m-1) F^(m-2).
__device__ inline double q_next_order(double ur, int n, int m, double f1, double f2) {
  return fma(-2.0 * (double)(m - 1) * ur, f1, (double)((n - m + 2) * (n + m - 1)) * f2);
}

// Q_n^m for n = m .. N+1 (zero elsewhere) from Q_N and Q_{N+1}, by the
// recurrence in n run downward (Q is its minimal solution upward).
template <int PMAX>
__device__ inline void q_column(double u, double sgn, int N, int m, double qN, double qN1,
                                const double* __restrict__ rcp, double (&Q)[PMAX + 4]) {
#pragma unroll
  for (int n = PMAX + 2; n >= 0; --n) {
    if (n == N + 1) {
      Q[n] = qN1;
    } else if (n == N) {
      Q[n] = qN;
    } else if (n < N && n >= m) {
      Q[n] = fma((double)(2 * n + 3) * u, Q[n + 1], sgn * (double)(n - m + 2) * Q[n + 2]) * rcp[n + m + 1];
    } else {
      Q[n] = 0.0;
    }
  }
}

// The downward recurrence in n of q_column with its coefficients per (n, m)
// from a table: Q_n = A_nm u Q_{n+1} + sgn B_nm Q_{n+2} with
// A_nm = (2n+3)/(n+m+1) and B_nm = (n-m+2)/(n+m+1).  Row h = n(n+1)/2 + m,
// n = 0 .. p, holds (A_nm, -B_nm) in the prolate half and (A_nm, B_nm) in the
// oblate half (kh = (p+1)(p+2)/2 rows each); with COLS = 3 a third column
// holds -sgn (n-m+1), the coefficient of Q_{n+1} in the u-derivative
// w dQ_n/du = -sgn (n-m+1) Q_{n+1} - (n+1) u Q_n.  Every (n, m) reads its own
// row, so with the orders unrolled no coefficient is shared between orders
// (which would keep it in a register across all of them).
template <int COLS>
__device__ inline void q_recurrence_table(int p, double* tab, int tid, int nthreads) {
  const int kh = (p + 1) * (p + 2) / 2;
  for (int k = tid; k < 2 * kh; k += nthreads) {
    const int h = k < kh ? k : k - kh;
    const double sgn = k < kh ? -1.0 : 1.0;
    int n = (int)((sqrt(8.0 * h + 1.0) - 1.0) * 0.5);
    n += (n + 1) * (n + 2) / 2 <= h ? 1 : 0;
    n -= n * (n + 1) / 2 > h ? 1 : 0;
    const int m = h - n * (n + 1) / 2;
    const double r = 1.0 / (double)(n + m + 1);
    tab[COLS * k] = (double)(2 * n + 3) * r;
    tab[COLS * k + 1] = sgn * (double)(n - m + 2) * r;
    if constexpr (COLS == 3) tab[3 * k + 2] = -sgn * (double)(n - m + 1);
  }
}

template <int PMAX, int COLS>
__device__ inline void q_column_tab(double u, int N, int m, double qN, double qN1, const double* __restrict__ tab,
                                    double (&Q)[PMAX + 4]) {
#pragma unroll
  for (int n = PMAX + 2; n >= 0; --n) {
    if (n == N + 1) {
      Q[n] = qN1;
    } else if (n == N) {
      Q[n] = qN;
    } else if (n < N && n >= m) {
      const int h = n * (n + 1) / 2 + m;
      Q[n] = fma(tab[COLS * h], u * Q[n + 1], tab[COLS * h + 1] * Q[n + 2]);
    } else {
      Q[n] = 0.0;
    }
  }
}

// Waves per workgroup of the near-field kernels built on expansion_orders
// (UNROLL): two waves (128 target nodes of one particle) share the LDS tables
// below; with expansion_terms one.
template <bool UNROLL>
constexpr int kNearWaves = UNROLL ? 2 : 1;

// LDS of those kernels with the orders unrolled (p = PMAX): per workgroup the
// normalised Ferrers recurrence (ab) and derivative (cd) coefficients through
// degree p+1 and the three-column recurrence table in n; per source its NSET
// expansions, set s at E[s K + l], each coefficient times the spectral ratio
// 1/Q_n^|m|(u0) of its (n, |m|).  Wave-uniform reads from LDS keep these
// values out of the scalar registers, which the unrolled orders would
// otherwise fill with hoisted loads.
template <int PMAX, int NSET>
struct NearTables {
  static constexpr int KM = (PMAX + 1) * (PMAX + 1), KHM = (PMAX + 1) * (PMAX + 2) / 2,
                       KH2M = (PMAX + 2) * (PMAX + 3) / 2;
  double E[NSET * KM];
  double ab[2 * KH2M];
  double cd[KHM];
  double qt[6 * KHM];

  __device__ void stage_fixed(const double* __restrict__ gab, const double* __restrict__ gcd, int tid, int nt) {
    for (int k = tid; k < 2 * KH2M; k += nt) ab[k] = gab[k];
    for (int k = tid; k < KHM; k += nt) cd[k] = gcd[k];
    q_recurrence_table<3>(PMAX, qt, tid, nt);
  }

  // Es: the source's first set (sets stride doubles apart); L: its spectra
  // rows (column 3 holds 1/Q_n^m(u0)).
  __device__ void stage_source(const double* __restrict__ Es, size_t stride, const double* __restrict__ L, int tid,
                               int nt) {
    for (int k = tid; k < NSET * KM; k += nt) {
      const int s = k / KM, l = k - s * KM;
      int n = (int)sqrt((double)l);
      n -= n * n > l ? 1 : 0;
      const int m = l - n * n - n;
      E[k] = Es[(size_t)s * stride + l] * L[(n * (n + 1) / 2 + (m < 0 ? -m : m)) * 4 + 3];
    }
  }
};

struct NoNearTables {};

template <int PMAX, bool UNROLL, int NSET>
using NearTablesFor = std::conditional_t<UNROLL, NearTables<PMAX, NSET>, NoNearTables>;

// What expansion_terms reads for one source: its coefficient sets (set s at
// E + s K), spectra rows L, the ab and cd tables and the recurrence table qt.
struct NearSourceView {
  const double* E;
  const double* L;
  const double* ab;
  const double* cd;
  const double* qt;
};

// Once per workgroup, before the first near_source: the fixed tables.
template <int PMAX, bool UNROLL, int NSET>
__device__ inline void near_tables_init(NearTablesFor<PMAX, UNROLL, NSET>& tb, const double* __restrict__ ab,
                                        const double* __restrict__ cd) {
  if constexpr (UNROLL) tb.stage_fixed(ab, cd, threadIdx.x, blockDim.x);
}

// One source's view: with the orders unrolled its sets are staged (scaled)
// in LDS between two barriers, which every wave of the workgroup reaches (all
// run the same source list); otherwise the global arrays as they are.
template <int PMAX, bool UNROLL, int NSET>
__device__ inline NearSourceView near_source(NearTablesFor<PMAX, UNROLL, NSET>& tb, bool oblate,
                                             const double* __restrict__ Ei, const double* __restrict__ Li,
                                             const double* __restrict__ ab, const double* __restrict__ cd, int K,
                                             int Kh) {
  if constexpr (UNROLL) {
    __syncthreads();  // the previous source's sets have been read
    tb.stage_source(Ei, (size_t)K, Li, threadIdx.x, blockDim.x);
    __syncthreads();
    return {tb.E, nullptr, tb.ab, tb.cd, tb.qt + (oblate ? 3 * Kh : 0)};
  } else {
    return {Ei, Li, ab, cd, nullptr};
  }
}

// A lab point in the spheroidal coordinates (u, v, phi) of source particle P
// (Table 1), from the sum of its distances to the focal points (prolate) or
// to the focal ring (oblate), 2 a cosh(mu): u = cosh(mu) resp. sinh(mu).
struct SpheroidalPoint {
  double u, w, sw;  // w = u^2 -+ 1, sw = sqrt(w)
  double v, sv;     // v and sqrt(1 - v^2)
  double c1, s1;    // cos(phi), sin(phi)
  double d[3];      // lab offset from the centre
};

// With axis_guard a point on the symmetry axis is moved off it by 1e-12 a (the
// v and phi directions of a gradient are singular there).  A point inside
// the spheroid sets kStatExterior in *bad.
__device__ inline SpheroidalPoint to_spheroidal(const Particle& P, double X0, double X1, double X2,
                                                bool axis_guard, unsigned* bad) {
  SpheroidalPoint q;
  q.d[0] = X0 - P.c[0];
  q.d[1] = X1 - P.c[1];
  q.d[2] = X2 - P.c[2];
  const double b0 = P.R[0] * q.d[0] + P.R[3] * q.d[1] + P.R[6] * q.d[2];
  const double b1 = P.R[1] * q.d[0] + P.R[4] * q.d[1] + P.R[7] * q.d[2];
  const double b2 = P.R[2] * q.d[0] + P.R[5] * q.d[1] + P.R[8] * q.d[2];
  const double a = P.a;
  const double rho0 = sqrt(b0 * b0 + b1 * b1);
  const double rho = axis_guard ? fmax(rho0, 1e-12 * a) : rho0;
  if (!P.oblate) {
    const double f1 = sqrt(rho * rho + (b2 - a) * (b2 - a));
    const double f2 = sqrt(rho * rho + (b2 + a) * (b2 + a));
    const double ch = (f1 + f2) / (2.0 * a);
    q.u = ch;
    q.w = (ch - 1.0) * (ch + 1.0);
  } else {
    const double f1 = sqrt((rho + a) * (rho + a) + b2 * b2);
    const double f2 = sqrt((rho - a) * (rho - a) + b2 * b2);
    const double ch = (f1 + f2) / (2.0 * a);
    q.u = sqrt((ch - 1.0) * (ch + 1.0));
    q.w = ch * ch;
  }
  if (!(q.u > P.u0)) *bad |= kStatExterior;
  q.sw = sqrt(q.w);
  q.v = b2 / (a * q.u);
  q.sv = rho / (a * q.sw);
  q.c1 = rho0 > 0.0 ? b0 / rho0 : 1.0;
  q.s1 = rho0 > 0.0 ? b1 / rho0 : 0.0;
  return q;
}

// The terms of an exterior expansion sum_l E[l] Q_n^|m|(u)/Q_n^|m|(u0) Y_l(v, phi)
// of one source particle at a mapped point, order by order: for every (n, m)
// with n <= p, f(lc, ls, m, a0, a1, a2, ap, b0, b1, b2, bp) receives the
// coefficient indices lc = n^2+n+m (cos(m phi)) and ls = n^2+n-m (sin(m phi),
// m > 0 only) and the basis values of the two: a0 the value, a1 its u, a2 its
// v and ap its phi derivative (b for the sine term).  L: the particle's
// spectra rows (column 3 holds 1/Q_n^m(u0)); ab, cd: normalised Ferrers
// recurrence and derivative coefficients through degree p+1; cap: the
// recurrence's step cap (near_depth).  Q and Q' come from the division-free
// backward recurrence (orders 0 and 1, then the order step).
template <int PMAX, typename F>
__device__ inline void expansion_terms(const SpheroidalPoint& q, bool oblate, const double* __restrict__ L,
                                       const double* __restrict__ ab, const double* __restrict__ cd,
                                       const double* __restrict__ rcp, int p, int cap, unsigned* bad, F&& f,
                                       bool lane_depth = false) {
  const int N1 = p + 1;
  const double u = q.u, v = q.v;
  const double inv_omv2 = 1.0 / (q.sv * q.sv);
  const double inv_w = 1.0 / q.w;
  const double sgn = oblate ? 1.0 : -1.0;
  int own = 0;
  const int Ld = near_depth(u, q.sw, N1, cap, kStatNumeric, bad, lane_depth ? &own : nullptr);
  double qn0[2], qn1[2];
  q_top_orders01(u, q.sw, sgn, N1, Ld, rcp, qn0, qn1, own);
  const double ur = u / q.sw;
  double fa2 = 0.0, fa1 = 0.0, fb2 = 0.0, fb1 = 0.0;
  double pbar = 0.28209479177387814347, cm = 1.0, sm = 0.0;
#pragma unroll 1
  for (int m = 0; m <= p; ++m) {
    if (m > 0) {
      pbar *= ab[m * (m + 3)] * q.sv;  // sqrt((2m+1)/(2m)), row n = m of the table
      const double cn = cm * q.c1 - sm * q.s1;
      sm = sm * q.c1 + cm * q.s1;
      cm = cn;
    }
    const double qN = m == 0 ? qn0[0] : (m == 1 ? qn0[1] : q_next_order(ur, N1, m, fa1, fa2));
    const double qN1 = m == 0 ? qn1[0] : (m == 1 ? qn1[1] : q_next_order(ur, N1 + 1, m, fb1, fb2));
    fa2 = fa1;
    fa1 = qN;
    fb2 = fb1;
    fb1 = qN1;
    double Q[PMAX + 4];
    q_column<PMAX>(u, sgn, N1, m, qN, qN1, rcp, Q);
    // the azimuthal factors of order m folded into the basis, so that each
    // set accumulates straight into its outputs (no per-order partial sums
    // per set: fewer registers for many sets)
    const double fm = m == 0 ? 1.0 : 1.41421356237309504880;
    const double fc = fm * cm, fs = fm * sm, fmc = (double)m * fc, fms = -(double)m * fs;
    // normalised Ferrers functions of v rolled forward in n: P_{n-1}, P_n and
    // (for the v-derivative) P_{n+1}
    double pm1 = 0.0, pn = pbar;
#pragma unroll
    for (int n = 0; n <= PMAX; ++n) {
      if (n >= m && n <= p) {
        const int h = n * (n + 1) / 2 + m;
        double pn1;
        if (n == m) {
          pn1 = ab[(m + 1) * (m + 2) + 2 * m] * v * pbar;  // sqrt(2m+3), row n = m+1
        } else {
          const int h1 = (n + 1) * (n + 2) / 2 + m;
          pn1 = ab[2 * h1] * (v * pn - ab[2 * h1 + 1] * pm1);
        }
        const double sc = L[h * 4 + 3];
        const double qr = Q[n] * sc;
        const double dq = ((-sgn) * (double)(n - m + 1) * Q[n + 1] - (double)(n + 1) * u * Q[n]) * inv_w * sc;
        const double dpn = ((double)(n + 1) * v * pn - cd[h] * pn1) * inv_omv2;
        const double t0 = pn * qr, t1 = pn * dq, t2 = dpn * qr;
        // cos(m phi) terms carry E_{n,m}, sin(m phi) terms E_{n,-m}; the
        // phi-derivative swaps them: d/dphi [c cos + s sin] = m (s cos - c sin)
        f(n * n + n + m, n * n + n - m, m, fc * t0, fc * t1, fc * t2, fms * t0, fs * t0, fs * t1, fs * t2, fmc * t0);
        pm1 = pn;
        pn = pn1;
      }
    }
  }
}

// The same expansion with the orders unrolled (p = PMAX), for kernels that
// keep per-order partial sums.  For every (n, m), m = 0 .. PMAX and
// n = m .. PMAX in ascending order, term(lc, ls, m, t0, tu, tv) receives the
// coefficient indices as above and
//   t0 = Pb_n^m(v) Q_n^m(u),  tu = Pb_n^m(v) w dQ_n^m/du,
//   tv = (1 - v^2) dPb_n^m/dv Q_n^m(u),
// without the factor 1/Q_n^m(u0) (the caller's coefficients carry it, as
// NearTables stages them) and without the azimuthal factor; after the
// degrees of order m, order_end(m, c, s) receives c = f_m cos(m phi) and
// s = f_m sin(m phi) (f_0 = 1, f_m = sqrt 2), and order_begin(m, c, s) the
// same before them.  With per-order sums
// A = sum_n E_{n,m} t and B = sum_n E_{n,-m} t an expansion adds c A + s B
// for t = t0 (its value), tu (w d/du) and tv ((1 - v^2) d/dv), and
// m (c B - s A) over t0 for d/dphi.  qt: the source kind's half of the
// three-column q_recurrence_table; ab and cd as for expansion_terms.
template <int PMAX, typename FB, typename FT, typename FO>
__device__ inline void expansion_orders(const SpheroidalPoint& q, bool oblate, const double* __restrict__ ab,
                                        const double* __restrict__ cd, const double* __restrict__ rcp,
                                        const double* __restrict__ qt, int cap, unsigned* bad, FB&& order_begin,
                                        FT&& term,
                                        FO&& order_end) {
  constexpr int N1 = PMAX + 1;
  const double u = q.u, v = q.v;
  const double sgn = oblate ? 1.0 : -1.0;
  const int Ld = near_depth(u, q.sw, N1, cap, kStatNumeric, bad);
  double qn0[2], qn1[2];
  q_top_orders01(u, q.sw, sgn, N1, Ld, rcp, qn0, qn1);
  const double ur = u / q.sw;
  double fa2 = 0.0, fa1 = 0.0, fb2 = 0.0, fb1 = 0.0;
  double pbar = 0.28209479177387814347, cm = 1.0, sm = 0.0;
  static_for<0, PMAX>([&](auto mc) {
    constexpr int m = decltype(mc)::value;
    __builtin_amdgcn_sched_barrier(0);  // orders one after the other: bounded live ranges
    if constexpr (m > 0) {
      pbar *= ab[m * (m + 3)] * q.sv;  // sqrt((2m+1)/(2m)), row n = m of the table
      const double cn = cm * q.c1 - sm * q.s1;
      sm = sm * q.c1 + cm * q.s1;
      cm = cn;
    }
    const double qN = m == 0 ? qn0[0] : (m == 1 ? qn0[1] : q_next_order(ur, N1, m, fa1, fa2));
    const double qN1 = m == 0 ? qn1[0] : (m == 1 ? qn1[1] : q_next_order(ur, N1 + 1, m, fb1, fb2));
    fa2 = fa1;
    fa1 = qN;
    fb2 = fb1;
    fb1 = qN1;
    double Q[PMAX + 4];
    q_column_tab<PMAX, 3>(u, N1, m, qN, qN1, qt, Q);
    const double fm = m == 0 ? 1.0 : 1.41421356237309504880;
    order_begin(m, fm * cm, fm * sm);
    // normalised Ferrers functions of v rolled forward in n: P_{n-1}, P_n, P_{n+1}
    double pm1 = 0.0, pn = pbar;
    static_for<m, PMAX>([&](auto nc) {
      constexpr int n = decltype(nc)::value;
      constexpr int h = n * (n + 1) / 2 + m;
      const double vp = v * pn;
      double pn1;
      if constexpr (n == m) {
        pn1 = ab[(m + 1) * (m + 2) + 2 * m] * vp;  // sqrt(2m+3), row n = m+1
      } else {
        constexpr int h1 = (n + 1) * (n + 2) / 2 + m;
        pn1 = ab[2 * h1] * fma(-ab[2 * h1 + 1], pm1, vp);
      }
      const double t0 = pn * Q[n];
      const double tu = pn * fma(qt[3 * h + 2], Q[n + 1], -(double)(n + 1) * (u * Q[n]));
      const double tv = fma(-cd[h], pn1, (double)(n + 1) * vp) * Q[n];
      term(n * n + n + m, n * n + n - m, m, t0, tu, tv);
      pm1 = pn;
      pn = pn1;
      __builtin_amdgcn_sched_barrier(0);  // a degree's loads stay after the previous degree's work
    });
    order_end(m, fm * cm, fm * sm);
  });
}

// NSET exterior expansions of one source particle at a mapped point, with
// their u, v and phi derivatives.  Es: coefficients of set s at E + s * stride.
// With lane_depth each lane's recurrence starts at its own depth.
template <int PMAX, int NSET>
__device__ inline void expansion_derivatives(const SpheroidalPoint& q, bool oblate, const double* __restrict__ E,
                                             size_t stride, const double* __restrict__ L,
                                             const double* __restrict__ ab, const double* __restrict__ cd,
                                             const double* __restrict__ rcp, int p, int cap, unsigned* bad,
                                             double (&Phi)[NSET], double (&Pu)[NSET], double (&Pv)[NSET],
                                             double (&Pp)[NSET], bool lane_depth = false) {
#pragma unroll
  for (int s = 0; s < NSET; ++s) Phi[s] = Pu[s] = Pv[s] = Pp[s] = 0.0;
  expansion_terms<PMAX>(q, oblate, L, ab, cd, rcp, p, cap, bad,
                        [&](int lc, int ls, int m, double a0, double a1, double a2, double ap, double b0, double b1,
                            double b2, double bp) {
#pragma unroll
                          for (int s = 0; s < NSET; ++s) {
                            const double ec = E[(size_t)s * stride + lc];
                            Phi[s] = fma(ec, a0, Phi[s]);
                            Pu[s] = fma(ec, a1, Pu[s]);
                            Pv[s] = fma(ec, a2, Pv[s]);
                            Pp[s] = fma(ec, ap, Pp[s]);
                            if (m > 0) {
                              const double es = E[(size_t)s * stride + ls];
                              Phi[s] = fma(es, b0, Phi[s]);
                              Pu[s] = fma(es, b1, Pu[s]);
                              Pv[s] = fma(es, b2, Pv[s]);
                              Pp[s] = fma(es, bp, Pp[s]);
                            }
                          }
                        },
                        lane_depth);
}

// The chain rule of lab_gradient as coefficients: the lab gradient of an
// expansion is g_r = al[r] Pu + be[r] Pv + ga[r] Pp.
__device__ inline void lab_gradient_coeffs(const Particle& P, double u, double su, double v, double sv, double c1,
                                           double s1, double al[3], double be[3], double ga[3]) {
  const double a = P.a;
  const double xu[3] = {a * u / su * sv * c1, a * u / su * sv * s1, a * v};
  const double xv[3] = {-a * su * v / sv * c1, -a * su * v / sv * s1, a * u};
  const double xp[3] = {-a * su * sv * s1, a * su * sv * c1, 0.0};
  const double hu2 = xu[0] * xu[0] + xu[1] * xu[1] + xu[2] * xu[2];
  const double hv2 = xv[0] * xv[0] + xv[1] * xv[1] + xv[2] * xv[2];
  const double hp2 = xp[0] * xp[0] + xp[1] * xp[1] + xp[2] * xp[2];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    al[r] = (P.R[3 * r] * xu[0] + P.R[3 * r + 1] * xu[1] + P.R[3 * r + 2] * xu[2]) / hu2;
    be[r] = (P.R[3 * r] * xv[0] + P.R[3 * r + 1] * xv[1] + P.R[3 * r + 2] * xv[2]) / hv2;
    ga[r] = (P.R[3 * r] * xp[0] + P.R[3 * r + 1] * xp[1]) / hp2;
  }
}

// Lab-frame gradient from the derivatives in (u, v, phi): the chain rule for
// the orthogonal coordinates of Table 1 in the body frame, rotated to the lab.
__device__ inline void lab_gradient(const Particle& P, double u, double su, double v, double sv, double c1,
                                    double s1, double Pu, double Pv, double Pp, double g[3]) {
  const double a = P.a;
  const double xu[3] = {a * u / su * sv * c1, a * u / su * sv * s1, a * v};
  const double xv[3] = {-a * su * v / sv * c1, -a * su * v / sv * s1, a * u};
  const double xp[3] = {-a * su * sv * s1, a * su * sv * c1, 0.0};
  const double hu2 = xu[0] * xu[0] + xu[1] * xu[1] + xu[2] * xu[2];
  const double hv2 = xv[0] * xv[0] + xv[1] * xv[1] + xv[2] * xv[2];
  const double hp2 = xp[0] * xp[0] + xp[1] * xp[1] + xp[2] * xp[2];
  const double fu = Pu / hu2, fv = Pv / hv2, fp = Pp / hp2;
  const double gb[3] = {xu[0] * fu + xv[0] * fv + xp[0] * fp, xu[1] * fu + xv[1] * fv + xp[1] * fp,
                        xu[2] * fu + xv[2] * fv};
#pragma unroll
  for (int r = 0; r < 3; ++r) g[r] = P.R[3 * r] * gb[0] + P.R[3 * r + 1] * gb[1] + P.R[3 * r + 2] * gb[2];
}

}  // namespace sbie
