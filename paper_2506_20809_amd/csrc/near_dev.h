// Legendre functions of the second kind for the near-field exterior
// expansions (Section 2.3, "Legendre function evaluation"; Theorems 1 and 2,
// exterior rows), shared by the Laplace and Stokes near-field kernels.  Real
// forms: prolate Q_n^m(u), oblate q_n^m(u) = i^(n+1) Q_n^m(iu); w = u^2 -+ 1,
// sgn = -1 (prolate) or +1 (oblate), N = p + 1.
#pragma once

#include <hip/hip_runtime.h>

namespace sbie {

// Depth L of the backward recurrence: the ratio of the minimal to the
// dominant solution shrinks by (u + sqrt(w))^-2 per degree; 2^-58 plus a
// margin, the largest over the wave (wave-uniform), in whole chunks of eight
// steps; past 1e5 steps the depth is capped and numeric_flag is set in *bad.
__device__ inline int near_depth(double u, double sw, int N, unsigned numeric_flag, unsigned* bad) {
  int steps = (int)ceil(20.1 / log(u + sw)) + 8;
  for (int off = 32; off >= 1; off >>= 1) steps = max(steps, __shfl_xor(steps, off, 64));
  steps = __builtin_amdgcn_readfirstlane(steps);
  if (steps > 100000) {
    steps = 100000;
    *bad |= numeric_flag;
  }
  steps = (steps + 7) & ~7;
  return N + steps;
}

// Q_N^m and Q_{N+1}^m for m = 0 and 1.  The minimal solution of the
// recurrence in n comes from backward recurrence from degree L (the continued
// fraction for Q_N/Q_{N-1} evaluated bottom-up), free of divisions with
// Q_n = s_n R_n and s_{n-1} = s_n/(n+m):
//   R_{n-1} = (2n+1) u R_n -+ ((n+1)^2 - m^2) R_{n+1},
// rescaled by 2^-600 whenever it grows past 2^600; the Casoratian at degree N
// against the forward P (division-free as Pt_n = (n-m)! P_n^m),
//   Pt_N Q_{N-1} -+ (N-m) Pt_{N-1} Q_N = (-1)^m (N+m-1)!,
// fixes the scale.  rcp[k] = 1/k.
__device__ inline void q_top_orders01(double u, double sw, double sgn, int N, int L, const double* __restrict__ rcp,
                                      double qN[2], double qN1[2]) {
  double qh[2] = {0.0, 0.0}, qc[2] = {1.0, 1.0};
  const double smsq[2] = {0.0, sgn};
  double c2n1 = (double)(2 * L + 1), snp = sgn * (double)(L + 1) * (double)(L + 1), sc = sgn * c2n1;
  const double dsc = -2.0 * sgn;
  for (int n = L; n > N; n -= 8) {
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

}  // namespace sbie
