// Associated Legendre functions off the cut, in real arithmetic, for the
// device (Section 2.3, "Legendre function evaluation").
//
// Prolate (x = u > 1): P_n^m(x), Q_n^m(x) of type 3.
// Oblate (z = i u, u > 0): the real functions p_n(u) = i^{-n} P_n^m(iu) and
// q_n(u) = i^{n+1} Q_n^m(iu).  Substituting into the recurrences of
// Section 2.3 gives
//   (n-m+1) p_{n+1} = (2n+1) u p_n + (n+m) p_{n-1},   p_m = (2m-1)!! (u^2+1)^{m/2},
//   (n-m+1) q_{n+1} = (n+m) q_{n-1} - (2n+1) u q_n,
//   Casoratian  p_n q_{n-1} + p_{n-1} q_n = (-1)^m (n+m-1)!/(n-m)!,
//   derivative  (u^2+1) p_n' = (n-m+1) p_{n+1} - (n+1) u p_n,
//               (u^2+1) q_n' = (m-n-1) q_{n+1} - (n+1) u q_n.
// The prolate derivative identity reads (u^2-1) F_n' = (n-m+1) F_{n+1} - (n+1) u F_n.
#pragma once

#include <hip/hip_runtime.h>

namespace sbie {

// Modified Lentz evaluation of f = a_N / (b_N + a_{N+1} / (b_{N+1} + ...)) with
//   prolate: a_k = -(k+m)/(k-m+1), b_k = -(2k+1) u/(k-m+1)   (f = Q_N/Q_{N-1})
//   oblate:  a_k =  (k+m)/(k-m+1), b_k =  (2k+1) u/(k-m+1)   (f = q_N/q_{N-1})
// Returns false when max_iter terms did not converge.
__device__ inline bool lentz_ratio(bool oblate, double u, int m, int N, int max_iter,
                                   double* out) {
  const double tiny = 1e-300;
  const double sgn = oblate ? 1.0 : -1.0;
  double f = tiny, C = tiny, D = 0.0;
  for (int it = 0, k = N; it < max_iter; ++it, ++k) {
    const double inv = 1.0 / (double)(k - m + 1);
    const double a = sgn * (double)(k + m) * inv;
    const double b = sgn * (double)(2 * k + 1) * u * inv;
    D = fma(a, D, b);
    if (D == 0.0) D = tiny;
    D = 1.0 / D;
    C = b + a / C;
    if (C == 0.0) C = tiny;
    const double delta = C * D;
    f *= delta;
    if (fabs(delta - 1.0) <= 2.3e-16) {
      *out = f;
      return true;
    }
  }
  *out = f;
  return false;
}

// Values for one order m at argument u: P[n], Q[n] for n = m..N and derivative
// values w0*P'[n], w0*Q'[n] (w0 = u^2 -+ 1) for n = m..N-1, written into
// arrays indexed by degree (size >= N+2).  Returns false on CF failure.
__device__ inline bool legendre_column(bool oblate, double u, int m, int N, int max_iter,
                                       double* P, double* Q, double* wdP, double* wdQ) {
  const double w = oblate ? fma(u, u, 1.0) : fma(u, u, -1.0);
  const double sw = sqrt(w);
  const double sgn = oblate ? 1.0 : -1.0;  // sign of the (n+m) term in the P recurrence
  double pmm = 1.0;
  for (int k = 1; k <= m; ++k) pmm *= (double)(2 * k - 1) * sw;
  P[m] = pmm;
  P[m + 1] = (double)(2 * m + 1) * u * pmm;
  for (int n = m + 1; n <= N; ++n)
    P[n + 1] = ((double)(2 * n + 1) * u * P[n] + sgn * (double)(n + m) * P[n - 1]) /
               (double)(n - m + 1);
  double H;
  if (!lentz_ratio(oblate, u, m, N, max_iter, &H)) return false;
  // Casoratian constant (-1)^m (N+m-1)!/(N-m)!  (1/N for m = 0)
  double cas = 1.0 / (double)N;
  for (int k = 1; k <= m; ++k) cas *= (double)(N + k - 1) * (double)(N - k + 1);
  if (m & 1) cas = -cas;
  const double den = oblate ? fma(H, P[N - 1], P[N]) : fma(-H, P[N - 1], P[N]);
  Q[N - 1] = cas / den;
  Q[N] = H * Q[N - 1];
  for (int n = N - 1; n >= m + 1; --n) {
    if (!oblate)
      Q[n - 1] = ((double)(2 * n + 1) * u * Q[n] - (double)(n - m + 1) * Q[n + 1]) / (double)(n + m);
    else
      Q[n - 1] = ((double)(n - m + 1) * Q[n + 1] + (double)(2 * n + 1) * u * Q[n]) / (double)(n + m);
  }
  for (int n = m; n <= N - 1; ++n) {
    if (!oblate) {
      wdP[n] = (double)(n - m + 1) * P[n + 1] - (double)(n + 1) * u * P[n];
      wdQ[n] = (double)(n - m + 1) * Q[n + 1] - (double)(n + 1) * u * Q[n];
    } else {
      wdP[n] = (double)(n - m + 1) * P[n + 1] - (double)(n + 1) * u * P[n];
      wdQ[n] = -(double)(n - m + 1) * Q[n + 1] - (double)(n + 1) * u * Q[n];
    }
  }
  return true;
}

}  // namespace sbie
