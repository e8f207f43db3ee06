// Stokes single layer through Laplace single layers (Section 4.3, Eq. (stokes)),
// viscosity 1:
//   u_k = 1/2 { S[sigma_k] - sum_j (x - c)_j d_k S[sigma_j] + d_k S[(y - c).sigma] }
// The identity holds for any origin c; each source particle uses its own
// centre, which keeps the three terms of the same size.  Per source particle
// there are four single-layer expansions (the three density components and
// rho = (y - c).sigma).  Self: values and exterior-limit gradients at the
// particle's own nodes (the gradient jump -f nu cancels in the combination);
// near: values and gradients of the neighbours' exterior expansions; far: the
// Stokeslet (1/8pi)(I/r + r r^T/r^3) by smooth quadrature (Section 4.3).
// With C = 4 components the pressure of the Stokeslet, kernel (1/4pi) r/r^3
// (r = x - y), follows as a fourth one: p = -sum_j d_j S[sigma_j] (the printed
// identity sum_j e_j . grad S[sigma_j] has the opposite sign); on the surface
// its exterior limit (the gradients' exterior limits).
#include <hip/hip_runtime.h>

#include <cmath>

#include "near_dev.h"
#include "sbie_internal.h"

namespace sbie {

namespace {

constexpr double kInv8Pi = 0.039788735772973833942220940843128591;
constexpr double kInv4Pi = 0.079577471545947667884441881686257181;

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

// Transform inputs of the four expansions (modified basis of Section 3.2:
// sqrt(u0^2 -+ v^2) times the density) and the far-field records
// (node - centre, W sigma).
template <typename R>
__global__ void k_stokes_prep(const Particle* __restrict__ part, const double* __restrict__ dens,
                              const double* __restrict__ x, const double* __restrict__ y,
                              const double* __restrict__ z, const double* __restrict__ w,
                              const double* __restrict__ wS, int p, int64_t N, double* __restrict__ f,
                              R* __restrict__ rec) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  const int Nphi = 2 * p + 2, T = (p + 1) * Nphi;
  const int i = (int)(g / T), t = (int)(g - (int64_t)i * T), j = t / Nphi;
  const double s0 = dens[g], s1 = dens[N + g], s2 = dens[2 * N + g];
  const double ox = x[g] - part[i].c[0], oy = y[g] - part[i].c[1], oz = z[g] - part[i].c[2];
  const double ws = wS[(size_t)i * (p + 1) + j];
  double* fr = f + (size_t)i * 4 * T + t;
  fr[0] = ws * s0;
  fr[T] = ws * s1;
  fr[2 * T] = ws * s2;
  fr[3 * T] = ws * fma(oz, s2, fma(oy, s1, ox * s0));
  const double wq = w[g];
  R* r = rec + 8 * g;
  r[0] = (R)ox;
  r[1] = (R)oy;
  r[2] = (R)oz;
  r[3] = (R)(wq * s0);
  r[4] = (R)(wq * s1);
  r[5] = (R)(wq * s2);
  r[6] = R(0);
  r[7] = R(0);
}

// E = lamS c (exterior single-layer coefficients) and Eu = E dR/du(u0).
__global__ void k_stokes_scale(const double* __restrict__ coef, const double* __restrict__ lam,
                               const double* __restrict__ dlr, int M, int p, double* __restrict__ E,
                               double* __restrict__ Eu) {
  const int K = (p + 1) * (p + 1), Kh = (p + 1) * (p + 2) / 2;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)4 * M * K) return;
  const int row = (int)(t / K), l = (int)(t - (int64_t)row * K);
  const int i = row / 4;
  const int n = (int)sqrt((double)l);
  const int m = l - n * n - n;
  const int h = n * (n + 1) / 2 + (m < 0 ? -m : m);
  const double e = lam[((size_t)i * Kh + h) * 4 + 2] * coef[t];
  E[t] = e;
  Eu[t] = e * dlr[(size_t)i * Kh + h];
}

// Cartesian (lab) gradients of the four expansions from their derivatives in
// (u, v, phi) and the combination of Eq. (stokes); with C = 4 also the
// pressure -sum_j d_j S[sigma_j] in out[3].  d = x - c (lab).
template <int C>
__device__ inline void stokes_from_derivatives(const Particle& P, double u, double su, double v, double sv,
                                               double c1, double s1, const double* Phi, const double* Pu,
                                               const double* Pv, const double* Pp, const double d[3],
                                               double (&out)[C]) {
  double grad[4][3];
#pragma unroll
  for (int s = 0; s < 4; ++s) lab_gradient(P, u, su, v, sv, c1, s1, Pu[s], Pv[s], Pp[s], grad[s]);
#pragma unroll
  for (int k = 0; k < 3; ++k)
    out[k] = 0.5 * (Phi[k] - d[0] * grad[0][k] - d[1] * grad[1][k] - d[2] * grad[2][k] + grad[3][k]);
  if constexpr (C == 4) out[3] = -(grad[0][0] + grad[1][1] + grad[2][2]);
}

// Self part at node g of particle i from the synthesised values U[0..3]
// (value, d/du exterior limit, d/dv, d/dphi) of the four expansions.
template <int C>
__global__ void k_stokes_self(const Particle* __restrict__ part, const double* __restrict__ gl,
                              const double* __restrict__ x, const double* __restrict__ y,
                              const double* __restrict__ z, const double* __restrict__ U, int M, int p,
                              int64_t N, double* __restrict__ out) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  const int Nphi = 2 * p + 2, T = (p + 1) * Nphi;
  const int i = (int)(g / T), t = (int)(g - (int64_t)i * T), j = t / Nphi, k = t - j * Nphi;
  const Particle P = part[i];
  const size_t plane = (size_t)4 * M * T;
  double Phi[4], Pu[4], Pv[4], Pp[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const size_t o = ((size_t)i * 4 + s) * T + t;
    Phi[s] = U[o];
    Pu[s] = U[plane + o];
    Pv[s] = U[2 * plane + o];
    Pp[s] = U[3 * plane + o];
  }
  const double v = gl[j];
  double s1, c1;
  sincospi(2.0 * k / Nphi, &s1, &c1);
  const double d[3] = {x[g] - P.c[0], y[g] - P.c[1], z[g] - P.c[2]};
  double o[C];
  stokes_from_derivatives<C>(P, P.u0, sqrt(P.w0), v, sqrt((1.0 - v) * (1.0 + v)), c1, s1, Phi, Pu, Pv, Pp, d, o);
#pragma unroll
  for (int c = 0; c < C; ++c) out[c * N + g] = o[c];
}

// Near part: one wave per (target particle, 64 target nodes); for every near
// source the target is mapped into the source frame, Q_n^m(u) and Q_n^m'(u)
// come from the same division-free backward recurrence as the Laplace near
// field, and the four expansions are summed with their u, v and phi
// derivatives.
template <int PMAX, bool EXACT, int C>
__global__ __launch_bounds__((64 * kNearWaves<kUnrollOrders<PMAX, EXACT>>)) __attribute__((amdgpu_waves_per_eu(3))) void k_near_stokes(
    const Particle* __restrict__ part, const double* __restrict__ x, const double* __restrict__ y,
    const double* __restrict__ z, const int32_t* __restrict__ near_ptr, const int32_t* __restrict__ near_src,
    const double* __restrict__ E, const double* __restrict__ lam, const double* __restrict__ ab,
    const double* __restrict__ cd, const double* __restrict__ rcp, int p_arg, int T, int chunks, int64_t N,
    unsigned* status, double* __restrict__ unear) {
  const int p = EXACT ? PMAX : p_arg;  // exact order: degree bounds known at compile time
  // one workgroup per (target particle, 64 W targets, range q of its
  // near-source list)
  constexpr int W = kNearWaves<kUnrollOrders<PMAX, EXACT>>;
  const int wgs = (chunks + W - 1) / W;
  const int q = blockIdx.x % kStokesNearSplit, rest = blockIdx.x / kStokesNearSplit;
  const int j = rest / wgs;
  const int t = (rest - j * wgs) * 64 * W + threadIdx.x;
  const bool live = t < T;
  const int64_t g = (int64_t)j * T + (live ? t : 0);
  const double X0 = x[g], X1 = y[g], X2 = z[g];
  const int K = (p + 1) * (p + 1), Kh = (p + 1) * (p + 2) / 2;
  __shared__ NearTablesFor<PMAX, kUnrollOrders<PMAX, EXACT>, 4> tb;
  near_tables_init<PMAX, kUnrollOrders<PMAX, EXACT>, 4>(tb, ab, cd);
  double acc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) acc[c] = 0.0;
  unsigned bad = 0u;
  const int cap = (int)status[1];  // the geometry's recurrence step cap
  const int n0 = near_ptr[j], nn = near_ptr[j + 1] - n0;
  const int s_begin = n0 + (nn * q) / kStokesNearSplit, s_end = n0 + (nn * (q + 1)) / kStokesNearSplit;
  for (int sidx = s_begin; sidx < s_end; ++sidx) {
    const int i = near_src[sidx];
    const Particle P = part[i];
    const SpheroidalPoint sp = to_spheroidal(P, X0, X1, X2, true, &bad);
    const NearSourceView src =
        near_source<PMAX, kUnrollOrders<PMAX, EXACT>, 4>(tb, P.oblate != 0, E + (size_t)i * 4 * K, lam + (size_t)i * Kh * 4, ab, cd, K, Kh);
    const double* Ei = src.E;
    // Eq. (stokes) is linear in the four expansions, so it is taken inside the
    // sum over (n, m), one basis evaluation for all of them: the values of
    // S[sigma_k]; grad (S[rho] - sum_j d_j S[sigma_j]) as the gradient of one
    // expansion with coefficients E3 - d.(E0, E1, E2) (d fixed at the
    // target); for the pressure -sum_j d_j S[sigma_j], one lab derivative of
    // each of the first three sets (the chain rule's coefficients applied to
    // the basis derivatives).
    double al[3], be[3], ga[3];
    lab_gradient_coeffs(P, sp.u, sp.sw, sp.v, sp.sv, sp.c1, sp.s1, al, be, ga);
    const double w0 = -sp.d[0], w1 = -sp.d[1], w2 = -sp.d[2];
    double Phi[3] = {0.0, 0.0, 0.0}, Gu = 0.0, Gv = 0.0, Gp = 0.0, pr = 0.0;
    if constexpr (kUnrollOrders<PMAX, EXACT>) {
      // per-order sums over n of the cosine (c) and sine (s) terms: values of
      // the three sets (v), the combined expansion's scaled derivatives (g)
      // and, for the pressure, the three sets' scaled u and v derivatives
      // (du, dv); folded with the azimuthal factors at the end of each order
      double vc[3] = {0.0, 0.0, 0.0}, vs[3] = {0.0, 0.0, 0.0};
      double guc = 0.0, gus = 0.0, gvc = 0.0, gvs = 0.0, g0c = 0.0, g0s = 0.0;
      double duc[3] = {0.0, 0.0, 0.0}, dus[3] = {0.0, 0.0, 0.0}, dvc[3] = {0.0, 0.0, 0.0}, dvs[3] = {0.0, 0.0, 0.0};
      double Pu[3] = {0.0, 0.0, 0.0}, Pv[3] = {0.0, 0.0, 0.0}, Pp[3] = {0.0, 0.0, 0.0};
      expansion_orders<PMAX>(
          sp, P.oblate != 0, src.ab, src.cd, rcp, src.qt, cap, &bad, [](int, double, double) {},
          [&](int lc, int ls, int m, double t0, double tu, double tv) {
            double e[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) e[k] = Ei[(size_t)k * K + lc];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
              vc[k] = fma(e[k], t0, vc[k]);
              if constexpr (C == 4) {
                duc[k] = fma(e[k], tu, duc[k]);
                dvc[k] = fma(e[k], tv, dvc[k]);
              }
            }
            const double fc = fma(w2, e[2], fma(w1, e[1], fma(w0, e[0], e[3])));
            guc = fma(fc, tu, guc);
            gvc = fma(fc, tv, gvc);
            g0c = fma(fc, t0, g0c);
            if (m > 0) {
#pragma unroll
              for (int k = 0; k < 4; ++k) e[k] = Ei[(size_t)k * K + ls];
#pragma unroll
              for (int k = 0; k < 3; ++k) {
                vs[k] = fma(e[k], t0, vs[k]);
                if constexpr (C == 4) {
                  dus[k] = fma(e[k], tu, dus[k]);
                  dvs[k] = fma(e[k], tv, dvs[k]);
                }
              }
              const double fs = fma(w2, e[2], fma(w1, e[1], fma(w0, e[0], e[3])));
              gus = fma(fs, tu, gus);
              gvs = fma(fs, tv, gvs);
              g0s = fma(fs, t0, g0s);
            }
          },
          [&](int m, double c, double s) {
            const double dm = (double)m;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
              Phi[k] = fma(c, vc[k], fma(s, vs[k], Phi[k]));
              if constexpr (C == 4) {
                Pu[k] = fma(c, duc[k], fma(s, dus[k], Pu[k]));
                Pv[k] = fma(c, dvc[k], fma(s, dvs[k], Pv[k]));
                Pp[k] = fma(dm, fma(c, vs[k], -s * vc[k]), Pp[k]);
                duc[k] = dus[k] = dvc[k] = dvs[k] = 0.0;
              }
              vc[k] = vs[k] = 0.0;
            }
            Gu = fma(c, guc, fma(s, gus, Gu));
            Gv = fma(c, gvc, fma(s, gvs, Gv));
            Gp = fma(dm, fma(c, g0s, -s * g0c), Gp);
            guc = gus = gvc = gvs = g0c = g0s = 0.0;
          });
      const double iw = 1.0 / sp.w, iv = 1.0 / (sp.sv * sp.sv);
      Gu *= iw;
      Gv *= iv;
      if constexpr (C == 4) {
#pragma unroll
        for (int k = 0; k < 3; ++k) pr -= fma(ga[k], Pp[k], fma(be[k], Pv[k] * iv, al[k] * (Pu[k] * iw)));
      }
    } else {
    expansion_terms<PMAX>(sp, P.oblate != 0, src.L, src.ab, src.cd, rcp, p, cap, &bad,
                          [&](int lc, int ls, int m, double a0, double a1, double a2, double ap, double b0,
                              double b1, double b2, double bp) {
#pragma unroll
                            for (int k = 0; k < 3; ++k) Phi[k] = fma(Ei[(size_t)k * K + lc], a0, Phi[k]);
                            const double fc = fma(w2, Ei[2 * K + lc], fma(w1, Ei[K + lc], fma(w0, Ei[lc], Ei[3 * K + lc])));
                            Gu = fma(fc, a1, Gu);
                            Gv = fma(fc, a2, Gv);
                            Gp = fma(fc, ap, Gp);
                            if constexpr (C == 4) {
#pragma unroll
                              for (int j = 0; j < 3; ++j)
                                pr = fma(Ei[(size_t)j * K + lc], -fma(ga[j], ap, fma(be[j], a2, al[j] * a1)), pr);
                            }
                            if (m > 0) {
#pragma unroll
                              for (int k = 0; k < 3; ++k) Phi[k] = fma(Ei[(size_t)k * K + ls], b0, Phi[k]);
                              const double fs =
                                  fma(w2, Ei[2 * K + ls], fma(w1, Ei[K + ls], fma(w0, Ei[ls], Ei[3 * K + ls])));
                              Gu = fma(fs, b1, Gu);
                              Gv = fma(fs, b2, Gv);
                              Gp = fma(fs, bp, Gp);
                              if constexpr (C == 4) {
#pragma unroll
                                for (int j = 0; j < 3; ++j)
                                  pr = fma(Ei[(size_t)j * K + ls], -fma(ga[j], bp, fma(be[j], b2, al[j] * b1)), pr);
                              }
                            }
                          });
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) acc[k] += 0.5 * (Phi[k] + fma(ga[k], Gp, fma(be[k], Gv, al[k] * Gu)));
    if constexpr (C == 4) acc[3] += pr;
  }
  if (bad) atomicOr(status, bad);
  if (live) {
#pragma unroll
    for (int c = 0; c < C; ++c) unear[((size_t)q * C + c) * N + g] = acc[c];
  }
}

template <typename R>
__device__ inline R rsq_r(R x);
template <>
__device__ inline float rsq_r<float>(float x) {
  return __builtin_amdgcn_rsqf(x);
}
template <>
__device__ inline double rsq_r<double>(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double e = fma(-x * y, y, 1.0);
  y = fma(0.5 * y, e, y);
  e = fma(-x * y, y, 1.0);
  return fma(0.5 * y, e, y);
}

// Far part: the Stokeslet summed over the far source nodes.  Grid as the
// Laplace far field (target tiles x source splits, split fastest); source
// records (node - centre, W sigma) are read with wave-uniform addresses; each
// source particle's tile sum is added per target under the exclusion flag,
// compensated (TwoSum) in FP32.
template <typename R, int TPT, int C>
__global__ __launch_bounds__(256) void k_far_stokes(const R* __restrict__ rec, const Particle* __restrict__ part,
                                                    const double* __restrict__ x, const double* __restrict__ y,
                                                    const double* __restrict__ z, const uint32_t* __restrict__ excl,
                                                    int words, int M, int T, int64_t N, int nsplit,
                                                    double* __restrict__ partial) {
  const int split = blockIdx.x % nsplit, tile = blockIdx.x / nsplit;
  const int s0 = (int)((int64_t)M * split / nsplit), s1 = (int)((int64_t)M * (split + 1) / nsplit);
  double tx[TPT], ty[TPT], tz[TPT];
  int tp[TPT];
  bool live[TPT];
  R acc[TPT][C], lo[TPT][C];
#pragma unroll
  for (int k = 0; k < TPT; ++k) {
    const int64_t gq = (int64_t)tile * 256 * TPT + k * 256 + threadIdx.x;
    live[k] = gq < N;
    const int64_t gg = live[k] ? gq : 0;
    tx[k] = x[gg];
    ty[k] = y[gg];
    tz[k] = z[gg];
    tp[k] = (int)(gg / T);
#pragma unroll
    for (int c = 0; c < C; ++c) acc[k][c] = lo[k][c] = R(0);
  }
  for (int s = s0; s < s1; ++s) {
    bool need[TPT];
    bool any = false;
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
      need[k] = live[k] && !((excl[(size_t)tp[k] * words + (s >> 5)] >> (s & 31)) & 1u);
      any |= need[k];
    }
    if (!__any(any)) continue;
    const double cx = part[s].c[0], cy = part[s].c[1], cz = part[s].c[2];
    R Dx[TPT], Dy[TPT], Dz[TPT], tmp[TPT][C];
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
      Dx[k] = (R)(tx[k] - cx);
      Dy[k] = (R)(ty[k] - cy);
      Dz[k] = (R)(tz[k] - cz);
#pragma unroll
      for (int c = 0; c < C; ++c) tmp[k][c] = R(0);
    }
    const R* rs = rec + (size_t)s * T * 8;
    for (int q = 0; q < T; ++q) {
      const R* r = rs + (size_t)q * 8;
      const R ox = r[0], oy = r[1], oz = r[2], q0 = r[3], q1 = r[4], q2 = r[5];
#pragma unroll
      for (int k = 0; k < TPT; ++k) {
        const R dx = Dx[k] - ox, dy = Dy[k] - oy, dz = Dz[k] - oz;
        const R r2 = fma(dz, dz, fma(dy, dy, dx * dx));
        const R ri = rsq_r<R>(r2);
        const R dot = fma(dz, q2, fma(dy, q1, dx * q0));
        const R f = dot * ri * ri * ri;
        tmp[k][0] = fma(q0, ri, fma(dx, f, tmp[k][0]));
        tmp[k][1] = fma(q1, ri, fma(dy, f, tmp[k][1]));
        tmp[k][2] = fma(q2, ri, fma(dz, f, tmp[k][2]));
        if constexpr (C == 4) tmp[k][3] += f;  // pressure: (r.q)/r^3, scaled by 1/(4 pi) below
      }
    }
#pragma unroll
    for (int k = 0; k < TPT; ++k)
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const R vv = need[k] ? tmp[k][c] : R(0);
        const R sum = acc[k][c] + vv;
        const R bp = sum - acc[k][c];
        lo[k][c] += (acc[k][c] - (sum - bp)) + (vv - bp);
        acc[k][c] = sum;
      }
  }
#pragma unroll
  for (int k = 0; k < TPT; ++k) {
    const int64_t gq = (int64_t)tile * 256 * TPT + k * 256 + threadIdx.x;
    if (!live[k]) continue;
#pragma unroll
    for (int c = 0; c < C; ++c)
      partial[((size_t)split * C + c) * N + gq] = ((double)acc[k][c] + (double)lo[k][c]) * (c < 3 ? kInv8Pi : kInv4Pi);
  }
}

// u = self + near slices + far slices in order (+ the pair kernel's running
// reverse totals racc [C][N], 1/8pi resp. 1/4pi applied here, when set).
template <int C>
__global__ void k_stokes_assemble(const double* __restrict__ uself, const double* __restrict__ unear,
                                  const double* __restrict__ partial, int nsplit, const double* __restrict__ racc,
                                  int64_t N, uint32_t parts, double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= C * N) return;
  const int c = (int)(t / N);
  const int64_t g = t - (int64_t)c * N;
  double u = 0.0;
  if (parts & SBIE_PARTS_SELF) u += uself[t];
  if (parts & SBIE_PARTS_NEAR)
    for (int q = 0; q < kStokesNearSplit; ++q) u += unear[(size_t)q * C * N + t];
  if (parts & SBIE_PARTS_FAR) {
    double f = 0.0;
    for (int s = 0; s < nsplit; ++s) f += partial[((size_t)s * C + c) * N + g];
    if (racc) f += racc[t] * (c < 3 ? kInv8Pi : kInv4Pi);
    u += f;
  }
  out[t] = u;
}

template <int PMAX, bool EXACT, int C>
void launch_near_stokes(sbie_geom* g, hipStream_t s) {
  const int chunks = (g->T + 63) / 64;
  constexpr int W = kNearWaves<kUnrollOrders<PMAX, EXACT>>;
  hipLaunchKernelGGL((k_near_stokes<PMAX, EXACT, C>), dim3(g->M * ((chunks + W - 1) / W) * kStokesNearSplit),
                     dim3(64 * W), 0, s, g->d_part, g->d_x, g->d_y, g->d_z,
                     g->d_near_ptr, g->d_near_src, g->d_stk_E, g->d_lam, g->d_ab, g->d_cd, g->d_rcp, g->p, g->T,
                     chunks, g->N, g->d_status, g->d_stk_near);
}

}  // namespace

#define SBIE_TRY_C(expr)            \
  do {                              \
    sbie_status _s = (expr);        \
    if (_s != SBIE_OK) return _s;   \
  } while (0)

sbie_status carve_stokes(sbie_geom* g, Carver& c) {
  const size_t MT4 = (size_t)4 * g->M * g->T, MK4 = (size_t)4 * g->M * g->K;
  const size_t N = (size_t)g->N;
  SBIE_TRY_C(c.take(&g->d_stk_f, MT4));
  SBIE_TRY_C(c.take(&g->d_stk_c, MK4));
  SBIE_TRY_C(c.take(&g->d_stk_E, 2 * MK4));
  SBIE_TRY_C(c.take(&g->d_stk_U, 4 * MT4));
  SBIE_TRY_C(c.take(&g->d_stk_src, 8 * N));
  // four components: velocity and pressure
  SBIE_TRY_C(c.take(&g->d_stk_part, (size_t)g->nsplit * 4 * N));
  SBIE_TRY_C(c.take(&g->d_stk_self, 4 * N));
  SBIE_TRY_C(c.take(&g->d_stk_near, (size_t)kStokesNearSplit * 4 * N));
  SBIE_TRY_C(c.take(&g->d_stk_io, 7 * N));
  // the pair kernel's source blocks, reverse sums and totals
  const size_t nb = (size_t)(g->T + 15) / 16;
  g->stk_rev_bytes = stokes_rev_bytes(g->M, g->T);
  SBIE_TRY_C(c.take(&g->d_stk_prec, (size_t)g->M * nb * stokes_record_doubles(false)));
  SBIE_TRY_C(c.take(&g->d_stk_rev, (size_t)(g->stk_rev_bytes / sizeof(double))));
  SBIE_TRY_C(c.take(&g->d_stk_racc, 4 * N));
  return SBIE_OK;
}

sbie_status stokes_buffers(sbie_geom* g) {
  if (g->stokes_ready) return SBIE_OK;
  Carver measure;
  SBIE_TRY_C(carve_stokes(g, measure));
  const size_t bytes = (measure.used + 255) & ~size_t(255);
  Carver c;
  const size_t start = (g->blk_used + 255) & ~size_t(255);
  if (g->blk && g->blk_bytes >= start + bytes) {
    // room reserved in the geometry's block, after its own buffers
    c.base = g->blk + start;
    c.size = g->blk_bytes - start;
  } else {
    hipError_t e = hipMalloc((void**)&g->stk_blk, bytes);
    if (e != hipSuccess) {
      g->stk_blk = nullptr;
      (void)hipGetLastError();
      set_error("device allocation of the Stokes work buffers failed");
      return SBIE_E_NOMEM;
    }
    g->footprint += bytes;
    c.base = g->stk_blk;
    c.size = bytes;
  }
  SBIE_TRY_C(carve_stokes(g, c));
  g->stokes_ready = true;
  return SBIE_OK;
}

sbie_status stokes_staging(sbie_geom* g, double** io) {
  SBIE_TRY_C(stokes_buffers(g));
  *io = g->d_stk_io;
  return SBIE_OK;
}

namespace {

template <int C>
sbie_status stokes_parts(sbie_geom* g, bool mixed, hipStream_t s, uint32_t parts, hipEvent_t* ev,
                         const double* d_dens, double* d_out);

}  // namespace

sbie_status apply_stokes(sbie_geom* g, int prec, const double* d_dens, double* d_out, hipStream_t s,
                         uint32_t parts, bool timed, bool pressure) {
  const int M = g->M, p = g->p, T = g->T, K = g->K;
  const int64_t N = g->N;
  const bool mixed = prec == SBIE_MIXED;
  const size_t MK4 = (size_t)4 * M * K;
  sbie_status st;
  SBIE_TRY_C(stokes_buffers(g));

  hipEvent_t* ev = nullptr;
  if (timed) {
    SBIE_TRY_C(next_timing_set(g, &ev));
    SBIE_HIP(hipEventRecord(ev[0], s));
  }
  const int B = 256;
  if (mixed)
    hipLaunchKernelGGL(k_stokes_prep<float>, dim3(cdiv(N, B)), dim3(B), 0, s, g->d_part, d_dens, g->d_x, g->d_y,
                       g->d_z, g->d_w, g->d_wS, p, N, g->d_stk_f, (float*)g->d_stk_src);
  else
    hipLaunchKernelGGL(k_stokes_prep<double>, dim3(cdiv(N, B)), dim3(B), 0, s, g->d_part, d_dens, g->d_x, g->d_y,
                       g->d_z, g->d_w, g->d_wS, p, N, g->d_stk_f, g->d_stk_src);
  SBIE_HIP(hipGetLastError());
  if (timed) SBIE_HIP(hipEventRecord(ev[1], s));
  if (parts & (SBIE_PARTS_SELF | SBIE_PARTS_NEAR)) {
    // forward transforms of the four densities per particle (rows i*4 + s).
    // The transforms run in FP64 in both precisions: the compensated FP32
    // form took as long here (0.52 against 0.51 ms per apply at 256 spheroids)
    // and its error, magnified where the three terms of the Stokeslet cancel,
    // set the mixed path's error on the surface.
    if ((st = gemm(false, g->d_stk_f, T, g->d_An, g->d_An32, K, g->d_stk_c, K, 4 * M, K, T, s)) != SBIE_OK)
      return st;
    hipLaunchKernelGGL(k_stokes_scale, dim3(cdiv((int64_t)MK4, B)), dim3(B), 0, s, g->d_stk_c, g->d_lam, g->d_dlr,
                       M, p, g->d_stk_E, g->d_stk_E + MK4);
    SBIE_HIP(hipGetLastError());
  }
  return pressure ? stokes_parts<4>(g, mixed, s, parts, ev, d_dens, d_out)
                  : stokes_parts<3>(g, mixed, s, parts, ev, d_dens, d_out);
}

namespace {

// Near (side stream when the geometry has one), self and far parts of C
// components, then the assembly into d_out [C][N].  The far part comes from
// the tree with SBIE_FAR_TREE (FP64 sums), else from the direct sum.
template <int C>
sbie_status stokes_parts(sbie_geom* g, bool mixed, hipStream_t s, uint32_t parts, hipEvent_t* ev,
                         const double* d_dens, double* d_out) {
  const int M = g->M, p = g->p, T = g->T, K = g->K;
  const int64_t N = g->N;
  const size_t MT4 = (size_t)4 * M * T, MK4 = (size_t)4 * M * K;
  const bool timed = ev != nullptr;
  const int B = 256;
  sbie_status st;
  // near field on the side stream, concurrently with the self and far parts
  const bool near = (parts & SBIE_PARTS_NEAR) && g->n_near > 0;
  const bool fork = near && g->side != nullptr;
  if (near) {
    if (fork) SBIE_TRY_C(fork_side(g, s));
    hipStream_t ns = fork ? g->side : s;
    if (timed) SBIE_HIP(hipEventRecord(ev[6], ns));
    dispatch_order(p, [&](auto pm, auto ex) { launch_near_stokes<decltype(pm)::value, decltype(ex)::value, C>(g, ns); });
    SBIE_HIP(hipGetLastError());
    if (timed) SBIE_HIP(hipEventRecord(ev[7], ns));
  } else if (timed) {
    SBIE_HIP(hipEventRecord(ev[6], s));
    SBIE_HIP(hipEventRecord(ev[7], s));
  }
  {
    if (parts & SBIE_PARTS_SELF) {
      double* U = g->d_stk_U;
      if ((st = gemm(false, g->d_stk_E, K, g->d_Sy, g->d_Sy32, T, U, T, 4 * M, T, K, s)) != SBIE_OK) return st;
      if ((st = gemm(false, g->d_stk_E + MK4, K, g->d_Sy, g->d_Sy32, T, U + MT4, T, 4 * M, T, K, s)) != SBIE_OK)
        return st;
      if ((st = gemm(false, g->d_stk_E, K, g->d_Sv, g->d_Sv32, T, U + 2 * MT4, T, 4 * M, T, K, s)) != SBIE_OK)
        return st;
      if ((st = gemm(false, g->d_stk_E, K, g->d_Sp, g->d_Sp32, T, U + 3 * MT4, T, 4 * M, T, K, s)) != SBIE_OK)
        return st;
      hipLaunchKernelGGL(k_stokes_self<C>, dim3(cdiv(N, B)), dim3(B), 0, s, g->d_part, g->d_gl, g->d_x, g->d_y,
                         g->d_z, g->d_stk_U, M, p, N, g->d_stk_self);
      SBIE_HIP(hipGetLastError());
    }
  }
  if (timed) SBIE_HIP(hipEventRecord(ev[2], s));
  if (timed) SBIE_HIP(hipEventRecord(ev[3], s));
  // far field: the tree, else the pair-symmetric matrix-core kernel (T >= 32),
  // else the one-sided vector-unit sum
  const bool tree = (parts & SBIE_FAR_TREE) != 0;
  const bool pairs = !tree && T >= 32;
  if ((parts & SBIE_PARTS_FAR) && tree) {
    SBIE_TRY_C(far_tree_stokes(g, C, d_dens, s));
  } else if ((parts & SBIE_PARTS_FAR) && pairs) {
    SBIE_TRY_C(far_stokes_pairs(g, C, mixed, d_dens, s));
  } else if (parts & SBIE_PARTS_FAR) {
    constexpr int TPT = 2;
    const dim3 grid(cdiv(N, 256 * TPT) * g->nsplit);
    if (mixed)
      hipLaunchKernelGGL((k_far_stokes<float, TPT, C>), grid, dim3(256), 0, s, (const float*)g->d_stk_src, g->d_part,
                         g->d_x, g->d_y, g->d_z, g->d_excl, g->excl_words, M, T, N, g->nsplit, g->d_stk_part);
    else
      hipLaunchKernelGGL((k_far_stokes<double, TPT, C>), grid, dim3(256), 0, s, (const double*)g->d_stk_src,
                         g->d_part, g->d_x, g->d_y, g->d_z, g->d_excl, g->excl_words, M, T, N, g->nsplit,
                         g->d_stk_part);
    SBIE_HIP(hipGetLastError());
  }
  if (timed) SBIE_HIP(hipEventRecord(ev[4], s));
  if (fork) SBIE_TRY_C(join_side(g, s));
  // with no near pairs the near part is empty and is left out of the sum
  const uint32_t sum_parts = g->n_near > 0 ? parts : (parts & ~(uint32_t)SBIE_PARTS_NEAR);
  const int nslices = pairs ? stokes_pair_splits(g, stokes_row_groups(T, !mixed)) : g->nsplit;
  hipLaunchKernelGGL(k_stokes_assemble<C>, dim3(cdiv(C * N, B)), dim3(B), 0, s, g->d_stk_self, g->d_stk_near,
                     g->d_stk_part, nslices, pairs ? (const double*)g->d_stk_racc : nullptr, N, sum_parts, d_out);
  SBIE_HIP(hipGetLastError());
  if (timed) SBIE_HIP(hipEventRecord(ev[5], s));
  return SBIE_OK;
}

}  // namespace

}  // namespace sbie
