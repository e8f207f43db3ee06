// Stokes double layer, the stresslet with the outward normal (viscosity 1):
//   D_stk[mu]_i(x) = 3/(4 pi) int (r.mu)(r.nu) r_i / |r|^5 dS_y,  r = x - y,
// normalised like the Laplace double layer (a constant mu gives -mu inside,
// -mu/2 on the surface).  Section 4.3 cites a decomposition into Laplace
// potentials without printing it; this one, with origin c at each source
// centre, follows from d_i (nu.r/r^3) and d_j (1/r) = -r_j/r^3:
//   D_stk[mu]_i = -sum_j (x-c)_j d_i D[mu_j] + d_i D[(y-c).mu] - sum_j d_j S[mu_j nu_i].
// Per source particle there are thirteen expansions: double layers of mu_1,
// mu_2, mu_3 and (y-c).mu (sets 0-3), single layers of mu_j nu_k (set
// 4 + 3k + j).  Self: exterior-limit gradients at the particle's own nodes,
// then the principal value D_stk+ - mu/2; near: gradients of the neighbours'
// exterior expansions; far: the stresslet by smooth quadrature.
#include <hip/hip_runtime.h>

#include <cmath>

#include "far_dev.h"
#include "near_dev.h"
#include "sbie_internal.h"

namespace sbie {

namespace {

constexpr double k3Over4Pi = 0.23873241463784300365332564505877154;
constexpr int kSets = 13;

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

// Transform inputs of the thirteen sets (rows i*13 + s; the single-layer sets
// in the modified basis sqrt(u0^2 -+ v^2)) and the far records (node - centre,
// W mu, nu_x, nu_y; nu_z stays in the geometry's normal array).
template <typename R>
__global__ void k_sdl_prep(const Particle* __restrict__ part, const double* __restrict__ dens,
                           const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ z,
                           const double* __restrict__ nx, const double* __restrict__ ny,
                           const double* __restrict__ nz, const double* __restrict__ w,
                           const double* __restrict__ wS, int p, int64_t N, double* __restrict__ f,
                           R* __restrict__ rec) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  const int Nphi = 2 * p + 2, T = (p + 1) * Nphi;
  const int i = (int)(g / T), t = (int)(g - (int64_t)i * T), j = t / Nphi;
  const double m[3] = {dens[g], dens[N + g], dens[2 * N + g]};
  const double nu[3] = {nx[g], ny[g], nz[g]};
  const double o[3] = {x[g] - part[i].c[0], y[g] - part[i].c[1], z[g] - part[i].c[2]};
  const double ws = wS[(size_t)i * (p + 1) + j];
  double* fr = f + (size_t)i * kSets * T + t;
  fr[0] = m[0];
  fr[T] = m[1];
  fr[2 * T] = m[2];
  fr[3 * T] = fma(o[2], m[2], fma(o[1], m[1], o[0] * m[0]));
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int c = 0; c < 3; ++c) fr[(size_t)(4 + 3 * k + c) * T] = ws * m[c] * nu[k];
  const double wq = w[g];
  R* r = rec + 8 * g;
  r[0] = (R)o[0];
  r[1] = (R)o[1];
  r[2] = (R)o[2];
  r[3] = (R)(wq * m[0]);
  r[4] = (R)(wq * m[1]);
  r[5] = (R)(wq * m[2]);
  r[6] = (R)nu[0];
  r[7] = (R)nu[1];
}

// E = lam c (double-layer sets: the exterior limit lam_D+; single-layer sets:
// lam_S) and Eu = E d/du ln Q(u0).
__global__ void k_sdl_scale(const double* __restrict__ coef, const double* __restrict__ lam,
                            const double* __restrict__ dlr, int M, int p, double* __restrict__ E,
                            double* __restrict__ Eu) {
  const int K = (p + 1) * (p + 1), Kh = (p + 1) * (p + 2) / 2;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)kSets * M * K) return;
  const int row = (int)(t / K), l = (int)(t - (int64_t)row * K);
  const int i = row / kSets, s = row - i * kSets;
  const int n = (int)sqrt((double)l);
  const int m = l - n * n - n;
  const int h = n * (n + 1) / 2 + (m < 0 ? -m : m);
  const double e = lam[((size_t)i * Kh + h) * 4 + (s < 4 ? 1 : 2)] * coef[t];
  E[t] = e;
  Eu[t] = e * dlr[(size_t)i * Kh + h];
}

// The decomposition from the lab gradients gD[4][3] and gS[9][3]; d = x - c.
__device__ inline void sdl_combine(const double (&gD)[4][3], const double (&gS)[9][3], const double d[3],
                                   double out[3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    double s = gD[3][i];
#pragma unroll
    for (int j = 0; j < 3; ++j) s = fma(-d[j], gD[j][i], s);
#pragma unroll
    for (int j = 0; j < 3; ++j) s -= gS[3 * i + j][j];
    out[i] = s;
  }
}

// Self part at node g: exterior-limit gradients of the thirteen expansions from
// U (d/du, d/dv, d/dphi), the decomposition, minus mu/2.
__global__ void k_sdl_self(const Particle* __restrict__ part, const double* __restrict__ gl,
                           const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ z,
                           const double* __restrict__ dens, const double* __restrict__ U, int M, int p, int64_t N,
                           double* __restrict__ out) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  const int Nphi = 2 * p + 2, T = (p + 1) * Nphi;
  const int i = (int)(g / T), t = (int)(g - (int64_t)i * T), j = t / Nphi, k = t - j * Nphi;
  const Particle P = part[i];
  const size_t plane = (size_t)kSets * M * T;
  const double v = gl[j];
  double s1, c1;
  sincospi(2.0 * k / Nphi, &s1, &c1);
  const double su = sqrt(P.w0), sv = sqrt((1.0 - v) * (1.0 + v));
  double gD[4][3], gS[9][3];
#pragma unroll
  for (int s = 0; s < kSets; ++s) {
    const size_t o = ((size_t)i * kSets + s) * T + t;
    double gr[3];
    lab_gradient(P, P.u0, su, v, sv, c1, s1, U[o], U[plane + o], U[2 * plane + o], gr);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (s < 4)
        gD[s][c] = gr[c];
      else
        gS[s - 4][c] = gr[c];
    }
  }
  const double d[3] = {x[g] - P.c[0], y[g] - P.c[1], z[g] - P.c[2]};
  double o3[3];
  sdl_combine(gD, gS, d, o3);
#pragma unroll
  for (int c = 0; c < 3; ++c) out[c * N + g] = o3[c] - 0.5 * dens[c * N + g];
}

// The orders are unrolled up to p = 12: the thirteen sets' work per (n, m)
// makes p = 16 too long for the instruction cache.
template <int PMAX, bool EXACT>
constexpr bool kSdlUnroll = EXACT && PMAX <= 12;

// Near part: one workgroup per (target particle, 64 W target nodes); the
// derivative recurrences run once for the four double-layer sets and once for
// the nine single-layer sets of every near source.
template <int PMAX, bool EXACT>
__global__ __launch_bounds__((64 * kNearWaves<kSdlUnroll<PMAX, EXACT>>))
__attribute__((amdgpu_waves_per_eu(3))) void k_near_sdl(
    const Particle* __restrict__ part, const double* __restrict__ x, const double* __restrict__ y,
    const double* __restrict__ z, const int32_t* __restrict__ near_ptr, const int32_t* __restrict__ near_src,
    const double* __restrict__ E, const double* __restrict__ lam, const double* __restrict__ ab,
    const double* __restrict__ cd, const double* __restrict__ rcp, int p_arg, int T, int chunks, int64_t N,
    unsigned* status, double* __restrict__ unear) {
  const int p = EXACT ? PMAX : p_arg;  // exact order: degree bounds known at compile time
  // one workgroup per (target particle, 64 W targets, range qr of its
  // near-source list)
  constexpr bool kU = kSdlUnroll<PMAX, EXACT>;
  constexpr int W = kNearWaves<kU>;
  const int wgs = (chunks + W - 1) / W;
  const int qr = blockIdx.x % kStokesNearSplit, rest = blockIdx.x / kStokesNearSplit;
  const int jt = rest / wgs;
  const int t = (rest - jt * wgs) * 64 * W + threadIdx.x;
  const bool live = t < T;
  const int64_t g = (int64_t)jt * T + (live ? t : 0);
  const double X0 = x[g], X1 = y[g], X2 = z[g];
  const int K = (p + 1) * (p + 1), Kh = (p + 1) * (p + 2) / 2;
  __shared__ NearTablesFor<PMAX, kU, kSets> tb;
  near_tables_init<PMAX, kU, kSets>(tb, ab, cd);
  double acc[3] = {0.0, 0.0, 0.0};
  unsigned bad = 0u;
  const int cap = (int)status[1];  // the geometry's recurrence step cap
  const int n0 = near_ptr[jt], nn = near_ptr[jt + 1] - n0;
  const int s_begin = n0 + (nn * qr) / kStokesNearSplit, s_end = n0 + (nn * (qr + 1)) / kStokesNearSplit;
  for (int sidx = s_begin; sidx < s_end; ++sidx) {
    const int i = near_src[sidx];
    const Particle P = part[i];
    const SpheroidalPoint q = to_spheroidal(P, X0, X1, X2, true, &bad);
    const NearSourceView src =
        near_source<PMAX, kU, kSets>(tb, P.oblate != 0, E + (size_t)i * kSets * K, lam + (size_t)i * Kh * 4, ab, cd, K,
                                     Kh);
    const double* Ei = src.E;
    // The decomposition is linear in the thirteen expansions, so it is taken
    // inside the sum over (n, m), one basis evaluation for all of them:
    //  - the double-layer part  grad (D[3] - sum_j d_j D[j])  is the gradient
    //    of one expansion with coefficients E3 - d.(E0, E1, E2) (d fixed at
    //    the target);
    //  - the single-layer part  -sum_j d_j S[4 + 3i + j]  needs one lab
    //    derivative of each set, the chain rule's coefficients applied to the
    //    basis derivatives.
    double al[3], be[3], ga[3];
    lab_gradient_coeffs(P, q.u, q.sw, q.v, q.sv, q.c1, q.s1, al, be, ga);
    const double w0 = -q.d[0], w1 = -q.d[1], w2 = -q.d[2];
    double Gu = 0.0, Gv = 0.0, Gp = 0.0, O[3] = {0.0, 0.0, 0.0};
    if constexpr (kU) {
      const double iw = 1.0 / q.w, iv = 1.0 / (q.sv * q.sv);
      double alw[3], bev[3];
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        alw[j] = al[j] * iw;
        bev[j] = be[j] * iv;
      }
      // per order, the lab derivative j of the cosine and sine terms of a
      // (scaled) basis function: x_j tu + y_j tv -+ z_j t0 with the azimuthal
      // factors and the chain rule's coefficients folded into x, y, z
      double xc[3], xs[3], yc[3], ys[3], zc[3], zs[3];
      // per-order sums of the double-layer part's combined expansion
      double guc = 0.0, gus = 0.0, gvc = 0.0, gvs = 0.0, g0c = 0.0, g0s = 0.0;
      expansion_orders<PMAX>(
          q, P.oblate != 0, src.ab, src.cd, rcp, src.qt, cap, &bad,
          [&](int m, double c, double s) {
#pragma unroll
            for (int j = 0; j < 3; ++j) {
              xc[j] = c * alw[j];
              xs[j] = s * alw[j];
              yc[j] = c * bev[j];
              ys[j] = s * bev[j];
              zc[j] = ((double)m * c) * ga[j];
              zs[j] = ((double)m * s) * ga[j];
            }
          },
          [&](int lc, int ls, int m, double t0, double tu, double tv) {
            const double fc = fma(w2, Ei[2 * K + lc], fma(w1, Ei[K + lc], fma(w0, Ei[lc], Ei[3 * K + lc])));
            guc = fma(fc, tu, guc);
            gvc = fma(fc, tv, gvc);
            g0c = fma(fc, t0, g0c);
            double dc[3];
#pragma unroll
            for (int j = 0; j < 3; ++j) dc[j] = fma(xc[j], tu, fma(yc[j], tv, -zs[j] * t0));
#pragma unroll
            for (int ii = 0; ii < 3; ++ii)
#pragma unroll
              for (int j = 0; j < 3; ++j) O[ii] = fma(-Ei[(size_t)(4 + 3 * ii + j) * K + lc], dc[j], O[ii]);
            if (m > 0) {
              const double fs = fma(w2, Ei[2 * K + ls], fma(w1, Ei[K + ls], fma(w0, Ei[ls], Ei[3 * K + ls])));
              gus = fma(fs, tu, gus);
              gvs = fma(fs, tv, gvs);
              g0s = fma(fs, t0, g0s);
              double ds[3];
#pragma unroll
              for (int j = 0; j < 3; ++j) ds[j] = fma(xs[j], tu, fma(ys[j], tv, zc[j] * t0));
#pragma unroll
              for (int ii = 0; ii < 3; ++ii)
#pragma unroll
                for (int j = 0; j < 3; ++j) O[ii] = fma(-Ei[(size_t)(4 + 3 * ii + j) * K + ls], ds[j], O[ii]);
            }
          },
          [&](int m, double c, double s) {
            Gu = fma(c, guc, fma(s, gus, Gu));
            Gv = fma(c, gvc, fma(s, gvs, Gv));
            Gp = fma((double)m, fma(c, g0s, -s * g0c), Gp);
            guc = gus = gvc = gvs = g0c = g0s = 0.0;
          });
      Gu *= iw;
      Gv *= iv;
    } else {
    expansion_terms<PMAX>(q, P.oblate != 0, src.L, src.ab, src.cd, rcp, p, cap, &bad,
                          [&](int lc, int ls, int m, double, double a1, double a2, double ap, double, double b1,
                              double b2, double bp) {
                            const double fc = fma(w2, Ei[2 * K + lc], fma(w1, Ei[K + lc], fma(w0, Ei[lc], Ei[3 * K + lc])));
                            Gu = fma(fc, a1, Gu);
                            Gv = fma(fc, a2, Gv);
                            Gp = fma(fc, ap, Gp);
                            double nc[3];
#pragma unroll
                            for (int j = 0; j < 3; ++j) nc[j] = -fma(ga[j], ap, fma(be[j], a2, al[j] * a1));
#pragma unroll
                            for (int ii = 0; ii < 3; ++ii)
#pragma unroll
                              for (int j = 0; j < 3; ++j) O[ii] = fma(Ei[(size_t)(4 + 3 * ii + j) * K + lc], nc[j], O[ii]);
                            if (m > 0) {
                              const double fs =
                                  fma(w2, Ei[2 * K + ls], fma(w1, Ei[K + ls], fma(w0, Ei[ls], Ei[3 * K + ls])));
                              Gu = fma(fs, b1, Gu);
                              Gv = fma(fs, b2, Gv);
                              Gp = fma(fs, bp, Gp);
                              double ns[3];
#pragma unroll
                              for (int j = 0; j < 3; ++j) ns[j] = -fma(ga[j], bp, fma(be[j], b2, al[j] * b1));
#pragma unroll
                              for (int ii = 0; ii < 3; ++ii)
#pragma unroll
                                for (int j = 0; j < 3; ++j)
                                  O[ii] = fma(Ei[(size_t)(4 + 3 * ii + j) * K + ls], ns[j], O[ii]);
                            }
                          });
    }
#pragma unroll
    for (int ii = 0; ii < 3; ++ii) acc[ii] += fma(ga[ii], Gp, fma(be[ii], Gv, al[ii] * Gu)) + O[ii];
  }
  if (bad) atomicOr(status, bad);
  if (live) {
    double* o = unear + (size_t)qr * 3 * N;
    o[g] = acc[0];
    o[N + g] = acc[1];
    o[2 * N + g] = acc[2];
  }
}

// Far part: the stresslet over the far source nodes (records: node - centre,
// W mu, nu_x, nu_y; nu_z read from the geometry's normal array); grid and
// compensation as the other direct sums.
template <typename R, int TPT>
__global__ __launch_bounds__(256) void k_far_sdl(const R* __restrict__ rec, const double* __restrict__ nzs,
                                                 const Particle* __restrict__ part, const double* __restrict__ x,
                                                 const double* __restrict__ y, const double* __restrict__ z,
                                                 const uint32_t* __restrict__ excl, int words, int M, int T,
                                                 int64_t N, int nsplit, double* __restrict__ partial) {
  const int split = blockIdx.x % nsplit, tile = blockIdx.x / nsplit;
  const int s0 = (int)((int64_t)M * split / nsplit), s1 = (int)((int64_t)M * (split + 1) / nsplit);
  double tx[TPT], ty[TPT], tz[TPT];
  int tp[TPT];
  bool live[TPT];
  R acc[TPT][3], lo[TPT][3];
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
    for (int c = 0; c < 3; ++c) acc[k][c] = lo[k][c] = R(0);
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
    R Dx[TPT], Dy[TPT], Dz[TPT], tmp[TPT][3];
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
      Dx[k] = (R)(tx[k] - cx);
      Dy[k] = (R)(ty[k] - cy);
      Dz[k] = (R)(tz[k] - cz);
#pragma unroll
      for (int c = 0; c < 3; ++c) tmp[k][c] = R(0);
    }
    const R* rs = rec + (size_t)s * T * 8;
    const double* ns = nzs + (size_t)s * T;
    for (int q = 0; q < T; ++q) {
      const R* r = rs + (size_t)q * 8;
      const R ox = r[0], oy = r[1], oz = r[2], m0 = r[3], m1 = r[4], m2 = r[5], n0 = r[6], n1 = r[7];
      const R n2 = (R)ns[q];
#pragma unroll
      for (int k = 0; k < TPT; ++k) {
        const R dx = Dx[k] - ox, dy = Dy[k] - oy, dz = Dz[k] - oz;
        const R r2 = fma(dz, dz, fma(dy, dy, dx * dx));
        const R ri = rsq_t<R>(r2);
        const R ri2 = ri * ri;
        const R dm = fma(dz, m2, fma(dy, m1, dx * m0));
        const R dn = fma(dz, n2, fma(dy, n1, dx * n0));
        const R wgt = dm * dn * ri * ri2 * ri2;
        tmp[k][0] = fma(wgt, dx, tmp[k][0]);
        tmp[k][1] = fma(wgt, dy, tmp[k][1]);
        tmp[k][2] = fma(wgt, dz, tmp[k][2]);
      }
    }
#pragma unroll
    for (int k = 0; k < TPT; ++k)
#pragma unroll
      for (int c = 0; c < 3; ++c) two_sum_add(acc[k][c], lo[k][c], need[k] ? tmp[k][c] : R(0));
  }
#pragma unroll
  for (int k = 0; k < TPT; ++k) {
    const int64_t gq = (int64_t)tile * 256 * TPT + k * 256 + threadIdx.x;
    if (!live[k]) continue;
#pragma unroll
    for (int c = 0; c < 3; ++c)
      partial[((size_t)split * 3 + c) * N + gq] = ((double)acc[k][c] + (double)lo[k][c]) * k3Over4Pi;
  }
}

__global__ void k_sdl_assemble(const double* __restrict__ uself, const double* __restrict__ unear,
                               const double* __restrict__ partial, int nsplit, const double* __restrict__ racc,
                               int64_t N, uint32_t parts, double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * N) return;
  const int c = (int)(t / N);
  const int64_t g = t - (int64_t)c * N;
  double u = 0.0;
  if (parts & SBIE_PARTS_SELF) u += uself[t];
  if (parts & SBIE_PARTS_NEAR)
    for (int q = 0; q < kStokesNearSplit; ++q) u += unear[(size_t)q * 3 * N + t];
  if (parts & SBIE_PARTS_FAR) {
    double f = 0.0;
    for (int s = 0; s < nsplit; ++s) f += partial[((size_t)s * 3 + c) * N + g];
    if (racc) f += racc[t] * k3Over4Pi;
    u += f;
  }
  out[t] = u;
}

template <int PMAX, bool EXACT>
void launch_near_sdl(sbie_geom* g, hipStream_t s) {
  const int chunks = (g->T + 63) / 64;
  constexpr int W = kNearWaves<kSdlUnroll<PMAX, EXACT>>;
  hipLaunchKernelGGL((k_near_sdl<PMAX, EXACT>), dim3(g->M * ((chunks + W - 1) / W) * kStokesNearSplit),
                     dim3(64 * W), 0, s, g->d_part, g->d_x, g->d_y, g->d_z,
                     g->d_near_ptr, g->d_near_src, g->d_sdl_E, g->d_lam, g->d_ab, g->d_cd, g->d_rcp, g->p, g->T,
                     chunks, g->N, g->d_status, g->d_sdl_near);
}

#define SBIE_TRY_D(expr)            \
  do {                              \
    sbie_status _s = (expr);        \
    if (_s != SBIE_OK) return _s;   \
  } while (0)

sbie_status carve_sdl(sbie_geom* g, Carver& c) {
  const size_t MT = (size_t)kSets * g->M * g->T, MK = (size_t)kSets * g->M * g->K;
  const size_t N = (size_t)g->N;
  SBIE_TRY_D(c.take(&g->d_sdl_f, MT));
  SBIE_TRY_D(c.take(&g->d_sdl_c, MK));
  SBIE_TRY_D(c.take(&g->d_sdl_E, 2 * MK));
  SBIE_TRY_D(c.take(&g->d_sdl_U, 3 * MT));
  SBIE_TRY_D(c.take(&g->d_sdl_src, 8 * N));
  SBIE_TRY_D(c.take(&g->d_sdl_part, (size_t)g->nsplit * 3 * N));
  SBIE_TRY_D(c.take(&g->d_sdl_self, 3 * N));
  SBIE_TRY_D(c.take(&g->d_sdl_near, (size_t)kStokesNearSplit * 3 * N));
  SBIE_TRY_D(c.take(&g->d_sdl_io, 6 * N));
  // the pair kernel's source blocks, reverse sums and totals
  const size_t nb = (size_t)(g->T + 15) / 16;
  g->sdl_rev_bytes = stokes_rev_bytes(g->M, g->T);
  SBIE_TRY_D(c.take(&g->d_sdl_prec, (size_t)g->M * nb * stokes_record_doubles(true)));
  SBIE_TRY_D(c.take(&g->d_sdl_rev, (size_t)(g->sdl_rev_bytes / sizeof(double))));
  SBIE_TRY_D(c.take(&g->d_sdl_racc, 3 * (size_t)N));
  return SBIE_OK;
}

sbie_status sdl_buffers(sbie_geom* g) {
  if (g->sdl_blk) return SBIE_OK;
  Carver measure;
  SBIE_TRY_D(carve_sdl(g, measure));
  const size_t bytes = (measure.used + 255) & ~size_t(255);
  if (hipMalloc((void**)&g->sdl_blk, bytes) != hipSuccess) {
    g->sdl_blk = nullptr;
    (void)hipGetLastError();
    set_error("device allocation of the Stokes double-layer work buffers failed");
    return SBIE_E_NOMEM;
  }
  g->footprint += bytes;
  Carver c;
  c.base = g->sdl_blk;
  c.size = bytes;
  return carve_sdl(g, c);
}

}  // namespace

sbie_status stokes_dl_staging(sbie_geom* g, double** io) {
  SBIE_TRY_D(sdl_buffers(g));
  *io = g->d_sdl_io;
  return SBIE_OK;
}

sbie_status apply_stokes_dl(sbie_geom* g, int prec, const double* d_dens, double* d_out, hipStream_t s,
                            uint32_t parts, bool timed) {
  const int M = g->M, p = g->p, T = g->T, K = g->K;
  const int64_t N = g->N;
  const bool mixed = prec == SBIE_MIXED;
  const size_t MT = (size_t)kSets * M * T, MK = (size_t)kSets * M * K;
  const int B = 256;
  sbie_status st;
  SBIE_TRY_D(sdl_buffers(g));
  hipEvent_t* ev = nullptr;
  if (timed) {
    SBIE_TRY_D(next_timing_set(g, &ev));
    SBIE_HIP(hipEventRecord(ev[0], s));
  }
  if (mixed)
    hipLaunchKernelGGL(k_sdl_prep<float>, dim3(cdiv(N, B)), dim3(B), 0, s, g->d_part, d_dens, g->d_x, g->d_y,
                       g->d_z, g->d_nx, g->d_ny, g->d_nz, g->d_w, g->d_wS, p, N, g->d_sdl_f,
                       reinterpret_cast<float*>(g->d_sdl_src));
  else
    hipLaunchKernelGGL(k_sdl_prep<double>, dim3(cdiv(N, B)), dim3(B), 0, s, g->d_part, d_dens, g->d_x, g->d_y,
                       g->d_z, g->d_nx, g->d_ny, g->d_nz, g->d_w, g->d_wS, p, N, g->d_sdl_f, g->d_sdl_src);
  SBIE_HIP(hipGetLastError());
  if (timed) SBIE_HIP(hipEventRecord(ev[1], s));
  if (parts & (SBIE_PARTS_SELF | SBIE_PARTS_NEAR)) {
    // FP64 transforms in both precisions, as for the single layer
    if ((st = gemm(false, g->d_sdl_f, T, g->d_An, g->d_An32, K, g->d_sdl_c, K, kSets * M, K, T, s)) != SBIE_OK)
      return st;
    hipLaunchKernelGGL(k_sdl_scale, dim3(cdiv((int64_t)MK, B)), dim3(B), 0, s, g->d_sdl_c, g->d_lam, g->d_dlr, M,
                       p, g->d_sdl_E, g->d_sdl_E + MK);
    SBIE_HIP(hipGetLastError());
  }
  if (parts & SBIE_PARTS_SELF) {
    double* U = g->d_sdl_U;
    if ((st = gemm(false, g->d_sdl_E + MK, K, g->d_Sy, g->d_Sy32, T, U, T, kSets * M, T, K, s)) != SBIE_OK)
      return st;
    if ((st = gemm(false, g->d_sdl_E, K, g->d_Sv, g->d_Sv32, T, U + MT, T, kSets * M, T, K, s)) != SBIE_OK)
      return st;
    if ((st = gemm(false, g->d_sdl_E, K, g->d_Sp, g->d_Sp32, T, U + 2 * MT, T, kSets * M, T, K, s)) != SBIE_OK)
      return st;
    hipLaunchKernelGGL(k_sdl_self, dim3(cdiv(N, B)), dim3(B), 0, s, g->d_part, g->d_gl, g->d_x, g->d_y, g->d_z,
                       d_dens, U, M, p, N, g->d_sdl_self);
    SBIE_HIP(hipGetLastError());
  }
  if (timed) SBIE_HIP(hipEventRecord(ev[2], s));
  const bool near = (parts & SBIE_PARTS_NEAR) && g->n_near > 0;
  if (timed) SBIE_HIP(hipEventRecord(ev[6], s));
  if (near) {
    dispatch_order(p, [&](auto pm, auto ex) { launch_near_sdl<decltype(pm)::value, decltype(ex)::value>(g, s); });
    SBIE_HIP(hipGetLastError());
  }
  if (timed) SBIE_HIP(hipEventRecord(ev[7], s));
  if (timed) SBIE_HIP(hipEventRecord(ev[3], s));
  // far field: the pair-symmetric matrix-core kernel (T >= 32), else the
  // one-sided vector-unit sum.  (At 256 spheroids the pair kernel took 8.35
  // against 9.02 ms in FP64 and, with three-piece bf16 products, 3.46 against
  // 3.95 ms in mixed precision; with FP32 products it took 4.21 ms there.)
  const bool pairs = T >= 32;
  if ((parts & SBIE_PARTS_FAR) && pairs) {
    SBIE_TRY_D(far_sdl_pairs(g, mixed, d_dens, s));
  } else if (parts & SBIE_PARTS_FAR) {
    constexpr int TPT = 2;
    const dim3 grid(cdiv(N, 256 * TPT) * g->nsplit);
    if (mixed)
      hipLaunchKernelGGL((k_far_sdl<float, TPT>), grid, dim3(256), 0, s, reinterpret_cast<const float*>(g->d_sdl_src),
                         g->d_nz, g->d_part, g->d_x, g->d_y, g->d_z, g->d_excl, g->excl_words, M, T, N, g->nsplit,
                         g->d_sdl_part);
    else
      hipLaunchKernelGGL((k_far_sdl<double, TPT>), grid, dim3(256), 0, s, g->d_sdl_src, g->d_nz, g->d_part, g->d_x,
                         g->d_y, g->d_z, g->d_excl, g->excl_words, M, T, N, g->nsplit, g->d_sdl_part);
    SBIE_HIP(hipGetLastError());
  }
  if (timed) SBIE_HIP(hipEventRecord(ev[4], s));
  const uint32_t sum_parts = g->n_near > 0 ? parts : (parts & ~(uint32_t)SBIE_PARTS_NEAR);
  const int nslices = pairs ? stokes_pair_splits(g, stokes_row_groups(T, !mixed)) : g->nsplit;
  hipLaunchKernelGGL(k_sdl_assemble, dim3(cdiv(3 * N, B)), dim3(B), 0, s, g->d_sdl_self, g->d_sdl_near,
                     g->d_sdl_part, nslices, pairs ? (const double*)g->d_sdl_racc : nullptr, N, sum_parts, d_out);
  SBIE_HIP(hipGetLastError());
  if (timed) SBIE_HIP(hipEventRecord(ev[5], s));
  return SBIE_OK;
}

}  // namespace sbie
