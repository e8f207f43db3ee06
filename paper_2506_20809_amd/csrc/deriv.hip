// Normal derivatives of the layer potentials at the nodes (Section 3.3): S'
// (Theorem 3, principal value on the surface) and D' (the derivative of the
// double layer along the target normal, which has no jump).  The parts follow
// Algorithm 1: a forward transform, diagonal spectra and an inverse transform
// for the self part, the gradient of each near neighbour's exterior expansion
// along the target normal, and the direct smooth-quadrature sum of the
// differentiated kernels for the far field.
#include <hip/hip_runtime.h>

#include <cmath>

#include "far_dev.h"
#include "near_dev.h"
#include "sbie_internal.h"

namespace sbie {

namespace {

constexpr double kInv4Pi = 0.079577471545947667884441881686257181;

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

// Transform input and far-field source records.
//  S': f = sqrt(u0^2 -+ v^2) sigma (modified basis), D': f = mu;
//  rec[g] = (node - centre, W dens, nu, 0) in R.
template <typename R, int OP>
__global__ void k_normal_prep(const Particle* __restrict__ part, const double* __restrict__ dens,
                              const double* __restrict__ x, const double* __restrict__ y,
                              const double* __restrict__ z, const double* __restrict__ nx,
                              const double* __restrict__ ny, const double* __restrict__ nz,
                              const double* __restrict__ w, const double* __restrict__ wS, int p, int64_t N,
                              double* __restrict__ f, R* __restrict__ rec) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  const int Nphi = 2 * p + 2, T = (p + 1) * Nphi;
  const int i = (int)(g / T), j = (int)((g - (int64_t)i * T) / Nphi);
  const double d = dens[g];
  f[g] = OP == SBIE_OP_SP ? wS[(size_t)i * (p + 1) + j] * d : d;
  const Particle& P = part[i];
  R* r = rec + 8 * g;
  r[0] = (R)(x[g] - P.c[0]);
  r[1] = (R)(y[g] - P.c[1]);
  r[2] = (R)(z[g] - P.c[2]);
  r[3] = (R)(w[g] * d);
  r[4] = (R)nx[g];
  r[5] = (R)ny[g];
  r[6] = (R)nz[g];
  r[7] = R(0);
}

// Self and exterior coefficients.  With h = sqrt(u0^2 -+ 1)/a and
// dlr = d/du ln Q_n^m(u) at u0 (real form for oblates):
//  S': the exterior limit is h lam_S dlr; the jump of the normal derivative of
//      the single layer is -sigma, i.e. -1 per mode of the modified basis, so
//      the principal value is h lam_S dlr + 1/2; exterior coefficients lam_S;
//  D': h lam_D+ dlr from either side; exterior coefficients lam_D+.
__global__ void k_normal_scale(const double* __restrict__ coef, const double* __restrict__ lam,
                               const double* __restrict__ dlr, const Particle* __restrict__ part, int M, int p,
                               int op, double* __restrict__ cself, double* __restrict__ E) {
  const int K = (p + 1) * (p + 1), Kh = (p + 1) * (p + 2) / 2;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)M * K) return;
  const int i = (int)(t / K), l = (int)(t - (int64_t)i * K);
  const int n = (int)sqrt((double)l);
  const int m = l - n * n - n;
  const int hh = n * (n + 1) / 2 + (m < 0 ? -m : m);
  const double* L = lam + ((size_t)i * Kh + hh) * 4;
  const double h = sqrt(part[i].w0) / part[i].a;
  const double dl = dlr[(size_t)i * Kh + hh];
  const double c = coef[t];
  if (op == SBIE_OP_SP) {
    cself[t] = fma(h * L[2], dl, 0.5) * c;
    E[t] = L[2] * c;
  } else {
    cself[t] = h * L[1] * dl * c;
    E[t] = L[1] * c;
  }
}

// Near part: one wave per (target particle, 64 target nodes, quarter of its
// near-source list); every near source's exterior expansion is differentiated
// in (u, v, phi) at the mapped target and its lab gradient is projected on the
// target's normal.
template <int PMAX, bool EXACT>
__global__ __launch_bounds__((64 * kNearWaves<kUnrollOrders<PMAX, EXACT>>)) __attribute__((amdgpu_waves_per_eu(3))) void k_near_normal(
    const Particle* __restrict__ part, const double* __restrict__ x, const double* __restrict__ y,
    const double* __restrict__ z, const double* __restrict__ nx, const double* __restrict__ ny,
    const double* __restrict__ nz, const int32_t* __restrict__ near_ptr, const int32_t* __restrict__ near_src,
    const double* __restrict__ E, const double* __restrict__ lam, const double* __restrict__ ab,
    const double* __restrict__ cd, const double* __restrict__ rcp, int p_arg, int T, int chunks, int64_t Nn,
    unsigned* status, double* __restrict__ unear) {
  const int p = EXACT ? PMAX : p_arg;  // exact order: degree bounds known at compile time
  // one workgroup per (target particle, 64 W target nodes, quarter of its
  // near-source list)
  constexpr int W = kNearWaves<kUnrollOrders<PMAX, EXACT>>;
  const int wgs = (chunks + W - 1) / W;
  const int q4 = blockIdx.x % kNearSplit, rest = blockIdx.x / kNearSplit;
  const int j = rest / wgs;
  const int t = (rest - j * wgs) * 64 * W + threadIdx.x;
  const bool live = t < T;
  const int64_t g = (int64_t)j * T + (live ? t : 0);
  const double X0 = x[g], X1 = y[g], X2 = z[g];
  const double n0 = nx[g], n1 = ny[g], n2 = nz[g];
  const int K = (p + 1) * (p + 1), Kh = (p + 1) * (p + 2) / 2;
  __shared__ NearTablesFor<PMAX, kUnrollOrders<PMAX, EXACT>, 1> tb;
  near_tables_init<PMAX, kUnrollOrders<PMAX, EXACT>, 1>(tb, ab, cd);
  double acc = 0.0;
  unsigned bad = 0u;
  const int cap = (int)status[1];  // the geometry's recurrence step cap
  const int l0 = near_ptr[j], nl = near_ptr[j + 1] - l0;
  const int s_begin = l0 + (nl * q4) / kNearSplit, s_end = l0 + (nl * (q4 + 1)) / kNearSplit;
  for (int sidx = s_begin; sidx < s_end; ++sidx) {
    const int i = near_src[sidx];
    const Particle P = part[i];
    const SpheroidalPoint q = to_spheroidal(P, X0, X1, X2, true, &bad);
    // the derivative along the target normal as one directional derivative of
    // the basis: nu.grad = (nu.al) d/du + (nu.be) d/dv + (nu.ga) d/dphi
    double al[3], be[3], ga[3];
    lab_gradient_coeffs(P, q.u, q.sw, q.v, q.sv, q.c1, q.s1, al, be, ga);
    const double cu = al[0] * n0 + al[1] * n1 + al[2] * n2;
    const double cv = be[0] * n0 + be[1] * n1 + be[2] * n2;
    const double cp = ga[0] * n0 + ga[1] * n1 + ga[2] * n2;
    const NearSourceView src =
        near_source<PMAX, kUnrollOrders<PMAX, EXACT>, 1>(tb, P.oblate != 0, E + (size_t)i * K, lam + (size_t)i * Kh * 4, ab, cd, K, Kh);
    const double* Ei = src.E;
    double dn = 0.0;
    if constexpr (kUnrollOrders<PMAX, EXACT>) {
      // per-order sums of the value and the scaled u and v derivatives of the
      // cosine (c) and sine (s) terms; the 1/w and 1/(1 - v^2) of the
      // derivatives folded into the direction once per source
      const double cuw = cu / q.w, cvw = cv / (q.sv * q.sv);
      double a0c = 0.0, a0s = 0.0, auc = 0.0, aus = 0.0, avc = 0.0, avs = 0.0;
      expansion_orders<PMAX>(
          q, P.oblate != 0, src.ab, src.cd, rcp, src.qt, cap, &bad, [](int, double, double) {},
          [&](int lc, int ls, int m, double t0, double tu, double tv) {
            const double ec = Ei[lc];
            a0c = fma(ec, t0, a0c);
            auc = fma(ec, tu, auc);
            avc = fma(ec, tv, avc);
            if (m > 0) {
              const double es = Ei[ls];
              a0s = fma(es, t0, a0s);
              aus = fma(es, tu, aus);
              avs = fma(es, tv, avs);
            }
          },
          [&](int m, double c, double s) {
            dn += fma(cuw, fma(c, auc, s * aus), fma(cvw, fma(c, avc, s * avs), cp * (double)m * fma(c, a0s, -s * a0c)));
            a0c = a0s = auc = aus = avc = avs = 0.0;
          });
    } else {
      expansion_terms<PMAX>(q, P.oblate != 0, src.L, src.ab, src.cd, rcp, p, cap, &bad,
                            [&](int lc, int ls, int m, double, double a1, double a2, double ap, double, double b1,
                                double b2, double bp) {
                              dn = fma(Ei[lc], fma(cp, ap, fma(cv, a2, cu * a1)), dn);
                              if (m > 0) dn = fma(Ei[ls], fma(cp, bp, fma(cv, b2, cu * b1)), dn);
                            });
    }
    acc += dn;
  }
  if (bad) atomicOr(status, bad);
  if (live) unear[(size_t)q4 * Nn + g] = acc;
}

// Far part: the differentiated kernels summed over the far source nodes, with
// d = x - y, q = W dens and the target normal nu_x:
//  S'  -q (nu_x.d) / r^3
//  D'   q (nu_x.nu_y / r^3 - 3 (nu_y.d)(nu_x.d) / r^5)
// Grid as the other direct sums (target tiles x source splits, split fastest);
// coordinates relative to the source centre; each source particle's tile sum
// is added per target under the exclusion flag with TwoSum.
template <typename R, int OP, int TPT>
__global__ __launch_bounds__(256) void k_far_normal(const R* __restrict__ rec, const Particle* __restrict__ part,
                                                    const double* __restrict__ x, const double* __restrict__ y,
                                                    const double* __restrict__ z, const double* __restrict__ nx,
                                                    const double* __restrict__ ny, const double* __restrict__ nz,
                                                    const uint32_t* __restrict__ excl, int words, int M, int T,
                                                    int64_t N, int nsplit, double* __restrict__ partial) {
  const int split = blockIdx.x % nsplit, tile = blockIdx.x / nsplit;
  const int s0 = (int)((int64_t)M * split / nsplit), s1 = (int)((int64_t)M * (split + 1) / nsplit);
  double tx[TPT], ty[TPT], tz[TPT];
  R tn[TPT][3], acc[TPT], lo[TPT];
  int tp[TPT];
  bool live[TPT];
#pragma unroll
  for (int k = 0; k < TPT; ++k) {
    const int64_t gq = (int64_t)tile * 256 * TPT + k * 256 + threadIdx.x;
    live[k] = gq < N;
    const int64_t gg = live[k] ? gq : 0;
    tx[k] = x[gg];
    ty[k] = y[gg];
    tz[k] = z[gg];
    tn[k][0] = (R)nx[gg];
    tn[k][1] = (R)ny[gg];
    tn[k][2] = (R)nz[gg];
    tp[k] = (int)(gg / T);
    acc[k] = lo[k] = R(0);
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
    R Dx[TPT], Dy[TPT], Dz[TPT], tmp[TPT];
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
      Dx[k] = (R)(tx[k] - cx);
      Dy[k] = (R)(ty[k] - cy);
      Dz[k] = (R)(tz[k] - cz);
      tmp[k] = R(0);
    }
    const R* rs = rec + (size_t)s * T * 8;
    for (int q = 0; q < T; ++q) {
      const R* r = rs + (size_t)q * 8;
      const R ox = r[0], oy = r[1], oz = r[2], qq = r[3];
#pragma unroll
      for (int k = 0; k < TPT; ++k) {
        const R dx = Dx[k] - ox, dy = Dy[k] - oy, dz = Dz[k] - oz;
        const R r2 = fma(dz, dz, fma(dy, dy, dx * dx));
        const R ri = rsq_t<R>(r2);
        const R ri3 = ri * ri * ri;
        const R nxd = fma(tn[k][2], dz, fma(tn[k][1], dy, tn[k][0] * dx));
        if (OP == SBIE_OP_SP) {
          tmp[k] = fma(-qq * nxd, ri3, tmp[k]);
        } else {
          const R m0 = r[4], m1 = r[5], m2 = r[6];
          const R nyd = fma(m2, dz, fma(m1, dy, m0 * dx));
          const R nn = fma(tn[k][2], m2, fma(tn[k][1], m1, tn[k][0] * m0));
          tmp[k] = fma(qq * ri3, fma(R(-3) * nyd * nxd, ri * ri, nn), tmp[k]);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < TPT; ++k) two_sum_add(acc[k], lo[k], need[k] ? tmp[k] : R(0));
  }
#pragma unroll
  for (int k = 0; k < TPT; ++k) {
    const int64_t gq = (int64_t)tile * 256 * TPT + k * 256 + threadIdx.x;
    if (live[k]) partial[(size_t)split * N + gq] = ((double)acc[k] + (double)lo[k]) * kInv4Pi;
  }
}

// u = u_self / sqrt(u0^2 -+ v^2) (the modified basis of the self expansions)
// + u_near + the far partials in split order (+ the running reverse sums of
// the pair-symmetric far field, when racc is set).
__global__ void k_normal_assemble(const double* __restrict__ uself, const double* __restrict__ wS,
                                  const double* __restrict__ unear, const double* __restrict__ partial, int nsplit,
                                  const double* __restrict__ racc, int p, int64_t N, uint32_t parts,
                                  double* __restrict__ out) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  const int Nphi = 2 * p + 2, T = (p + 1) * Nphi;
  const int i = (int)(g / T), j = (int)((g - (int64_t)i * T) / Nphi);
  double u = 0.0;
  if (parts & SBIE_PARTS_SELF) u += uself[g] / wS[(size_t)i * (p + 1) + j];
  if (parts & SBIE_PARTS_NEAR)
    for (int q = 0; q < kNearSplit; ++q) u += unear[(size_t)q * N + g];
  if (parts & SBIE_PARTS_FAR) {
    double f = 0.0;
    for (int s = 0; s < nsplit; ++s) f += partial[(size_t)s * N + g];
    if (racc) f += racc[g] * kInv4Pi;
    u += f;
  }
  out[g] = u;
}

template <int PMAX, bool EXACT>
void launch_near_normal(sbie_geom* g, hipStream_t s) {
  const int chunks = (g->T + 63) / 64;
  constexpr int W = kNearWaves<kUnrollOrders<PMAX, EXACT>>;
  hipLaunchKernelGGL((k_near_normal<PMAX, EXACT>), dim3(g->M * ((chunks + W - 1) / W) * kNearSplit), dim3(64 * W), 0,
                     s, g->d_part, g->d_x,
                     g->d_y, g->d_z, g->d_nx, g->d_ny, g->d_nz, g->d_near_ptr, g->d_near_src, g->d_E, g->d_lam,
                     g->d_ab, g->d_cd, g->d_rcp, g->p, g->T, chunks, g->N, g->d_status, g->d_unear);
}

template <typename R, int OP>
void launch_normal_prep(sbie_geom* g, const double* d_dens, hipStream_t s) {
  hipLaunchKernelGGL((k_normal_prep<R, OP>), dim3(cdiv(g->N, 256)), dim3(256), 0, s, g->d_part, d_dens, g->d_x,
                     g->d_y, g->d_z, g->d_nx, g->d_ny, g->d_nz, g->d_w, g->d_wS, g->p, g->N, g->d_f,
                     reinterpret_cast<R*>(g->d_src));
}

template <typename R, int OP>
void launch_far_normal(sbie_geom* g, hipStream_t s) {
  constexpr int TPT = 2;
  const dim3 grid(cdiv(g->N, 256 * TPT) * g->nsplit);
  hipLaunchKernelGGL((k_far_normal<R, OP, TPT>), grid, dim3(256), 0, s, reinterpret_cast<const R*>(g->d_src),
                     g->d_part, g->d_x, g->d_y, g->d_z, g->d_nx, g->d_ny, g->d_nz, g->d_excl, g->excl_words, g->M,
                     g->T, g->N, g->nsplit, g->d_partial);
}

}  // namespace

sbie_status normal_records(sbie_geom* g, int op, int prec, const double* d_dens, hipStream_t s) {
  const bool mixed = prec == SBIE_MIXED;
  if (op == SBIE_OP_SP)
    mixed ? launch_normal_prep<float, SBIE_OP_SP>(g, d_dens, s) : launch_normal_prep<double, SBIE_OP_SP>(g, d_dens, s);
  else
    mixed ? launch_normal_prep<float, SBIE_OP_DP>(g, d_dens, s) : launch_normal_prep<double, SBIE_OP_DP>(g, d_dens, s);
  SBIE_HIP(hipGetLastError());
  return SBIE_OK;
}

sbie_status normal_expansions(sbie_geom* g, int op, int prec, hipStream_t s) {
  const int M = g->M, p = g->p, T = g->T, K = g->K;
  sbie_status st = gemm(prec == SBIE_MIXED, g->d_f, T, g->d_An, g->d_An32, K, g->d_coef, K, M, K, T, s);
  if (st) return st;
  hipLaunchKernelGGL(k_normal_scale, dim3(cdiv((int64_t)M * K, 256)), dim3(256), 0, s, g->d_coef, g->d_lam,
                     g->d_dlr, g->d_part, M, p, op, g->d_cself, g->d_E);
  SBIE_HIP(hipGetLastError());
  return SBIE_OK;
}

sbie_status apply_normal(sbie_geom* g, int op, int prec, const double* d_dens, double* d_out, hipStream_t s,
                         uint32_t parts, bool timed) {
  const int M = g->M, p = g->p, T = g->T, K = g->K;
  const int64_t N = g->N;
  const bool mixed = prec == SBIE_MIXED;
  hipEvent_t* ev = nullptr;
  if (timed) {
    sbie_status st = next_timing_set(g, &ev);
    if (st) return st;
    SBIE_HIP(hipEventRecord(ev[0], s));
  }
  sbie_status st0 = normal_records(g, op, prec, d_dens, s);
  if (st0) return st0;
  if (timed) SBIE_HIP(hipEventRecord(ev[1], s));
  if (parts & (SBIE_PARTS_SELF | SBIE_PARTS_NEAR)) {
    sbie_status st = normal_expansions(g, op, prec, s);
    if (st) return st;
  }
  if (parts & SBIE_PARTS_SELF) {
    sbie_status st = gemm(mixed, g->d_cself, K, g->d_Sy, g->d_Sy32, T, g->d_uself, T, M, T, K, s);
    if (st) return st;
  }
  if (timed) SBIE_HIP(hipEventRecord(ev[2], s));
  if (timed) SBIE_HIP(hipEventRecord(ev[6], s));
  if ((parts & SBIE_PARTS_NEAR) && g->n_near > 0) {
    dispatch_order(p, [&](auto pm, auto ex) { launch_near_normal<decltype(pm)::value, decltype(ex)::value>(g, s); });
    SBIE_HIP(hipGetLastError());
  }
  if (timed) SBIE_HIP(hipEventRecord(ev[7], s));
  // far field through the tree (SBIE_FAR_TREE, FP64 sums), else on the
  // pair-symmetric matrix-core kernel (T >= 32), small T on the vector-unit sums
  const bool tree = (parts & SBIE_FAR_TREE) != 0;
  const bool pairs = !tree && T >= 32;
  if ((parts & SBIE_PARTS_FAR) && tree) {
    if (timed) SBIE_HIP(hipEventRecord(ev[3], s));
    sbie_status st = far_tree_normal(g, op, d_dens, s);
    if (st) return st;
    if (timed) SBIE_HIP(hipEventRecord(ev[4], s));
  } else if ((parts & SBIE_PARTS_FAR) && pairs) {
    sbie_status st = far_mfma(g, op, prec, d_dens, s, timed ? ev[3] : nullptr, timed ? ev[4] : nullptr);
    if (st) return st;
  } else {
    if (timed) SBIE_HIP(hipEventRecord(ev[3], s));
    if (parts & SBIE_PARTS_FAR) {
      if (op == SBIE_OP_SP)
        mixed ? launch_far_normal<float, SBIE_OP_SP>(g, s) : launch_far_normal<double, SBIE_OP_SP>(g, s);
      else
        mixed ? launch_far_normal<float, SBIE_OP_DP>(g, s) : launch_far_normal<double, SBIE_OP_DP>(g, s);
      SBIE_HIP(hipGetLastError());
    }
    if (timed) SBIE_HIP(hipEventRecord(ev[4], s));
  }
  const uint32_t sum_parts = g->n_near > 0 ? parts : (parts & ~(uint32_t)SBIE_PARTS_NEAR);
  const int nslices = pairs ? far_launch_splits(g, far_row_groups(g, !mixed)) : g->nsplit;
  hipLaunchKernelGGL(k_normal_assemble, dim3(cdiv(N, 256)), dim3(256), 0, s, g->d_uself, g->d_wS, g->d_unear,
                     g->d_partial, nslices, pairs ? (const double*)g->d_racc : nullptr, p, N, sum_parts, d_out);
  SBIE_HIP(hipGetLastError());
  if (timed) SBIE_HIP(hipEventRecord(ev[5], s));
  return SBIE_OK;
}

}  // namespace sbie
