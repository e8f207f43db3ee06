// Particle-to-target evaluation (Section 4, the particle-to-target variant of
// Algorithm 1): S or D of a nodal density, and its gradient (Eq.
// (dSLevalformula) and the same construction for D), at arbitrary points
// outside every particle.  Each (target, source particle) pair is classified
// on its own by the exact distance from the point to the surface: near
// sources contribute their exterior expansion (value and derivatives in
// (u, v, phi), mapped to the lab gradient), far ones the smooth quadrature.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>

#include "far_dev.h"
#include "near_dev.h"
#include "sbie_internal.h"

namespace sbie {

namespace {

constexpr double kInv4Pi = 0.079577471545947667884441881686257181;
constexpr double kHalfPi = 1.57079632679489661923132169163975144;

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

__global__ void k_targets_soa(const double* __restrict__ pts, int64_t n, double* __restrict__ tx,
                              double* __restrict__ ty, double* __restrict__ tz) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  tx[t] = pts[3 * t];
  ty[t] = pts[3 * t + 1];
  tz[t] = pts[3 * t + 2];
}

// Distance from a meridian-plane point (rho, z >= 0) outside the ellipse
// (A cos t, C sin t) to the ellipse.  The foot of the normal has t in
// [0, pi/2] where g(t) = (A^2 - C^2) sin t cos t - rho A sin t + z C cos t
// vanishes; g(0) >= 0 >= g(pi/2) and the root is unique outside the ellipse,
// so 64 halvings of the bracket locate it to the resolution of t.
__device__ inline double meridian_distance(double rho, double z, double A, double C) {
  double lo = 0.0, hi = kHalfPi;
  const double e = (A - C) * (A + C);
  for (int it = 0; it < 64; ++it) {
    const double mid = 0.5 * (lo + hi);
    double sn, cs;
    sincos(mid, &sn, &cs);
    const double gm = fma(e * sn, cs, fma(-rho * A, sn, z * C * cs));
    if (gm > 0.0)
      lo = mid;
    else
      hi = mid;
  }
  double sn, cs;
  sincos(0.5 * (lo + hi), &sn, &cs);
  const double dr = rho - A * cs, dz = z - C * sn;
  return sqrt(dr * dr + dz * dz);
}

// Near flags near[t][w] (bit b of word w: particle 32w + b) by the rule
// distance < eta * diam(source); the circumsphere bound |x - c| - diam/2
// settles most pairs without the exact distance.  A point inside a particle
// sets kStatExterior.  One wave per (target, 64 particles), a lane per
// particle, so that only the particles near the wave's one target take the
// exact distance (a wave of 64 targets would run it for the union of their
// candidates); the flags are the wave's ballot.  The units run grid-stride.
__global__ __launch_bounds__(256) void k_classify_targets(const Particle* __restrict__ part, int M, int words,
                                                          double eta, const double* __restrict__ tx,
                                                          const double* __restrict__ ty,
                                                          const double* __restrict__ tz, int64_t n,
                                                          uint32_t* __restrict__ mask, unsigned* status) {
  const int chunks = (M + 63) / 64;
  const int lane = threadIdx.x & 63;
  const int64_t units = n * chunks;
  const int64_t stride = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t u = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); u < units; u += stride) {
    const int64_t t = u / chunks;
    const int c = (int)(u - t * chunks);
    const int i = 64 * c + lane;
    const double X0 = tx[t], X1 = ty[t], X2 = tz[t];
    bool near = false, inside = false;
    if (i < M) {
      const Particle& P = part[i];
      const double d0 = X0 - P.c[0], d1 = X1 - P.c[1], d2 = X2 - P.c[2];
      const double lim = eta * P.diam;
      // |x - c| - diam/2 >= lim, squared (no square root for the far pairs)
      const double rr = lim + 0.5 * P.diam;
      if (fma(d2, d2, fma(d1, d1, d0 * d0)) < rr * rr) {
        const double b0 = P.R[0] * d0 + P.R[3] * d1 + P.R[6] * d2;
        const double b1 = P.R[1] * d0 + P.R[4] * d1 + P.R[7] * d2;
        const double b2 = P.R[2] * d0 + P.R[5] * d1 + P.R[8] * d2;
        const double rho = sqrt(b0 * b0 + b1 * b1), z = fabs(b2);
        if ((rho / P.A) * (rho / P.A) + (z / P.C) * (z / P.C) <= 1.0)
          inside = near = true;
        else
          near = meridian_distance(rho, z, P.A, P.C) < lim;
      }
    }
    const uint64_t bits = __ballot(near);
    if (lane == 0) {
      mask[(size_t)t * words + 2 * c] = (uint32_t)bits;
      if (2 * c + 1 < words) mask[(size_t)t * words + 2 * c + 1] = (uint32_t)(bits >> 32);
    }
    if (__any(inside) && lane == 0) atomicOr(status, kStatExterior);
  }
}

// Sort key of each target: its first near particle, or M with none (whose
// near part is then zero, written here).
__global__ void k_target_keys(const uint32_t* __restrict__ mask, int words, int M, int64_t n,
                              uint32_t* __restrict__ key, double* __restrict__ nearv) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  uint32_t k = (uint32_t)M;
  for (int w = 0; w < words; ++w) {
    const uint32_t m = mask[(size_t)t * words + w];
    if (m) {
      k = 32u * (uint32_t)w + (uint32_t)__builtin_ctz(m);
      break;
    }
  }
  key[t] = k;
  if (k == (uint32_t)M)
    for (int c = 0; c < 4; ++c) nearv[(size_t)c * n + t] = 0.0;
}

__global__ void k_fill_u32(uint32_t* __restrict__ a, int64_t count, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) a[i] = v;
}

__global__ void k_key_count(const uint32_t* __restrict__ key, int64_t n, uint32_t* __restrict__ cnt) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) atomicAdd(&cnt[key[t]], 1u);
}

// Exclusive prefix sums of cnt[0..nb) in place, by one workgroup of 256 lanes
// in blocks of 256 values; cnt[nb] receives the total of cnt[0..nb-1) (the
// targets with a near particle, whose keys are below nb - 1 = M).
__global__ __launch_bounds__(256) void k_key_offsets(uint32_t* __restrict__ cnt, int nb) {
  __shared__ uint32_t s[256];
  __shared__ uint32_t carry;
  const int tid = threadIdx.x;
  if (tid == 0) carry = 0u;
  __syncthreads();
  for (int base = 0; base < nb; base += 256) {
    const int i = base + tid;
    const uint32_t v = i < nb ? cnt[i] : 0u;
    s[tid] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      const uint32_t add = tid >= off ? s[tid - off] : 0u;
      __syncthreads();
      s[tid] += add;
      __syncthreads();
    }
    const uint32_t c0 = carry;
    if (i < nb) cnt[i] = c0 + s[tid] - v;
    if (i == nb - 1) cnt[nb] = c0 + s[tid] - v;
    __syncthreads();
    if (tid == 255) carry = c0 + s[255];
    __syncthreads();
  }
}

// perm: targets grouped by key (the order within a group is immaterial: every
// target's result depends on its own point only).
__global__ void k_key_scatter(const uint32_t* __restrict__ key, int64_t n, uint32_t* __restrict__ off,
                              uint32_t* __restrict__ perm) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) perm[atomicAdd(&off[key[t]], 1u)] = (uint32_t)t;
}

// Near part: one wave per 64 targets of the key order (slots below *nnear:
// the targets with a near particle, grouped by their first one, so that a
// wave's targets share their near particles).  The wave visits every particle
// that is near to any of its lanes; all lanes evaluate the expansion (each
// lane's recurrence from its own depth), lanes whose target is not near that
// particle map a stand-in point two diameters from its centre and discard the
// result.  out[4][n]: value and lab gradient, at the targets' own indices.
template <int PMAX>
__global__ __launch_bounds__(64) void k_near_targets(
    const Particle* __restrict__ part, const double* __restrict__ tx, const double* __restrict__ ty,
    const double* __restrict__ tz, int64_t n, const uint32_t* __restrict__ perm, const uint32_t* __restrict__ nnear,
    const uint32_t* __restrict__ mask, int words, int M,
    const double* __restrict__ E, const double* __restrict__ lam, const double* __restrict__ ab,
    const double* __restrict__ cd, const double* __restrict__ rcp, int p, unsigned* status,
    double* __restrict__ out) {
  const int64_t slot = (int64_t)blockIdx.x * 64;
  const int64_t nn = (int64_t)*nnear;
  if (slot >= nn) return;  // wave-uniform
  const bool live = slot + threadIdx.x < nn;
  const int64_t t = live ? (int64_t)perm[slot + threadIdx.x] : 0;
  const int64_t tt = t;
  const double X0 = tx[tt], X1 = ty[tt], X2 = tz[tt];
  const int K = (p + 1) * (p + 1), Kh = (p + 1) * (p + 2) / 2;
  double v = 0.0, g0 = 0.0, g1 = 0.0, g2 = 0.0;
  unsigned bad = 0u;
  const int cap = (int)status[1];  // the geometry's recurrence step cap
  for (int w = 0; w < words; ++w) {
    const uint32_t mine = live ? mask[(size_t)tt * words + w] : 0u;
    uint32_t all = mine;
    for (int off = 32; off >= 1; off >>= 1) all |= (uint32_t)__shfl_xor((int)all, off, 64);
    all = __builtin_amdgcn_readfirstlane(all);
    while (all) {
      const int b = __builtin_ctz(all);
      all &= all - 1u;
      const int i = 32 * w + b;
      if (i >= M) break;
      const bool use = (mine >> b) & 1u;
      const Particle P = part[i];
      const double px = use ? X0 : P.c[0] + 2.0 * P.diam;
      const double py = use ? X1 : P.c[1];
      const double pz = use ? X2 : P.c[2];
      unsigned lb = 0u;
      const SpheroidalPoint q = to_spheroidal(P, px, py, pz, true, &lb);
      double Phi[1], Pu[1], Pv[1], Pp[1];
      expansion_derivatives<PMAX, 1>(q, P.oblate != 0, E + (size_t)i * K, (size_t)K, lam + (size_t)i * Kh * 4, ab,
                                     cd, rcp, p, cap, &lb, Phi, Pu, Pv, Pp, true);
      double gr[3];
      lab_gradient(P, q.u, q.sw, q.v, q.sv, q.c1, q.s1, Pu[0], Pv[0], Pp[0], gr);
      if (use) {
        v += Phi[0];
        g0 += gr[0];
        g1 += gr[1];
        g2 += gr[2];
        bad |= lb;
      }
    }
  }
  if (bad) atomicOr(status, bad);
  if (live) {
    out[t] = v;
    out[n + t] = g0;
    out[2 * n + t] = g1;
    out[3 * n + t] = g2;
  }
}

// Far part, with d = x - y and q = W dens (records (node - centre, q, nu)):
//  S  value q/r,            gradient -q d/r^3
//  D  value q (nu.d)/r^3,   gradient q (nu/r^3 - 3 (nu.d) d/r^5)
// Target tiles x source splits (split fastest); coordinates relative to the
// source centre; each source particle's tile sum is added per target under
// its far flag with TwoSum.  partial[split][4][n].
template <typename R, int OP, int TPT>
__global__ __launch_bounds__(256) void k_far_targets(const R* __restrict__ rec, const Particle* __restrict__ part,
                                                     const double* __restrict__ tx, const double* __restrict__ ty,
                                                     const double* __restrict__ tz, int64_t n,
                                                     const uint32_t* __restrict__ mask, int words, int M, int T,
                                                     int nsplit, double* __restrict__ partial) {
  const int split = blockIdx.x % nsplit, tile = blockIdx.x / nsplit;
  const int s0 = (int)((int64_t)M * split / nsplit), s1 = (int)((int64_t)M * (split + 1) / nsplit);
  double px[TPT], py[TPT], pz[TPT];
  int64_t tq[TPT];
  bool live[TPT];
  R acc[TPT][4], lo[TPT][4];
#pragma unroll
  for (int k = 0; k < TPT; ++k) {
    const int64_t t = (int64_t)tile * 256 * TPT + k * 256 + threadIdx.x;
    live[k] = t < n;
    tq[k] = live[k] ? t : 0;
    px[k] = tx[tq[k]];
    py[k] = ty[tq[k]];
    pz[k] = tz[tq[k]];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[k][c] = lo[k][c] = R(0);
  }
  for (int s = s0; s < s1; ++s) {
    bool need[TPT];
    bool any = false;
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
      need[k] = live[k] && !((mask[(size_t)tq[k] * words + (s >> 5)] >> (s & 31)) & 1u);
      any |= need[k];
    }
    if (!__any(any)) continue;
    const double cx = part[s].c[0], cy = part[s].c[1], cz = part[s].c[2];
    R Dx[TPT], Dy[TPT], Dz[TPT], tmp[TPT][4];
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
      Dx[k] = (R)(px[k] - cx);
      Dy[k] = (R)(py[k] - cy);
      Dz[k] = (R)(pz[k] - cz);
#pragma unroll
      for (int c = 0; c < 4; ++c) tmp[k][c] = R(0);
    }
    const R* rs = rec + (size_t)s * T * 8;
    for (int j = 0; j < T; ++j) {
      const R* r = rs + (size_t)j * 8;
      const R ox = r[0], oy = r[1], oz = r[2], qq = r[3];
#pragma unroll
      for (int k = 0; k < TPT; ++k) {
        const R dx = Dx[k] - ox, dy = Dy[k] - oy, dz = Dz[k] - oz;
        const R r2 = fma(dz, dz, fma(dy, dy, dx * dx));
        const R ri = rsq_t<R>(r2);
        const R ri2 = ri * ri;
        const R a = qq * ri * ri2;  // q / r^3
        if (OP == SBIE_OP_S) {
          tmp[k][0] = fma(qq, ri, tmp[k][0]);
          tmp[k][1] = fma(-a, dx, tmp[k][1]);
          tmp[k][2] = fma(-a, dy, tmp[k][2]);
          tmp[k][3] = fma(-a, dz, tmp[k][3]);
        } else {
          const R m0 = r[4], m1 = r[5], m2 = r[6];
          const R nd = fma(m2, dz, fma(m1, dy, m0 * dx));
          const R bb = R(-3) * a * nd * ri2;
          tmp[k][0] = fma(a, nd, tmp[k][0]);
          tmp[k][1] = fma(a, m0, fma(bb, dx, tmp[k][1]));
          tmp[k][2] = fma(a, m1, fma(bb, dy, tmp[k][2]));
          tmp[k][3] = fma(a, m2, fma(bb, dz, tmp[k][3]));
        }
      }
    }
#pragma unroll
    for (int k = 0; k < TPT; ++k)
#pragma unroll
      for (int c = 0; c < 4; ++c) two_sum_add(acc[k][c], lo[k][c], need[k] ? tmp[k][c] : R(0));
  }
#pragma unroll
  for (int k = 0; k < TPT; ++k) {
    if (!live[k]) continue;
#pragma unroll
    for (int c = 0; c < 4; ++c)
      partial[((size_t)split * 4 + c) * n + tq[k]] = ((double)acc[k][c] + (double)lo[k][c]) * kInv4Pi;
  }
}

// value = near + far partials (split order); gradient likewise, written [n][3].
__global__ void k_targets_combine(const double* __restrict__ nearv, const double* __restrict__ partial, int nsplit,
                                  int64_t n, double* __restrict__ val, double* __restrict__ grad) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  double o[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    double f = 0.0;
    for (int s = 0; s < nsplit; ++s) f += partial[((size_t)s * 4 + c) * n + t];
    o[c] = nearv[(size_t)c * n + t] + f;
  }
  val[t] = o[0];
  if (grad) {
    grad[3 * t] = o[1];
    grad[3 * t + 1] = o[2];
    grad[3 * t + 2] = o[3];
  }
}

struct DevMem {
  void* p = nullptr;
  ~DevMem() {
    if (p) (void)hipFree(p);
  }
};

sbie_status dev_alloc(DevMem& b, size_t bytes) {
  if (hipMalloc(&b.p, std::max<size_t>(bytes, 256)) != hipSuccess) {
    b.p = nullptr;
    (void)hipGetLastError();
    set_error("device allocation of " + std::to_string(bytes) + " bytes for the target evaluation failed");
    return SBIE_E_NOMEM;
  }
  return SBIE_OK;
}

template <typename R, int OP>
void launch_far_targets(const sbie_geom* g, const double* tx, const double* ty, const double* tz, int64_t n,
                        const uint32_t* mask, int nsplit, double* partial, hipStream_t s) {
  constexpr int TPT = 2;
  hipLaunchKernelGGL((k_far_targets<R, OP, TPT>), dim3(cdiv(n, 256 * TPT) * nsplit), dim3(256), 0, s,
                     reinterpret_cast<const R*>(g->d_src), g->d_part, tx, ty, tz, n, mask, g->excl_words, g->M,
                     g->T, nsplit, partial);
}

template <int PMAX>
void launch_near_targets(const sbie_geom* g, const double* tx, const double* ty, const double* tz, int64_t n,
                         const uint32_t* perm, const uint32_t* nnear, const uint32_t* mask, double* out,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_near_targets<PMAX>, dim3(cdiv(n, 64)), dim3(64), 0, s, g->d_part, tx, ty, tz, n, perm, nnear,
                     mask, g->excl_words, g->M, g->d_E, g->d_lam, g->d_ab, g->d_cd, g->d_rcp, g->p, g->d_status,
                     out);
}

// Work buffers of one evaluation at n points: target coordinates (SoA),
// per-target near masks, near values and gradients, far partials per split,
// sort keys, the key order and the per-key counts.
struct TargetWork {
  double* xyz = nullptr;    // [3][n]
  uint32_t* mask = nullptr; // [n][words]
  double* nearv = nullptr;  // [4][n]
  double* partial = nullptr;  // [nsplit][4][n]
  uint32_t* key = nullptr;  // [n]
  uint32_t* perm = nullptr; // [n]
  uint32_t* cnt = nullptr;  // [M + 2]: per-key counts, then offsets; [M + 1] the targets with a near particle
};

int target_splits(const sbie_geom* g, int64_t n) {
  const int64_t tiles = (n + 511) / 512;
  return (int)std::min<int64_t>({(int64_t)g->M, 64, std::max<int64_t>(1, (2048 + tiles - 1) / tiles)});
}

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Bytes of the work buffers, each 256-byte aligned, as carved by carve_work.
size_t target_work_bytes(const sbie_geom* g, int64_t n) {
  const size_t un = (size_t)n;
  return align256(sizeof(double) * 3 * un) + align256(sizeof(uint32_t) * un * g->excl_words) +
         align256(sizeof(double) * 4 * un) + align256(sizeof(double) * 4 * (size_t)target_splits(g, n) * un) +
         2 * align256(sizeof(uint32_t) * un) + align256(sizeof(uint32_t) * ((size_t)g->M + 2));
}

TargetWork carve_work(const sbie_geom* g, int64_t n, char* base) {
  const size_t un = (size_t)n;
  TargetWork w;
  w.xyz = reinterpret_cast<double*>(base);
  base += align256(sizeof(double) * 3 * un);
  w.mask = reinterpret_cast<uint32_t*>(base);
  base += align256(sizeof(uint32_t) * un * g->excl_words);
  w.nearv = reinterpret_cast<double*>(base);
  base += align256(sizeof(double) * 4 * un);
  w.partial = reinterpret_cast<double*>(base);
  base += align256(sizeof(double) * 4 * (size_t)target_splits(g, n) * un);
  w.key = reinterpret_cast<uint32_t*>(base);
  base += align256(sizeof(uint32_t) * un);
  w.perm = reinterpret_cast<uint32_t*>(base);
  base += align256(sizeof(uint32_t) * un);
  w.cnt = reinterpret_cast<uint32_t*>(base);
  return w;
}

// S or D at n device points [n][3] into val [n] and, if non-NULL, grad [n][3],
// with the work buffers w.  Every work buffer is written before it is read.
sbie_status eval_targets(sbie_geom* g, int op, int prec, const double* d_dens, int64_t n, const double* d_pts,
                         double* d_val, double* d_grad, const TargetWork& w, hipStream_t s) {
  const int nop = op == SBIE_OP_S ? SBIE_OP_SP : SBIE_OP_DP;  // records and exterior coefficients of S / D
  sbie_status st = normal_records(g, nop, prec, d_dens, s);
  if (st) return st;
  // The exterior coefficients come from the FP64 transform in both
  // precisions: evaluated close to a surface, the expansions' gradients
  // magnify the compensated FP32 transform's error in the high orders about
  // tenfold, and the transform is a small share of the call.
  if ((st = normal_expansions(g, nop, SBIE_FP64, s))) return st;
  const int words = g->excl_words;
  const int nsplit = target_splits(g, n);
  double* tx = w.xyz;
  double* ty = tx + n;
  double* tz = ty + n;
  hipLaunchKernelGGL(k_targets_soa, dim3(cdiv(n, 256)), dim3(256), 0, s, d_pts, n, tx, ty, tz);
  SBIE_HIP(hipGetLastError());
  {
    const int64_t units = n * (int64_t)((g->M + 63) / 64);
    const int64_t blocks = std::min<int64_t>(cdiv(units, 4), 262144);
    hipLaunchKernelGGL(k_classify_targets, dim3((unsigned)blocks), dim3(256), 0, s, g->d_part, g->M, words, g->eta,
                       tx, ty, tz, n, w.mask, g->d_status);
  }
  SBIE_HIP(hipGetLastError());
  // the targets grouped by their first near particle (counting sort), so that
  // a wave of the near kernel visits few particles
  const int nb = g->M + 1;
  hipLaunchKernelGGL(k_target_keys, dim3(cdiv(n, 256)), dim3(256), 0, s, w.mask, words, g->M, n, w.key, w.nearv);
  hipLaunchKernelGGL(k_fill_u32, dim3(cdiv((int64_t)nb + 1, 256)), dim3(256), 0, s, w.cnt, (int64_t)nb + 1, 0u);
  hipLaunchKernelGGL(k_key_count, dim3(cdiv(n, 256)), dim3(256), 0, s, w.key, n, w.cnt);
  hipLaunchKernelGGL(k_key_offsets, dim3(1), dim3(256), 0, s, w.cnt, nb);
  hipLaunchKernelGGL(k_key_scatter, dim3(cdiv(n, 256)), dim3(256), 0, s, w.key, n, w.cnt, w.perm);
  SBIE_HIP(hipGetLastError());
  const uint32_t* nnear = w.cnt + nb;
  if (g->p <= 8)
    launch_near_targets<8>(g, tx, ty, tz, n, w.perm, nnear, w.mask, w.nearv, s);
  else if (g->p <= 16)
    launch_near_targets<16>(g, tx, ty, tz, n, w.perm, nnear, w.mask, w.nearv, s);
  else
    launch_near_targets<32>(g, tx, ty, tz, n, w.perm, nnear, w.mask, w.nearv, s);
  SBIE_HIP(hipGetLastError());
  const bool mixed = prec == SBIE_MIXED;
  const uint32_t* mk = w.mask;
  double* pa = w.partial;
  if (op == SBIE_OP_S)
    mixed ? launch_far_targets<float, SBIE_OP_S>(g, tx, ty, tz, n, mk, nsplit, pa, s)
          : launch_far_targets<double, SBIE_OP_S>(g, tx, ty, tz, n, mk, nsplit, pa, s);
  else
    mixed ? launch_far_targets<float, SBIE_OP_D>(g, tx, ty, tz, n, mk, nsplit, pa, s)
          : launch_far_targets<double, SBIE_OP_D>(g, tx, ty, tz, n, mk, nsplit, pa, s);
  SBIE_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_targets_combine, dim3(cdiv(n, 256)), dim3(256), 0, s, (const double*)w.nearv, pa, nsplit, n,
                     d_val, d_grad);
  SBIE_HIP(hipGetLastError());
  return SBIE_OK;
}

// Allocation-free variant's work space: one array per GPU, in device memory
// for the life of the process.  In host code `scratch` names a host-side
// stand-in; its device address comes from hipGetSymbolAddress, once per
// device, and only that address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[SBIE_TARGETS_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

sbie_status scratch_address(int device, char** out) {
  if (device < 0 || device >= kMaxDevices) {
    set_error("device ordinal out of range for the static work space");
    return SBIE_E_INVALID;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return device_error(e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[device] = static_cast<char*>(ptr);
  }
  *out = g_scratch_ptr[device];
  return SBIE_OK;
}

}  // namespace

}  // namespace sbie

using namespace sbie;

extern "C" sbie_status sbie_eval_targets(sbie_geom* g, sbie_op op, sbie_precision prec, const double* density,
                                         int64_t npts, const double* pts, double* val, double* grad, void* stream,
                                         uint32_t flags) {
  if (!g) {
    set_error("geometry is NULL");
    return SBIE_E_INVALID;
  }
  if (op != SBIE_OP_S && op != SBIE_OP_D) {
    set_error("target evaluation takes SBIE_OP_S or SBIE_OP_D");
    return SBIE_E_INVALID;
  }
  if (prec != SBIE_FP64 && prec != SBIE_MIXED) {
    set_error("unknown precision");
    return SBIE_E_INVALID;
  }
  if (npts < 0 || npts > ((int64_t)1 << 31)) {
    set_error("npts must be in [0, 2^31]");
    return SBIE_E_INVALID;
  }
  if (npts == 0) return SBIE_OK;
  if (!density || !pts || !val) {
    set_error("density, pts or val is NULL");
    return SBIE_E_INVALID;
  }
  SBIE_HIP(hipSetDevice(g->ctx->device));
  hipStream_t s = stream ? (hipStream_t)stream : g->ctx->stream;
  const int64_t N = g->N;
  const bool devptr = (flags & SBIE_DEVICE_PTRS) != 0;
  sbie_status st;
  DevMem io;
  const double* dd = density;
  const double* dp = pts;
  double* dv = val;
  double* dg = grad;
  if (!devptr) {
    if ((st = dev_alloc(io, sizeof(double) * ((size_t)N + 7 * (size_t)npts)))) return st;
    double* b = (double*)io.p;
    SBIE_HIP(hipMemcpyAsync(b, density, sizeof(double) * N, hipMemcpyHostToDevice, s));
    SBIE_HIP(hipMemcpyAsync(b + N, pts, sizeof(double) * 3 * npts, hipMemcpyHostToDevice, s));
    dd = b;
    dp = b + N;
    dv = b + N + 3 * npts;
    dg = grad ? b + N + 4 * npts : nullptr;
  }
  DevMem work;
  if ((st = dev_alloc(work, target_work_bytes(g, npts)))) return st;
  st = eval_targets(g, (int)op, (int)prec, dd, npts, dp, dv, dg, carve_work(g, npts, (char*)work.p), s);
  if (st) {
    (void)hipStreamSynchronize(s);  // queued work may still use the buffers freed on return
    return st;
  }
  // the work buffers are freed on return
  SBIE_HIP(hipStreamSynchronize(s));
  if (!devptr) {
    SBIE_HIP(hipMemcpyAsync(val, dv, sizeof(double) * npts, hipMemcpyDeviceToHost, s));
    if (grad) SBIE_HIP(hipMemcpyAsync(grad, dg, sizeof(double) * 3 * npts, hipMemcpyDeviceToHost, s));
    SBIE_HIP(hipStreamSynchronize(s));
  }
  return sbie_geom_sync(g, s);
}

extern "C" sbie_status sbie_eval_targets_noalloc(sbie_geom* g, sbie_op op, sbie_precision prec,
                                                 const double* density, int64_t npts, const double* pts,
                                                 double* val, double* grad, void* stream, uint32_t flags) {
  if (!g) {
    set_error("geometry is NULL");
    return SBIE_E_INVALID;
  }
  if (op != SBIE_OP_S && op != SBIE_OP_D) {
    set_error("target evaluation takes SBIE_OP_S or SBIE_OP_D");
    return SBIE_E_INVALID;
  }
  if (prec != SBIE_FP64 && prec != SBIE_MIXED) {
    set_error("unknown precision");
    return SBIE_E_INVALID;
  }
  if (!(flags & SBIE_DEVICE_PTRS)) {
    set_error("the allocation-free evaluation takes device pointers only (SBIE_DEVICE_PTRS)");
    return SBIE_E_INVALID;
  }
  if (npts < 0 || npts > ((int64_t)1 << 31)) {
    set_error("npts must be in [0, 2^31]");
    return SBIE_E_INVALID;
  }
  if (npts == 0) return SBIE_OK;
  if (!density || !pts || !val) {
    set_error("density, pts or val is NULL");
    return SBIE_E_INVALID;
  }
  const size_t need = target_work_bytes(g, npts);
  if (need > (size_t)SBIE_TARGETS_SCRATCH_BYTES) {
    set_error("the work buffers for " + std::to_string(npts) + " points need " + std::to_string(need) +
              " bytes, more than the static work space of " + std::to_string((size_t)SBIE_TARGETS_SCRATCH_BYTES));
    return SBIE_E_BUDGET;
  }
  SBIE_HIP(hipSetDevice(g->ctx->device));
  char* ws = nullptr;
  sbie_status st = scratch_address(g->ctx->device, &ws);
  if (st) return st;
  hipStream_t s = stream ? (hipStream_t)stream : g->ctx->stream;
  st = eval_targets(g, (int)op, (int)prec, density, npts, pts, val, grad, carve_work(g, npts, ws), s);
  if (st) return st;
  return sbie_geom_sync(g, s);
}
