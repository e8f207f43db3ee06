// The operator apply of Algorithm 1 (and its single-layer variant): forward
// transform, diagonal self interaction with inverse transform, near-field
// exterior expansions, far-field direct sum, assembly.
#include <hip/hip_runtime.h>

#include <cmath>

#include "near_dev.h"
#include "sbie_internal.h"

namespace sbie {

namespace {

constexpr double kInv4Pi = 0.079577471545947667884441881686257181;

using d4 = double __attribute__((ext_vector_type(4)));
using f4 = float __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------- prep

// Transform input and far-field source records.
//  S: f = sqrt(u0^2 -+ v^2) sigma (modified basis, Section 3.2), record (x, y, z, W sigma)
//  D: f = mu, record (x, y, z, W mu nu)
template <int OP>
__global__ void k_prep_f64(const double* __restrict__ dens, const double* __restrict__ x,
                           const double* __restrict__ y, const double* __restrict__ z,
                           const double* __restrict__ nx, const double* __restrict__ ny,
                           const double* __restrict__ nz, const double* __restrict__ w,
                           const double* __restrict__ wS, int p, int64_t N, double* f, double* src) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  const int Nphi = 2 * p + 2, T = (p + 1) * Nphi;
  const double d = dens[g];
  const double q = w[g] * d;
  if (OP == SBIE_OP_S) {
    const int i = (int)(g / T), j = (int)((g - (int64_t)i * T) / Nphi);
    f[g] = wS[(size_t)i * (p + 1) + j] * d;
    double* r = src + 4 * g;
    r[0] = x[g];
    r[1] = y[g];
    r[2] = z[g];
    r[3] = q;
  } else {
    f[g] = d;
    double* r = src + 8 * g;
    r[0] = x[g];
    r[1] = y[g];
    r[2] = z[g];
    r[3] = q * nx[g];
    r[4] = q * ny[g];
    r[5] = q * nz[g];
    r[6] = 0.0;
    r[7] = 0.0;
  }
}

// ---------------------------------------------------------------- transforms (MFMA f64)

// C[rows x cols] = A[rows x kd] * B[kd x cols], row-major.  A workgroup of four
// waves computes a 64 x 64 tile; each wave a 16 x 64 strip as four 16 x 16
// v_mfma_f64_16x16x4f64 accumulators.  Operand layout of the 16x16x4 f64 MFMA
// (measured on gfx950): lane l supplies A[l%16][l/16] and B[l/16][l%16];
// accumulator element r of lane l is C[l/16 + 4*r][l%16].
__global__ __launch_bounds__(256) void k_gemm_f64(const double* __restrict__ A, int lda,
                                                  const double* __restrict__ B, int ldb,
                                                  double* __restrict__ C, int ldc, int rows,
                                                  int cols, int kd) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row0 = blockIdx.y * 64 + wave * 16;
  const int col0 = blockIdx.x * 64;
  const int li = lane & 15, lk = lane >> 4;
  d4 acc[4];
  for (int b = 0; b < 4; ++b) acc[b] = d4{0.0, 0.0, 0.0, 0.0};
  const int r = row0 + li;
  for (int k0 = 0; k0 < kd; k0 += 4) {
    const int k = k0 + lk;
    const double av = (r < rows && k < kd) ? A[(size_t)r * lda + k] : 0.0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int c = col0 + 16 * b + li;
      const double bv = (c < cols && k < kd) ? B[(size_t)k * ldb + c] : 0.0;
      acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[b], 0, 0, 0);
    }
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int c = col0 + 16 * b + li;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int rr = row0 + lk + 4 * e;
      if (rr < rows && c < cols) C[(size_t)rr * ldc + c] = acc[b][e];
    }
  }
}

// The same contraction on the FP32 matrix cores (v_mfma_f32_16x16x4f32:
// accumulator element r of lane l is C[4*(l/16) + r][l%16]), for the mixed
// path.  A is read in double and rounded once; every 32 terms of the inner
// dimension form an FP32 tile that is added into an (hi, lo) pair with TwoSum,
// and the result is written in double.
__global__ __launch_bounds__(256) void k_gemm_f32c(const double* __restrict__ A, int lda,
                                                   const float* __restrict__ B, int ldb,
                                                   double* __restrict__ C, int ldc, int rows, int cols,
                                                   int kd) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row0 = blockIdx.y * 64 + wave * 16;
  const int col0 = blockIdx.x * 64;
  const int li = lane & 15, lk = lane >> 4;
  f4 hi[4], lo[4];
  for (int b = 0; b < 4; ++b) hi[b] = lo[b] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  const int r = row0 + li;
  for (int k0 = 0; k0 < kd; k0 += 32) {
    f4 t[4];
    for (int b = 0; b < 4; ++b) t[b] = f4{0.0f, 0.0f, 0.0f, 0.0f};
    const int kend = k0 + 32 < kd ? k0 + 32 : kd;
    for (int kk = k0; kk < kend; kk += 4) {
      const int k = kk + lk;
      const float av = (r < rows && k < kd) ? (float)A[(size_t)r * lda + k] : 0.0f;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int c = col0 + 16 * b + li;
        const float bv = (c < cols && k < kd) ? B[(size_t)k * ldb + c] : 0.0f;
        t[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, t[b], 0, 0, 0);
      }
    }
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float s = hi[b][e] + t[b][e];
        const float bp = s - hi[b][e];
        lo[b][e] += (hi[b][e] - (s - bp)) + (t[b][e] - bp);
        hi[b][e] = s;
      }
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int c = col0 + 16 * b + li;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int rr = row0 + 4 * lk + e;
      if (rr < rows && c < cols) C[(size_t)rr * ldc + c] = (double)hi[b][e] + (double)lo[b][e];
    }
  }
}

// Nodal single-layer density from the synthesis of modified-basis
// coefficients: sigma = f / sqrt(u0^2 -+ v^2) (Section 3.2), in place.
__global__ void k_unweight_f64(const double* __restrict__ wS, int p, int64_t N, double* f) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  const int Nphi = 2 * p + 2, T = (p + 1) * Nphi;
  const int i = (int)(g / T), j = (int)((g - (int64_t)i * T) / Nphi);
  f[g] = f[g] / wS[(size_t)i * (p + 1) + j];
}

// Diagonal spectra: self coefficients and exterior coefficients per particle.
__global__ void k_scale_coef(const double* __restrict__ coef, const double* __restrict__ lam, int M,
                             int p, int op, double* cself, double* E) {
  const int K = (p + 1) * (p + 1), Kh = (p + 1) * (p + 2) / 2;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)M * K) return;
  const int i = (int)(t / K), l = (int)(t - (int64_t)i * K);
  const int n = (int)sqrt((double)l);
  const int m = l - n * n - n;
  const int h = n * (n + 1) / 2 + (m < 0 ? -m : m);
  const double* L = lam + ((size_t)i * Kh + h) * 4;
  const double c = coef[t];
  if (op == SBIE_OP_S) {
    cself[t] = L[2] * c;
    E[t] = L[2] * c;
  } else {
    cself[t] = L[0] * c;
    E[t] = L[1] * c;
  }
}

// ---------------------------------------------------------------- near field

// One wave per (target particle, 64 target nodes, quarter of its near-source
// list).  Each lane maps its target into the frame of every near source i of
// the quarter (ascending i), finds (u, v, phi) from
// the focal distances and sums E_l Q_n^|m|(u)/Q_n^|m|(u0) Y_l(v, phi).  The
// paper's Legendre algorithm (continued fraction for Q_N/Q_{N-1}, Casoratian,
// backward recurrence; Section 2.3) gives Q_N and Q_{N+1} for orders 0 and 1
// (the continued fraction in Miller's form: the backward recurrence itself
// from a depth where it has converged to double precision); higher orders
// follow from the recurrence in the order at fixed degree, and every column
// Q_n^m, n = m..N+1, from the backward recurrence in n.  All in FP64.
//
// With EXACT the order is PMAX itself (p_arg is ignored): every comparison of
// a degree with p and N = p+1 is then settled at compile time, which keeps the
// unrolled loops free of runtime predicates (otherwise held, and spilled, as
// scalar masks).
//
// With NR > 1 the first nr <= NR densities' expansions (density r's at
// E + r e_stride) share every basis evaluation, in workgroups of two waves
// (128 target nodes); density r's partials go to unear + r kNearSplit Nn.
template <int PMAX, bool EXACT, int NR = 1>
__device__ __forceinline__ void near_f64_body(
    const Particle* __restrict__ part, const double* __restrict__ x, const double* __restrict__ y,
    const double* __restrict__ z, const int32_t* __restrict__ near_ptr,
    const int32_t* __restrict__ near_src, const double* __restrict__ E,
    const double* __restrict__ lam, const double* __restrict__ ab, const double* __restrict__ rcp, int p_arg,
    int T, int chunks, int64_t Nn, unsigned* status, double* __restrict__ unear, int bid, int nr = 1,
    size_t e_stride = 0) {
  const int p = EXACT ? PMAX : p_arg;
  constexpr int W = NR > 1 ? 2 : 1;
  const int wgs = (chunks + W - 1) / W;
  const int q4 = bid % kNearSplit, rest = bid / kNearSplit;
  const int j = rest / wgs;
  const int t = (rest - j * wgs) * 64 * W + threadIdx.x;
  const bool live = t < T;
  const int64_t g = (int64_t)j * T + (live ? t : 0);
  const double X0 = x[g], X1 = y[g], X2 = z[g];
  const int K = (p + 1) * (p + 1), Kh = (p + 1) * (p + 2) / 2, N = p + 1;
  // Tables read with wave-uniform addresses, staged in LDS so that they stay
  // out of the scalar registers: the Ferrers recurrence table and 1/k (once),
  // each source's exterior coefficients times the spectral ratios 1/Q_n^|m|(u0).
  // The coefficients of the recurrence in n come from their own table.
  constexpr int KM = (PMAX + 1) * (PMAX + 1), KHM = (PMAX + 1) * (PMAX + 2) / 2;
  constexpr int KH2M = (PMAX + 2) * (PMAX + 3) / 2, RM = 2 * PMAX + 8;
  __shared__ double s_E[NR * KM], s_ab[2 * KH2M], s_rcp[RM], s_qt[4 * KHM];
  const int Kh2 = (p + 2) * (p + 3) / 2;
  for (int k = threadIdx.x; k < 2 * Kh2; k += 64 * W) s_ab[k] = ab[k];
  for (int k = threadIdx.x; k < RM; k += 64 * W) s_rcp[k] = rcp[k];
  q_recurrence_table<2>(p, s_qt, threadIdx.x, 64 * W);
  const int cap = (int)status[1];  // the geometry's recurrence step cap
  double acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r] = 0.0;
  unsigned bad = 0u;
  const int n0 = near_ptr[j], nn = near_ptr[j + 1] - n0;
  const int s_begin = n0 + (nn * q4) / kNearSplit, s_end = n0 + (nn * (q4 + 1)) / kNearSplit;
  for (int s = s_begin; s < s_end; ++s) {
    const int i = near_src[s];
    const Particle P = part[i];
    __syncthreads();  // the previous source's tables have been read
    for (int k = threadIdx.x; k < NR * K; k += 64 * W) {
      const int r = NR == 1 ? 0 : k / K, l = k - r * K;
      int n = (int)sqrt((double)l);
      n -= n * n > l ? 1 : 0;
      const int m = l - n * n - n;
      s_E[r * KM + l] = r < nr ? E[r * e_stride + (size_t)i * K + l] *
                                     lam[((size_t)i * Kh + n * (n + 1) / 2 + (m < 0 ? -m : m)) * 4 + 3]
                               : 0.0;
    }
    __syncthreads();
    const double* Ei = s_E;
    // lab -> body frame of the source
    const double d0 = X0 - P.c[0], d1 = X1 - P.c[1], d2 = X2 - P.c[2];
    const double b0 = P.R[0] * d0 + P.R[3] * d1 + P.R[6] * d2;
    const double b1 = P.R[1] * d0 + P.R[4] * d1 + P.R[7] * d2;
    const double b2 = P.R[2] * d0 + P.R[5] * d1 + P.R[8] * d2;
    const double rho = sqrt(b0 * b0 + b1 * b1);
    const double a = P.a;
    // sum of the distances to the focal points (prolate) or to the focal ring
    // (oblate) is 2 a cosh(mu): u = cosh(mu) resp. u = sinh(mu)
    double u, w;
    if (!P.oblate) {
      const double f1 = sqrt(rho * rho + (b2 - a) * (b2 - a));
      const double f2 = sqrt(rho * rho + (b2 + a) * (b2 + a));
      const double ch = (f1 + f2) / (2.0 * a);
      u = ch;
      w = (ch - 1.0) * (ch + 1.0);
    } else {
      const double f1 = sqrt((rho + a) * (rho + a) + b2 * b2);
      const double f2 = sqrt((rho - a) * (rho - a) + b2 * b2);
      const double ch = (f1 + f2) / (2.0 * a);
      u = sqrt((ch - 1.0) * (ch + 1.0));
      w = ch * ch;
    }
    if (!(u > P.u0)) bad |= kStatExterior;
    const double sw = sqrt(w);
    const double v = b2 / (a * u);
    const double sv = rho / (a * sw);  // sqrt(1 - v^2)
    const double c1 = rho > 0.0 ? b0 / rho : 1.0, s1 = rho > 0.0 ? b1 / rho : 0.0;
    const double sgn = P.oblate ? 1.0 : -1.0;
    const int L = near_depth(u, sw, N, cap, kStatNumeric, &bad);
    // Q_N^m, Q_{N+1}^m: orders 0 and 1 from the backward recurrence and the
    // Casoratian, higher orders by the upward recurrence in m
    double qn0[2], qn1[2];
    q_top_orders01(u, sw, sgn, N, L, s_rcp, qn0, qn1);
    const double ur = u / sw;
    double fa2 = 0.0, fa1 = 0.0, fb2 = 0.0, fb1 = 0.0;  // F^(m-2), F^(m-1) at degrees N and N+1
    double pbar = 0.28209479177387814347;  // normalised Ferrers Pb_m^m(v), 1/sqrt(4 pi) at m = 0
    double cm = 1.0, sm = 0.0;             // cos(m phi), sin(m phi)
    for_orders<PMAX, kUnrollOrders<PMAX, EXACT>>(p, [&](auto mc) {
      const int m = mc;
      __builtin_amdgcn_sched_barrier(0);  // orders one after the other: bounded live ranges
      if (m > 0) {
        pbar *= s_ab[m * (m + 3)] * sv;  // sqrt((2m+1)/(2m)), row n = m
        const double cn = cm * c1 - sm * s1;
        sm = sm * c1 + cm * s1;
        cm = cn;
      }
      const double qN = m == 0 ? qn0[0] : (m == 1 ? qn0[1] : q_next_order(ur, N, m, fa1, fa2));
      const double qN1 = m == 0 ? qn1[0] : (m == 1 ? qn1[1] : q_next_order(ur, N + 1, m, fb1, fb2));
      fa2 = fa1;
      fa1 = qN;
      fb2 = fb1;
      fb1 = qN1;
      double Q[PMAX + 4];
      q_column_tab<PMAX, 2>(u, N, m, qN, qN1, s_qt + (P.oblate ? 2 * Kh : 0), Q);
      // contraction with the normalised Ferrers functions, forward in n
      double sc[NR], ss[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) sc[r] = ss[r] = 0.0;
      double p2 = 0.0, p1 = pbar;
#pragma unroll
      for (int n = 0; n <= PMAX; ++n) {
        if (n >= m && n <= p) {
          double pn;
          if (n == m) {
            pn = pbar;
          } else if (n == m + 1) {
            pn = s_ab[(m + 1) * (m + 2) + 2 * m] * v * pbar;  // sqrt(2m+3), row n = m+1
            p2 = p1;
            p1 = pn;
          } else {
            const int h = n * (n + 1) / 2 + m;
            pn = s_ab[2 * h] * (v * p1 - s_ab[2 * h + 1] * p2);
            p2 = p1;
            p1 = pn;
          }
          const double t0 = pn * Q[n];
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            sc[r] = fma(Ei[r * KM + n * n + n + m], t0, sc[r]);
            if (m > 0) ss[r] = fma(Ei[r * KM + n * n + n - m], t0, ss[r]);
          }
        }
      }
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        if (m == 0)
          acc[r] += sc[r];
        else
          acc[r] += 1.41421356237309504880 * (sc[r] * cm + ss[r] * sm);
      }
    });
  }
  if (bad) atomicOr(status, bad);
  if (live) {
#pragma unroll
    for (int r = 0; r < NR; ++r)
      if (r < nr) unear[((size_t)r * kNearSplit + q4) * Nn + g] = acc[r];
  }
}

template <int PMAX, bool EXACT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void k_near_f64(
    const Particle* __restrict__ part, const double* __restrict__ x, const double* __restrict__ y,
    const double* __restrict__ z, const int32_t* __restrict__ near_ptr,
    const int32_t* __restrict__ near_src, const double* __restrict__ E,
    const double* __restrict__ lam, const double* __restrict__ ab, const double* __restrict__ rcp, int p_arg,
    int T, int chunks, int64_t Nn, unsigned* status, double* __restrict__ unear) {
  near_f64_body<PMAX, EXACT>(part, x, y, z, near_ptr, near_src, E, lam, ab, rcp, p_arg, T, chunks, Nn, status,
                             unear, (int)blockIdx.x);
}

// Up to four densities' near fields of one geometry, sharing the basis.
template <int PMAX, bool EXACT>
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(3))) void k_near_f64_multi(
    const Particle* __restrict__ part, const double* __restrict__ x, const double* __restrict__ y,
    const double* __restrict__ z, const int32_t* __restrict__ near_ptr,
    const int32_t* __restrict__ near_src, const double* __restrict__ E, size_t e_stride, int nr,
    const double* __restrict__ lam, const double* __restrict__ ab, const double* __restrict__ rcp, int p_arg,
    int T, int chunks, int64_t Nn, unsigned* status, double* __restrict__ unear) {
  near_f64_body<PMAX, EXACT, 4>(part, x, y, z, near_ptr, near_src, E, lam, ab, rcp, p_arg, T, chunks, Nn, status,
                                unear, (int)blockIdx.x, nr, e_stride);
}

// Several geometries' near fields (one order) in one launch: job j owns the
// workgroups [wg_begin_j, wg_begin_{j+1}) and runs those of its own launch.
template <int PMAX, bool EXACT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void k_near_f64_batch(const NearJob* __restrict__ jobs, int njobs) {
  const int bid = (int)blockIdx.x;
  int lo = 0, hi = njobs - 1;  // the last job starting at or before bid
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (jobs[mid].wg_begin <= bid) lo = mid;
    else hi = mid - 1;
  }
  const NearJob& J = jobs[lo];
  near_f64_body<PMAX, EXACT>(J.part, J.x, J.y, J.z, J.near_ptr, J.near_src, J.E, J.lam, J.ab, J.rcp, J.p, J.T,
                             J.chunks, J.N, J.status, J.unear, bid - J.wg_begin);
}

// ---------------------------------------------------------------- far field (FP64)

__device__ inline double rsqrt_f64(double r2) {
  double yv = __builtin_amdgcn_rsq(r2);
  const double h = r2 * yv;
  const double e = fma(-h, yv, 1.0);
  yv = fma(0.5 * yv, e, yv);
  const double h2 = r2 * yv;
  const double e2 = fma(-h2, yv, 1.0);
  return fma(0.5 * yv, e2, yv);
}

// Direct far-field sum.  The grid is (target tiles) x (source splits) with the
// split as the fastest index, so consecutive workgroups -- which the hardware
// spreads round-robin over the eight XCDs -- take different source ranges and
// each XCD's L2 holds one slice of the sources.  A workgroup of 256 lanes owns
// 256*TPT targets; every source particle of its split is skipped per target
// when it is the target's own particle or in its near field (exclusion mask).
// Source records are read with wave-uniform addresses (scalar loads); each
// source particle's contribution is summed on its own before it is added.
template <int OP, int TPT>
__global__ __launch_bounds__(256) void k_far_f64(
    const double* __restrict__ src, const double* __restrict__ x, const double* __restrict__ y,
    const double* __restrict__ z, const uint32_t* __restrict__ excl, int words, int M, int T,
    int64_t N, int nsplit, double* __restrict__ partial) {
  const int split = blockIdx.x % nsplit;
  const int tile = blockIdx.x / nsplit;
  const int s0 = (int)((int64_t)M * split / nsplit), s1 = (int)((int64_t)M * (split + 1) / nsplit);
  double tx[TPT], ty[TPT], tz[TPT], acc[TPT];
  int tp[TPT];
  bool live[TPT];
#pragma unroll
  for (int k = 0; k < TPT; ++k) {
    const int64_t g = (int64_t)tile * 256 * TPT + k * 256 + threadIdx.x;
    live[k] = g < N;
    const int64_t gg = live[k] ? g : 0;
    tx[k] = x[gg];
    ty[k] = y[gg];
    tz[k] = z[gg];
    tp[k] = (int)(gg / T);
    acc[k] = 0.0;
  }
  constexpr int SW = (OP == SBIE_OP_S) ? 4 : 8;
  for (int s = s0; s < s1; ++s) {
    bool need[TPT];
    bool any = false;
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
      need[k] = live[k] && !((excl[(size_t)tp[k] * words + (s >> 5)] >> (s & 31)) & 1u);
      any |= need[k];
    }
    if (!__any(any)) continue;
    double tmp[TPT];
#pragma unroll
    for (int k = 0; k < TPT; ++k) tmp[k] = 0.0;
    const double* rs = src + (size_t)s * T * SW;
    for (int q = 0; q < T; ++q) {
      const double* r = rs + (size_t)q * SW;
      const double sx = r[0], sy = r[1], sz = r[2];
      if (OP == SBIE_OP_S) {
        const double sq = r[3];
#pragma unroll
        for (int k = 0; k < TPT; ++k) {
          const double dx = tx[k] - sx, dy = ty[k] - sy, dz = tz[k] - sz;
          const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
          tmp[k] = fma(sq, rsqrt_f64(r2), tmp[k]);
        }
      } else {
        const double qx = r[3], qy = r[4], qz = r[5];
#pragma unroll
        for (int k = 0; k < TPT; ++k) {
          const double dx = tx[k] - sx, dy = ty[k] - sy, dz = tz[k] - sz;
          const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
          const double ri = rsqrt_f64(r2);
          const double ri3 = ri * ri * ri;
          const double dot = fma(qz, dz, fma(qy, dy, qx * dx));
          tmp[k] = fma(dot, ri3, tmp[k]);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < TPT; ++k) acc[k] += need[k] ? tmp[k] : 0.0;
  }
#pragma unroll
  for (int k = 0; k < TPT; ++k) {
    const int64_t g = (int64_t)tile * 256 * TPT + k * 256 + threadIdx.x;
    if (live[k]) partial[(size_t)split * N + g] = acc[k] * kInv4Pi;
  }
}

// ---------------------------------------------------------------- assembly

// u = u_self + u_near + sum over the forward far partials (split order) + the
// running reverse sums of the pair-symmetric far field (racc, when set).
__global__ void k_assemble_f64(const double* __restrict__ uself, const double* __restrict__ unear,
                               const double* __restrict__ partial, int nsplit, const double* __restrict__ racc,
                               int64_t N, uint32_t parts, double* __restrict__ out) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  double u = 0.0;
  if (parts & SBIE_PARTS_SELF) u += uself[g];
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

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

sbie_status launch_gemm(const double* A, int lda, const double* B, int ldb, double* C, int ldc, int rows,
                        int cols, int kd, hipStream_t s) {
  hipLaunchKernelGGL(k_gemm_f64, dim3(cdiv(cols, 64), cdiv(rows, 64)), dim3(256), 0, s, A, lda, B, ldb, C, ldc,
                     rows, cols, kd);
  SBIE_HIP(hipGetLastError());
  return SBIE_OK;
}

sbie_status launch_gemm32(const double* A, int lda, const float* B, int ldb, double* C, int ldc, int rows,
                          int cols, int kd, hipStream_t s) {
  hipLaunchKernelGGL(k_gemm_f32c, dim3(cdiv(cols, 64), cdiv(rows, 64)), dim3(256), 0, s, A, lda, B, ldb, C, ldc,
                     rows, cols, kd);
  SBIE_HIP(hipGetLastError());
  return SBIE_OK;
}

template <int PMAX, bool EXACT>
void launch_near(sbie_geom* g, hipStream_t s) {
  const int chunks = (g->T + 63) / 64;
  hipLaunchKernelGGL((k_near_f64<PMAX, EXACT>), dim3(g->M * chunks * kNearSplit), dim3(64), 0, s, g->d_part, g->d_x,
                     g->d_y, g->d_z, g->d_near_ptr, g->d_near_src, g->d_E, g->d_lam, g->d_ab, g->d_rcp, g->p, g->T,
                     chunks, g->N, g->d_status, g->d_unear);
}

// nr densities' near fields: density r's coefficients at E + r M K, its
// partials at unear + r kNearSplit N
template <int PMAX, bool EXACT>
void launch_near_multi(sbie_geom* g, const double* E, int nr, double* unear, hipStream_t s) {
  const int chunks = (g->T + 63) / 64;
  hipLaunchKernelGGL((k_near_f64_multi<PMAX, EXACT>), dim3(g->M * ((chunks + 1) / 2) * kNearSplit), dim3(128), 0, s,
                     g->d_part, g->d_x, g->d_y, g->d_z, g->d_near_ptr, g->d_near_src, E, (size_t)g->M * g->K, nr,
                     g->d_lam, g->d_ab, g->d_rcp, g->p, g->T, chunks, g->N, g->d_status, unear);
}

}  // namespace

sbie_status next_timing_set(sbie_geom* g, hipEvent_t** ev) {
  Timing& tm = g->timing;
  if (tm.used == tm.sets.size()) {
    std::vector<hipEvent_t> set(8, nullptr);
    for (int e = 0; e < 8; ++e) SBIE_HIP(hipEventCreate(&set[e]));
    tm.sets.push_back(set);
  }
  *ev = tm.sets[tm.used++].data();
  return SBIE_OK;
}

sbie_status fork_side(sbie_geom* g, hipStream_t s) {
  SBIE_HIP(hipEventRecord(g->ev_fork, s));
  SBIE_HIP(hipStreamWaitEvent(g->side, g->ev_fork, 0));
  return SBIE_OK;
}

sbie_status join_side(sbie_geom* g, hipStream_t s) {
  SBIE_HIP(hipEventRecord(g->ev_join, g->side));
  SBIE_HIP(hipStreamWaitEvent(s, g->ev_join, 0));
  return SBIE_OK;
}

sbie_status apply_laplace(sbie_geom* g, int op, int prec, const double* d_dens, double* d_out, hipStream_t s,
                          uint32_t parts, bool timed) {
  if (op == SBIE_OP_SP || op == SBIE_OP_DP) return apply_normal(g, op, prec, d_dens, d_out, s, parts, timed);
  const int M = g->M, p = g->p, T = g->T, K = g->K;
  const int64_t N = g->N;
  const int B = 256;
  hipEvent_t* ev = nullptr;
  if (timed) {
    sbie_status st = next_timing_set(g, &ev);
    if (st) return st;
    SBIE_HIP(hipEventRecord(ev[0], s));
  }
  // coefficients given (SBIE_INPUT_COEFFS): the transform step is skipped, and
  // the far field's nodal density is their synthesis at the nodes, in FP64
  const bool coef_in = (parts & SBIE_INPUT_COEFFS) != 0;
  const double* coef = g->d_coef;
  if (coef_in) {
    coef = d_dens;
    sbie_status st = launch_gemm(coef, K, g->d_Sy, T, g->d_dens, T, M, T, K, s);
    if (st) return st;
    if (op == SBIE_OP_S) {
      hipLaunchKernelGGL(k_unweight_f64, dim3(cdiv(N, B)), dim3(B), 0, s, g->d_wS, p, N, g->d_dens);
      SBIE_HIP(hipGetLastError());
    }
    d_dens = g->d_dens;
  }
  // prep: transform input and far-field source records
  if (op == SBIE_OP_S)
    hipLaunchKernelGGL(k_prep_f64<SBIE_OP_S>, dim3(cdiv(N, B)), dim3(B), 0, s, d_dens, g->d_x, g->d_y, g->d_z,
                       g->d_nx, g->d_ny, g->d_nz, g->d_w, g->d_wS, p, N, g->d_f, g->d_src);
  else
    hipLaunchKernelGGL(k_prep_f64<SBIE_OP_D>, dim3(cdiv(N, B)), dim3(B), 0, s, d_dens, g->d_x, g->d_y, g->d_z,
                       g->d_nx, g->d_ny, g->d_nz, g->d_w, g->d_wS, p, N, g->d_f, g->d_src);
  SBIE_HIP(hipGetLastError());
  if (timed) SBIE_HIP(hipEventRecord(ev[1], s));
  // part (a) forward transform, part (b) spectra and inverse transform
  const bool mixed = prec == SBIE_MIXED;
  if (parts & (SBIE_PARTS_SELF | SBIE_PARTS_NEAR)) {
    if (!coef_in) {
      sbie_status st = mixed ? launch_gemm32(g->d_f, T, g->d_An32, K, g->d_coef, K, M, K, T, s)
                             : launch_gemm(g->d_f, T, g->d_An, K, g->d_coef, K, M, K, T, s);
      if (st) return st;
    }
    hipLaunchKernelGGL(k_scale_coef, dim3(cdiv((int64_t)M * K, B)), dim3(B), 0, s, coef, g->d_lam, M, p, op,
                       g->d_cself, g->d_E);
    SBIE_HIP(hipGetLastError());
  }
  if (parts & SBIE_PARTS_SELF) {
    sbie_status st = mixed ? launch_gemm32(g->d_cself, K, g->d_Sy32, T, g->d_uself, T, M, T, K, s)
                           : launch_gemm(g->d_cself, K, g->d_Sy, T, g->d_uself, T, M, T, K, s);
    if (st) return st;
  }
  if (timed) SBIE_HIP(hipEventRecord(ev[2], s));
  // part (c) near field, on the apply's stream: the pair-symmetric far kernel
  // fills every compute unit, so running the two concurrently gains nothing
  // measurable (1-2%) and would blur the far kernel's own timing
  const bool near = (parts & SBIE_PARTS_NEAR) && g->n_near > 0;
  if (near) {
    if (timed) SBIE_HIP(hipEventRecord(ev[6], s));
    dispatch_order(p, [&](auto pm, auto ex) { launch_near<decltype(pm)::value, decltype(ex)::value>(g, s); });
    SBIE_HIP(hipGetLastError());
    if (timed) SBIE_HIP(hipEventRecord(ev[7], s));
  } else if (timed) {
    SBIE_HIP(hipEventRecord(ev[6], s));
    SBIE_HIP(hipEventRecord(ev[7], s));
  }
  // part (d) far field: through the tree (SBIE_FAR_TREE), else the
  // pair-symmetric matrix-core kernel (T >= 32, i.e. p >= 3), else the
  // vector-unit sum in FP64
  const bool tree = (parts & SBIE_FAR_TREE) != 0;
  if ((parts & SBIE_PARTS_FAR) && tree) {
    if (timed) SBIE_HIP(hipEventRecord(ev[3], s));
    sbie_status st = far_tree(g, op, prec == SBIE_MIXED, s);
    if (st) return st;
    if (timed) SBIE_HIP(hipEventRecord(ev[4], s));
  } else if ((parts & SBIE_PARTS_FAR) && T >= 32) {
    sbie_status st = far_mfma(g, op, prec, d_dens, s, timed ? ev[3] : nullptr, timed ? ev[4] : nullptr);
    if (st) return st;
  } else if (parts & SBIE_PARTS_FAR) {
    if (timed) SBIE_HIP(hipEventRecord(ev[3], s));
    constexpr int TPT = 2;
    const unsigned tiles = cdiv(N, 256 * TPT);
    if (op == SBIE_OP_S)
      hipLaunchKernelGGL((k_far_f64<SBIE_OP_S, TPT>), dim3(tiles * g->nsplit), dim3(256), 0, s, g->d_src, g->d_x,
                         g->d_y, g->d_z, g->d_excl, g->excl_words, M, T, N, g->nsplit, g->d_partial);
    else
      hipLaunchKernelGGL((k_far_f64<SBIE_OP_D, TPT>), dim3(tiles * g->nsplit), dim3(256), 0, s, g->d_src, g->d_x,
                         g->d_y, g->d_z, g->d_excl, g->excl_words, M, T, N, g->nsplit, g->d_partial);
    SBIE_HIP(hipGetLastError());
    if (timed) SBIE_HIP(hipEventRecord(ev[4], s));
  } else if (timed) {
    SBIE_HIP(hipEventRecord(ev[3], s));
    SBIE_HIP(hipEventRecord(ev[4], s));
  }
  // with no near pairs the near part is empty and is left out of the sum
  const uint32_t sum_parts = g->n_near > 0 ? parts : (parts & ~(uint32_t)SBIE_PARTS_NEAR);
  // the pair kernel writes the forward slices [0, its splits) and the reverse
  // totals; the tree and the vector-unit sum write all nsplit slices
  const bool pairs = !tree && T >= 32;
  const int nslices = pairs ? far_launch_splits(g, far_row_groups(g, !mixed)) : g->nsplit;
  hipLaunchKernelGGL(k_assemble_f64, dim3(cdiv(N, B)), dim3(B), 0, s, g->d_uself, g->d_unear, g->d_partial, nslices,
                     pairs ? (const double*)g->d_racc : nullptr, N, sum_parts, d_out);
  SBIE_HIP(hipGetLastError());
  if (timed) SBIE_HIP(hipEventRecord(ev[5], s));
  return SBIE_OK;
}

sbie_status apply_laplace_batch(sbie_geom* const* gs, int n, int op, int prec, const double* const* d_dens,
                                double* const* d_out, BatchJobs* jobs, hipStream_t s) {
  if (n < 1) return SBIE_OK;
  if (n > jobs->cap) {
    set_error("batch larger than its job tables");
    return SBIE_E_INVALID;
  }
  const int B = 256;
  const bool mixed = prec == SBIE_MIXED;
  const int p = gs[0]->p;
  // each geometry's prep, forward transform, spectra, self part and far
  // strengths: the kernels of apply_laplace, in its order
  for (int k = 0; k < n; ++k) {
    sbie_geom* g = gs[k];
    const int M = g->M, T = g->T, K = g->K;
    const int64_t N = g->N;
    if (g->p != p || !far_batch_fits(g)) {
      set_error("batched geometries must share the order and fit one far-field launch");
      return SBIE_E_INVALID;
    }
    if (op == SBIE_OP_S)
      hipLaunchKernelGGL(k_prep_f64<SBIE_OP_S>, dim3(cdiv(N, B)), dim3(B), 0, s, d_dens[k], g->d_x, g->d_y, g->d_z,
                         g->d_nx, g->d_ny, g->d_nz, g->d_w, g->d_wS, p, N, g->d_f, g->d_src);
    else
      hipLaunchKernelGGL(k_prep_f64<SBIE_OP_D>, dim3(cdiv(N, B)), dim3(B), 0, s, d_dens[k], g->d_x, g->d_y, g->d_z,
                         g->d_nx, g->d_ny, g->d_nz, g->d_w, g->d_wS, p, N, g->d_f, g->d_src);
    SBIE_HIP(hipGetLastError());
    sbie_status st = mixed ? launch_gemm32(g->d_f, T, g->d_An32, K, g->d_coef, K, M, K, T, s)
                           : launch_gemm(g->d_f, T, g->d_An, K, g->d_coef, K, M, K, T, s);
    if (st) return st;
    hipLaunchKernelGGL(k_scale_coef, dim3(cdiv((int64_t)M * K, B)), dim3(B), 0, s, g->d_coef, g->d_lam, M, p, op,
                       g->d_cself, g->d_E);
    SBIE_HIP(hipGetLastError());
    st = mixed ? launch_gemm32(g->d_cself, K, g->d_Sy32, T, g->d_uself, T, M, T, K, s)
               : launch_gemm(g->d_cself, K, g->d_Sy, T, g->d_uself, T, M, T, K, s);
    if (st) return st;
    if ((st = far_strengths(g, op, prec, d_dens[k], s))) return st;
  }
  // one near launch over the geometries with near pairs
  int nn = 0, near_wg = 0;
  for (int k = 0; k < n; ++k) {
    sbie_geom* g = gs[k];
    if (g->n_near == 0) continue;
    NearJob& J = jobs->h_near[nn++];
    J.part = g->d_part;
    J.x = g->d_x;
    J.y = g->d_y;
    J.z = g->d_z;
    J.near_ptr = g->d_near_ptr;
    J.near_src = g->d_near_src;
    J.E = g->d_E;
    J.lam = g->d_lam;
    J.ab = g->d_ab;
    J.rcp = g->d_rcp;
    J.p = g->p;
    J.T = g->T;
    J.chunks = (g->T + 63) / 64;
    J.wg_begin = near_wg;
    J.N = g->N;
    J.status = g->d_status;
    J.unear = g->d_unear;
    near_wg += g->M * J.chunks * kNearSplit;
  }
  // one far launch over all of them
  int far_wg = 0;
  for (int k = 0; k < n; ++k) far_wg += far_batch_job(gs[k], op, prec, far_wg, &jobs->h_far[k]);
  SBIE_HIP(hipMemcpyAsync(jobs->d_near, jobs->h_near, sizeof(NearJob) * nn, hipMemcpyHostToDevice, s));
  SBIE_HIP(hipMemcpyAsync(jobs->d_far, jobs->h_far, sizeof(FarJob) * n, hipMemcpyHostToDevice, s));
  if (nn > 0) {
    dispatch_order(p, [&](auto pm, auto ex) {
      hipLaunchKernelGGL((k_near_f64_batch<decltype(pm)::value, decltype(ex)::value>), dim3((unsigned)near_wg),
                         dim3(64), 0, s, jobs->d_near, nn);
    });
    SBIE_HIP(hipGetLastError());
  }
  sbie_status st = far_batch_launch(gs, n, jobs->d_far, far_wg, op, prec, s);
  if (st) return st;
  // each geometry's assembly (forward slices of its own split count, reverse totals)
  for (int k = 0; k < n; ++k) {
    sbie_geom* g = gs[k];
    const uint32_t sum_parts = g->n_near > 0 ? SBIE_PARTS_ALL : (SBIE_PARTS_ALL & ~(uint32_t)SBIE_PARTS_NEAR);
    const int nslices = far_launch_splits(g, far_row_groups(g, !mixed));
    hipLaunchKernelGGL(k_assemble_f64, dim3(cdiv(g->N, B)), dim3(B), 0, s, g->d_uself, g->d_unear, g->d_partial,
                       nslices, (const double*)g->d_racc, g->N, sum_parts, d_out[k]);
    SBIE_HIP(hipGetLastError());
  }
  return SBIE_OK;
}

sbie_status multi_buffers(sbie_geom* g) {
  if (g->multi) return SBIE_OK;
  const size_t N = (size_t)g->N, MK = (size_t)g->M * g->K, R4 = 4;
  const uint64_t rev_bytes = multi_rev_bytes(g->M, g->T);
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t sz[] = {al(8 * R4 * MK), al(8 * R4 * N), al(8 * R4 * kNearSplit * N), al(8 * R4 * g->nsplit * N),
                       al(8 * R4 * N), al(8 * multi_rec_values(g->M, g->T)), al(rev_bytes), al(8 * 2 * R4 * N)};
  size_t total = 0;
  for (size_t v : sz) total += v;
  MultiWork* mw = new (std::nothrow) MultiWork;
  if (!mw) return SBIE_E_NOMEM;
  if (hipMalloc((void**)&mw->blk, total) != hipSuccess) {
    (void)hipGetLastError();
    delete mw;
    set_error("device allocation of the multi-density work buffers failed");
    return SBIE_E_NOMEM;
  }
  char* p = mw->blk;
  double** dst[] = {&mw->E, &mw->uself, &mw->unear, &mw->partial, &mw->racc, &mw->rec, &mw->rev, &mw->io};
  for (int i = 0; i < 8; ++i) {
    *dst[i] = reinterpret_cast<double*>(p);
    p += sz[i];
  }
  mw->bytes = total;
  mw->rev_bytes = rev_bytes;
  g->footprint += total;
  g->multi = mw;
  return SBIE_OK;
}

sbie_status apply_laplace_multi(sbie_geom* g, int op, int prec, int nr, const double* d_dens, double* d_out,
                                hipStream_t s, uint32_t parts) {
  if (nr < 2 || nr > 4 || g->T < 32 || (op != SBIE_OP_S && op != SBIE_OP_D)) {
    set_error("the multi-density apply takes S or D, 2 to 4 densities and T >= 32");
    return SBIE_E_INVALID;
  }
  sbie_status st = multi_buffers(g);
  if (st) return st;
  MultiWork& mw = *g->multi;
  const int M = g->M, p = g->p, T = g->T, K = g->K;
  const int64_t N = g->N;
  const int B = 256;
  const bool mixed = prec == SBIE_MIXED;
  const bool near = (parts & SBIE_PARTS_NEAR) && g->n_near > 0;
  // per density: prep, forward transform, spectra and self part,
  // the kernels of apply_laplace into the density's own buffers
  for (int k = 0; k < nr; ++k) {
    const double* dk = d_dens + (size_t)k * N;
    double* Ek = mw.E + (size_t)k * M * K;
    if (op == SBIE_OP_S)
      hipLaunchKernelGGL(k_prep_f64<SBIE_OP_S>, dim3(cdiv(N, B)), dim3(B), 0, s, dk, g->d_x, g->d_y, g->d_z,
                         g->d_nx, g->d_ny, g->d_nz, g->d_w, g->d_wS, p, N, g->d_f, g->d_src);
    else
      hipLaunchKernelGGL(k_prep_f64<SBIE_OP_D>, dim3(cdiv(N, B)), dim3(B), 0, s, dk, g->d_x, g->d_y, g->d_z,
                         g->d_nx, g->d_ny, g->d_nz, g->d_w, g->d_wS, p, N, g->d_f, g->d_src);
    SBIE_HIP(hipGetLastError());
    if (parts & (SBIE_PARTS_SELF | SBIE_PARTS_NEAR)) {
      st = mixed ? launch_gemm32(g->d_f, T, g->d_An32, K, g->d_coef, K, M, K, T, s)
                 : launch_gemm(g->d_f, T, g->d_An, K, g->d_coef, K, M, K, T, s);
      if (st) return st;
      hipLaunchKernelGGL(k_scale_coef, dim3(cdiv((int64_t)M * K, B)), dim3(B), 0, s, g->d_coef, g->d_lam, M, p, op,
                         g->d_cself, Ek);
      SBIE_HIP(hipGetLastError());
    }
    if (parts & SBIE_PARTS_SELF) {
      st = mixed ? launch_gemm32(g->d_cself, K, g->d_Sy32, T, mw.uself + (size_t)k * N, T, M, T, K, s)
                 : launch_gemm(g->d_cself, K, g->d_Sy, T, mw.uself + (size_t)k * N, T, M, T, K, s);
      if (st) return st;
    }
  }
  // the near fields of all densities at once: one basis evaluation per
  // (near pair, target, n, m) serves every density
  if (near) {
    dispatch_order(p, [&](auto pm, auto ex) {
      launch_near_multi<decltype(pm)::value, decltype(ex)::value>(g, mw.E, nr, mw.unear, s);
    });
    SBIE_HIP(hipGetLastError());
  }
  // the far field of all densities at once
  const int nsl = multi_splits(g, multi_row_groups(T, !mixed, op));
  if (parts & SBIE_PARTS_FAR) {
    st = far_multi(g, op, mixed, nr, d_dens, s);
    if (st) return st;
  }
  const uint32_t sum_parts = near ? parts : (parts & ~(uint32_t)SBIE_PARTS_NEAR);
  for (int k = 0; k < nr; ++k) {
    hipLaunchKernelGGL(k_assemble_f64, dim3(cdiv(N, B)), dim3(B), 0, s, mw.uself + (size_t)k * N,
                       mw.unear + (size_t)k * kNearSplit * N, mw.partial + (size_t)k * nsl * N, nsl,
                       (const double*)(mw.racc + (size_t)k * N), N, sum_parts, d_out + (size_t)k * N);
    SBIE_HIP(hipGetLastError());
  }
  return SBIE_OK;
}

}  // namespace sbie

namespace sbie {

sbie_status transform_only(sbie_geom* g, int op, const double* d_dens, double* d_coef, hipStream_t s) {
  const int64_t N = g->N;
  const int B = 256;
  if (op == SBIE_OP_S)
    hipLaunchKernelGGL(k_prep_f64<SBIE_OP_S>, dim3(cdiv(N, B)), dim3(B), 0, s, d_dens, g->d_x, g->d_y, g->d_z,
                       g->d_nx, g->d_ny, g->d_nz, g->d_w, g->d_wS, g->p, N, g->d_f, g->d_src);
  else
    hipLaunchKernelGGL(k_prep_f64<SBIE_OP_D>, dim3(cdiv(N, B)), dim3(B), 0, s, d_dens, g->d_x, g->d_y, g->d_z,
                       g->d_nx, g->d_ny, g->d_nz, g->d_w, g->d_wS, g->p, N, g->d_f, g->d_src);
  SBIE_HIP(hipGetLastError());
  return launch_gemm(g->d_f, g->T, g->d_An, g->K, d_coef, g->K, g->M, g->K, g->T, s);
}

}  // namespace sbie

namespace sbie {

sbie_status gemm(bool mixed, const double* A, int lda, const double* B64, const float* B32, int ldb, double* C,
                 int ldc, int rows, int cols, int kd, hipStream_t s) {
  return mixed ? launch_gemm32(A, lda, B32, ldb, C, ldc, rows, cols, kd, s)
               : launch_gemm(A, lda, B64, ldb, C, ldc, rows, cols, kd, s);
}

}  // namespace sbie
