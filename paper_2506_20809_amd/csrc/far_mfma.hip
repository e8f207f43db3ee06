// Far-field direct sum (part (d), Section 4.1 smooth quadrature; Algorithm 1,
// lines 6-8) with the pair distances formed on the matrix cores.
//
// For a target t and a source y = c_s + o in source particle s (centre c_s,
// offset o), with D = t - c_s:
//     |t - y|^2 = |D|^2 - 2 D.o + |o|^2 = [Dx Dy Dz |D|^2] . [-2ox -2oy -2oz 1] + |o|^2,
// a K = 4 contraction between a target row and a source column, so a 16x16x4
// MFMA yields 256 squared distances per instruction with the per-source |o|^2
// as the accumulator input.  The double layer's dipole term is a second
// contraction  d.(t - y) = [Dx Dy Dz |D|^2] . [dx dy dz 0] - d.o.  The vector
// units then only take the reciprocal square root and accumulate.
//
// Sources are padded per particle to a multiple of 16 nodes with zero-strength
// points at the particle centre, and each 16-source block stores its B operand
// in lane order so a lane reads one value.  A wave owns 64 consecutive targets
// as four 16-row blocks; every source particle of the workgroup's split is a
// tile, staged through LDS once per workgroup, whose sum is kept apart and then
// added per target unless the source particle is the target's own or in its
// near field.  FP32 tiles are added into (hi, lo) pairs with TwoSum; the final
// cross-lane reduction is in FP64.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "sbie_internal.h"

namespace sbie {

namespace {

constexpr double kInv4PiD = 0.079577471545947667884441881686257181;

using f4 = float __attribute__((ext_vector_type(4)));
using d4 = double __attribute__((ext_vector_type(4)));

template <typename R>
struct Mfma;

template <>
struct Mfma<float> {
  using V = f4;
  // accumulator element e of lane l holds row 4*(l/16) + e, column l%16
  static __device__ inline int row(int lg, int e) { return 4 * lg + e; }
  static __device__ inline V mma(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ inline float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
};

template <>
struct Mfma<double> {
  using V = d4;
  // accumulator element e of lane l holds row l/16 + 4*e, column l%16
  static __device__ inline int row(int lg, int e) { return lg + 4 * e; }
  static __device__ inline V mma(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // hardware reciprocal square root refined by one Newton step
  static __device__ inline double rsq(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double h = x * y;
    const double e = fma(-h, y, 1.0);
    return fma(0.5 * y, e, y);
  }
};

constexpr int kChunk = 40;  // 16-source blocks staged in LDS at a time

// geo: per block 80 values (B operand in lane order, then |o|^2 per source);
// app: per block 16 values W sigma (S) or 80 values ((W mu nu, 0) in lane
// order, then -W mu nu.o) (D).  A workgroup of four waves owns 256 targets; the
// blocks of each source particle are staged through LDS and read by all four.
template <typename R, int OP>
__global__ __launch_bounds__(256) void k_far_mfma(const R* __restrict__ geo, const R* __restrict__ app,
                                                  const Particle* __restrict__ part, const double* __restrict__ x,
                                                  const double* __restrict__ y, const double* __restrict__ z,
                                                  const uint32_t* __restrict__ excl, int words, int M, int T,
                                                  int T16, int64_t N, int nsplit, double* __restrict__ partial) {
  using MM = Mfma<R>;
  using V = typename MM::V;
  constexpr int GEO = 80, APP = (OP == SBIE_OP_S) ? 16 : 80;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R* lds = reinterpret_cast<R*>(smem_raw);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int split = blockIdx.x % nsplit, tile = blockIdx.x / nsplit;
  const int s0 = (int)((int64_t)M * split / nsplit), s1 = (int)((int64_t)M * (split + 1) / nsplit);
  const int nb = T16 / 16;
  const int64_t wg0 = (int64_t)tile * 256;
  const int pw0 = (int)(wg0 / T);
  const int pw1 = (int)(((wg0 + 255 < N) ? (wg0 + 255) : (N - 1)) / T);
  const int64_t base = wg0 + wave * 64;
  const bool wave_live = base < N;

  // A-operand rows: targets base + 16 rb + li
  double tc[4][3];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) {
    int64_t t = base + 16 * rb + li;
    if (t >= N) t = N - 1;
    tc[rb][0] = x[t];
    tc[rb][1] = y[t];
    tc[rb][2] = z[t];
  }
  // target particles spanned by the wave's 64 rows (T >= 32: at most three)
  const int tp0 = (int)((wave_live ? base : wg0) / T);
  const int b1 = (int)((int64_t)(tp0 + 1) * T - base);  // first local row of particle tp0+1
  const int b2 = b1 + T;                                 // first local row of particle tp0+2
  const int64_t nrows = !wave_live ? 0 : ((N - base < 64) ? (N - base) : 64);

  R acc[4][4], lo[4][4];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[rb][e] = lo[rb][e] = R(0);

  for (int s = s0; s < s1; ++s) {
    const uint32_t bit = 1u << (s & 31);
    const int wd = s >> 5;
    // workgroup-uniform: does any target particle of the workgroup need source s?
    bool wg_need = false;
    for (int tp = pw0; tp <= pw1; ++tp) wg_need |= !(excl[(size_t)tp * words + wd] & bit);
    if (!wg_need) continue;
    bool need[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int tp = tp0 + q;
      const int first = q == 0 ? 0 : (q == 1 ? b1 : b2);
      need[q] = tp < M && first < nrows && !(excl[(size_t)tp * words + wd] & bit);
    }
    const bool wave_need = need[0] || need[1] || need[2];
    const double cx = part[s].c[0], cy = part[s].c[1], cz = part[s].c[2];
    R a[4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      const double dx = tc[rb][0] - cx, dy = tc[rb][1] - cy, dz = tc[rb][2] - cz;
      const double v = lg == 0 ? dx : (lg == 1 ? dy : (lg == 2 ? dz : fma(dz, dz, fma(dy, dy, dx * dx))));
      a[rb] = (R)v;
    }
    R tmp[4][4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int e = 0; e < 4; ++e) tmp[rb][e] = R(0);
    for (int c0 = 0; c0 < nb; c0 += kChunk) {
      const int nbc = nb - c0 < kChunk ? nb - c0 : kChunk;
      __syncthreads();  // the previous chunk has been consumed
      {
        using C16 = typename std::conditional<sizeof(R) == 4, float4, double2>::type;
        constexpr int PER = 16 / sizeof(R);
        const C16* gs = reinterpret_cast<const C16*>(geo + ((size_t)s * nb + c0) * GEO);
        C16* ld = reinterpret_cast<C16*>(lds);
        for (int i = tid; i < nbc * GEO / PER; i += 256) ld[i] = gs[i];
        const C16* as = reinterpret_cast<const C16*>(app + ((size_t)s * nb + c0) * APP);
        C16* la = reinterpret_cast<C16*>(lds + kChunk * GEO);
        for (int i = tid; i < nbc * APP / PER; i += 256) la[i] = as[i];
      }
      __syncthreads();
      if (wave_need) {
        for (int ib = 0; ib < nbc; ++ib) {
          const R bv = lds[ib * GEO + lane];
          const R cw = lds[ib * GEO + 64 + li];
          const V cinit = {cw, cw, cw, cw};
          if (OP == SBIE_OP_S) {
            const R qv = lds[kChunk * GEO + ib * 16 + li];
            V r2[4];
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) r2[rb] = MM::mma(a[rb], bv, cinit);
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
#pragma unroll
              for (int e = 0; e < 4; ++e) tmp[rb][e] = fma(qv, MM::rsq(r2[rb][e]), tmp[rb][e]);
          } else {
            const R dv = lds[kChunk * GEO + ib * 80 + lane];
            const R dw = lds[kChunk * GEO + ib * 80 + 64 + li];
            const V c2 = {dw, dw, dw, dw};
#pragma unroll
            for (int rb = 0; rb < 4; ++rb) {
              const V r2 = MM::mma(a[rb], bv, cinit);
              const V dt = MM::mma(a[rb], dv, c2);
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                const R ri = MM::rsq(r2[e]);
                tmp[rb][e] = fma(dt[e] * ri, ri * ri, tmp[rb][e]);
              }
            }
          }
        }
      }
    }
    if (!wave_need) continue;
    // add the tile under the per-target exclusion, compensated for FP32
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = 16 * rb + MM::row(lg, e);
        const bool nd = r < b1 ? need[0] : (r < b2 ? need[1] : need[2]);
        const R v = nd ? tmp[rb][e] : R(0);
        const R sum = acc[rb][e] + v;
        const R bp = sum - acc[rb][e];
        lo[rb][e] += (acc[rb][e] - (sum - bp)) + (v - bp);
        acc[rb][e] = sum;
      }
  }
  if (!wave_live) return;
  // reduce each row over the 16 columns held by lanes with the same l/16 (FP64)
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      double v = (double)acc[rb][e] + (double)lo[rb][e];
#pragma unroll
      for (int off = 1; off < 16; off <<= 1) v += __shfl_xor(v, off, 64);
      const int r = 16 * rb + MM::row(lg, e);
      if (li == 0 && r < nrows) partial[(size_t)split * N + base + r] = v * kInv4PiD;
    }
}

// Per-geometry source operands.  One thread per (padded) source q of particle
// s: o = node - centre (FP64 difference rounded once); padding sits at the
// centre (o = 0).  Block b = q/16 of particle s holds, at (s*nb + b)*80, the B
// operand entry [k][j] at 16k + j and |o_j|^2 at 64 + j.
template <typename R>
__global__ void k_far_records(const Particle* __restrict__ part, const double* __restrict__ x,
                              const double* __restrict__ y, const double* __restrict__ z, int M, int T, int T16,
                              R* __restrict__ geo) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)M * T16) return;
  const int s = (int)(t / T16), q = (int)(t - (int64_t)s * T16);
  double ox = 0.0, oy = 0.0, oz = 0.0;
  if (q < T) {
    const int64_t g = (int64_t)s * T + q;
    ox = x[g] - part[s].c[0];
    oy = y[g] - part[s].c[1];
    oz = z[g] - part[s].c[2];
  }
  R* b = geo + (t / 16) * 80 + (t % 16);
  b[0] = (R)(-2.0 * ox);
  b[16] = (R)(-2.0 * oy);
  b[32] = (R)(-2.0 * oz);
  b[48] = R(1);
  b[64] = (R)fma(oz, oz, fma(oy, oy, ox * ox));
}

// Per-apply source strengths: S W sigma per source; D per block (W mu nu, 0) in
// lane order and -W mu nu.o.
template <typename R, int OP>
__global__ void k_far_strengths(const Particle* __restrict__ part, const double* __restrict__ dens,
                                const double* __restrict__ x, const double* __restrict__ y,
                                const double* __restrict__ z, const double* __restrict__ nx,
                                const double* __restrict__ ny, const double* __restrict__ nz,
                                const double* __restrict__ w, int M, int T, int T16, R* __restrict__ app) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)M * T16) return;
  const int s = (int)(t / T16), q = (int)(t - (int64_t)s * T16);
  double wq = 0.0;
  int64_t g = 0;
  if (q < T) {
    g = (int64_t)s * T + q;
    wq = w[g] * dens[g];
  }
  if (OP == SBIE_OP_S) {
    app[t] = (R)wq;
  } else {
    double dx = 0.0, dy = 0.0, dz = 0.0, dot = 0.0;
    if (q < T) {
      dx = wq * nx[g];
      dy = wq * ny[g];
      dz = wq * nz[g];
      const double ox = x[g] - part[s].c[0], oy = y[g] - part[s].c[1], oz = z[g] - part[s].c[2];
      dot = fma(dz, oz, fma(dy, oy, dx * ox));
    }
    R* b = app + (t / 16) * 80 + (t % 16);
    b[0] = (R)dx;
    b[16] = (R)dy;
    b[32] = (R)dz;
    b[48] = R(0);
    b[64] = (R)(-dot);
  }
}

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

template <typename R>
sbie_status launch_far(sbie_geom* g, int op, const double* d_dens, const R* geo, R* app, hipStream_t s,
                       hipEvent_t ev_begin, hipEvent_t ev_end) {
  const int64_t n16 = (int64_t)g->M * g->T16;
  const dim3 pre(cdiv(n16, 256)), blk(256);
  if (op == SBIE_OP_S)
    hipLaunchKernelGGL((k_far_strengths<R, SBIE_OP_S>), pre, blk, 0, s, g->d_part, d_dens, g->d_x, g->d_y, g->d_z,
                       g->d_nx, g->d_ny, g->d_nz, g->d_w, g->M, g->T, g->T16, app);
  else
    hipLaunchKernelGGL((k_far_strengths<R, SBIE_OP_D>), pre, blk, 0, s, g->d_part, d_dens, g->d_x, g->d_y, g->d_z,
                       g->d_nx, g->d_ny, g->d_nz, g->d_w, g->M, g->T, g->T16, app);
  SBIE_HIP(hipGetLastError());
  if (ev_begin) SBIE_HIP(hipEventRecord(ev_begin, s));
  const dim3 grid(cdiv(g->N, 256) * g->nsplit);
  const size_t lds = (size_t)kChunk * (80 + (op == SBIE_OP_S ? 16 : 80)) * sizeof(R);
  if (op == SBIE_OP_S)
    hipLaunchKernelGGL((k_far_mfma<R, SBIE_OP_S>), grid, blk, lds, s, geo, app, g->d_part, g->d_x, g->d_y, g->d_z,
                       g->d_excl, g->excl_words, g->M, g->T, g->T16, g->N, g->nsplit, g->d_partial);
  else
    hipLaunchKernelGGL((k_far_mfma<R, SBIE_OP_D>), grid, blk, lds, s, geo, app, g->d_part, g->d_x, g->d_y, g->d_z,
                       g->d_excl, g->excl_words, g->M, g->T, g->T16, g->N, g->nsplit, g->d_partial);
  SBIE_HIP(hipGetLastError());
  if (ev_end) SBIE_HIP(hipEventRecord(ev_end, s));
  return SBIE_OK;
}

}  // namespace

sbie_status far_records(sbie_geom* g, hipStream_t s) {
  const int64_t n = (int64_t)g->M * g->T16;
  hipLaunchKernelGGL(k_far_records<float>, dim3(cdiv(n, 256)), dim3(256), 0, s, g->d_part, g->d_x, g->d_y, g->d_z,
                     g->M, g->T, g->T16, g->d_srec32);
  SBIE_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_far_records<double>, dim3(cdiv(n, 256)), dim3(256), 0, s, g->d_part, g->d_x, g->d_y, g->d_z,
                     g->M, g->T, g->T16, g->d_srec64);
  SBIE_HIP(hipGetLastError());
  return SBIE_OK;
}

sbie_status far_mfma(sbie_geom* g, int op, int prec, const double* d_dens, hipStream_t s, hipEvent_t ev_begin,
                     hipEvent_t ev_end) {
  if (prec == SBIE_MIXED)
    return launch_far<float>(g, op, d_dens, g->d_srec32, g->d_fstr32, s, ev_begin, ev_end);
  return launch_far<double>(g, op, d_dens, g->d_srec64, g->d_fstr64, s, ev_begin, ev_end);
}

}  // namespace sbie
