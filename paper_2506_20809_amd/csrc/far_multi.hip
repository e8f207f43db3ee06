// Pair-symmetric far field of S or D for several densities at once (the
// far-field step of Algorithm 1 applied to NR right-hand sides on one
// geometry): each node pair's 1/r (and, for D, 1/r^3) is computed once and
// serves every density in both directions.
//
// The structure is that of the Stokes pair kernel (far_stokes.hip): the
// workgroups of particle a visit each partner b once, keep a's forward sums in
// registers, and reduce the reverse sums into b's nodes over a's rows into
// rev[b][slot][rg][k][t], folded slot by slot.  Per 16 x 16 tile the matrix
// cores take, with D = x - c_b and o = y - c_b,
//     |d|^2   = [D |D|^2] . [-2o 1] + |o|^2,
// and for the double layer, per density k (dipoles m = W mu_k nu),
//     m_b.d   = [D 1] . [m_b  -m_b.o]          (forward, kernel m_b.d / r^3)
//     m_a.d   = [m_a/2  m_a.D] . [-2o 1]       (reverse, kernel m_a.(y - x) / r^3),
// d = x - y; the single layer needs no product beyond |d|^2 (q/r both ways).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "sbie_internal.h"
#include "x3.h"

namespace sbie {

namespace {

constexpr double kInv4PiM = 0.079577471545947667884441881686257181;
// most waves per workgroup: the FP64 single layer's kernels fit four per
// SIMD, the others are run at three
template <typename R, int OP>
struct MultiWaves {
  static constexpr int W = (OP == SBIE_OP_S && sizeof(R) == 8) ? 16 : 12;
};
constexpr int kMaxRhs = 4;   // densities per launch

using d4m = double __attribute__((ext_vector_type(4)));

template <typename R>
struct MultiShape;
template <>
struct MultiShape<float> {
  static constexpr int RB = 2;
  using V = f4;
  static __device__ inline int row(int lg, int e) { return 4 * lg + e; }
  static __device__ inline V mma(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  static __device__ inline float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
};
template <>
struct MultiShape<double> {
  static constexpr int RB = 1;
  using V = d4m;
  static __device__ inline int row(int lg, int e) { return lg + 4 * e; }
  static __device__ inline V mma(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline double rsq(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double h = x * y;
    const double e = fma(-h, y, 1.0);
    return fma(0.5 * y, e, y);
  }
};

// values per 16-source block: [-2o 1] (64, lane order), |o|^2 per column (16),
// then per density: S q per column (16), D [m  -m.o] (64, lane order)
template <int OP, int NR>
struct MultiLayout {
  static constexpr int PER = OP == SBIE_OP_S ? 16 : 64;
  static constexpr int GEO = 80 + NR * PER;
};
// source blocks staged in LDS at a time (static LDS under 64 KB)
template <typename R, int OP>
struct MultiChunk {
  static constexpr int CH = sizeof(R) == 8 ? 6 : (OP == SBIE_OP_S ? 16 : 12);
};

__device__ inline double lane_sum16(double v) {
#pragma unroll
  for (int off = 1; off < 16; off <<= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Per-block records from the densities dens[k][N] (one thread per lane of a block).
template <typename R, int OP, int NR>
__global__ void k_multi_records(const Particle* __restrict__ part, const double* __restrict__ dens,
                                const double* __restrict__ x, const double* __restrict__ y,
                                const double* __restrict__ z, const double* __restrict__ nx,
                                const double* __restrict__ ny, const double* __restrict__ nz,
                                const double* __restrict__ w, int M, int T, int nb, int64_t N, R* __restrict__ rec) {
  using L = MultiLayout<OP, NR>;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)M * nb * 64) return;
  const int lane = (int)(i & 63);
  const int64_t blk = i >> 6;
  const int b = (int)(blk / nb), ib = (int)(blk - (int64_t)b * nb);
  const int lg = lane >> 4, li = lane & 15, r = ib * 16 + li;
  double o[3] = {0.0, 0.0, 0.0}, nv[3] = {0.0, 0.0, 0.0}, wq = 0.0;
  int64_t g = 0;
  if (r < T) {
    g = (int64_t)b * T + r;
    o[0] = x[g] - part[b].c[0];
    o[1] = y[g] - part[b].c[1];
    o[2] = z[g] - part[b].c[2];
    nv[0] = nx[g];
    nv[1] = ny[g];
    nv[2] = nz[g];
    wq = w[g];
  }
  R* out = rec + blk * L::GEO;
  out[lane] = lg < 3 ? (R)(-2.0 * o[lg]) : R(1);
  if (lg == 0) out[64 + li] = (R)(o[0] * o[0] + o[1] * o[1] + o[2] * o[2]);
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    const double q = r < T ? wq * dens[(int64_t)k * N + g] : 0.0;
    if (OP == SBIE_OP_S) {
      if (lg == 0) out[80 + 16 * k + li] = (R)q;
    } else {
      const double m[3] = {q * nv[0], q * nv[1], q * nv[2]};
      out[80 + 64 * k + lane] = lg < 3 ? (R)m[lg] : (R)(-(m[0] * o[0] + m[1] * o[1] + m[2] * o[2]));
    }
  }
}

// The pair kernel for NR densities: work index (XCD-ordered) -> (particle a,
// row group rg, split of a's partner offsets), as the Stokes pair kernel; the
// forward sums of density k go to fwd[k][split][N] (first launch: written),
// the reverse sums to rev[b][k - kbase][rg][k][t].
template <typename R, int OP, int NR>
__global__ __launch_bounds__(64 * (MultiWaves<R, OP>::W)) void k_far_multi_pairs(
    const R* __restrict__ rec, const Particle* __restrict__ part, const double* __restrict__ x,
    const double* __restrict__ y, const double* __restrict__ z, const double* __restrict__ nx,
    const double* __restrict__ ny, const double* __restrict__ nz, const double* __restrict__ dens,
    const double* __restrict__ w, const uint32_t* __restrict__ excl, int words, int M, int T, int64_t N, int nsplit,
    int RG, int kbase, int kend, int first, double* __restrict__ fwd, R* __restrict__ rev) {
  using SS = MultiShape<R>;
  using V = typename SS::V;
  using L = MultiLayout<OP, NR>;
  constexpr int RB = SS::RB, CH = MultiChunk<R, OP>::CH, GEO = L::GEO, WMAX = MultiWaves<R, OP>::W;
  const int W = (int)(blockDim.x >> 6);
  constexpr bool F32 = sizeof(R) == 4;
  constexpr bool DL = OP == SBIE_OP_D;
  __shared__ R lds_rec[CH * GEO];
  __shared__ R lds_rev[WMAX * NR * CH * 16];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 15, lg = lane >> 4;
  const int x16 = (lane ^ 16) << 2, x32 = (lane ^ 32) << 2;
  const int wid = xcd_work_index();
  const int split = wid % nsplit, rest = wid / nsplit;
  const int rg = rest % RG, a = rest / RG;
  const int nb = (T + 15) / 16;
  const int gb0 = (int)((int64_t)rg * nb / RG), cnt = (int)((int64_t)(rg + 1) * nb / RG) - gb0;
  const int rb0 = gb0 + (wave * cnt) / W;
  const int nown = __builtin_amdgcn_readfirstlane(gb0 + ((wave + 1) * cnt) / W - rb0);
  const int H = (M - 1) / 2;
  const bool even = (M & 1) == 0;
  const int P = H + ((even && a < M / 2) ? 1 : 0);
  const int klo = kbase < P ? kbase : P, khi = kend < P ? kend : P;
  const int k0 = klo + (int)((int64_t)(khi - klo) * split / nsplit);
  const int k1 = klo + (int)((int64_t)(khi - klo) * (split + 1) / nsplit);
  const int KS = kend - kbase;
  const Particle& Pa = part[a];

  // rows: the A-operand row li (component lg of its position and, for D, of
  // its dipoles), the accumulator rows' strengths (S); rows past the wave's
  // own blocks are zero-strength points at a's centre
  const int cl = lg < 3 ? lg : 0;
  const double* xyz = cl == 0 ? x : (cl == 1 ? y : z);
  const double* nrm = cl == 0 ? nx : (cl == 1 ? ny : nz);
  double tcl[RB];
  R mA[DL ? RB : 1][NR], qacc[DL ? 1 : RB][4][NR];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    const int bk = rb0 + rb;
    const int ra = bk * 16 + li;
    const bool la = rb < nown && ra < T;
    const int64_t ga = (int64_t)a * T + (la ? ra : 0);
    tcl[rb] = la ? xyz[ga] : Pa.c[cl];
    if constexpr (DL) {
#pragma unroll
      for (int k = 0; k < NR; ++k)
        mA[rb][k] = (la && lg < 3) ? (R)(w[ga] * dens[(int64_t)k * N + ga] * nrm[ga]) : R(0);
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = bk * 16 + SS::row(lg, e);
        const bool lr = rb < nown && r < T;
        const int64_t g = (int64_t)a * T + (lr ? r : 0);
        const double wq = lr ? w[g] : 0.0;
#pragma unroll
        for (int k = 0; k < NR; ++k) qacc[rb][e][k] = (R)(wq * dens[(int64_t)k * N + g]);
      }
    }
  }

  double accF[(4 * RB * NR + 15) / 16];
#pragma unroll
  for (int h = 0; h < (4 * RB * NR + 15) / 16; ++h) accF[h] = 0.0;
  double accD[F32 ? 1 : RB][4][NR];
#pragma unroll
  for (int rb = 0; rb < (F32 ? 1 : RB); ++rb)
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int k = 0; k < NR; ++k) accD[rb][e][k] = 0.0;

  for (int kk = k0; kk < k1; ++kk) {
    const int b = kk < H ? (a + 1 + kk) % M : a + M / 2;
    const bool need_f = !((excl[(size_t)a * words + (b >> 5)] >> (b & 31)) & 1u);
    const bool need_r = !((excl[(size_t)b * words + (a >> 5)] >> (a & 31)) & 1u);
    R* rout = rev + (((size_t)b * KS + (kk - kbase)) * RG + rg) * (size_t)NR * T;
    if (!need_f && !need_r) {
      for (int t = tid; t < NR * T; t += blockDim.x) rout[t] = R(0);
      continue;
    }
    const double cb = part[b].c[cl];
    R aop[RB], a1[RB], a3[DL ? RB : 1][NR];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const double dl = lg < 3 ? tcl[rb] - cb : 0.0;
      double d2 = dl * dl;
      d2 += lane_value(d2, x16);
      d2 += lane_value(d2, x32);
      aop[rb] = (R)(lg < 3 ? dl : d2);
      a1[rb] = lg < 3 ? (R)dl : R(1);
      if constexpr (DL) {
#pragma unroll
        for (int k = 0; k < NR; ++k) {
          double md = lg < 3 ? (double)mA[rb][k] * dl : 0.0;
          md += lane_value(md, x16);
          md += lane_value(md, x32);
          a3[rb][k] = lg < 3 ? R(0.5) * mA[rb][k] : (R)md;
        }
      }
    }
    R tf[F32 ? RB : 1][4][NR];
#pragma unroll
    for (int rb = 0; rb < (F32 ? RB : 1); ++rb)
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int k = 0; k < NR; ++k) tf[rb][e][k] = R(0);
    auto fref = [&](int rb, int e, int k) -> R& {
      if constexpr (F32) return tf[rb][e][k];
      else return accD[rb][e][k];
    };
    auto partner = [&](auto nf_c) {
      constexpr bool NF = decltype(nf_c)::value;
      for (int c0 = 0; c0 < nb; c0 += CH) {
        const int nbc = nb - c0 < CH ? nb - c0 : CH;
        __syncthreads();  // the previous chunk's operands and reverse sums are consumed
        {
          const R* gsrc = rec + ((size_t)b * nb + c0) * GEO;
          for (int i = tid; i < nbc * GEO; i += blockDim.x) lds_rec[i] = gsrc[i];
        }
        __syncthreads();
        for (int ib = 0; ib < nbc; ++ib) {
          const R* Lb = lds_rec + ib * GEO;
          const R bgeo = Lb[lane], o2 = Lb[64 + li];
          R qb[NR];
#pragma unroll
          for (int k = 0; k < NR; ++k) qb[k] = DL ? Lb[80 + 64 * k + lane] : Lb[80 + 16 * k + li];
          const V zero = {R(0), R(0), R(0), R(0)};
          V r2[RB], df[DL ? RB : 1][NR], dr[DL ? RB : 1][NR];
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) {
            r2[rb] = SS::mma(aop[rb], bgeo, V{o2, o2, o2, o2});
            if constexpr (DL) {
#pragma unroll
              for (int k = 0; k < NR; ++k) {
                if (NF) df[rb][k] = SS::mma(a1[rb], qb[k], zero);
                dr[rb][k] = SS::mma(a3[rb][k], bgeo, zero);
              }
            }
          }
          R rv[NR];
#pragma unroll
          for (int k = 0; k < NR; ++k) rv[k] = R(0);
#pragma unroll
          for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const R ri = SS::rsq(r2[rb][e]);
              if constexpr (DL) {
                const R ri3 = ri * ri * ri;
#pragma unroll
                for (int k = 0; k < NR; ++k) {
                  if (NF) fref(rb, e, k) = fma(df[rb][k][e], ri3, fref(rb, e, k));
                  rv[k] = fma(dr[rb][k][e], ri3, rv[k]);
                }
              } else {
#pragma unroll
                for (int k = 0; k < NR; ++k) {
                  if (NF) fref(rb, e, k) = fma(qb[k], ri, fref(rb, e, k));
                  rv[k] = fma(qacc[DL ? 0 : rb][e][k], ri, rv[k]);
                }
              }
            }
#pragma unroll
          for (int k = 0; k < NR; ++k) {
            rv[k] += lane_value(rv[k], x16);
            rv[k] += lane_value(rv[k], x32);
          }
          if (lg == 0)
#pragma unroll
            for (int k = 0; k < NR; ++k) lds_rev[((wave * NR + k) * CH + ib) * 16 + li] = rv[k];
        }
        __syncthreads();
        // reverse sums over the waves, in wave order (the double layer's
        // reverse kernel is m_a.(y - x) = -m_a.d)
        for (int idx = tid; idx < NR * nbc * 16; idx += blockDim.x) {
          const int k = idx / (nbc * 16), col = idx - k * (nbc * 16);
          const int t = c0 * 16 + col;
          if (t >= T) continue;
          R sum = R(0);
          for (int wv = 0; wv < W; ++wv) sum += lds_rev[(wv * NR + k) * CH * 16 + col];
          rout[(size_t)k * T + t] = need_r ? (DL ? -sum : sum) : R(0);
        }
      }
    };
    if (need_f) partner(std::true_type{});
    else partner(std::false_type{});
    if (!need_f) continue;
    if constexpr (F32) {
      // this partner's tiles summed over their 16 columns, into FP64:
      // elements f = (rb*4 + e)*NR + k in arrays of 16, lane li keeping element li
#pragma unroll
      for (int h = 0; h < (4 * RB * NR + 15) / 16; ++h) {
        float v[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const int f = 16 * h + j;
          const int rb = f / (4 * NR), e = (f / NR) % 4, k = f % NR;
          v[j] = rb < RB ? (float)tf[rb < RB ? rb : 0][e][k] : 0.0f;
        }
        accF[h] += row_group_sums(v, lane);
      }
    }
  }
  auto put = [&](int rb, int e, int k, double v) {
    if (rb >= nown) return;
    const int r = (rb0 + rb) * 16 + SS::row(lg, e);
    if (r >= T) return;
    double* f = fwd + ((size_t)k * nsplit + split) * N + (int64_t)a * T + r;
    *f = (first ? 0.0 : *f) + v * kInv4PiM;
  };
  if constexpr (F32) {
#pragma unroll
    for (int h = 0; h < (4 * RB * NR + 15) / 16; ++h) {
      const int f = 16 * h + li;
      const int rb = f / (4 * NR), e = (f / NR) % 4, k = f % NR;
      if (rb < RB) put(rb, e, k, accF[h]);
    }
  } else {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int k = 0; k < NR; ++k) {
          const double v = lane_sum16(accD[rb][e][k]);
          if (li == 0) put(rb, e, k, v);
        }
  }
}

// Each target's reverse slots of a launch into its running totals racc [NR][N].
template <typename R>
__global__ void k_far_multi_fold(const R* __restrict__ rev, int M, int T, int RG, int NR, int kbase, int kend,
                                 int first, int64_t N, double* __restrict__ racc) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  const int b = (int)(g / T), t = (int)(g - (int64_t)b * T);
  const int H = (M - 1) / 2;
  const int slots = H + (((M & 1) == 0 && b >= M / 2) ? 1 : 0);
  const int KS = kend - kbase;
  const int hi = kend < slots ? kend : slots;
  for (int k = 0; k < NR; ++k) {
    double r = first ? 0.0 : racc[(size_t)k * N + g];
    for (int s = kbase; s < hi; ++s)
      for (int rg = 0; rg < RG; ++rg)
        r += (double)rev[((((size_t)b * KS + (s - kbase)) * RG + rg) * NR + k) * T + t];
    racc[(size_t)k * N + g] = r;
  }
}

template <typename R, int OP, int NR>
sbie_status launch_multi(sbie_geom* g, const double* d_dens, hipStream_t s) {
  const int M = g->M, T = g->T, nb = (T + 15) / 16;
  const int RG = multi_row_groups(T, sizeof(R) == 8, OP);
  MultiWork& mw = *g->multi;
  R* rec = reinterpret_cast<R*>(mw.rec);
  hipLaunchKernelGGL((k_multi_records<R, OP, NR>), dim3((unsigned)(((int64_t)M * nb * 64 + 255) / 256)), dim3(256), 0,
                     s, g->d_part, d_dens, g->d_x, g->d_y, g->d_z, g->d_nx, g->d_ny, g->d_nz, g->d_w, M, T, nb,
                     g->N, rec);
  SBIE_HIP(hipGetLastError());
  const int PMAX = (M - 1) / 2 + ((M & 1) == 0 ? 1 : 0);
  const int KS = multi_rev_slots(M, T, NR, OP, (int)sizeof(R), mw.rev_bytes);
  const int nsplit = multi_splits(g, RG);
  R* rev = reinterpret_cast<R*>(mw.rev);
  const dim3 grid((unsigned)((int64_t)M * RG * nsplit)), fold((unsigned)((g->N + 255) / 256));
  for (int kbase = 0; kbase == 0 || kbase < PMAX; kbase += KS) {
    const int kend = kbase + KS, first = kbase == 0 ? 1 : 0;
    hipLaunchKernelGGL((k_far_multi_pairs<R, OP, NR>), grid, dim3(64 * multi_waves(T, sizeof(R) == 8, OP)), 0, s, rec,
                       g->d_part, g->d_x,
                       g->d_y, g->d_z, g->d_nx, g->d_ny, g->d_nz, d_dens, g->d_w, g->d_excl, g->excl_words, M, T,
                       g->N, nsplit, RG, kbase, kend, first, mw.partial, rev);
    SBIE_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_far_multi_fold<R>, fold, dim3(256), 0, s, rev, M, T, RG, NR, kbase, kend, first, g->N,
                       mw.racc);
    SBIE_HIP(hipGetLastError());
  }
  return SBIE_OK;
}

template <typename R, int OP>
sbie_status launch_multi_n(sbie_geom* g, int nr, const double* d_dens, hipStream_t s) {
  switch (nr) {
    case 2: return launch_multi<R, OP, 2>(g, d_dens, s);
    case 3: return launch_multi<R, OP, 3>(g, d_dens, s);
    default: return launch_multi<R, OP, 4>(g, d_dens, s);
  }
}

}  // namespace

// Row groups hold up to Wg * RB blocks: Wg = 16 for the FP64 single layer,
// else 12.  FP32 launches take twelve waves whatever the group's size (more
// resident waves measured faster than fewer stand-in rows); FP64 launches the
// fewest waves that hold the largest group.
int multi_row_groups(int T, bool fp64, int op) {
  const int nb = (T + 15) / 16;
  const int Wg = (op == SBIE_OP_S && fp64) ? MultiWaves<double, SBIE_OP_S>::W : 12;
  const int gb = Wg * (fp64 ? MultiShape<double>::RB : MultiShape<float>::RB);
  return (nb + gb - 1) / gb;
}

int multi_waves(int T, bool fp64, int op) {
  if (!fp64) return 12;
  const int nb = (T + 15) / 16, RG = multi_row_groups(T, fp64, op);
  const int cnt = (nb + RG - 1) / RG;
  return (cnt + MultiShape<double>::RB - 1) / MultiShape<double>::RB;
}

int multi_rev_slots(int M, int T, int NR, int op, int bytes_per_value, uint64_t cap_bytes) {
  const int pmax = (M - 1) / 2 + ((M & 1) == 0 ? 1 : 0);
  if (pmax < 1) return 1;
  const uint64_t per_slot = (uint64_t)M * multi_row_groups(T, bytes_per_value == 8, op) * NR * T * bytes_per_value;
  int k = (int)(cap_bytes / (per_slot > 0 ? per_slot : 1));
  if (k > pmax) k = pmax;
  if (k < 1) k = 1;
  const int launches = (pmax + k - 1) / k;
  return (pmax + launches - 1) / launches;
}

int multi_splits(const sbie_geom* g, int RG) {
  const int want = (int)((512 + (int64_t)g->M * RG - 1) / ((int64_t)g->M * RG));
  const int pmax = (g->M - 1) / 2 + ((g->M & 1) == 0 ? 1 : 0);
  int n = want < g->nsplit ? want : g->nsplit;
  if (n > pmax) n = pmax;
  return n < 1 ? 1 : n;
}

uint64_t multi_rev_bytes(int M, int T) {
  const int pmax = (M - 1) / 2 + ((M & 1) == 0 ? 1 : 0);
  // the largest per-slot size: FP64, the double layer's (smaller) row groups
  const uint64_t per_slot = (uint64_t)M * multi_row_groups(T, true, SBIE_OP_D) * kMaxRhs * T * sizeof(double);
  const uint64_t all = per_slot * (uint64_t)(pmax > 0 ? pmax : 1);
  const uint64_t cap = all < kRevBudget ? all : kRevBudget;
  return cap < per_slot ? per_slot : cap;
}

size_t multi_rec_values(int M, int T) {
  return (size_t)M * ((T + 15) / 16) * MultiLayout<SBIE_OP_D, kMaxRhs>::GEO;
}

sbie_status far_multi(sbie_geom* g, int op, bool mixed, int nr, const double* d_dens, hipStream_t s) {
  if (nr < 2 || nr > kMaxRhs) {
    set_error("the multi-density far field takes 2 to 4 densities");
    return SBIE_E_INVALID;
  }
  if (mixed)
    return op == SBIE_OP_S ? launch_multi_n<float, SBIE_OP_S>(g, nr, d_dens, s)
                           : launch_multi_n<float, SBIE_OP_D>(g, nr, d_dens, s);
  return op == SBIE_OP_S ? launch_multi_n<double, SBIE_OP_S>(g, nr, d_dens, s)
                         : launch_multi_n<double, SBIE_OP_D>(g, nr, d_dens, s);
}

}  // namespace sbie
