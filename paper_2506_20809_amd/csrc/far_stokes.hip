// Pair-symmetric far field of the Stokes single layer (Section 4.3: the
// Stokeslet (1/8pi)(q/r + (d.q) d/r^3), d = x - y, q = W sigma, by smooth
// quadrature over the far node pairs; far-field step of Algorithm 1), with its
// pressure (1/4pi)(d.q)/r^3 as a fourth component.
//
// The Stokeslet is even in d, so one evaluation of 1/r per node pair serves
// both directions, as in the Laplace pair kernel: every unordered pair of
// particles (a, b) is visited once, by the workgroups that own a's rows; the
// forward sums into a's targets stay in registers across the partners, the
// reverse sums into b's targets are reduced over a's rows (lanes, then waves
// in order) into rev[b][slot][rg][c][t] and folded slot by slot.  The pressure
// kernel is odd in d: its reverse term changes sign.
//
// The matrix cores take the contractions over a K = 4 operand pair, 256 node
// pairs per product, with D = x - c_b and o = y - c_b:
//     |d|^2   = [D |D|^2] . [-2o 1] + |o|^2
//     d.q_b   = [D 1] . [q_b  -q_b.o]
//     d.q_a   = [q_a/2  q_a.D] . [-2o 1]
// and the vector units the components d_i = D_i - o_i (one add per node pair
// and component, cheaper on this chip than a product per component: a
// 16x16x4 product costs about as much as twelve vector instructions of the
// wave), 1/r, 1/r^3 and the multiply-adds of the two directions' velocity
// terms.  Rows of a (and sources of b) are padded to 16 with zero-strength
// points at the particle's centre.
//
// The same kernel (SDL) takes the far field of the Stokes double layer
// (Section 4.3): the stresslet (3/4pi)(d.m)(d.nu) d/r^5 with m = W mu, which is
// odd in d, so its reverse term changes sign.  Its products per tile are |d|^2
// and the four dots d.m_b = [D 1].[m_b -m_b.o], d.nu_b likewise, and
// d.m_a = [m_a/2 m_a.D].[-2o 1], d.nu_a likewise; the vector units take d_i,
// 1/r^5 and the weights.  Five FP32 products per tile would cost more than the
// one-sided sum, so in the mixed path they are three-piece bf16 products
// (x3.h), half the matrix-core time for the same FP32 accuracy of each dot.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "sbie_internal.h"
#include "x3.h"

namespace sbie {

namespace {

constexpr double kInv8PiS = 0.039788735772973833942220940843128591;
constexpr double kInv4PiS = 0.079577471545947667884441881686257181;
constexpr double k3Over4PiS = 0.23873241463784300365332564505877154;

using d4s = double __attribute__((ext_vector_type(4)));

// values per 16-source block: [-2o 1] B operand (64, lane order), |o|^2 per
// column (16), [q  -q.o] B operand (64), 16 unused
constexpr int kSGeo = 160;
// the stresslet's: [-2o 1] (64), |o|^2 (16), [m  -m.o] (64), [nu  -nu.o] (64)
constexpr int kSDGeo = 208;

// The stresslet's mixed path takes its products in the three-piece bf16 form
// (x3.h): its source blocks (kSDGeo floats in HBM) are split as they are
// staged in LDS, per block, in floats, the B operands as one u4 per lane:
// [-2o 1] with |o|^2 in its extra slots (0..255), [m -m.o] (256..511),
// [nu -nu.o] (512..767); then -o_i per column [3][16].  (The Stokeslet keeps
// the FP32 products: with them its far field is about three times closer to
// the FP64 one, for about 4% more time.)
struct SdlX3 {
  static constexpr int MO = 768, SIZE = 816;
};

// values per staged source block in LDS
template <typename R, bool SDL>
constexpr int stokes_geo() {
  return SDL ? (sizeof(R) == 4 ? SdlX3::SIZE : kSDGeo) : kSGeo;
}
constexpr int kSWaves = 12;  // most waves per workgroup (three per SIMD), each holding up to RB row blocks

template <typename R>
struct StokesShape;
template <>
struct StokesShape<float> {
  static constexpr int RB = 2;      // row blocks per wave
  static constexpr int CHUNK = 16;  // source blocks staged at a time
  using V = f4;
  static __device__ inline int row(int lg, int e) { return 4 * lg + e; }
  static __device__ inline V mma(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  static __device__ inline float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
};
template <>
struct StokesShape<double> {
  static constexpr int RB = 1;
  static constexpr int CHUNK = 8;
  using V = d4s;
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

__device__ inline double lane_sum_fp64(double v) {
#pragma unroll
  for (int off = 1; off < 16; off <<= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Source blocks of every particle: the B operands and per-column terms of
// the products above, from the density [3][N] (one thread per lane of a
// block).
template <typename R>
__global__ void k_stokes_pair_records(const Particle* __restrict__ part, const double* __restrict__ dens,
                                      const double* __restrict__ x, const double* __restrict__ y,
                                      const double* __restrict__ z, const double* __restrict__ w, int M, int T,
                                      int nb, int64_t N, R* __restrict__ rec) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)M * nb * 64) return;
  const int lane = (int)(i & 63);
  const int64_t blk = i >> 6;
  const int b = (int)(blk / nb), ib = (int)(blk - (int64_t)b * nb);
  const int lg = lane >> 4, li = lane & 15, r = ib * 16 + li;
  double o[3] = {0.0, 0.0, 0.0}, q[3] = {0.0, 0.0, 0.0};
  if (r < T) {
    const int64_t g = (int64_t)b * T + r;
    o[0] = x[g] - part[b].c[0];
    o[1] = y[g] - part[b].c[1];
    o[2] = z[g] - part[b].c[2];
    const double wq = w[g];
    for (int k = 0; k < 3; ++k) q[k] = wq * dens[(int64_t)k * N + g];
  }
  R* out = rec + blk * kSGeo;
  out[lane] = lg < 3 ? (R)(-2.0 * o[lg]) : R(1);
  out[80 + lane] = lg < 3 ? (R)q[lg] : (R)(-(q[0] * o[0] + q[1] * o[1] + q[2] * o[2]));
  if (lg == 0) {
    out[64 + li] = (R)(o[0] * o[0] + o[1] * o[1] + o[2] * o[2]);
    out[144 + li] = R(0);
  }
}

// The stresslet's source blocks: m = W mu from the density [3][N] and the
// normals (one thread per lane of a block).
template <typename R>
__global__ void k_sdl_pair_records(const Particle* __restrict__ part, const double* __restrict__ dens,
                                   const double* __restrict__ x, const double* __restrict__ y,
                                   const double* __restrict__ z, const double* __restrict__ w,
                                   const double* __restrict__ nx, const double* __restrict__ ny,
                                   const double* __restrict__ nz, int M, int T, int nb, int64_t N,
                                   R* __restrict__ rec) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)M * nb * 64) return;
  const int lane = (int)(i & 63);
  const int64_t blk = i >> 6;
  const int b = (int)(blk / nb), ib = (int)(blk - (int64_t)b * nb);
  const int lg = lane >> 4, li = lane & 15, r = ib * 16 + li;
  double o[3] = {0.0, 0.0, 0.0}, m[3] = {0.0, 0.0, 0.0}, nu[3] = {0.0, 0.0, 0.0};
  if (r < T) {
    const int64_t g = (int64_t)b * T + r;
    o[0] = x[g] - part[b].c[0];
    o[1] = y[g] - part[b].c[1];
    o[2] = z[g] - part[b].c[2];
    const double wq = w[g];
    for (int k = 0; k < 3; ++k) m[k] = wq * dens[(int64_t)k * N + g];
    nu[0] = nx[g];
    nu[1] = ny[g];
    nu[2] = nz[g];
  }
  R* out = rec + blk * kSDGeo;
  out[lane] = lg < 3 ? (R)(-2.0 * o[lg]) : R(1);
  out[80 + lane] = lg < 3 ? (R)m[lg] : (R)(-(m[0] * o[0] + m[1] * o[1] + m[2] * o[2]));
  out[144 + lane] = lg < 3 ? (R)nu[lg] : (R)(-(nu[0] * o[0] + nu[1] * o[1] + nu[2] * o[2]));
  if (lg == 0) out[64 + li] = (R)(o[0] * o[0] + o[1] * o[1] + o[2] * o[2]);
}

// The pair kernel.  Work index (XCD-ordered) -> (particle a, row group rg,
// split of a's partner offsets); a row group is a balanced share of a's 16-row
// blocks, spread over the waves as whole blocks (at most RB per wave).  One
// launch covers the partner offsets [kbase, kend); its forward sums are added
// to the split's slice [split][C][N] (first launch: written), its reverse
// sums go to rev[b][k - kbase][rg][c][t] (a dropped direction writes zeros).
// With SDL the stresslet (C = 3; nx, ny, nz the normals) instead of the
// Stokeslet (C = 3, or 4 with the pressure; no normals).
template <typename R, int C, bool SDL>
__global__ __launch_bounds__(64 * kSWaves) void k_far_stokes_pairs(
    const R* __restrict__ rec, const Particle* __restrict__ part, const double* __restrict__ x,
    const double* __restrict__ y, const double* __restrict__ z, const double* __restrict__ dens,
    const double* __restrict__ w, const double* __restrict__ nx, const double* __restrict__ ny,
    const double* __restrict__ nz, const uint32_t* __restrict__ excl, int words, int M, int T, int64_t N,
    int nsplit, int RG, int kbase, int kend, int first, double* __restrict__ fwd, R* __restrict__ rev) {
  using SS = StokesShape<R>;
  using V = typename SS::V;
  constexpr int RB = SS::RB, CH = SS::CHUNK;
  constexpr bool F32 = sizeof(R) == 4;
  constexpr bool X3 = F32 && SDL;  // three-piece products
  constexpr int GEO = stokes_geo<R, SDL>();
  __shared__ __align__(16) R lds_rec[CH * GEO];
  __shared__ R lds_rev[kSWaves * C * CH * 16];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int W = (int)(blockDim.x >> 6);
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
  // an A operand: the value itself, or its three-piece form (with `extra`,
  // the slots that add the B operand's per-column term)
  using AOp = std::conditional_t<X3, u4, R>;
  auto aform = [&](R v, bool extra) -> AOp {
    if constexpr (X3) return split_a(v, lg, extra);
    else return v;
  };

  // rows: the A-operand row li (component lg of its position and strength)
  // and the accumulator rows' strengths
  const int cl = lg < 3 ? lg : 0;
  const double* xyz = cl == 0 ? x : (cl == 1 ? y : z);
  double tcl[RB];
  // row li's strength component lg (Stokeslet q, stresslet m) and, for the
  // stresslet, its normal's; the Stokeslet's accumulator rows' strengths
  R qA[RB], nA[SDL ? RB : 1], qacc[SDL ? 1 : RB][4][3];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    const int bk = rb0 + rb;
    const int ra = bk * 16 + li;
    const bool la = rb < nown && ra < T;
    const int64_t ga = (int64_t)a * T + (la ? ra : 0);
    tcl[rb] = la ? xyz[ga] : Pa.c[cl];
    qA[rb] = (la && lg < 3) ? (R)(w[ga] * dens[(int64_t)lg * N + ga]) : R(0);
    if constexpr (SDL) {
      const double* nxyz = cl == 0 ? nx : (cl == 1 ? ny : nz);
      nA[rb] = (la && lg < 3) ? (R)nxyz[ga] : R(0);
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = bk * 16 + SS::row(lg, e);
        const bool lr = rb < nown && r < T;
        const int64_t g = (int64_t)a * T + (lr ? r : 0);
        const double wq = lr ? w[g] : 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) qacc[rb][e][k] = (R)(wq * dens[(int64_t)k * N + g]);
      }
    }
  }

  // forward sums over the admitted partners: FP32 per partner, folded into
  // FP64 (the per-partner sums over the 16 columns packed two arrays of 16
  // per lane); FP64 directly, columns summed at the end
  double accF[2] = {0.0, 0.0};
  double accD[F32 ? 1 : RB][4][C];
#pragma unroll
  for (int rb = 0; rb < (F32 ? 1 : RB); ++rb)
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int c = 0; c < C; ++c) accD[rb][e][c] = 0.0;

  for (int k = k0; k < k1; ++k) {
    const int b = k < H ? (a + 1 + k) % M : a + M / 2;
    const bool need_f = !((excl[(size_t)a * words + (b >> 5)] >> (b & 31)) & 1u);
    const bool need_r = !((excl[(size_t)b * words + (a >> 5)] >> (a & 31)) & 1u);
    R* rout = rev + (((size_t)b * KS + (k - kbase)) * RG + rg) * (size_t)C * T;
    if (!need_f && !need_r) {
      for (int t = tid; t < C * T; t += blockDim.x) rout[t] = R(0);
      continue;
    }
    const double cb = part[b].c[cl];
    // A operands: [D |D|^2], [D 1], [q_a/2  q_a.D] (stresslet: m_a) and, for
    // the stresslet, [nu_a/2  nu_a.D]; D_i of this lane's accumulator rows,
    // from the lanes holding them in [D 1] (row r, component i at lane r + 16 i)
    AOp aop[RB], a1[RB], a3[RB], a4[SDL ? RB : 1];
    R d1[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const double dl = lg < 3 ? tcl[rb] - cb : 0.0;
      double d2 = dl * dl;
      d2 += lane_value(d2, x16);
      d2 += lane_value(d2, x32);
      double qd = lg < 3 ? (double)qA[rb] * dl : 0.0;
      qd += lane_value(qd, x16);
      qd += lane_value(qd, x32);
      d1[rb] = lg < 3 ? (R)dl : R(1);
      aop[rb] = aform((R)(lg < 3 ? dl : d2), true);
      a1[rb] = aform(d1[rb], false);
      a3[rb] = aform(lg < 3 ? R(0.5) * qA[rb] : (R)qd, false);
      if constexpr (SDL) {
        double nd = lg < 3 ? (double)nA[rb] * dl : 0.0;
        nd += lane_value(nd, x16);
        nd += lane_value(nd, x32);
        a4[rb] = aform(lg < 3 ? R(0.5) * nA[rb] : (R)nd, false);
      }
    }
    R Dv[RB][4][3];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int i = 0; i < 3; ++i) Dv[rb][e][i] = lane_value(d1[rb], (SS::row(lg, e) + 16 * i) << 2);
    // this partner's forward tiles (FP32); FP64 adds into accD directly
    R tf[F32 ? RB : 1][4][C];
#pragma unroll
    for (int rb = 0; rb < (F32 ? RB : 1); ++rb)
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int c = 0; c < C; ++c) tf[rb][e][c] = R(0);
    auto fref = [&](int rb, int e, int c) -> R& {
      if constexpr (F32) return tf[rb][e][c];
      else return accD[rb][e][c];
    };
    // the partner's source blocks, one code path per admitted forward
    // direction (NF, wave-uniform); every wave takes RB row blocks, the ones
    // past its own being zero-strength rows at a's centre whose results are
    // dropped
    auto partner = [&](auto nf_c) {
      constexpr bool NF = decltype(nf_c)::value;
      for (int c0 = 0; c0 < nb; c0 += CH) {
        const int nbc = nb - c0 < CH ? nb - c0 : CH;
        __syncthreads();  // the previous chunk's operands and reverse sums are consumed
        if constexpr (X3) {
          // one thread per source column: its three B operands in the
          // three-piece form, and -o_i (half of the [-2o 1] operand)
          const float* gsrc = rec + ((size_t)b * nb + c0) * kSDGeo;
          for (int i = tid; i < nbc * 16; i += blockDim.x) {
            const float* r = gsrc + (i >> 4) * kSDGeo;
            const int j = i & 15;
            float* L = lds_rec + (i >> 4) * GEO;
            u4* LB = reinterpret_cast<u4*>(L) + j;
            u4 ops[4];
            const float g4[4] = {r[j], r[16 + j], r[32 + j], r[48 + j]};
            split_b_column(g4, r[64 + j], ops);
#pragma unroll
            for (int k = 0; k < 4; ++k) LB[16 * k] = ops[k];
            const float m4[4] = {r[80 + j], r[96 + j], r[112 + j], r[128 + j]};
            split_b_column(m4, 0.0f, ops);
#pragma unroll
            for (int k = 0; k < 4; ++k) LB[64 + 16 * k] = ops[k];
            const float n4[4] = {r[144 + j], r[160 + j], r[176 + j], r[192 + j]};
            split_b_column(n4, 0.0f, ops);
#pragma unroll
            for (int k = 0; k < 4; ++k) LB[128 + 16 * k] = ops[k];
#pragma unroll
            for (int k = 0; k < 3; ++k) L[SdlX3::MO + 16 * k + j] = 0.5f * r[16 * k + j];
          }
        } else {
          const R* gsrc = rec + ((size_t)b * nb + c0) * GEO;
          for (int i = tid; i < nbc * GEO; i += blockDim.x) lds_rec[i] = gsrc[i];
        }
        __syncthreads();
        for (int ib = 0; ib < nbc; ++ib) {
          const R* L = lds_rec + ib * GEO;
          // -o_i and q_b of column li
          R mo[3], qb[3];
          V r2[RB], df[RB], dr[RB], dfn[SDL ? RB : 1], drn[SDL ? RB : 1];
          if constexpr (X3) {
            const u4* LB = reinterpret_cast<const u4*>(L);
            const u4 bgeo = LB[lane];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
              mo[i] = L[SdlX3::MO + 16 * i + li];
              qb[i] = R(0);
            }
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
              r2[rb] = mma_x3(aop[rb], bgeo);
              if (NF) df[rb] = mma_x3(a1[rb], LB[64 + lane]);
              dr[rb] = mma_x3(a3[rb], bgeo);
              if (NF) dfn[rb] = mma_x3(a1[rb], LB[128 + lane]);
              drn[rb] = mma_x3(a4[rb], bgeo);
            }
          } else {
            const R bgeo = L[lane], bq = L[80 + lane];
            const R o2 = L[64 + li];
            // -o_i is half of the [-2o 1] operand
#pragma unroll
            for (int i = 0; i < 3; ++i) {
              mo[i] = R(0.5) * L[16 * i + li];
              qb[i] = SDL ? R(0) : L[80 + 16 * i + li];
            }
            const V zero = {R(0), R(0), R(0), R(0)};
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
              r2[rb] = SS::mma(aop[rb], bgeo, V{o2, o2, o2, o2});
              if (NF) df[rb] = SS::mma(a1[rb], bq, zero);
              dr[rb] = SS::mma(a3[rb], bgeo, zero);
              if constexpr (SDL) {
                if (NF) dfn[rb] = SS::mma(a1[rb], L[144 + lane], zero);
                drn[rb] = SS::mma(a4[rb], bgeo, zero);
              }
            }
          }
          R rv[C];
#pragma unroll
          for (int c = 0; c < C; ++c) rv[c] = R(0);
#pragma unroll
          for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              // q_i/r + (d.q) d_i/r^3 = (q_i + ((d.q)/r^2) d_i) / r
              const R ri = SS::rsq(r2[rb][e]);
              const R ri2 = ri * ri;
              R dd[3];
#pragma unroll
              for (int i = 0; i < 3; ++i) dd[i] = Dv[rb][e][i] + mo[i];
              if constexpr (SDL) {
                // (d.m)(d.nu) d / r^5 forward; reversed, d changes sign
                const R ri5 = ri * ri2 * ri2;
                if (NF) {
                  const R wf = df[rb][e] * dfn[rb][e] * ri5;
#pragma unroll
                  for (int i = 0; i < 3; ++i) fref(rb, e, i) = fma(wf, dd[i], fref(rb, e, i));
                }
                const R wr = dr[rb][e] * drn[rb][e] * ri5;
#pragma unroll
                for (int i = 0; i < 3; ++i) rv[i] = fma(-wr, dd[i], rv[i]);
              } else {
                if (NF) {
                  const R ff = df[rb][e] * ri2;
#pragma unroll
                  for (int i = 0; i < 3; ++i) fref(rb, e, i) = fma(ri, fma(ff, dd[i], qb[i]), fref(rb, e, i));
                  if constexpr (C == 4) fref(rb, e, 3) = fma(ff, ri, fref(rb, e, 3));
                }
                const R fr = dr[rb][e] * ri2;
#pragma unroll
                for (int i = 0; i < 3; ++i) rv[i] = fma(ri, fma(fr, dd[i], qacc[rb][e][i]), rv[i]);
                if constexpr (C == 4) rv[3] = fma(-fr, ri, rv[3]);  // the pressure kernel is odd in d
              }
            }
          // the four lane groups holding the same column
#pragma unroll
          for (int c = 0; c < C; ++c) {
            rv[c] += lane_value(rv[c], x16);
            rv[c] += lane_value(rv[c], x32);
          }
          if (lg == 0)
#pragma unroll
            for (int c = 0; c < C; ++c) lds_rev[((wave * C + c) * CH + ib) * 16 + li] = rv[c];
        }
        __syncthreads();
        // reverse sums over the waves, in wave order
        for (int idx = tid; idx < C * nbc * 16; idx += blockDim.x) {
          const int c = idx / (nbc * 16), col = idx - c * (nbc * 16);
          const int t = c0 * 16 + col;
          if (t >= T) continue;
          R sum = R(0);
          for (int wv = 0; wv < W; ++wv) sum += lds_rev[(wv * C + c) * CH * 16 + col];
          rout[(size_t)c * T + t] = need_r ? sum : R(0);
        }
      }
    };
    if (need_f) partner(std::true_type{});
    else partner(std::false_type{});
    if (!need_f) continue;
    if constexpr (F32) {
      // this partner's tiles summed over their 16 columns, into FP64: two
      // arrays of 16 elements f = (rb*4 + e)*C + c, lane li keeping element li
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        float v[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
          const int f = 16 * h + j;
          const int rb = f / (4 * C), e = (f / C) % 4, c = f % C;
          v[j] = (rb < RB) ? (float)tf[rb < RB ? rb : 0][e][c] : 0.0f;
        }
        accF[h] += row_group_sums(v, lane);
      }
    }
  }
  // forward partials
  auto put = [&](int rb, int e, int c, double v) {
    if (rb >= nown) return;
    const int r = (rb0 + rb) * 16 + SS::row(lg, e);
    if (r >= T) return;
    double* f = fwd + ((size_t)split * C + c) * N + (int64_t)a * T + r;
    *f = (first ? 0.0 : *f) + v * (SDL ? k3Over4PiS : (c < 3 ? kInv8PiS : kInv4PiS));
  };
  if constexpr (F32) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int f = 16 * h + li;
      const int rb = f / (4 * C), e = (f / C) % 4, c = f % C;
      if (rb < RB) put(rb, e, c, accF[h]);
    }
  } else {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const double v = lane_sum_fp64(accD[rb][e][c]);
          if (li == 0) put(rb, e, c, v);
        }
  }
}

// Each target's reverse slots of a launch, slot then row group, added in FP64
// to its running totals racc [C][N] (first launch: from zero).
template <typename R>
__global__ void k_far_stokes_fold(const R* __restrict__ rev, int M, int T, int RG, int C, int kbase, int kend,
                                  int first, int64_t N, double* __restrict__ racc) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  const int b = (int)(g / T), t = (int)(g - (int64_t)b * T);
  const int H = (M - 1) / 2;
  const int slots = H + (((M & 1) == 0 && b >= M / 2) ? 1 : 0);
  const int KS = kend - kbase;
  const int hi = kend < slots ? kend : slots;
  for (int c = 0; c < C; ++c) {
    double r = first ? 0.0 : racc[(size_t)c * N + g];
    for (int k = kbase; k < hi; ++k)
      for (int rg = 0; rg < RG; ++rg)
        r += (double)rev[((((size_t)b * KS + (k - kbase)) * RG + rg) * C + c) * T + t];
    racc[(size_t)c * N + g] = r;
  }
}

// The pair kernel's launches over the partner offsets, each followed by its
// fold: source blocks into prec, reverse sums of a launch in rev (rev_bytes),
// forward sums into the first stokes_pair_splits slices of fwd [slices][C][N],
// reverse totals into racc [C][N].
template <typename R, int C, bool SDL>
sbie_status launch_stokes_pairs(sbie_geom* g, const double* d_dens, hipStream_t s, double* prec, double* rev_buf,
                                uint64_t rev_bytes, double* fwd, double* racc) {
  const int M = g->M, T = g->T, nb = (T + 15) / 16;
  const int RG = stokes_row_groups(T, sizeof(R) == 8);
  R* rec = reinterpret_cast<R*>(prec);
  const dim3 rgrid((unsigned)(((int64_t)M * nb * 64 + 255) / 256));
  if constexpr (SDL)
    hipLaunchKernelGGL(k_sdl_pair_records<R>, rgrid, dim3(256), 0, s, g->d_part, d_dens, g->d_x, g->d_y, g->d_z,
                       g->d_w, g->d_nx, g->d_ny, g->d_nz, M, T, nb, g->N, rec);
  else
    hipLaunchKernelGGL(k_stokes_pair_records<R>, rgrid, dim3(256), 0, s, g->d_part, d_dens, g->d_x, g->d_y, g->d_z,
                       g->d_w, M, T, nb, g->N, rec);
  SBIE_HIP(hipGetLastError());
  const int PMAX = (M - 1) / 2 + ((M & 1) == 0 ? 1 : 0);
  const int KS = stokes_rev_slots(M, T, C, (int)sizeof(R), rev_bytes);
  const int nsplit = stokes_pair_splits(g, RG);
  R* rev = reinterpret_cast<R*>(rev_buf);
  const dim3 grid((unsigned)((int64_t)M * RG * nsplit)), fold((unsigned)((g->N + 255) / 256));
  for (int kbase = 0; kbase == 0 || kbase < PMAX; kbase += KS) {
    const int kend = kbase + KS, first = kbase == 0 ? 1 : 0;
    hipLaunchKernelGGL((k_far_stokes_pairs<R, C, SDL>), grid, dim3(64 * kSWaves), 0, s, rec, g->d_part, g->d_x,
                       g->d_y, g->d_z, d_dens, g->d_w, g->d_nx, g->d_ny, g->d_nz, g->d_excl, g->excl_words, M, T,
                       g->N, nsplit, RG, kbase, kend, first, fwd, rev);
    SBIE_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_far_stokes_fold<R>, fold, dim3(256), 0, s, rev, M, T, RG, C, kbase, kend, first, g->N,
                       racc);
    SBIE_HIP(hipGetLastError());
  }
  return SBIE_OK;
}

}  // namespace

size_t stokes_record_doubles(bool sdl) { return sdl ? (size_t)kSDGeo : (size_t)kSGeo; }

int stokes_row_groups(int T, bool fp64) {
  const int nb = (T + 15) / 16;
  const int gb = kSWaves * (fp64 ? StokesShape<double>::RB : StokesShape<float>::RB);
  return (nb + gb - 1) / gb;
}

int stokes_rev_slots(int M, int T, int C, int bytes_per_value, uint64_t cap_bytes) {
  const int pmax = (M - 1) / 2 + ((M & 1) == 0 ? 1 : 0);
  if (pmax < 1) return 1;
  const uint64_t per_slot = (uint64_t)M * stokes_row_groups(T, bytes_per_value == 8) * C * T * bytes_per_value;
  int k = (int)(cap_bytes / (per_slot > 0 ? per_slot : 1));
  if (k > pmax) k = pmax;
  if (k < 1) k = 1;
  const int launches = (pmax + k - 1) / k;
  return (pmax + launches - 1) / launches;
}

int stokes_pair_splits(const sbie_geom* g, int RG) {
  const int want = (int)((512 + (int64_t)g->M * RG - 1) / ((int64_t)g->M * RG));
  const int pmax = (g->M - 1) / 2 + ((g->M & 1) == 0 ? 1 : 0);
  int n = want < g->nsplit ? want : g->nsplit;
  if (n > pmax) n = pmax;
  return n < 1 ? 1 : n;
}

uint64_t stokes_rev_bytes(int M, int T) {
  // every slot at once if that fits the budget, else the budget (FP64, four
  // components); at least one slot
  const int pmax = (M - 1) / 2 + ((M & 1) == 0 ? 1 : 0);
  const uint64_t per_slot = (uint64_t)M * stokes_row_groups(T, true) * 4 * T * sizeof(double);
  const uint64_t all = per_slot * (uint64_t)(pmax > 0 ? pmax : 1);
  const uint64_t cap = all < kStokesRevBudget ? all : kStokesRevBudget;
  return cap < per_slot ? per_slot : cap;
}

sbie_status far_stokes_pairs(sbie_geom* g, int C, bool mixed, const double* d_dens, hipStream_t s) {
  double *pr = g->d_stk_prec, *rv = g->d_stk_rev, *fw = g->d_stk_part, *ra = g->d_stk_racc;
  const uint64_t rb = g->stk_rev_bytes;
  if (mixed)
    return C == 4 ? launch_stokes_pairs<float, 4, false>(g, d_dens, s, pr, rv, rb, fw, ra)
                  : launch_stokes_pairs<float, 3, false>(g, d_dens, s, pr, rv, rb, fw, ra);
  return C == 4 ? launch_stokes_pairs<double, 4, false>(g, d_dens, s, pr, rv, rb, fw, ra)
                : launch_stokes_pairs<double, 3, false>(g, d_dens, s, pr, rv, rb, fw, ra);
}

sbie_status far_sdl_pairs(sbie_geom* g, bool mixed, const double* d_dens, hipStream_t s) {
  double *pr = g->d_sdl_prec, *rv = g->d_sdl_rev, *fw = g->d_sdl_part, *ra = g->d_sdl_racc;
  const uint64_t rb = g->sdl_rev_bytes;
  return mixed ? launch_stokes_pairs<float, 3, true>(g, d_dens, s, pr, rv, rb, fw, ra)
               : launch_stokes_pairs<double, 3, true>(g, d_dens, s, pr, rv, rb, fw, ra);
}

}  // namespace sbie
