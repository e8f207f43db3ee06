// Far-field direct sum (part (d), Section 4.1 smooth quadrature; far-field step
// of Algorithm 1) with the pair distances formed on the matrix cores.
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
//
// In mixed precision the single and double layers take their K = 4 products
// on the bf16 matrix cores, each FP32 operand split exactly into three bf16
// pieces (see split3 below): a 16x16x32 bf16 product gives the FP32 products'
// values at half the issue time of the 16x16x4 FP32 one.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "sbie_internal.h"
#include "x3.h"

namespace sbie {

namespace {

constexpr double kInv4PiD = 0.079577471545947667884441881686257181;

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

// Values per 16-source block of the geometry records (geo) and the per-apply
// strengths (app), in HBM (GEO_G, APP_G) and as staged in LDS (GEO, APP).  In
// HBM every block holds one R per lane of its B operands and the accumulator
// input per column after them.  The mixed single and double layers take their
// products in the three-piece form: the staging splits each B operand into
// one u4 per lane, so that HBM holds the compact FP32 values only.
template <typename R, int OP>
struct FarLayout {
  static constexpr bool X3 = sizeof(R) == 4 && (OP == SBIE_OP_S || OP == SBIE_OP_D);
  static constexpr int GEO_G = 80;
  static constexpr int APP_G = OP == SBIE_OP_S ? 16 : (OP == SBIE_OP_SP ? 128 : 80);
  static constexpr int GEO = X3 ? 256 : GEO_G;
  static constexpr int APP = X3 && OP == SBIE_OP_D ? 256 : APP_G;
};

constexpr int kChunk = 40;  // 16-source blocks staged in LDS at a time
// Workgroup shape of the pair kernel: up to WMAX waves (three per SIMD, which
// the registers allow), each holding up to RBMAX blocks of 16 target rows; a
// particle's rows are split into groups of WMAX*RBMAX blocks, spread evenly
// over the waves so that every SIMD carries the same work.  (FP64 at eight
// waves of five blocks, two per SIMD, took 7% (S) and 5% (D) longer; at
// sixteen waves of three, four per SIMD with a few spilled registers, 7%.)
template <typename R>
struct PairShape {
  static constexpr int WMAX = 12;
  static constexpr int RBMAX = 4;
  static constexpr int GB = WMAX * RBMAX;  // row blocks per group
  // row blocks whose matrix-core products are issued together
  static constexpr int batch(bool) { return 4; }
};

// Pair-symmetric far field.  Every unordered pair of particles (a, b) is
// visited once, by the workgroup that owns a's target rows: a visits the
// partners b = a+1 .. a+H (mod M), H = (M-1)/2, and for even M the partner
// a + M/2 when a < M/2.  The reciprocal distance of each node pair serves both
// directions: the forward sum into a's targets from b's sources stays in
// registers across the partners, and the reverse sum into b's targets from
// a's sources is reduced over a's rows (lanes, then waves in order).  A
// direction whose source is excluded for its target particle (self, near
// field) is dropped.
//
// One launch covers the partner offsets k in [kbase, kend) (k = (b - a - 1)
// mod M is also the slot of handler a in b's list).  Its reverse sums go to
// rev[b][k - kbase][rg][t] (a dropped direction writes zeros), which
// k_far_fold adds, slot by slot, into b's running totals before the next
// launch reuses the slots: memory for kend - kbase slots instead of H + 1.
// The forward sums of the launch are added to the split's running partial
// (first launch: written).
//
// Squared distances come off the matrix cores as in a K = 4 contraction: with
// D = x - c_b and o = y - c_b,  |x - y|^2 = [D |D|^2] . [-2o 1] + |o|^2.  The
// double layer's forward dot d_b.(x - y) is [D |D|^2] . [d_b 0] - d_b.o, and
// its reverse dot d_a.(x - y) is [d_a/2  d_a.D] . [-2o 1].  For S' (the
// derivative along the target normal, strengths q = W sigma) the forward dot
// q_b nu_a.(x - y) is [nu_a/2  nu_a.D] . [-2 q_b o  q_b] and the reverse dot
// q_a nu_b.(x - y) is [q_a D  q_a] . [nu_b  -nu_b.o]; the forward kernel is
// q_b nu_a.(y - x)/r^3, the reverse q_a nu_b.(x - y)/r^3.  D' has the
// symmetric kernel B = nu_a.nu_b/r^3 - 3 (nu_a.d)(nu_b.d)/r^5, d = x - y, with
// nu_a.nu_b = [nu_a 0] . [nu_b  -nu_b.o], nu_b.d = [D 1] . [nu_b  -nu_b.o] and
// nu_a.d = [nu_a/2  nu_a.D] . [-2o 1]; forward q_b B, reverse q_a B.
//
// Rows of a are padded to 16 with zero-strength points at a's centre.
template <typename R, int OP>
__device__ __forceinline__ void far_pairs_body(const R* __restrict__ geo, const R* __restrict__ app,
                                               const Particle* __restrict__ part, const double* __restrict__ x,
                                               const double* __restrict__ y, const double* __restrict__ z,
                                               const uint32_t* __restrict__ excl, int words, int M, int T, int T16,
                                               int64_t N, int nsplit, int RG, int kbase, int kend, int first,
                                               double* __restrict__ fwd, R* __restrict__ rev, int wid) {
  using MM = Mfma<R>;
  using V = typename MM::V;
  using L = FarLayout<R, OP>;
  constexpr bool X3 = L::X3;
  using AOp = typename std::conditional<X3, u4, R>::type;  // A operand of one row block
  using BOp = typename std::conditional<X3, u4, R>::type;  // B operand of one source block
  constexpr int GEO = L::GEO, APP = L::APP, GEO_G = L::GEO_G, APP_G = L::APP_G;
  constexpr bool NORMALS = OP == SBIE_OP_SP || OP == SBIE_OP_DP;  // rows carry their normals
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R* lds_geo = reinterpret_cast<R*>(smem_raw);
  R* lds_app = lds_geo + kChunk * GEO;
  R* lds_rev = lds_app + kChunk * APP;  // [wave][kChunk*16] reverse column sums
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform, for the compiler
  const int li = lane & 15, lg = lane >> 4;
  const int x16 = (lane ^ 16) << 2, x32 = (lane ^ 32) << 2;  // partner lanes of the column sums
  const int split = wid % nsplit, rest = wid / nsplit;
  const int rg = rest % RG, a = rest / RG;
  const int nb = T16 / 16;
  constexpr int GB = PairShape<R>::GB, RB = PairShape<R>::RBMAX;
  const int W = blockDim.x >> 6;
  const int rbg = rg * GB;                                     // first row block of the group
  const int cnt = nb - rbg < GB ? nb - rbg : GB;               // row blocks of the group
  // With cnt = base*W + 1 and base < RB, wave w owns base blocks (slots
  // 0 .. base-1) and every wave holds the last block in slot base, taking it
  // against its W-th of each chunk's source blocks: every SIMD then carries
  // the same work.  Otherwise the blocks are spread as evenly as whole blocks
  // allow.
  const int base = cnt / W, rem = cnt - base * W;
  const int nx = (rem == 1 && base > 0 && base < RB) ? 1 : 0;  // shared blocks
  const int rb0 = nx > 0 ? rbg + wave * base : rbg + (wave * cnt) / W;  // first owned block
  const int nown = nx > 0 ? base : rbg + ((wave + 1) * cnt) / W - rb0;  // owned blocks
  const int xb0 = rbg + W * base;                                        // first shared block
  const int nrb = nown + nx;                                             // slots in use
  const int nown_u = __builtin_amdgcn_readfirstlane(nown);  // wave-uniform, for the compiler
  const int nx_u = __builtin_amdgcn_readfirstlane(nx);
  const int H = (M - 1) / 2;
  const bool even = (M & 1) == 0;
  const int P = H + ((even && a < M / 2) ? 1 : 0);
  // this launch's partner offsets of particle a, split nsplit ways
  const int klo = kbase < P ? kbase : P, khi = kend < P ? kend : P;
  const int k0 = klo + (int)((int64_t)(khi - klo) * split / nsplit);
  const int k1 = klo + (int)((int64_t)(khi - klo) * (split + 1) / nsplit);
  const int KS = kend - kbase;  // slots of the launch
  const Particle& Pa = part[a];

  // A-operand row li of each row block: lane group lg < 3 keeps component lg
  // of the target (tcl) and of its d_a resp. nu_a (dal, zero in group 3);
  // |D|^2 and the dots are summed across the lane groups per partner.
  // Accumulator rows: the single layer's and D''s strengths (qa), S''s
  // strength of the A-operand row (qr).
  // (The three-piece double layer, short of registers, keeps tcl and dal in
  // LDS after the reverse sums, read back per partner.)
  constexpr bool STASH = X3 && OP == SBIE_OP_D;
  double* lds_tc0 = reinterpret_cast<double*>(lds_rev + kChunk * 16 * W);  // [W][RB][64]
  R* lds_da0 = reinterpret_cast<R*>(lds_tc0 + W * RB * 64);                   // [W][RB][64]
  double* lds_tc = lds_tc0 + wave * RB * 64 + lane;
  R* lds_da = lds_da0 + wave * RB * 64 + lane;
  double tcl[RB];
  R dal[RB];
  R qa[RB][4];
  R qr[RB];
  const int cl = lg < 3 ? lg : 0;
  const double* xyz = cl == 0 ? x : (cl == 1 ? y : z);
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    const int bk = rb < nown ? rb0 + rb : xb0 + (rb - nown);  // block of slot rb (if rb < nrb)
    const int r = bk * 16 + li;
    const double tv = (rb < nrb && r < T) ? xyz[(int64_t)a * T + r] : Pa.c[cl];
    const size_t blk = (size_t)a * nb + (rb < nrb ? bk : 0);
    R dv = R(0);
    if (rb < nrb && lg < 3) {
      if constexpr (OP == SBIE_OP_D || OP == SBIE_OP_DP)
        dv = app[blk * APP_G + 16 * lg + li];
      else if constexpr (OP == SBIE_OP_SP)
        dv = app[blk * APP_G + 64 + 16 * lg + li];
    }
    if constexpr (STASH) {
      lds_tc[rb * 64] = tv;
      lds_da[rb * 64] = dv;
    } else {
      tcl[rb] = tv;
      dal[rb] = dv;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
      qa[rb][e] = rb >= nrb ? R(0)
                  : OP == SBIE_OP_S ? app[blk * 16 + MM::row(lg, e)]
                  : OP == SBIE_OP_DP ? app[blk * 80 + 64 + MM::row(lg, e)] : R(0);
    qr[rb] = (OP == SBIE_OP_SP && rb < nrb) ? app[blk * 128 + 48 + li] : R(0);
  }

  // forward sums of the accumulator rows over the admitted partners (FP64).
  // FP32 (four slots, sixteen elements k = 4*slot + e per lane): each
  // partner's tiles are first summed over their 16 columns, lane li of every
  // row group keeping element li, so one accumulator per lane (acc1); FP64:
  // every element per lane (acc), the columns summed at the end.
  constexpr bool ROWSUM = sizeof(R) == 4 && RB == 4;
  double acc1 = 0.0;
  double acc[ROWSUM ? 1 : RB][4];
#pragma unroll
  for (int rb = 0; rb < (ROWSUM ? 1 : RB); ++rb)
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[rb][e] = 0.0;

  // A operand of this lane's row from a value; `extra` picks up the B
  // column's accumulator term in the three-piece form
  auto mk_a = [&](double v, bool extra) -> AOp {
    if constexpr (X3) return split_a((float)v, lg, extra);
    else return (R)v;
  };
  auto ldb = [&](const R* blk) -> BOp {
    if constexpr (X3) return reinterpret_cast<const u4*>(blk)[lane];
    else return blk[lane];
  };
  // one K = 4 product; the three-piece form carries c in its extra slots
  auto mm = [&](AOp av, BOp bv, V c) -> V {
    if constexpr (X3) return mma_x3(av, bv);
    else return MM::mma(av, bv, c);
  };

  for (int k = k0; k < k1; ++k) {
    const int b = k < H ? (a + 1 + k) % M : a + M / 2;
    const bool need_f = !((excl[(size_t)a * words + (b >> 5)] >> (b & 31)) & 1u);
    const bool need_r = !((excl[(size_t)b * words + (a >> 5)] >> (a & 31)) & 1u);
    R* rout = rev + (((size_t)b * KS + (k - kbase)) * RG + rg) * T;
    if (!need_f && !need_r) {
      for (int t = tid; t < T; t += blockDim.x) rout[t] = R(0);
      continue;
    }
    const double cb = part[b].c[cl];
    // A operands of this wave's rows against partner b: [D |D|^2] with
    // D = x - c_b; double layer also [d_a/2  d_a.D]; S' [nu_a/2  nu_a.D] and
    // [q_a D  q_a]; D' [D 1]
    AOp aop[RB], a3[RB];
    R aq[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      if (rb >= nown_u + nx_u) break;
      const double tv = STASH ? lds_tc[rb * 64] : tcl[rb];
      const double dl = lg < 3 ? tv - cb : 0.0;
      double d2 = dl * dl;
      d2 += lane_value(d2, x16);
      d2 += lane_value(d2, x32);
      aop[rb] = mk_a(lg < 3 ? dl : d2, true);
      if (OP == SBIE_OP_D || NORMALS) {
        const R da = STASH ? lds_da[rb * 64] : dal[rb];
        double dd = (double)da * dl;
        dd += lane_value(dd, x16);
        dd += lane_value(dd, x32);
        a3[rb] = mk_a(lg < 3 ? (double)(R(0.5) * da) : dd, false);
      }
      if (OP == SBIE_OP_SP) aq[rb] = lg < 3 ? (R)((double)qr[rb] * dl) : qr[rb];
      if (OP == SBIE_OP_DP) aq[rb] = lg < 3 ? (R)dl : R(1);
    }
    R tmp[RB][4];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int e = 0; e < 4; ++e) tmp[rb][e] = R(0);
    for (int c0 = 0; c0 < nb; c0 += kChunk) {
      const int nbc = nb - c0 < kChunk ? nb - c0 : kChunk;
      // No barrier is needed before the staging: the previous operands were
      // last read before the barrier that precedes the previous reverse
      // reduction, and the reverse sums are next written only after the
      // barrier below, which every thread reaches after its reduction.
      {
        using C16 = typename std::conditional<sizeof(R) == 4, float4, double2>::type;
        constexpr int PER = 16 / sizeof(R);
        // a block's B operand in the three-piece form: lane 16k + j takes term k
        // of column j and the column's accumulator input (value 64 + j); one
        // thread per column
        auto stage_x3 = [&](const R* src, R* dst) {
          u4* ld = reinterpret_cast<u4*>(dst);
          for (int i = tid; i < nbc * 16; i += blockDim.x) {
            const R* r = src + (i >> 4) * 80;
            const int j = i & 15;
            const float xk[4] = {(float)r[j], (float)r[16 + j], (float)r[32 + j], (float)r[48 + j]};
            u4 o[4];
            split_b_column(xk, (float)r[64 + j], o);
            u4* d = ld + (i >> 4) * 64 + j;
#pragma unroll
            for (int k = 0; k < 4; ++k) d[16 * k] = o[k];
          }
        };
        const R* gsrc = geo + ((size_t)b * nb + c0) * GEO_G;
        if constexpr (X3) {
          stage_x3(gsrc, lds_geo);
        } else {
          const C16* gs = reinterpret_cast<const C16*>(gsrc);
          C16* ld = reinterpret_cast<C16*>(lds_geo);
          for (int i = tid; i < nbc * GEO / PER; i += blockDim.x) ld[i] = gs[i];
        }
        const R* asrc = app + ((size_t)b * nb + c0) * APP_G;
        if constexpr (X3 && OP == SBIE_OP_D) {
          stage_x3(asrc, lds_app);
        } else {
          const C16* as = reinterpret_cast<const C16*>(asrc);
          C16* la = reinterpret_cast<C16*>(lds_app);
          for (int i = tid; i < nbc * APP / PER; i += blockDim.x) la[i] = as[i];
        }
      }
      __syncthreads();
      // the tiles of source block ib for the first NR slots, unrolled so that
      // the matrix-core products of all NR blocks are issued before their
      // vector work (NR is wave-uniform: one branch per wave)
      auto tiles = [&](auto nr, int ib) {
        constexpr int NR = decltype(nr)::value;
        {
          const BOp bv = ldb(lds_geo + ib * GEO);
          V cinit = {R(0), R(0), R(0), R(0)};
          if constexpr (!X3) {
            const R cw = lds_geo[ib * GEO + 64 + li];
            cinit = V{cw, cw, cw, cw};
          }
          const V zero = {R(0), R(0), R(0), R(0)};
          R rsum = R(0);  // reverse sum for source column li over this lane's rows
          // row blocks in batches of G: the batch's matrix-core products first,
          // then its vector work (G bounded by the registers)
          // (D': four products per block; the double layer's three-piece operands)
          constexpr int G = (OP == SBIE_OP_DP || (X3 && OP == SBIE_OP_D)) ? 2 : PairShape<R>::batch(OP == SBIE_OP_S);
          if (OP == SBIE_OP_S) {
            const R qb = lds_app[ib * 16 + li];
#pragma unroll
            for (int g0 = 0; g0 < NR; g0 += G) {
              V r2[G];
#pragma unroll
              for (int j = 0; j < G; ++j)
                if (g0 + j < NR) r2[j] = mm(aop[g0 + j], bv, cinit);
#pragma unroll
              for (int j = 0; j < G; ++j)
                if (g0 + j < NR)
#pragma unroll
                  for (int e = 0; e < 4; ++e) {
                    const R ri = MM::rsq(r2[j][e]);
                    tmp[g0 + j][e] = fma(qb, ri, tmp[g0 + j][e]);
                    rsum = fma(qa[g0 + j][e], ri, rsum);
                  }
            }
          } else if constexpr (OP == SBIE_OP_DP) {
            const R bn = lds_app[ib * 80 + lane];
            const R qb = lds_app[ib * 80 + 64 + li];
#pragma unroll
            for (int g0 = 0; g0 < NR; g0 += G) {
              V r2[G], nn[G], nyd[G], nxd[G];
#pragma unroll
              for (int j = 0; j < G; ++j)
                if (g0 + j < NR) {
                  r2[j] = mm(aop[g0 + j], bv, cinit);
                  nn[j] = MM::mma(dal[g0 + j], bn, zero);
                  nyd[j] = MM::mma(aq[g0 + j], bn, zero);
                  nxd[j] = mm(a3[g0 + j], bv, zero);
                }
#pragma unroll
              for (int j = 0; j < G; ++j)
                if (g0 + j < NR)
#pragma unroll
                  for (int e = 0; e < 4; ++e) {
                    const R ri = MM::rsq(r2[j][e]);
                    const R ri2 = ri * ri;
                    const R w = fma(R(-3) * nyd[j][e], nxd[j][e] * ri2, nn[j][e]);
                    const R bk = w * ri2 * ri;
                    tmp[g0 + j][e] = fma(qb, bk, tmp[g0 + j][e]);
                    rsum = fma(qa[g0 + j][e], bk, rsum);
                  }
            }
          } else if constexpr (OP == SBIE_OP_SP) {
            const R bq = lds_app[ib * 128 + lane];
            const R bn = lds_app[ib * 128 + 64 + lane];
#pragma unroll
            for (int g0 = 0; g0 < NR; g0 += G) {
              V r2[G], df[G], dr[G];
#pragma unroll
              for (int j = 0; j < G; ++j)
                if (g0 + j < NR) {
                  r2[j] = mm(aop[g0 + j], bv, cinit);
                  df[j] = mm(a3[g0 + j], bq, zero);
                  dr[j] = MM::mma(aq[g0 + j], bn, zero);
                }
#pragma unroll
              for (int j = 0; j < G; ++j)
                if (g0 + j < NR)
#pragma unroll
                  for (int e = 0; e < 4; ++e) {
                    const R ri = MM::rsq(r2[j][e]);
                    const R ri3 = ri * ri * ri;
                    tmp[g0 + j][e] = fma(-df[j][e], ri3, tmp[g0 + j][e]);
                    rsum = fma(dr[j][e], ri3, rsum);
                  }
            }
          } else {
            const BOp dv = ldb(lds_app + ib * APP);
            V c2 = zero;
            if constexpr (!X3) {
              const R dw = lds_app[ib * 80 + 64 + li];
              c2 = V{dw, dw, dw, dw};
            }
#pragma unroll
            for (int g0 = 0; g0 < NR; g0 += G) {
              V r2[G], df[G], dr[G];
#pragma unroll
              for (int j = 0; j < G; ++j)
                if (g0 + j < NR) {
                  r2[j] = mm(aop[g0 + j], bv, cinit);
                  df[j] = mm(aop[g0 + j], dv, c2);
                  dr[j] = mm(a3[g0 + j], bv, zero);
                }
#pragma unroll
              for (int j = 0; j < G; ++j)
                if (g0 + j < NR)
#pragma unroll
                  for (int e = 0; e < 4; ++e) {
                    const R ri = MM::rsq(r2[j][e]);
                    const R ri3 = ri * ri * ri;
                    tmp[g0 + j][e] = fma(df[j][e], ri3, tmp[g0 + j][e]);
                    rsum = fma(dr[j][e], ri3, rsum);
                  }
            }
          }
          // sum the four lane groups holding the same column
          rsum += lane_value(rsum, x16);
          rsum += lane_value(rsum, x32);
          if (lg == 0) lds_rev[wave * (kChunk * 16) + ib * 16 + li] = rsum;
        }
      };
      if constexpr (sizeof(R) == 8) {
        // FP64: one row block at a time under a wave-uniform guard (the
        // batched form does not fit the FP64 operands in registers)
        const int xlo = nx_u > 0 ? (nbc * wave) / W : 0, xhi = nx_u > 0 ? (nbc * (wave + 1)) / W : 0;
        if (nrb > 0) {
          for (int ib = 0; ib < nbc; ++ib) {
            const int nr = (ib >= xlo && ib < xhi) ? nown_u + nx_u : nown_u;
            const R bv = lds_geo[ib * GEO + lane];
            const R cw = lds_geo[ib * GEO + 64 + li];
            const V cinit = {cw, cw, cw, cw};
            const V zero = {R(0), R(0), R(0), R(0)};
            // the source block's strengths: S W sigma; D (W mu nu, 0) and
            // -W mu nu.o; S' (-2 q o, q) and (nu, -nu.o); D' (nu, -nu.o) and q
            R u0, u1 = R(0);
            if constexpr (OP == SBIE_OP_S) {
              u0 = lds_app[ib * 16 + li];
            } else if constexpr (OP == SBIE_OP_SP) {
              u0 = lds_app[ib * 128 + lane];
              u1 = lds_app[ib * 128 + 64 + lane];
            } else {
              u0 = lds_app[ib * 80 + lane];
              u1 = lds_app[ib * 80 + 64 + li];
            }
            R rsum = R(0);
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
              if (rb < nr) {
                if (OP == SBIE_OP_S) {
                  const V r2 = MM::mma(aop[rb], bv, cinit);
#pragma unroll
                  for (int e = 0; e < 4; ++e) {
                    const R ri = MM::rsq(r2[e]);
                    tmp[rb][e] = fma(u0, ri, tmp[rb][e]);
                    rsum = fma(qa[rb][e], ri, rsum);
                  }
                } else if (OP == SBIE_OP_DP) {
                  const V r2 = MM::mma(aop[rb], bv, cinit);
                  const V nn = MM::mma(dal[rb], u0, zero);
                  const V nyd = MM::mma(aq[rb], u0, zero);
                  const V nxd = MM::mma(a3[rb], bv, zero);
#pragma unroll
                  for (int e = 0; e < 4; ++e) {
                    const R ri = MM::rsq(r2[e]);
                    const R ri2 = ri * ri;
                    const R w = fma(R(-3) * nyd[e], nxd[e] * ri2, nn[e]);
                    const R bk = w * ri2 * ri;
                    tmp[rb][e] = fma(u1, bk, tmp[rb][e]);
                    rsum = fma(qa[rb][e], bk, rsum);
                  }
                } else if (OP == SBIE_OP_SP) {
                  const V r2 = MM::mma(aop[rb], bv, cinit);
                  const V df = MM::mma(a3[rb], u0, zero);
                  const V dr = MM::mma(aq[rb], u1, zero);
#pragma unroll
                  for (int e = 0; e < 4; ++e) {
                    const R ri = MM::rsq(r2[e]);
                    const R ri3 = ri * ri * ri;
                    tmp[rb][e] = fma(-df[e], ri3, tmp[rb][e]);
                    rsum = fma(dr[e], ri3, rsum);
                  }
                } else {
                  const V c2 = {u1, u1, u1, u1};
                  const V r2 = MM::mma(aop[rb], bv, cinit);
                  const V df = MM::mma(aop[rb], u0, c2);
                  const V dr = MM::mma(a3[rb], bv, zero);
#pragma unroll
                  for (int e = 0; e < 4; ++e) {
                    const R ri = MM::rsq(r2[e]);
                    const R ri3 = ri * ri * ri;
                    tmp[rb][e] = fma(df[e], ri3, tmp[rb][e]);
                    rsum = fma(dr[e], ri3, rsum);
                  }
                }
              }
            }
            rsum += lane_value(rsum, x16);
            rsum += lane_value(rsum, x32);
            if (lg == 0) lds_rev[wave * (kChunk * 16) + ib * 16 + li] = rsum;
          }
        } else {
          for (int c = lane; c < nbc * 16; c += 64) lds_rev[wave * (kChunk * 16) + c] = R(0);
        }
      } else {
        // source blocks against the owned slots, and against the shared slot
        // too in this wave's slice [xlo, xhi) of the chunk; one case per
        // (wave-uniform) slot count
        const int xlo = (nbc * wave) / W, xhi = (nbc * (wave + 1)) / W;
        auto run = [&](auto no) {
          constexpr int NO = decltype(no)::value;
          if (nx_u == 0) {
            for (int ib = 0; ib < nbc; ++ib) tiles(no, ib);
          } else {
            constexpr int NT = NO + 1 < RB ? NO + 1 : RB;
            for (int ib = 0; ib < xlo; ++ib) tiles(no, ib);
            for (int ib = xlo; ib < xhi; ++ib) tiles(std::integral_constant<int, NT>{}, ib);
            for (int ib = xhi; ib < nbc; ++ib) tiles(no, ib);
          }
        };
        switch (nown_u) {
          case 0:
            for (int c = lane; c < nbc * 16; c += 64) lds_rev[wave * (kChunk * 16) + c] = R(0);
            break;
          case 1:
            run(std::integral_constant<int, 1>{});
            break;
          case 2:
            run(std::integral_constant<int, 2>{});
            break;
          case 3:
            run(std::integral_constant<int, 3>{});
            break;
          case 4:
            if constexpr (RB > 4)
              run(std::integral_constant<int, 4>{});
            else  // nown = RB, so no shared block
              for (int ib = 0; ib < nbc; ++ib) tiles(std::integral_constant<int, RB>{}, ib);
            break;
          default:  // nown = RB, so no shared block
            for (int ib = 0; ib < nbc; ++ib) tiles(std::integral_constant<int, RB>{}, ib);
            break;
        }
      }
      __syncthreads();
      // reverse sums over the group's waves, in wave order
      for (int c = tid; c < nbc * 16; c += blockDim.x) {
        const int t = c0 * 16 + c;
        if (t >= T) continue;
        R sum = R(0);
        for (int w = 0; w < W; ++w) sum += lds_rev[w * (kChunk * 16) + c];
        // the double layer's reverse kernel is d_a.(y - x) = -d_a.(x - y)
        rout[t] = need_r ? (OP == SBIE_OP_D ? -sum : sum) : R(0);
      }
    }
    if (!need_f) continue;
    // forward tile sum added under the exclusion
    if constexpr (ROWSUM) {
      float v[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) v[k] = tmp[k >> 2][k & 3];
      acc1 += row_group_sums(v, lane);
    } else {
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        if (rb >= nown_u + nx_u) break;
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[rb][e] += (double)tmp[rb][e];
      }
    }
  }
  // forward partials: each row summed over its 16 columns; the shared blocks'
  // partials then summed over the waves in wave order (LDS reused: every wave
  // has passed its last read of the staged operands at the barrier)
  double* lds_x = reinterpret_cast<double*>(smem_raw);  // [W][nx*16]
  if (nx_u > 0) __syncthreads();
  if constexpr (ROWSUM) {
    const int rb = li >> 2, row = MM::row(lg, li & 3);
    if (rb < nown) {
      const int r = (rb0 + rb) * 16 + row;
      if (r < T) {
        double* f = fwd + (size_t)split * N + (int64_t)a * T + r;
        *f = (first ? 0.0 : *f) + acc1 * kInv4PiD;
      }
    } else if (rb < nrb) {
      lds_x[wave * (nx * 16) + (rb - nown) * 16 + row] = acc1;
    }
  } else {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        double v = acc[rb][e];
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) v += __shfl_xor(v, off, 64);
        const int row = MM::row(lg, e);
        if (rb < nown) {
          const int r = (rb0 + rb) * 16 + row;
          if (li == 0 && r < T) {
            double* f = fwd + (size_t)split * N + (int64_t)a * T + r;
            *f = (first ? 0.0 : *f) + v * kInv4PiD;
          }
        } else if (rb < nrb && li == 0) {
          lds_x[wave * (nx * 16) + (rb - nown) * 16 + row] = v;
        }
      }
  }
  if (nx_u > 0) {
    __syncthreads();
    for (int c = tid; c < nx * 16; c += blockDim.x) {
      const int r = xb0 * 16 + c;
      double v = 0.0;
      for (int w = 0; w < W; ++w) v += lds_x[w * (nx * 16) + c];
      if (r < T) {
        double* f = fwd + (size_t)split * N + (int64_t)a * T + r;
        *f = (first ? 0.0 : *f) + v * kInv4PiD;
      }
    }
  }
}

template <typename R, int OP>
__global__ __launch_bounds__(64 * PairShape<R>::WMAX) void k_far_pairs(const R* __restrict__ geo, const R* __restrict__ app,
                                                   const Particle* __restrict__ part, const double* __restrict__ x,
                                                   const double* __restrict__ y, const double* __restrict__ z,
                                                   const uint32_t* __restrict__ excl, int words, int M, int T,
                                                   int T16, int64_t N, int nsplit, int RG, int kbase, int kend,
                                                   int first, double* __restrict__ fwd, R* __restrict__ rev) {
  far_pairs_body<R, OP>(geo, app, part, x, y, z, excl, words, M, T, T16, N, nsplit, RG, kbase, kend, first, fwd,
                        rev, xcd_work_index());
}

// Several geometries' pair-kernel work in one launch (served sessions of one
// order and operator): job j owns the work indices [wg_begin_j, wg_begin_{j+1})
// and runs exactly the workgroups its own launch would, so its sums are
// bitwise those of its own launch.  Every job's far field fits one launch
// (all partner offsets, first = 1).
template <typename R, int OP>
__global__ __launch_bounds__(64 * PairShape<R>::WMAX) void k_far_pairs_batch(const FarJob* __restrict__ jobs,
                                                                            int njobs) {
  const int wid = xcd_work_index();
  int lo = 0, hi = njobs - 1;  // the last job starting at or before wid
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (jobs[mid].wg_begin <= wid) lo = mid;
    else hi = mid - 1;
  }
  const FarJob& J = jobs[lo];
  far_pairs_body<R, OP>(static_cast<const R*>(J.geo), static_cast<const R*>(J.app), J.part, J.x, J.y, J.z, J.excl,
                        J.words, J.M, J.T, J.T16, J.N, J.nsplit, J.RG, 0, J.kend, 1, J.fwd, static_cast<R*>(J.rev),
                        wid - J.wg_begin);
}

// After a launch over the partner offsets [kbase, kend): each target's reverse
// slots of the launch (the slots with a handler: k < H, and k = H for even M
// when the target is in the upper half), slot then row group, added in FP64 to
// its running total (first launch: from zero).  Over the launches the totals
// take the slots in ascending order, as one pass over all of them would.
template <typename R>
__global__ void k_far_fold(const R* __restrict__ rev, int M, int T, int RG, int kbase, int kend, int first,
                           int64_t N, double* __restrict__ racc) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  const int b = (int)(g / T), t = (int)(g - (int64_t)b * T);
  const int H = (M - 1) / 2;
  const int slots = H + (((M & 1) == 0 && b >= M / 2) ? 1 : 0);
  const int KS = kend - kbase;
  const int hi = kend < slots ? kend : slots;
  double r = first ? 0.0 : racc[g];
  for (int k = kbase; k < hi; ++k)
    for (int rg = 0; rg < RG; ++rg) r += (double)rev[(((size_t)b * KS + (k - kbase)) * RG + rg) * T + t];
  racc[g] = r;
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
// lane order and -W mu nu.o;
// S' per block (-2 q o, q) and (nu, -nu.o) in lane order, q = W sigma; D' per
// block (nu, -nu.o) in lane order and q = W mu.
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
  } else if (OP == SBIE_OP_DP) {
    double ox = 0.0, oy = 0.0, oz = 0.0, n0 = 0.0, n1 = 0.0, n2 = 0.0;
    if (q < T) {
      ox = x[g] - part[s].c[0];
      oy = y[g] - part[s].c[1];
      oz = z[g] - part[s].c[2];
      n0 = nx[g];
      n1 = ny[g];
      n2 = nz[g];
    }
    R* b = app + (t / 16) * 80 + (t % 16);
    b[0] = (R)n0;
    b[16] = (R)n1;
    b[32] = (R)n2;
    b[48] = (R)(-fma(n2, oz, fma(n1, oy, n0 * ox)));
    b[64] = (R)wq;
  } else if (OP == SBIE_OP_SP) {
    double ox = 0.0, oy = 0.0, oz = 0.0, n0 = 0.0, n1 = 0.0, n2 = 0.0;
    if (q < T) {
      ox = x[g] - part[s].c[0];
      oy = y[g] - part[s].c[1];
      oz = z[g] - part[s].c[2];
      n0 = nx[g];
      n1 = ny[g];
      n2 = nz[g];
    }
    R* b = app + (t / 16) * 128 + (t % 16);
    b[0] = (R)(-2.0 * wq * ox);
    b[16] = (R)(-2.0 * wq * oy);
    b[32] = (R)(-2.0 * wq * oz);
    b[48] = (R)wq;
    b[64] = (R)n0;
    b[80] = (R)n1;
    b[96] = (R)n2;
    b[112] = (R)(-fma(n2, oz, fma(n1, oy, n0 * ox)));
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

// Workgroup size and dynamic LDS of the pair kernel for g's order and op.
template <typename R>
void pair_launch_shape(const sbie_geom* g, int op, dim3* wg, size_t* lds) {
  using PS = PairShape<R>;
  const int nb = g->T16 / 16;
  const int blocks = nb < PS::GB ? nb : PS::GB;
  *wg = dim3((unsigned)(64 * (blocks < PS::WMAX ? blocks : PS::WMAX)));
  int ngeo = 0, napp = 0;
  switch (op) {
    case SBIE_OP_S: ngeo = FarLayout<R, SBIE_OP_S>::GEO; napp = FarLayout<R, SBIE_OP_S>::APP; break;
    case SBIE_OP_D: ngeo = FarLayout<R, SBIE_OP_D>::GEO; napp = FarLayout<R, SBIE_OP_D>::APP; break;
    case SBIE_OP_SP: ngeo = FarLayout<R, SBIE_OP_SP>::GEO; napp = FarLayout<R, SBIE_OP_SP>::APP; break;
    default: ngeo = FarLayout<R, SBIE_OP_DP>::GEO; napp = FarLayout<R, SBIE_OP_DP>::APP; break;
  }
  *lds = (size_t)kChunk * (ngeo + napp + 16 * (wg->x / 64)) * sizeof(R);
  if (op == SBIE_OP_D && FarLayout<R, SBIE_OP_D>::X3)  // the double layer's row stash
    *lds += (size_t)(wg->x / 64) * PS::RBMAX * 64 * (sizeof(double) + sizeof(R));
}

template <typename R>
sbie_status launch_strengths(sbie_geom* g, int op, const double* d_dens, R* app, hipStream_t s) {
  const int64_t n16 = (int64_t)g->M * g->T16;
  const dim3 pre(cdiv(n16, 256)), blk(256);
  if (op == SBIE_OP_S)
    hipLaunchKernelGGL((k_far_strengths<R, SBIE_OP_S>), pre, blk, 0, s, g->d_part, d_dens, g->d_x, g->d_y, g->d_z,
                       g->d_nx, g->d_ny, g->d_nz, g->d_w, g->M, g->T, g->T16, app);
  else
    hipLaunchKernelGGL((k_far_strengths<R, SBIE_OP_D>), pre, blk, 0, s, g->d_part, d_dens, g->d_x, g->d_y, g->d_z,
                       g->d_nx, g->d_ny, g->d_nz, g->d_w, g->M, g->T, g->T16, app);
  SBIE_HIP(hipGetLastError());
  return SBIE_OK;
}

template <typename R>
sbie_status launch_far(sbie_geom* g, int op, const double* d_dens, const R* geo, R* app, hipStream_t s,
                       hipEvent_t ev_begin, hipEvent_t ev_end) {
  const int64_t n16 = (int64_t)g->M * g->T16;
  const dim3 pre(cdiv(n16, 256)), blk(256);
  if (op == SBIE_OP_S)
    hipLaunchKernelGGL((k_far_strengths<R, SBIE_OP_S>), pre, blk, 0, s, g->d_part, d_dens, g->d_x, g->d_y, g->d_z,
                       g->d_nx, g->d_ny, g->d_nz, g->d_w, g->M, g->T, g->T16, app);
  else if (op == SBIE_OP_SP)
    hipLaunchKernelGGL((k_far_strengths<R, SBIE_OP_SP>), pre, blk, 0, s, g->d_part, d_dens, g->d_x, g->d_y, g->d_z,
                       g->d_nx, g->d_ny, g->d_nz, g->d_w, g->M, g->T, g->T16, app);
  else if (op == SBIE_OP_DP)
    hipLaunchKernelGGL((k_far_strengths<R, SBIE_OP_DP>), pre, blk, 0, s, g->d_part, d_dens, g->d_x, g->d_y, g->d_z,
                       g->d_nx, g->d_ny, g->d_nz, g->d_w, g->M, g->T, g->T16, app);
  else
    hipLaunchKernelGGL((k_far_strengths<R, SBIE_OP_D>), pre, blk, 0, s, g->d_part, d_dens, g->d_x, g->d_y, g->d_z,
                       g->d_nx, g->d_ny, g->d_nz, g->d_w, g->M, g->T, g->T16, app);
  SBIE_HIP(hipGetLastError());
  if (ev_begin) SBIE_HIP(hipEventRecord(ev_begin, s));
  using PS = PairShape<R>;
  const int RG = far_row_groups(g, sizeof(R) == 8);
  const int nb = g->T16 / 16;
  const int blocks = nb < PS::GB ? nb : PS::GB;
  const dim3 grid((unsigned)((int64_t)g->M * RG * far_launch_splits(g, RG))),
      wg((unsigned)(64 * (blocks < PS::WMAX ? blocks : PS::WMAX)));
  int ngeo = 0, napp = 0;
  switch (op) {
    case SBIE_OP_S: ngeo = FarLayout<R, SBIE_OP_S>::GEO; napp = FarLayout<R, SBIE_OP_S>::APP; break;
    case SBIE_OP_D: ngeo = FarLayout<R, SBIE_OP_D>::GEO; napp = FarLayout<R, SBIE_OP_D>::APP; break;
    case SBIE_OP_SP: ngeo = FarLayout<R, SBIE_OP_SP>::GEO; napp = FarLayout<R, SBIE_OP_SP>::APP; break;
    default: ngeo = FarLayout<R, SBIE_OP_DP>::GEO; napp = FarLayout<R, SBIE_OP_DP>::APP; break;
  }
  size_t lds = (size_t)kChunk * (ngeo + napp + 16 * (wg.x / 64)) * sizeof(R);
  if (op == SBIE_OP_D && FarLayout<R, SBIE_OP_D>::X3)  // the double layer's row stash
    lds += (size_t)(wg.x / 64) * PS::RBMAX * 64 * (sizeof(double) + sizeof(R));
  R* rev = reinterpret_cast<R*>(g->d_rev);
  const int KS = g->rev_slots, PMAX = (g->M - 1) / 2 + ((g->M & 1) == 0 ? 1 : 0);
  const int nsplit = far_launch_splits(g, RG);
  const dim3 fold((unsigned)cdiv(g->N, 256));
  // (at least one launch: with no partners it writes the zero forward slices
  // and reverse totals that the assembly reads)
  for (int kbase = 0; kbase == 0 || kbase < PMAX; kbase += KS) {
    const int kend = kbase + KS, first = kbase == 0 ? 1 : 0;
    if (op == SBIE_OP_S)
      hipLaunchKernelGGL((k_far_pairs<R, SBIE_OP_S>), grid, wg, lds, s, geo, app, g->d_part, g->d_x, g->d_y,
                         g->d_z, g->d_excl, g->excl_words, g->M, g->T, g->T16, g->N, nsplit, RG, kbase, kend, first,
                         g->d_partial, rev);
    else if (op == SBIE_OP_SP)
      hipLaunchKernelGGL((k_far_pairs<R, SBIE_OP_SP>), grid, wg, lds, s, geo, app, g->d_part, g->d_x, g->d_y,
                         g->d_z, g->d_excl, g->excl_words, g->M, g->T, g->T16, g->N, nsplit, RG, kbase, kend, first,
                         g->d_partial, rev);
    else if (op == SBIE_OP_DP)
      hipLaunchKernelGGL((k_far_pairs<R, SBIE_OP_DP>), grid, wg, lds, s, geo, app, g->d_part, g->d_x, g->d_y,
                         g->d_z, g->d_excl, g->excl_words, g->M, g->T, g->T16, g->N, nsplit, RG, kbase, kend, first,
                         g->d_partial, rev);
    else
      hipLaunchKernelGGL((k_far_pairs<R, SBIE_OP_D>), grid, wg, lds, s, geo, app, g->d_part, g->d_x, g->d_y,
                         g->d_z, g->d_excl, g->excl_words, g->M, g->T, g->T16, g->N, nsplit, RG, kbase, kend, first,
                         g->d_partial, rev);
    SBIE_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_far_fold<R>, fold, dim3(256), 0, s, rev, g->M, g->T, RG, kbase, kend, first, g->N,
                       g->d_racc);
    SBIE_HIP(hipGetLastError());
  }
  if (ev_end) SBIE_HIP(hipEventRecord(ev_end, s));
  return SBIE_OK;
}

}  // namespace

int far_row_groups(const sbie_geom* g, bool fp64) {
  const int T16 = 16 * ((g->T + 15) / 16);
  const int GB = fp64 ? PairShape<double>::GB : PairShape<float>::GB;
  return (T16 / 16 + GB - 1) / GB;
}

int far_launch_splits(const sbie_geom* g, int RG) {
  const int want = (int)((512 + (int64_t)g->M * RG - 1) / ((int64_t)g->M * RG));
  const int by_work = g->rev_slots / 4 > 1 ? g->rev_slots / 4 : 1;
  int n = want < g->nsplit ? want : g->nsplit;
  n = n < by_work ? n : by_work;
  return n > 1 ? n : 1;
}

int far_rev_slots(int M, int T) {
  const int nb = (T + 15) / 16;
  const int RG = (nb + PairShape<double>::GB - 1) / PairShape<double>::GB;  // the FP64 sizing covers FP32
  const int pmax = (M - 1) / 2 + ((M & 1) == 0 ? 1 : 0);
  if (pmax < 1) return 1;  // one particle: no partners, one launch writes the zero sums
  const size_t per_slot = (size_t)M * RG * T * sizeof(double);
  int k = (int)(kRevBudget / (per_slot > 0 ? per_slot : 1));
  if (k > pmax) k = pmax;
  if (k < 1) k = 1;
  // as many launches as the budget needs, their partner ranges balanced
  const int launches = (pmax + k - 1) / k;
  return (pmax + launches - 1) / launches;
}

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

bool far_batch_fits(const sbie_geom* g) {
  const int pmax = (g->M - 1) / 2 + ((g->M & 1) == 0 ? 1 : 0);
  return g->T >= 32 && pmax <= g->rev_slots;
}

sbie_status far_strengths(sbie_geom* g, int op, int prec, const double* d_dens, hipStream_t s) {
  if (prec == SBIE_MIXED) return launch_strengths<float>(g, op, d_dens, g->d_fstr32, s);
  return launch_strengths<double>(g, op, d_dens, g->d_fstr64, s);
}

int far_batch_job(const sbie_geom* g, int op, int prec, int wg_begin, FarJob* job) {
  const bool mixed = prec == SBIE_MIXED;
  const int RG = far_row_groups(g, !mixed);
  const int nsplit = far_launch_splits(g, RG);
  job->geo = mixed ? (const void*)g->d_srec32 : (const void*)g->d_srec64;
  job->app = mixed ? (const void*)g->d_fstr32 : (const void*)g->d_fstr64;
  job->part = g->d_part;
  job->x = g->d_x;
  job->y = g->d_y;
  job->z = g->d_z;
  job->excl = g->d_excl;
  job->words = g->excl_words;
  job->M = g->M;
  job->T = g->T;
  job->T16 = g->T16;
  job->N = g->N;
  job->nsplit = nsplit;
  job->RG = RG;
  job->kend = g->rev_slots;
  job->wg_begin = wg_begin;
  job->fwd = g->d_partial;
  job->rev = g->d_rev;
  (void)op;
  return g->M * RG * nsplit;
}

sbie_status far_batch_launch(sbie_geom* const* gs, int n, const FarJob* d_jobs, int total_wg, int op, int prec,
                             hipStream_t s) {
  if (n < 1) return SBIE_OK;
  const bool mixed = prec == SBIE_MIXED;
  dim3 wg;
  size_t lds = 0;
  if (mixed) pair_launch_shape<float>(gs[0], op, &wg, &lds);
  else pair_launch_shape<double>(gs[0], op, &wg, &lds);
  const dim3 grid((unsigned)total_wg);
  if (mixed && op == SBIE_OP_S)
    hipLaunchKernelGGL((k_far_pairs_batch<float, SBIE_OP_S>), grid, wg, lds, s, d_jobs, n);
  else if (mixed)
    hipLaunchKernelGGL((k_far_pairs_batch<float, SBIE_OP_D>), grid, wg, lds, s, d_jobs, n);
  else if (op == SBIE_OP_S)
    hipLaunchKernelGGL((k_far_pairs_batch<double, SBIE_OP_S>), grid, wg, lds, s, d_jobs, n);
  else
    hipLaunchKernelGGL((k_far_pairs_batch<double, SBIE_OP_D>), grid, wg, lds, s, d_jobs, n);
  SBIE_HIP(hipGetLastError());
  // each geometry's reverse sums into its totals, as after its own single launch
  for (int k = 0; k < n; ++k) {
    sbie_geom* g = gs[k];
    const int RG = far_row_groups(g, !mixed);
    const dim3 fold((unsigned)cdiv(g->N, 256));
    if (mixed)
      hipLaunchKernelGGL(k_far_fold<float>, fold, dim3(256), 0, s, reinterpret_cast<const float*>(g->d_rev), g->M,
                         g->T, RG, 0, g->rev_slots, 1, g->N, g->d_racc);
    else
      hipLaunchKernelGGL(k_far_fold<double>, fold, dim3(256), 0, s, (const double*)g->d_rev, g->M, g->T, RG, 0,
                         g->rev_slots, 1, g->N, g->d_racc);
    SBIE_HIP(hipGetLastError());
  }
  return SBIE_OK;
}

}  // namespace sbie
