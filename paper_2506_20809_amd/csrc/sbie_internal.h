// Internal declarations of the HIP library behind include/sbie.h.
#pragma once

#include <type_traits>

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/sbie.h"

namespace sbie {

constexpr int kMaxP = 32;
constexpr int kRcpN = 16384;  // reciprocal table length (near-field recurrences)
constexpr size_t kRevBudget = size_t(128) << 20;  // reverse sums of one pair-kernel launch, bytes
constexpr size_t kStokesRevBudget = size_t(128) << 20;  // the same for the Stokes pair kernel
constexpr double kPi = 3.14159265358979323846264338327950288;

// Per-particle parameters on the device (Section 2.1, Table 1).
struct Particle {
  double c[3];   // centre
  double R[9];   // body -> lab rotation, row-major
  double a;      // focal parameter
  double u0;     // coordinate of the surface
  double A, C;   // semi-axes
  double diam;   // twice the largest semi-axis
  double w0;     // u0^2 - 1 (prolate) or u0^2 + 1 (oblate)
  int oblate;
  int pad;
};

// The near sources of each target particle are split into kNearSplit
// consecutive ranges, one wave each, whose partial sums the assembly adds in
// range order (balances particles with many and few neighbours).
constexpr int kNearSplit = 4;
// The Stokes near kernels (four or thirteen expansions per source, many
// registers, few waves otherwise) split each list eight ways.
constexpr int kStokesNearSplit = 8;

// One geometry's share of a batched far-field launch (served sessions of one
// order, operator and precision): the arguments of its own pair-kernel launch
// over all partner offsets, and its first work index in the batch.
struct FarJob {
  const void* geo;
  const void* app;
  const Particle* part;
  const double *x, *y, *z;
  const uint32_t* excl;
  int words, M, T, T16;
  int64_t N;
  int nsplit, RG, kend, wg_begin;
  double* fwd;
  void* rev;
};

// One geometry's share of a batched near-field launch (Laplace S and D).
struct NearJob {
  const Particle* part;
  const double *x, *y, *z;
  const int32_t *near_ptr, *near_src;
  const double *E, *lam, *ab, *rcp;
  int p, T, chunks, wg_begin;
  int64_t N;
  unsigned* status;
  double* unear;
};

// Order dispatch of the near-field kernels: the orders 8, 12, 16 and 32 get
// kernels of their exact order (f(PMAX, true)), whose degree loops then carry
// no runtime bounds; other orders the next larger of 8, 16, 32 (f(PMAX, false)).
template <typename F>
inline void dispatch_order(int p, F&& f) {
  using std::integral_constant;
  if (p == 8) f(integral_constant<int, 8>{}, std::true_type{});
  else if (p == 12) f(integral_constant<int, 12>{}, std::true_type{});
  else if (p == 16) f(integral_constant<int, 16>{}, std::true_type{});
  else if (p == 32) f(integral_constant<int, 32>{}, std::true_type{});
  else if (p < 8) f(integral_constant<int, 8>{}, std::false_type{});
  else if (p < 16) f(integral_constant<int, 16>{}, std::false_type{});
  else f(integral_constant<int, 32>{}, std::false_type{});
}

// Status word written by kernels (bit flags).
enum : unsigned { kStatNumeric = 1u, kStatOverlap = 2u, kStatExterior = 4u };

// The largest number of near-field backward-recurrence steps past degree p+1,
// and each geometry's default cap (sbie_geom_set_depth_cap lowers it).
constexpr int kMaxNearDepth = 100000;

struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
};

// One set of eight events per timed apply (per right-hand side), reused across
// accumulation windows: 0 start, 1 after prep, 2 after transforms and self,
// 3/4 around the far-field kernel, 5 end (all on the apply's stream), 6/7
// around the near field (on the side stream).
struct Timing {
  std::vector<std::vector<hipEvent_t>> sets;
  size_t used = 0;
};

// Tree far field (tree.hip): host plan and device state.
struct TreePlan {
  int nc = 0, order = 0;
  double theta = 0.0;
  std::vector<double> box;                // [nc][6] lo, hi of every cluster
  std::vector<int32_t> first, count;      // [nc] range of the permutation
  std::vector<int32_t> perm;              // [M] particles in cluster order
  std::vector<int64_t> pptr, dptr;        // [M+1] per target particle
  std::vector<int32_t> pidx, didx;        // clusters through proxies; source particles summed directly
};

// Work buffers of the multi-density S and D apply (up to four densities at
// once), allocated on its first use and held with the geometry.
struct MultiWork {
  char* blk = nullptr;
  size_t bytes = 0;
  double* E = nullptr;        // [4][M][K] exterior coefficients per density
  double* uself = nullptr;    // [4][N]
  double* unear = nullptr;    // [4][kNearSplit][N]
  double* partial = nullptr;  // [4][nsplit][N] forward far partials
  double* racc = nullptr;     // [4][N] reverse totals
  double* rec = nullptr;      // per-block source records (multi_rec_values doubles)
  double* rev = nullptr;      // reverse sums of one launch (rev_bytes)
  uint64_t rev_bytes = 0;
  double* io = nullptr;       // [2][4][N] staging of host densities and results
};

struct FarTree {
  double theta = 0.0;
  int nc = 0, order = 0, leaf = 0, nused = 0;  // nused: clusters taken through proxies by some target
  int64_t n_proxy = 0, n_direct = 0;     // (target, cluster) and (target, source particle) pairs
  int64_t proxy_evals = 0, direct_evals = 0, charge_evals = 0;  // node-level work per apply
  size_t bytes = 0;
  char* blk = nullptr;                   // one device block holding everything below
  bool blk_owned = true;                 // false: the block came from a TreeAlloc
  double* d_box = nullptr;               // [nused][6]
  int npiece = 0;                        // workgroups of the proxy charges (pieces of used clusters)
  int32_t *d_piece = nullptr;            // [npiece][3] cluster slot, first, count (in the permutation)
  int32_t *d_cptr = nullptr;             // [nused+1] pieces by cluster slot
  int32_t *d_perm = nullptr;
  int64_t *d_pptr = nullptr, *d_dptr = nullptr;
  int32_t *d_pidx = nullptr, *d_didx = nullptr;  // pidx holds used-cluster slots
  double* d_q = nullptr;                 // [nused][n3p][4] proxy points and charges of the current apply
  double* d_qpart = nullptr;             // [npiece][(order+1)^3][1 or 3] their partial sums (3: dipole moments)
  // mixed path: the single layer's three-piece matrix-core records (64 lanes
  // x 4 words per 16 sources; n3b = ceil((order+1)^3 / 16), T16 = ceil(T / 16))
  uint32_t* d_prec = nullptr;            // [nused][n3b][64][4] proxies - box centre
  uint32_t* d_srec = nullptr;            // [M][T16][64][4] nodes - particle centre
  uint32_t* d_pdrec = nullptr;           // [nused][n3b][64][4] double layer dipole proxies of the current apply
  float* d_q32 = nullptr;                // [nused][16 n3b] single layer proxy charges of the current apply
  float* d_sq32 = nullptr;               // [M][16 T16] single layer node strengths of the current apply
  float* d_src32 = nullptr;              // [N][8] double layer's direct sources: node - particle centre, W mu nu
};

}  // namespace sbie

struct sbie_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::atomic<int> live_geoms{0};  // geometries created on this context and not yet destroyed
  bool closing = false;   // sbie_ctx_destroy called while geometries were live
};

struct sbie_geom {
  sbie_ctx* ctx = nullptr;
  int M = 0, p = 0, T = 0, K = 0, Kh = 0, Nphi = 0;
  int64_t N = 0;
  double eta = 1.0;
  int64_t n_near = 0;
  int64_t far_pairs = 0;

  // host copies
  std::vector<sbie::Particle> h_part;
  std::vector<int32_t> h_near_ptr, h_near_src;  // CSR by target particle

  // device, geometry
  sbie::Particle* d_part = nullptr;
  double *d_x = nullptr, *d_y = nullptr, *d_z = nullptr;     // nodes (SoA)
  double *d_nx = nullptr, *d_ny = nullptr, *d_nz = nullptr;  // unit outward normals
  double* d_w = nullptr;                                     // quadrature weights
  float* d_off32 = nullptr;       // [N][4] node - centre (float), for the mixed far field
  double* d_gl = nullptr;         // [2(p+1)] GL nodes, weights
  double* d_An = nullptr;         // [T][K] analysis matrix (weights folded in)
  double* d_Sy = nullptr;         // [K][T] synthesis matrix
  float* d_An32 = nullptr;        // FP32 copies for the mixed path
  float* d_Sy32 = nullptr;
  double* d_Sv = nullptr;         // [K][T] dY_l/dv at the nodes
  double* d_Sp = nullptr;         // [K][T] dY_l/dphi at the nodes
  float* d_Sv32 = nullptr;
  float* d_Sp32 = nullptr;
  double* d_dlr = nullptr;        // [M][Kh] d/du (Q(u)/Q(u0)) at u0
  double* d_cd = nullptr;         // [Kh] sqrt((2n+1)(n+m+1)(n-m+1)/(2n+3)), Ferrers derivative
  // Stokes single layer work buffers (allocated on the first Stokes apply)
  double* d_stk_f = nullptr;      // [4M][T] transform inputs (3 components and rho)
  double* d_stk_c = nullptr;      // [4M][K] coefficients
  double* d_stk_E = nullptr;      // [2][4M][K] exterior coefficients and their u-derivative form
  double* d_stk_U = nullptr;      // [4][4M][T] value, d/du, d/dv, d/dphi at the nodes
  double* d_stk_src = nullptr;    // [N][8] far-field records / [nsplit][3][N] partials follow
  double* d_stk_part = nullptr;   // [nsplit][4][N] (velocity and pressure)
  double* d_stk_self = nullptr;   // [4][N]
  double* d_stk_near = nullptr;   // [kStokesNearSplit][4][N] near partials per source-list range
  double* d_stk_io = nullptr;     // [7][N] staging of host densities and velocities
  double* d_stk_prec = nullptr;   // [M][T16/16][stokes_record_doubles] source blocks of the pair kernel
  double* d_stk_rev = nullptr;    // reverse sums of one pair-kernel launch (stk_rev_bytes)
  double* d_stk_racc = nullptr;   // [4][N] running reverse totals
  uint64_t stk_rev_bytes = 0;
  // Stokes double layer (stokes_dl.hip), in its own block carved on first use
  char* sdl_blk = nullptr;
  double* d_sdl_f = nullptr;      // [13M][T] transform inputs of the 13 expansion sets
  double* d_sdl_c = nullptr;      // [13M][K] coefficients
  double* d_sdl_E = nullptr;      // [2][13M][K] exterior coefficients and their d/du form
  double* d_sdl_U = nullptr;      // [3][13M][T] d/du (exterior), d/dv, d/dphi at the nodes
  double* d_sdl_src = nullptr;    // [N][8] far records (node - centre, W mu, nu_x, nu_y)
  double* d_sdl_part = nullptr;   // [nsplit][3][N]
  double* d_sdl_self = nullptr;   // [3][N]
  double* d_sdl_near = nullptr;   // [kStokesNearSplit][3][N] near partials per source-list range
  double* d_sdl_io = nullptr;     // [6][N] host staging
  double* d_sdl_prec = nullptr;   // [M][T16/16][stokes_record_doubles] source blocks of the stresslet pair kernel
  double* d_sdl_rev = nullptr;    // reverse sums of one stresslet pair-kernel launch (sdl_rev_bytes)
  double* d_sdl_racc = nullptr;   // [3][N] running reverse totals
  uint64_t sdl_rev_bytes = 0;
  double* d_wS = nullptr;         // [M][p+1] sqrt(u0^2 -+ v_j^2)
  double* d_lam = nullptr;        // [M][Kh][4]: D principal value, D exterior, S, 1/Q_n^m(z0)
  double* d_ab = nullptr;         // [Kh][2] normalised Ferrers recurrence coefficients
  int32_t *d_near_ptr = nullptr, *d_near_src = nullptr;
  uint32_t* d_excl = nullptr;     // [M][ceil(M/32)] bit i of row j: source i excluded for target j
  int excl_words = 0;
  unsigned* d_status = nullptr;   // [0] sticky status bits, [1] near-field recurrence step cap

  // device, work
  double* d_f = nullptr;          // [M][T] transform input
  double* d_coef = nullptr;       // [M][K]
  double* d_cself = nullptr;      // [M][K]
  double* d_E = nullptr;          // [M][K] exterior coefficients
  double* d_uself = nullptr;      // [N]
  double* d_unear = nullptr;      // [kNearSplit][N] near-field partials (source-list quarters)
  double* d_src = nullptr;        // [N][8] far-field source records
  double* d_partial = nullptr;    // [nsplit][N]
  double* d_dens = nullptr;       // [N] staging for host densities
  double* d_out = nullptr;        // [N] staging for host potentials
  // matrix-core far field: sources padded per particle to T16 = 16*ceil(T/16)
  int T16 = 0;
  // per 16-source block b of particle s, 80 values at (s*nb + b)*80: the MFMA B
  // operand in lane order ([k][j] at 16k+j; (-2 o_x, -2 o_y, -2 o_z, 1) for
  // source j, o = node - centre) followed by |o_j|^2, j = 0..15
  float* d_srec32 = nullptr;      // [M*T16*5]
  double* d_srec64 = nullptr;
  // per-apply strengths per block: S 16 values W sigma_j at (s*nb + b)*16;
  // D 80 values at (s*nb + b)*80: (W mu nu_j, 0) in lane order, then -W mu nu_j.o_j
  // (the mixed S and D kernels split them into the three-piece form as they
  // stage them in LDS)
  float* d_fstr32 = nullptr;      // [M*T16*8] per-apply far strengths (S 1, D 5, S' 8 per source)
  double* d_fstr64 = nullptr;     // [M*T16*8]
  double* d_rcp = nullptr;        // [kRcpN] reciprocals 1/k for the near-field recurrences
  // pair-symmetric far field, run as launches over chunks of rev_slots partner
  // offsets: each launch's reverse sums [M][rev_slots][RG][T] (FP64, or FP32 in
  // the first half for the mixed path), RG target-row groups, folded after the
  // launch into the running FP64 reverse sums racc [N]
  double* d_rev = nullptr;
  double* d_racc = nullptr;
  int rev_slots = 0;
  double* d_eta = nullptr;        // [M] completion scalings of the last completed apply / solve
  double* d_qint = nullptr;       // [M] eta_i * integral of the density over particle i
  int nsplit = 8;
  uint64_t footprint = 0;
  // device memory: one block carved into every buffer above (owned, or lent by
  // a server arena), and a second owned block for the Stokes buffers when the
  // first has no room reserved for them
  char* blk = nullptr;
  size_t blk_bytes = 0, blk_used = 0;
  bool blk_owned = false;
  char* stk_blk = nullptr;
  bool stokes_ready = false;
  uint8_t* d_near_scratch = nullptr;  // [M][M] near flags of the classification

  sbie::Timing timing;
  sbie::FarTree* tree = nullptr;  // tree far field, built by sbie_geom_far_tree
  sbie::MultiWork* multi = nullptr;  // multi-density apply buffers
  // the near field runs on a side stream, concurrently with the far field
  // (plain geometries; served sessions keep one stream per lane)
  bool fork_near = true;
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
};

namespace sbie {

void set_error(const std::string& msg);
sbie_status device_error(hipError_t e, const char* what);

// Tree far field (tree.hip).  plan_tree is host code: excl [M][words], bit s
// of row t set iff source particle s is excluded for target particle t.
sbie_status plan_tree(int M, int T, const double* centers, const double* radii, const uint32_t* excl, int words,
                      double theta, int order, int leaf, TreePlan* out);
// Device memory for a tree from the caller (served sessions carve it from
// their server's arena): fn returns a block of the given size, or nullptr when
// none is free; the tree then does not free it.
struct TreeAlloc {
  char* (*fn)(void* ctx, size_t bytes) = nullptr;
  void* ctx = nullptr;
};
sbie_status build_tree(sbie_geom* g, double theta, int order, int leaf, const TreeAlloc* alloc = nullptr);
void free_tree(sbie_geom* g);
sbie_status far_tree(sbie_geom* g, int op, bool mixed, hipStream_t s);
sbie_status far_tree_normal(sbie_geom* g, int op, const double* d_dens, hipStream_t s);
sbie_status far_tree_stokes(sbie_geom* g, int C, const double* d_dens, hipStream_t s);

// Stokes pair kernel (far_stokes.hip): row groups of a particle's 16-row
// blocks, partner slots per launch within cap_bytes of reverse sums, forward
// splits (at most the geometry's nsplit), the reverse buffer's size, and the
// far field of C = 3 (velocity) or 4 (with the pressure) components into
// d_stk_part's first stokes_pair_splits slices and d_stk_racc.
int stokes_row_groups(int T, bool fp64);
int stokes_rev_slots(int M, int T, int C, int bytes_per_value, uint64_t cap_bytes);
int stokes_pair_splits(const sbie_geom* g, int RG);
uint64_t stokes_rev_bytes(int M, int T);
// doubles per 16-source block of the Stokeslet (or stresslet) pair kernel's
// source records (FP64 values; the mixed path's FP32 values use half)
size_t stokes_record_doubles(bool sdl);
sbie_status far_stokes_pairs(sbie_geom* g, int C, bool mixed, const double* d_dens, hipStream_t s);
// The Stokes double layer's far field (the stresslet) through the same pair
// kernel: forward sums into d_sdl_part's first stokes_pair_splits slices,
// reverse totals into d_sdl_racc (to be scaled by 3/(4 pi)).
sbie_status far_sdl_pairs(sbie_geom* g, bool mixed, const double* d_dens, hipStream_t s);

// Multi-density S and D (far_multi.hip, apply.hip): the pair kernel's row
// groups, slots, splits and buffer sizes for up to four densities, its far
// field of nr = 2..4 densities d_dens [nr][N] into the work's partials and
// totals, the work's allocation, and the whole apply of nr densities
// (d_dens [nr][N] -> d_out [nr][N], device pointers; T >= 32).
int multi_row_groups(int T, bool fp64, int op);
int multi_waves(int T, bool fp64, int op);
int multi_rev_slots(int M, int T, int NR, int op, int bytes_per_value, uint64_t cap_bytes);
int multi_splits(const sbie_geom* g, int RG);
uint64_t multi_rev_bytes(int M, int T);
size_t multi_rec_values(int M, int T);
sbie_status far_multi(sbie_geom* g, int op, bool mixed, int nr, const double* d_dens, hipStream_t s);
sbie_status multi_buffers(sbie_geom* g);
sbie_status apply_laplace_multi(sbie_geom* g, int op, int prec, int nr, const double* d_dens, double* d_out,
                                hipStream_t s, uint32_t parts);

// Carves 256-byte aligned buffers out of one device block; with no block it
// only measures.
struct Carver {
  char* base = nullptr;
  size_t size = 0, used = 0;
  template <typename Tp>
  sbie_status take(Tp** p, size_t count) {
    used = (used + 255) & ~size_t(255);
    const size_t bytes = count * sizeof(Tp);
    if (base) {
      if (used + bytes > size) {
        set_error("device block too small for the geometry's buffers");
        return SBIE_E_NOMEM;
      }
      *p = reinterpret_cast<Tp*>(base + used);
    }
    used += bytes;
    return SBIE_OK;
  }
};

// Buffers of a geometry (setup tables, work buffers, classification scratch)
// and of the Stokes single layer, in carving order; measuring with an empty
// Carver gives the exact block size.
sbie_status carve_geometry(sbie_geom* g, Carver& c);
sbie_status carve_stokes(sbie_geom* g, Carver& c);
// Exact device bytes of a geometry of M particles at order p (with the Stokes
// buffers if stokes), as carved.
uint64_t plan_bytes(int M, int p, bool stokes);
// Allocates (or carves from the block's reserve) the Stokes buffers once.
sbie_status stokes_buffers(sbie_geom* g);

#define SBIE_HIP(call)                                              \
  do {                                                              \
    hipError_t _e = (call);                                         \
    if (_e != hipSuccess) return ::sbie::device_error(_e, #call);   \
  } while (0)

// geometry construction (capi.hip): host checks and per-particle parameters;
// a geometry on ctx's stream, in a lent device block (blk) or in one of its own
// (blk == nullptr); destruction
sbie_status check_particles(const double* centers, const double* quats, const double* A, const double* C,
                            int32_t M, int32_t p, double eta, std::vector<Particle>* out);
sbie_status make_geometry(sbie_ctx* ctx, std::vector<Particle>&& parts, int32_t p, double eta, char* blk,
                          size_t blk_bytes, bool fork_near, sbie_geom** out);
void destroy_geometry(sbie_geom* g);

// setup kernels (setup.hip)
sbie_status setup_geometry(sbie_geom* g, hipStream_t s);

// apply kernels (apply.hip)
sbie_status apply_laplace(sbie_geom* g, int op, int prec, const double* d_dens, double* d_out,
                          hipStream_t s, uint32_t parts, bool timed);
sbie_status transform_only(sbie_geom* g, int op, const double* d_dens, double* d_coef, hipStream_t s);
// C[rows x cols] = A[rows x kd] B[kd x cols] on the matrix cores (FP64, or FP32 with compensated tiles)
sbie_status gemm(bool mixed, const double* A, int lda, const double* B64, const float* B32, int ldb, double* C,
                 int ldc, int rows, int cols, int kd, hipStream_t s);

// timing event set of the next timed apply (apply.hip)
sbie_status next_timing_set(sbie_geom* g, hipEvent_t** ev);
// fork the side stream from s (after all work queued on s) and join it back
sbie_status fork_side(sbie_geom* g, hipStream_t s);
sbie_status join_side(sbie_geom* g, hipStream_t s);

// Stokes double layer (stokes_dl.hip); density and output [3][N]
sbie_status apply_stokes_dl(sbie_geom* g, int prec, const double* d_dens, double* d_out, hipStream_t s,
                            uint32_t parts, bool timed);
sbie_status stokes_dl_staging(sbie_geom* g, double** io);

// S' and D' (deriv.hip); apply_laplace dispatches these ops to it
sbie_status apply_normal(sbie_geom* g, int op, int prec, const double* d_dens, double* d_out, hipStream_t s,
                         uint32_t parts, bool timed);

// Transform input f and far records rec[g] = (node - centre, W dens, nu, 0)
// (float in d_src for SBIE_MIXED, else double) for op SBIE_OP_SP (modified
// basis, the records of S) or SBIE_OP_DP (those of D); then the forward
// transform with the self coefficients of S'/D' in d_cself and the exterior
// coefficients of S (lam_S c) resp. D (lam_D+ c) in d_E.
sbie_status normal_records(sbie_geom* g, int op, int prec, const double* d_dens, hipStream_t s);
sbie_status normal_expansions(sbie_geom* g, int op, int prec, hipStream_t s);

// completed double-layer operator and its GMRES solve (solve.hip)
double completion_eta(const Particle& P, int completion);

// Stokes single layer (stokes.hip); density [3][N], output [3][N], or [4][N]
// with the pressure
sbie_status apply_stokes(sbie_geom* g, int prec, const double* d_dens, double* d_out, hipStream_t s,
                         uint32_t parts, bool timed, bool pressure);
// device staging of 7N doubles (density [3][N], output up to [4][N]) for
// host-pointer Stokes applies (allocated once)
sbie_status stokes_staging(sbie_geom* g, double** io);

// matrix-core far field (far_mfma.hip); target-row groups per particle of
// the FP64 or the FP32 pair kernel
int far_row_groups(const sbie_geom* g, bool fp64);
// partner offsets per launch of the pair kernel: as many as keep one launch's
// reverse sums within kRevBudget bytes (at least 1, at most every partner)
int far_rev_slots(int M, int T);
// Splits of each pair-kernel launch's partner offsets over workgroups (and so
// the forward partial slices [0, splits) it writes): enough that a launch has
// about 512 workgroups (two per compute unit), at most the geometry's nsplit
// slices, and at least four partners per split.
int far_launch_splits(const sbie_geom* g, int RG);

// Batched far field of several geometries of one order, operator (S or D)
// and precision, each in one launch's worth of partner offsets: whether g
// qualifies, its per-apply source strengths, its job (returns its workgroup
// count), and the batched launch over the jobs (a device copy) with each
// geometry's fold of its reverse sums after it.
bool far_batch_fits(const sbie_geom* g);

// Job tables of batched applies: pinned host staging and device copies of up
// to cap jobs each.  The host side is rewritten by the next batch, so the
// stream must have consumed the previous copies (the served lanes synchronise
// after every batch).
struct BatchJobs {
  int cap = 0;
  FarJob *h_far = nullptr, *d_far = nullptr;
  NearJob *h_near = nullptr, *d_near = nullptr;
};

// S or D applied to n geometries of one order at once (served sessions): each
// geometry's transform, self part and strengths, then one near launch and one
// far launch over all of them, then each geometry's folds and assembly.  The
// kernels, data and order of every geometry's arithmetic are those of
// apply_laplace with all parts, so each result is bitwise the same.  Every
// geometry must satisfy far_batch_fits and share the order.
sbie_status far_strengths(sbie_geom* g, int op, int prec, const double* d_dens, hipStream_t s);
int far_batch_job(const sbie_geom* g, int op, int prec, int wg_begin, FarJob* job);
sbie_status far_batch_launch(sbie_geom* const* gs, int n, const FarJob* d_jobs, int total_wg, int op, int prec,
                             hipStream_t s);
sbie_status apply_laplace_batch(sbie_geom* const* gs, int n, int op, int prec, const double* const* d_dens,
                                double* const* d_out, BatchJobs* jobs, hipStream_t s);
sbie_status far_records(sbie_geom* g, hipStream_t s);
sbie_status far_mfma(sbie_geom* g, int op, int prec, const double* d_dens, hipStream_t s, hipEvent_t ev_begin,
                     hipEvent_t ev_end);

}  // namespace sbie
