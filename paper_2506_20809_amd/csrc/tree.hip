// Tree far field: a barycentric Lagrange treecode in the role of the FMM that
// Section 4.1 uses for the far field (the far-field step of Algorithm 1).
//
// Source particles are clustered by recursive bisection of their centres.  A
// cluster's box holds the bounding spheres of its particles.  For a target
// particle t (centre c_t, bounding radius r_t) a cluster C (box centre b,
// half-diagonal rho) is taken through proxies when
//     rho + r_t < theta |c_t - b|,
// C has more nodes than proxies and none of its particles is excluded for t
// (t itself or a source whose near field holds t); otherwise its children
// are visited, and at a leaf its particles that are not excluded are summed
// directly.  Every (target, far source particle) pair is thus covered exactly
// once, and excluded pairs never.
//
// Proxies of C are the tensor grid of Chebyshev points of the second kind,
// (n+1)^3 points s_k in its box.  The Laplace kernel G(x, y) = 1/(4 pi |x-y|)
// is interpolated in y by the barycentric Lagrange basis L_k, so
//     sum_j q_j G(x, y_j)            ~ sum_k qhat_k G(x, s_k),  qhat_k = sum_j q_j L_k(y_j)
//     sum_j d_j . grad_y G(x, y_j)   ~ sum_k qhat_k G(x, s_k),  qhat_k = sum_j d_j . grad L_k(y_j)
// for the single layer (q = W sigma) and the double layer (d = W mu nu).  The
// error falls geometrically in n at a rate set by theta.
//
// Any kernel smooth in the source point interpolates the same way: the
// Stokeslet (Section 4.3) takes vector charges qhat_k = sum_j q_j L_k(y_j) (q =
// W sigma) and is evaluated at the proxies as it stands, and so is its
// pressure kernel.
//
// The interpolation is in the source point only, so the same proxies serve the
// derivatives in the target (Theorem 3's S' and D', the target normal nu_x):
//     nu_x . grad_x sum_k qhat_k G(x, s_k) = -sum_k qhat_k nu_x.(x - s_k) / (4 pi |x - s_k|^3),
// with the single layer's charges for S' and the double layer's for D'.
//
// The plan is host code (no device needed).  The proxy charges are FP64
// kernels, one workgroup per piece of a cluster; the sums take a target
// particle per group of workgroups, in FP64, or in mixed precision with the
// squared distances on the matrix cores (the double layer's proxies then
// carry its dipole moments, Dhat_k = sum_j L_k(y_j) d_j, evaluated against
// grad_y G(x, s_k), in which nothing cancels).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "sbie_internal.h"
#include "x3.h"

namespace sbie {

namespace {

constexpr double kInv4PiT = 0.079577471545947667884441881686257181;
constexpr int kTreeMaxOrder = 12;
constexpr int kChargeParts = 4;  // particles per workgroup of the proxy charges
constexpr int kTreeDipoles = 2;  // charge kind beside SBIE_OP_S and SBIE_OP_D: the double layer's dipole moments

struct TreeNode {
  int first = 0, count = 0;  // range of the permutation
  int child[2] = {-1, -1};
  double lo[3], hi[3];
};

sbie_status invalid(const char* msg) {
  set_error(msg);
  return SBIE_E_INVALID;
}

}  // namespace

// Plan of the tree far field.  excl: [M][words], bit s of row t set iff source
// particle s is excluded for target particle t.
sbie_status plan_tree(int M, int T, const double* centers, const double* radii, const uint32_t* excl, int words,
                      double theta, int order, int leaf, TreePlan* out) {
  if (M < 1 || T < 1 || !centers || !radii || !excl || words < (M + 31) / 32)
    return invalid("tree plan: bad particle arrays");
  if (!(theta > 0.0 && theta < 1.0)) return invalid("tree plan: theta must be in (0, 1)");
  if (order < 2 || order > kTreeMaxOrder) return invalid("tree plan: order must be in [2, 12]");
  if (leaf < 1) return invalid("tree plan: leaf must be >= 1");
  for (int i = 0; i < M; ++i)
    if (!std::isfinite(centers[3 * i]) || !std::isfinite(centers[3 * i + 1]) || !std::isfinite(centers[3 * i + 2]) ||
        !(radii[i] > 0.0) || !std::isfinite(radii[i]))
      return invalid("tree plan: non-finite centre or radius <= 0");
  const int64_t n3 = (int64_t)(order + 1) * (order + 1) * (order + 1);
  auto excluded = [&](int t, int s) { return (excl[(size_t)t * words + (s >> 5)] >> (s & 31)) & 1u; };

  std::vector<int> perm(M);
  std::iota(perm.begin(), perm.end(), 0);
  std::vector<TreeNode> nodes;
  nodes.reserve(2 * (size_t)M);
  // depth-first construction: a cluster's box bounds its particles' spheres;
  // it splits at the median of its centres along their longest extent
  struct Item {
    int first, count, parent, side;
  };
  std::vector<Item> stack{{0, M, -1, 0}};
  while (!stack.empty()) {
    const Item it = stack.back();
    stack.pop_back();
    const int k = (int)nodes.size();
    nodes.emplace_back();
    TreeNode& nd = nodes.back();
    nd.first = it.first;
    nd.count = it.count;
    if (it.parent >= 0) nodes[it.parent].child[it.side] = k;
    double clo[3], chi[3];
    for (int d = 0; d < 3; ++d) {
      nd.lo[d] = clo[d] = INFINITY;
      nd.hi[d] = chi[d] = -INFINITY;
    }
    for (int i = it.first; i < it.first + it.count; ++i) {
      const int s = perm[i];
      for (int d = 0; d < 3; ++d) {
        const double c = centers[3 * s + d];
        nd.lo[d] = std::min(nd.lo[d], c - radii[s]);
        nd.hi[d] = std::max(nd.hi[d], c + radii[s]);
        clo[d] = std::min(clo[d], c);
        chi[d] = std::max(chi[d], c);
      }
    }
    if (it.count > leaf) {
      int dim = 0;
      for (int d = 1; d < 3; ++d)
        if (chi[d] - clo[d] > chi[dim] - clo[dim]) dim = d;
      std::sort(perm.begin() + it.first, perm.begin() + it.first + it.count, [&](int a, int b) {
        const double ca = centers[3 * a + dim], cb = centers[3 * b + dim];
        return ca < cb || (ca == cb && a < b);
      });
      const int h = it.count / 2;
      // the second half is pushed first so that the first half is built next
      stack.push_back({it.first + h, it.count - h, k, 1});
      stack.push_back({it.first, h, k, 0});
    }
  }

  out->nc = (int)nodes.size();
  out->box.resize((size_t)out->nc * 6);
  out->first.resize(out->nc);
  out->count.resize(out->nc);
  for (int k = 0; k < out->nc; ++k) {
    for (int d = 0; d < 3; ++d) {
      out->box[6 * (size_t)k + d] = nodes[k].lo[d];
      out->box[6 * (size_t)k + 3 + d] = nodes[k].hi[d];
    }
    out->first[k] = nodes[k].first;
    out->count[k] = nodes[k].count;
  }
  out->perm = perm;
  out->pptr.assign(M + 1, 0);
  out->dptr.assign(M + 1, 0);
  out->pidx.clear();
  out->didx.clear();
  std::vector<int> visit;
  for (int t = 0; t < M; ++t) {
    visit.assign(1, 0);
    const double* ct = centers + 3 * t;
    while (!visit.empty()) {
      const int k = visit.back();
      visit.pop_back();
      const TreeNode& nd = nodes[k];
      double dist2 = 0.0, diag2 = 0.0;
      for (int d = 0; d < 3; ++d) {
        const double b = 0.5 * (nd.lo[d] + nd.hi[d]);
        dist2 += (ct[d] - b) * (ct[d] - b);
        diag2 += (nd.hi[d] - nd.lo[d]) * (nd.hi[d] - nd.lo[d]);
      }
      bool take = 0.5 * std::sqrt(diag2) + radii[t] < theta * std::sqrt(dist2) && (int64_t)nd.count * T > n3;
      for (int i = nd.first; take && i < nd.first + nd.count; ++i)
        if (excluded(t, perm[i])) take = false;
      if (take) {
        out->pidx.push_back(k);
      } else if (nd.child[0] >= 0) {
        visit.push_back(nd.child[1]);
        visit.push_back(nd.child[0]);
      } else {
        for (int i = nd.first; i < nd.first + nd.count; ++i)
          if (!excluded(t, perm[i])) out->didx.push_back(perm[i]);
      }
    }
    out->pptr[t + 1] = (int64_t)out->pidx.size();
    out->dptr[t + 1] = (int64_t)out->didx.size();
  }
  out->order = order;
  out->theta = theta;
  return SBIE_OK;
}

namespace {

// 1/sqrt(x): the hardware estimate and one Newton step
__device__ inline double rsqrt_tree(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double h = x * y;
  const double e = fma(-h, y, 1.0);
  return fma(0.5 * y, e, y);
}

// Chebyshev points of the second kind s_k = cos(pi k / n) on [-1, 1] and
// their barycentric weights (-1)^k, halved at both ends, into cs[0..n] and
// cw[0..n] (LDS, filled by the first n+1 lanes)
__device__ inline void cheb_table(int n, double* cs, double* cw) {
  const int k = threadIdx.x;
  if (k <= n) {
    cs[k] = cospi((double)k / (double)n);
    cw[k] = ((k & 1) ? -1.0 : 1.0) * ((k == 0 || k == n) ? 0.5 : 1.0);
  }
}

// Lagrange basis L_k(u), k = 0..n, on the Chebyshev points, and (DERIV) its
// derivative, by the barycentric formulas; at a Chebyshev point itself the
// basis is the unit vector and the derivative the differentiation-matrix row
template <bool DERIV>
__device__ inline void lagrange(int n, const double* cs, const double* cw, double u, double* L, double* dL) {
  int hit = -1;
  for (int k = 0; k <= n; ++k)
    if (u == cs[k]) hit = k;
  if (hit < 0) {
    double A = 0.0, B = 0.0;
    for (int k = 0; k <= n; ++k) {
      const double r = 1.0 / (u - cs[k]);
      const double a = cw[k] * r;
      L[k] = a;
      A += a;
      B += a * r;
    }
    const double iA = 1.0 / A;
    for (int k = 0; k <= n; ++k) {
      const double l = L[k] * iA;
      L[k] = l;
      if (DERIV) dL[k] = l * (B * iA - 1.0 / (u - cs[k]));
    }
  } else {
    double sum = 0.0;
    for (int k = 0; k <= n; ++k) {
      L[k] = k == hit ? 1.0 : 0.0;
      if (DERIV && k != hit) {
        dL[k] = (cw[k] / cw[hit]) / (cs[hit] - cs[k]);
        sum += dL[k];
      }
    }
    if (DERIV) dL[hit] = -sum;
  }
}

// Partial proxy charges: one workgroup per piece of a used cluster (at most
// kChargeParts of its particles; piece = (cluster slot, first, count) in the
// permutation), qhat_k over the piece's nodes, 64 nodes at a time through
// LDS.  Source records: S (x, y, z, W sigma) in 4 doubles, D (x, y, z, W mu nu)
// in 8.  Kind kTreeDipoles takes the double layer's dipole moments instead,
// Dhat_k = sum_j L_k(y_j) d_j (three per proxy): the far field is then
// sum_k Dhat_k . grad_y G(x, s_k), in which nothing cancels.
template <int OP>
__global__ __launch_bounds__(256) void k_tree_charges(const double* __restrict__ box, const int32_t* __restrict__ piece,
                                                     const int32_t* __restrict__ perm, const double* __restrict__ src,
                                                     int T, int n, double* __restrict__ qpart) {
  constexpr bool DIP = OP == kTreeDipoles;
  constexpr int SW = OP == SBIE_OP_S ? 4 : 8;
  constexpr int NC = 64, NB = kTreeMaxOrder + 1;
  // S: q Lx, Ly, Lz; D: Lx, Ly, Lz, d_x dLx, d_y dLy, d_z dLz; dipoles: Lx, Ly, Lz
  constexpr int NSET = OP == SBIE_OP_D ? 6 : 3;
  constexpr int NA = DIP ? 3 : 1;  // accumulators per proxy
  __shared__ double basis[NSET][NC][NB];
  __shared__ double dip[DIP ? NC : 1][3];
  __shared__ double cs[NB], cw[NB];
  const int pc = blockIdx.x, tid = threadIdx.x;
  const int c = piece[3 * pc], pfirst = piece[3 * pc + 1], pcount = piece[3 * pc + 2];
  const int n1 = n + 1, n3 = n1 * n1 * n1;
  cheb_table(n, cs, cw);
  __syncthreads();
  double lo[3], sc[3];
  for (int d = 0; d < 3; ++d) {
    lo[d] = box[6 * c + d];
    sc[d] = 2.0 / (box[6 * c + 3 + d] - lo[d]);  // d u / d y
  }
  constexpr int KPT = (NB * NB * NB + 255) / 256;
  double acc[KPT][NA];
#pragma unroll
  for (int m = 0; m < KPT; ++m)
#pragma unroll
    for (int w = 0; w < NA; ++w) acc[m][w] = 0.0;
  const int64_t nodes = (int64_t)pcount * T;
  for (int64_t j0 = 0; j0 < nodes; j0 += NC) {
    if (tid < NC) {
      const int64_t j = j0 + tid;
      if (j < nodes) {
        const int part = perm[pfirst + (int)(j / T)];
        const double* r = src + ((int64_t)part * T + j % T) * SW;
        for (int d = 0; d < 3; ++d)
          lagrange<OP == SBIE_OP_D>(n, cs, cw, (r[d] - lo[d]) * sc[d] - 1.0, basis[d][tid],
                                    basis[OP == SBIE_OP_D ? 3 + d : d][tid]);
        // S: the strength folded into the x basis; D: the dipole component
        // (times d u / d y) into each derivative
        if (OP == SBIE_OP_S) {
          for (int k = 0; k < n1; ++k) basis[0][tid][k] *= r[3];
        } else if (OP == SBIE_OP_D) {
          for (int d = 0; d < 3; ++d)
            for (int k = 0; k < n1; ++k) basis[3 + d][tid][k] *= r[3 + d] * sc[d];
        } else {
          for (int d = 0; d < 3; ++d) dip[tid][d] = r[3 + d];
        }
      } else {
        for (int w = 0; w < NSET; ++w)
          for (int k = 0; k < n1; ++k) basis[w][tid][k] = 0.0;
        if (DIP)
          for (int d = 0; d < 3; ++d) dip[tid][d] = 0.0;
      }
    }
    __syncthreads();
    const int jn = nodes - j0 < NC ? (int)(nodes - j0) : NC;
#pragma unroll
    for (int m = 0; m < KPT; ++m) {
      const int k = tid + 256 * m;
      if (k < n3) {
        const int k1 = k / (n1 * n1), k2 = (k / n1) % n1, k3 = k % n1;
        double a[NA];
#pragma unroll
        for (int w = 0; w < NA; ++w) a[w] = acc[m][w];
        for (int j = 0; j < jn; ++j) {
          if (OP == SBIE_OP_S) {
            a[0] = fma(basis[0][j][k1] * basis[1][j][k2], basis[2][j][k3], a[0]);
          } else if (OP == SBIE_OP_D) {
            const double lx = basis[0][j][k1], ly = basis[1][j][k2], lz = basis[2][j][k3];
            a[0] = fma(basis[3][j][k1] * ly, lz, a[0]);
            a[0] = fma(lx * basis[4][j][k2], lz, a[0]);
            a[0] = fma(lx * ly, basis[5][j][k3], a[0]);
          } else {
            const double l = basis[0][j][k1] * basis[1][j][k2] * basis[2][j][k3];
#pragma unroll
            for (int w = 0; w < NA; ++w) a[w] = fma(l, dip[j][w], a[w]);
          }
        }
#pragma unroll
        for (int w = 0; w < NA; ++w) acc[m][w] = a[w];
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int m = 0; m < KPT; ++m) {
    const int k = tid + 256 * m;
    if (k < n3)
#pragma unroll
      for (int w = 0; w < NA; ++w) qpart[((int64_t)pc * n3 + k) * NA + w] = acc[m][w];
  }
}

// Proxy table of each used cluster: [n3p][4] = (point, charge), the charge
// its pieces' partial charges added in piece order; n3p = n3 rounded up to
// four, the padding zero charges at a distant point.  With q32 (mixed path)
// also the FP32 charges alone, nq = 16 n3b per cluster, zero past n3; the
// grid covers nq entries per cluster (n3p without q32).
__global__ void k_tree_proxies(const double* __restrict__ box, const int32_t* __restrict__ pptr,
                               const double* __restrict__ qpart, int nused, int n, int n3p, int nq,
                               double* __restrict__ prox, float* __restrict__ q32) {
  __shared__ double cs[kTreeMaxOrder + 1], cw[kTreeMaxOrder + 1];
  cheb_table(n, cs, cw);
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nused * nq) return;
  const int n1 = n + 1, n3 = n1 * n1 * n1;
  const int c = (int)(i / nq), k = (int)(i - (int64_t)c * nq);
  double* o = prox + 4 * ((int64_t)c * n3p + k);
  if (k >= n3) {
    if (k < n3p) {
      o[0] = o[1] = o[2] = 1e30;
      o[3] = 0.0;
    }
    if (q32) q32[i] = 0.0f;
    return;
  }
  const int idx[3] = {k / (n1 * n1), (k / n1) % n1, k % n1};
  for (int d = 0; d < 3; ++d) {
    const double lo = box[6 * c + d], hi = box[6 * c + 3 + d];
    o[d] = lo + 0.5 * (cs[idx[d]] + 1.0) * (hi - lo);
  }
  double q = 0.0;
  for (int p = pptr[c]; p < pptr[c + 1]; ++p) q += qpart[(int64_t)p * n3 + k];
  o[3] = q;
  if (q32) q32[i] = (float)q;
}

// Vector-charge proxy table of each used cluster for the Stokeslet, [nused][n3p]
// records (s, qhat, 0, 0) of 8 doubles, the charges its pieces' partial
// charges (kind kTreeDipoles) added in piece order; padding at a distant point
// with zero charge.
__global__ void k_tree_proxies3(const double* __restrict__ box, const int32_t* __restrict__ pptr,
                                const double* __restrict__ qpart, int nused, int n, int n3p,
                                double* __restrict__ prox) {
  __shared__ double cs[kTreeMaxOrder + 1], cw[kTreeMaxOrder + 1];
  cheb_table(n, cs, cw);
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nused * n3p) return;
  const int n1 = n + 1, n3 = n1 * n1 * n1;
  const int c = (int)(i / n3p), k = (int)(i - (int64_t)c * n3p);
  double* o = prox + 8 * i;
  o[6] = o[7] = 0.0;
  if (k >= n3) {
    o[0] = o[1] = o[2] = 1e30;
    o[3] = o[4] = o[5] = 0.0;
    return;
  }
  const int idx[3] = {k / (n1 * n1), (k / n1) % n1, k % n1};
  for (int d = 0; d < 3; ++d) {
    const double lo = box[6 * c + d], hi = box[6 * c + 3 + d];
    o[d] = lo + 0.5 * (cs[idx[d]] + 1.0) * (hi - lo);
  }
  double q[3] = {0.0, 0.0, 0.0};
  for (int p = pptr[c]; p < pptr[c + 1]; ++p)
    for (int w = 0; w < 3; ++w) q[w] += qpart[((int64_t)p * n3 + k) * 3 + w];
  for (int w = 0; w < 3; ++w) o[3 + w] = q[w];
}

// Matrix-core form of the mixed path.  Sources are the rows of a 16x16x32 bf16
// product in the three-piece form, target nodes its columns: source record
// [-2 s, |s|^2] against [t, 1] with |t|^2 in the extra slots gives |t - s|^2
// for 16 x 16 pairs, s and t rounded to FP32 once, relative to the source
// set's origin (a cluster's box centre, a source particle's centre).  One
// record per 16 sources, 64 lanes x 4 words; padding sources sit at the
// origin with zero strength.

// the A-operand words of lane group lg for a source at s (FP32)
__device__ inline u4 tree_point_record(float sx, float sy, float sz, int lg) {
  const double s2 = fma((double)sz, (double)sz, fma((double)sy, (double)sy, (double)sx * sx));
  const float v = lg == 0 ? -2.0f * sx : (lg == 1 ? -2.0f * sy : (lg == 2 ? -2.0f * sz : (float)s2));
  return split_a(v, lg, true);
}

// proxy records of every used cluster, [nused][n3b][64]: the Chebyshev points
// relative to the box centre
__global__ void k_tree_proxy_records(const double* __restrict__ box, int nused, int n, int n3b, u4* __restrict__ rec) {
  __shared__ double cs[kTreeMaxOrder + 1], cw[kTreeMaxOrder + 1];
  cheb_table(n, cs, cw);
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int nq = 16 * n3b;
  if (i >= (int64_t)nused * nq) return;
  const int n1 = n + 1, n3 = n1 * n1 * n1;
  const int c = (int)(i / nq), k = (int)(i - (int64_t)c * nq);
  float r[3] = {0.0f, 0.0f, 0.0f};
  if (k < n3) {
    const int idx[3] = {k / (n1 * n1), (k / n1) % n1, k % n1};
    for (int d = 0; d < 3; ++d) r[d] = (float)(0.5 * cs[idx[d]] * (box[6 * c + 3 + d] - box[6 * c + d]));
  }
  u4* o = rec + (i / 16) * 64 + (k % 16);
  for (int lg = 0; lg < 4; ++lg) o[16 * lg] = tree_point_record(r[0], r[1], r[2], lg);
}

// Per-apply dipole records of every used cluster for the mixed double layer,
// [nused][n3b][64]: [Dhat, -Dhat.s] with s as in the proxy records (no extra
// term), whose product with the target column [t - b, 1] is Dhat.(t - b - s);
// the pieces' moments added in piece order; zero past n3.
__global__ void k_tree_dipole_records(const double* __restrict__ box, const int32_t* __restrict__ pptr,
                                      const double* __restrict__ qpart, int nused, int n, int n3b,
                                      u4* __restrict__ rec) {
  __shared__ double cs[kTreeMaxOrder + 1], cw[kTreeMaxOrder + 1];
  cheb_table(n, cs, cw);
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int nq = 16 * n3b;
  if (i >= (int64_t)nused * nq) return;
  const int n1 = n + 1, n3 = n1 * n1 * n1;
  const int c = (int)(i / nq), k = (int)(i - (int64_t)c * nq);
  double d[3] = {0.0, 0.0, 0.0}, dot = 0.0;
  if (k < n3) {
    const int idx[3] = {k / (n1 * n1), (k / n1) % n1, k % n1};
    for (int p = pptr[c]; p < pptr[c + 1]; ++p)
      for (int w = 0; w < 3; ++w) d[w] += qpart[((int64_t)p * n3 + k) * 3 + w];
    for (int w = 0; w < 3; ++w) {
      const float sw = (float)(0.5 * cs[idx[w]] * (box[6 * c + 3 + w] - box[6 * c + w]));
      dot = fma(d[w], (double)sw, dot);
    }
  }
  u4* o = rec + (i / 16) * 64 + (k % 16);
  for (int lg = 0; lg < 4; ++lg) o[16 * lg] = split_a((float)(lg < 3 ? d[lg] : -dot), lg, false);
}

// node records of every particle as a direct source, [M][T16][64]: nodes
// relative to the particle centre
__global__ void k_tree_node_records(const double* __restrict__ x, const double* __restrict__ y,
                                    const double* __restrict__ z, const Particle* __restrict__ part, int M, int T,
                                    int T16, u4* __restrict__ rec) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)M * T16 * 16) return;
  const int s = (int)(i / (T16 * 16)), q = (int)(i - (int64_t)s * T16 * 16);
  float r[3] = {0.0f, 0.0f, 0.0f};
  if (q < T) {
    const int64_t g = (int64_t)s * T + q;
    r[0] = (float)(x[g] - part[s].c[0]);
    r[1] = (float)(y[g] - part[s].c[1]);
    r[2] = (float)(z[g] - part[s].c[2]);
  }
  u4* o = rec + (i / 16) * 64 + (q % 16);
  for (int lg = 0; lg < 4; ++lg) o[16 * lg] = tree_point_record(r[0], r[1], r[2], lg);
}

// Per-apply FP32 strengths W sigma of the direct sources for the mixed single
// layer, [M][T16*16] (zero past T).
__global__ void k_tree_strengths32(const double* __restrict__ src, int M, int T, int T16, float* __restrict__ q32) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)M * T16 * 16) return;
  const int s = (int)(i / (T16 * 16)), q = (int)(i - (int64_t)s * T16 * 16);
  q32[i] = q < T ? (float)src[((int64_t)s * T + q) * 4 + 3] : 0.0f;
}

// The mixed-precision single layer of a target particle (split over nsplit
// workgroups like k_tree_eval).  The particle's target nodes are staged in
// LDS; a wave takes four 16-node column blocks at a time as B operands,
// rebuilt for each source set from the targets' FP32 offsets from its origin.
// Per 16-source record and column block one product gives the 256 squared
// distances; lane l holds sources 4*(l/16) + e (e = 0..3) of column l%16 and
// adds their four FP32 terms into its FP64 sum, and the four lane groups are
// added at the end.  The vector unit bounds it (about 12 vector instructions
// per product, the matrix cores a sixth busy), so occupancy pays: registers are capped for eight
// waves per SIMD (a few spilled outside the record loop), seven for the
// dipole proxies' two products.
//
// DIP: the double layer's proxies alone, through their dipole records: a
// second product of [Dhat, -Dhat.s] with the same columns gives
// Dhat.(t - s) for the weight r^-3 (the target's offset from the box centre
// is at most (1 + theta) / (1 - theta) times its distance from a proxy, so
// the difference loses little); the direct sums are k_tree_eval32_d's.
template <bool DIP>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(DIP ? 7 : 8, 8))) void k_tree_eval_x3(
    const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ z,
    const Particle* __restrict__ part, const double* __restrict__ box, const int64_t* __restrict__ pptr,
    const int32_t* __restrict__ pidx, const int64_t* __restrict__ dptr, const int32_t* __restrict__ didx,
    const u4* __restrict__ prec, const float* __restrict__ pq32, const u4* __restrict__ pdrec,
    const u4* __restrict__ srec, const float* __restrict__ sq32, int T, int T16, int n3b, int nsplit, int64_t N,
    double* __restrict__ out) {
  extern __shared__ double tsh[];  // [3][T]
  const int t = blockIdx.x / nsplit, split = blockIdx.x % nsplit;
  for (int i = threadIdx.x; i < T; i += blockDim.x) {
    const int64_t g = (int64_t)t * T + i;
    tsh[i] = x[g];
    tsh[T + i] = y[g];
    tsh[2 * T + i] = z[g];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, lg = lane >> 4, li = lane & 15;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), nw = blockDim.x >> 6;
  const int64_t p0 = pptr[t], np = pptr[t + 1] - p0, d0 = dptr[t], nd = dptr[t + 1] - d0;
  const int64_t pa = p0 + np * split / nsplit, pb = p0 + np * (split + 1) / nsplit;
  const int64_t da = d0 + nd * split / nsplit, db = d0 + nd * (split + 1) / nsplit;
  for (int cb0 = 4 * wave; cb0 < T16; cb0 += 4 * nw) {
    const int ncb = min(4, T16 - cb0);  // column blocks of this wave (uniform)
    u4 B[4];
    // columns past T repeat the last node and are not written
    auto columns = [&](double ox, double oy, double oz) {
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        const int i = min(16 * (cb0 + cb) + li, T - 1);
        const float fx = (float)(tsh[i] - ox), fy = (float)(tsh[T + i] - oy), fz = (float)(tsh[2 * T + i] - oz);
        const float e = (float)fma((double)fz, (double)fz, fma((double)fy, (double)fy, (double)fx * fx));
        B[cb] = split_b(lg == 0 ? fx : (lg == 1 ? fy : (lg == 2 ? fz : 1.0f)), lg, e);
      }
    };
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    auto blocks = [&](const u4* R, const float* Q, int nblk) {
#pragma unroll 2
      for (int bk = 0; bk < nblk; ++bk) {
        const u4 a = R[64 * bk + lane];
        const f4 q = reinterpret_cast<const f4*>(Q + 16 * bk)[lg];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
          if (cb < ncb) {
            const f4 r2 = mma_x3(a, B[cb]);
            const float v = q.x * __builtin_amdgcn_rsqf(r2.x) + q.y * __builtin_amdgcn_rsqf(r2.y) +
                            q.z * __builtin_amdgcn_rsqf(r2.z) + q.w * __builtin_amdgcn_rsqf(r2.w);
            acc[cb] += (double)v;
          }
        }
      }
    };
    auto dipoles = [&](const u4* R, const u4* R2, int nblk) {
      for (int bk = 0; bk < nblk; ++bk) {
        const u4 a = R[64 * bk + lane], a2 = R2[64 * bk + lane];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
          if (cb < ncb) {
            const f4 r2 = mma_x3(a, B[cb]);
            const f4 dt = mma_x3(a2, B[cb]);
            float v = 0.0f;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const float ri = __builtin_amdgcn_rsqf(r2[e]);
              v = fmaf(dt[e], ri * ri * ri, v);
            }
            acc[cb] += (double)v;
          }
        }
      }
    };
    for (int64_t m = pa; m < pb; ++m) {
      const int c = pidx[m];
      columns(0.5 * (box[6 * c] + box[6 * c + 3]), 0.5 * (box[6 * c + 1] + box[6 * c + 4]),
              0.5 * (box[6 * c + 2] + box[6 * c + 5]));
      if constexpr (DIP)
        dipoles(prec + (size_t)c * n3b * 64, pdrec + (size_t)c * n3b * 64, n3b);
      else
        blocks(prec + (size_t)c * n3b * 64, pq32 + (size_t)c * n3b * 16, n3b);
    }
    for (int64_t m = DIP ? db : da; m < db; ++m) {
      const int s = didx[m];
      columns(part[s].c[0], part[s].c[1], part[s].c[2]);
      blocks(srec + (size_t)s * T16 * 64, sq32 + (size_t)s * T16 * 16, T16);
    }
    // the four lane groups of a column, then lane l keeps column block l/16
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      acc[cb] += lane_value(acc[cb], (lane ^ 16) << 2);
      acc[cb] += lane_value(acc[cb], (lane ^ 32) << 2);
    }
    const double v = lg == 0 ? acc[0] : (lg == 1 ? acc[1] : (lg == 2 ? acc[2] : acc[3]));
    const int i = 16 * cb0 + lane;
    if (lg < ncb && i < T) out[(size_t)split * N + (int64_t)t * T + i] = v * kInv4PiT;
  }
}

// FP32 records of the direct sources for the mixed double layer: node -
// particle centre and W mu nu, 8 floats per node (the last two as stored).
__global__ void k_tree_src32_d(const double* __restrict__ src, const Particle* __restrict__ part, int T, int64_t N,
                               float* __restrict__ src32) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  const double* r = src + g * 8;
  const double* c = part[g / T].c;
  float* o = src32 + g * 8;
  for (int d = 0; d < 3; ++d) o[d] = (float)(r[d] - c[d]);
  for (int w = 3; w < 8; ++w) o[w] = (float)r[w];
}

// The mixed-precision double layer (split over nsplit workgroups like
// k_tree_eval, one target per lane).  Its proxy charges cancel strongly
// within a cluster (they come from dipoles), so the proxy sums are FP64.  The
// direct sums take FP32 differences from the source particle's centre, the
// target's offset from it rounded once per particle, FP32 terms four per
// step added into the FP64 sum.  (On the matrix cores, d.(t - s) as
// d.t - d.s cancels and costs the bar its margin.)
//
// ADD: the direct sums alone, added into the slices (after the dipole
// proxies of k_tree_eval_x3).
template <int TPT, bool ADD>
__global__ __launch_bounds__(1024) void k_tree_eval32_d(const double* __restrict__ x, const double* __restrict__ y,
                                                        const double* __restrict__ z, const float* __restrict__ src32,
                                                        const Particle* __restrict__ part,
                                                        const double* __restrict__ prox,
                                                        const int64_t* __restrict__ pptr,
                                                        const int32_t* __restrict__ pidx,
                                                        const int64_t* __restrict__ dptr,
                                                        const int32_t* __restrict__ didx, int T, int n3p, int nsplit,
                                                        int64_t N, double* __restrict__ out) {
  const int t = blockIdx.x / nsplit, split = blockIdx.x % nsplit, tid = threadIdx.x;
  const int64_t p0 = pptr[t], np = pptr[t + 1] - p0, d0 = dptr[t], nd = dptr[t + 1] - d0;
  double tx[TPT], ty[TPT], tz[TPT], acc[TPT];
#pragma unroll
  for (int k = 0; k < TPT; ++k) {
    const int i = tid + k * blockDim.x;
    const int64_t g = (int64_t)t * T + (i < T ? i : 0);
    tx[k] = x[g];
    ty[k] = y[g];
    tz[k] = z[g];
    acc[k] = 0.0;
  }
  for (int64_t m = p0 + np * split / nsplit; !ADD && m < p0 + np * (split + 1) / nsplit; ++m) {
    const double* P = prox + (int64_t)pidx[m] * n3p * 4;
    for (int k = 0; k < n3p; k += 4) {
#pragma unroll
      for (int e = 0; e < TPT; ++e) {
        double a[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const double* r = P + 4 * (k + u);
          const double dx = tx[e] - r[0], dy = ty[e] - r[1], dz = tz[e] - r[2];
          a[u] = r[3] * rsqrt_tree(fma(dz, dz, fma(dy, dy, dx * dx)));
        }
        acc[e] += (a[0] + a[1]) + (a[2] + a[3]);
      }
    }
  }
  for (int64_t m = d0 + nd * split / nsplit; m < d0 + nd * (split + 1) / nsplit; ++m) {
    const int s = didx[m];
    const float* rs = src32 + (int64_t)s * T * 8;
    const double* cc = part[s].c;
    float rx[TPT], ry[TPT], rz[TPT];
#pragma unroll
    for (int e = 0; e < TPT; ++e) {
      rx[e] = (float)(tx[e] - cc[0]);
      ry[e] = (float)(ty[e] - cc[1]);
      rz[e] = (float)(tz[e] - cc[2]);
    }
    int j = 0;
    for (; j + 4 <= T; j += 4) {
#pragma unroll
      for (int e = 0; e < TPT; ++e) {
        float a[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const float* r = rs + (int64_t)(j + u) * 8;
          const float dx = rx[e] - r[0], dy = ry[e] - r[1], dz = rz[e] - r[2];
          const float ri = __builtin_amdgcn_rsqf(fmaf(dz, dz, fmaf(dy, dy, dx * dx)));
          const float dot = fmaf(r[5], dz, fmaf(r[4], dy, r[3] * dx));
          a[u] = dot * (ri * ri * ri);
        }
        acc[e] += (double)((a[0] + a[1]) + (a[2] + a[3]));
      }
    }
    for (; j < T; ++j) {
      const float* r = rs + (int64_t)j * 8;
#pragma unroll
      for (int e = 0; e < TPT; ++e) {
        const float dx = rx[e] - r[0], dy = ry[e] - r[1], dz = rz[e] - r[2];
        const float ri = __builtin_amdgcn_rsqf(fmaf(dz, dz, fmaf(dy, dy, dx * dx)));
        const float dot = fmaf(r[5], dz, fmaf(r[4], dy, r[3] * dx));
        acc[e] += (double)(dot * (ri * ri * ri));
      }
    }
  }
#pragma unroll
  for (int k = 0; k < TPT; ++k) {
    const int i = tid + k * blockDim.x;
    if (i < T) {
      double* o = out + (size_t)split * N + (int64_t)t * T + i;
      *o = ADD ? *o + acc[k] * kInv4PiT : acc[k] * kInv4PiT;
    }
  }
}

// Far field of a target particle, its interaction lists split over nsplit
// workgroups (split s takes the s-th of the accepted clusters and of the
// direct particles, and writes slice s of the partial sums): the accepted
// clusters through their proxy tables, then the direct far particles'
// records.  Source points are read with wave-uniform addresses (scalar loads
// through the constant cache), four per step into four partial sums.  Lane l
// holds targets l, l + blockDim, ... of the particle (TPT of them).
template <int OP, int TPT>
__global__ __launch_bounds__(1024) void k_tree_eval(const double* __restrict__ x, const double* __restrict__ y,
                                                    const double* __restrict__ z, const double* __restrict__ src,
                                                    const double* __restrict__ prox, const int64_t* __restrict__ pptr,
                                                    const int32_t* __restrict__ pidx, const int64_t* __restrict__ dptr,
                                                    const int32_t* __restrict__ didx, int T, int n3p, int nsplit,
                                                    int64_t N, double* __restrict__ out) {
  constexpr int SW = OP == SBIE_OP_S ? 4 : 8;
  const int t = blockIdx.x / nsplit, split = blockIdx.x % nsplit, tid = threadIdx.x;
  const int64_t p0 = pptr[t], np = pptr[t + 1] - p0, d0 = dptr[t], nd = dptr[t + 1] - d0;
  double tx[TPT], ty[TPT], tz[TPT], acc[TPT];
#pragma unroll
  for (int k = 0; k < TPT; ++k) {
    const int i = tid + k * blockDim.x;
    const int64_t g = (int64_t)t * T + (i < T ? i : 0);
    tx[k] = x[g];
    ty[k] = y[g];
    tz[k] = z[g];
    acc[k] = 0.0;
  }
  // proxies of the accepted clusters: point charges, four per step
  for (int64_t m = p0 + np * split / nsplit; m < p0 + np * (split + 1) / nsplit; ++m) {
    const double* P = prox + (int64_t)pidx[m] * n3p * 4;
    for (int k = 0; k < n3p; k += 4) {
#pragma unroll
      for (int e = 0; e < TPT; ++e) {
        double a[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const double* r = P + 4 * (k + u);
          const double dx = tx[e] - r[0], dy = ty[e] - r[1], dz = tz[e] - r[2];
          a[u] = r[3] * rsqrt_tree(fma(dz, dz, fma(dy, dy, dx * dx)));
        }
        acc[e] += (a[0] + a[1]) + (a[2] + a[3]);
      }
    }
  }
  // direct far particles
  for (int64_t m = d0 + nd * split / nsplit; m < d0 + nd * (split + 1) / nsplit; ++m) {
    const double* rs = src + (int64_t)didx[m] * T * SW;
    int j = 0;
    for (; j + 4 <= T; j += 4) {
#pragma unroll
      for (int e = 0; e < TPT; ++e) {
        double a[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const double* r = rs + (int64_t)(j + u) * SW;
          const double dx = tx[e] - r[0], dy = ty[e] - r[1], dz = tz[e] - r[2];
          const double ri = rsqrt_tree(fma(dz, dz, fma(dy, dy, dx * dx)));
          if (OP == SBIE_OP_S) {
            a[u] = r[3] * ri;
          } else {
            const double dot = fma(r[5], dz, fma(r[4], dy, r[3] * dx));
            a[u] = dot * (ri * ri * ri);
          }
        }
        acc[e] += (a[0] + a[1]) + (a[2] + a[3]);
      }
    }
    for (; j < T; ++j) {
      const double* r = rs + (int64_t)j * SW;
#pragma unroll
      for (int e = 0; e < TPT; ++e) {
        const double dx = tx[e] - r[0], dy = ty[e] - r[1], dz = tz[e] - r[2];
        const double ri = rsqrt_tree(fma(dz, dz, fma(dy, dy, dx * dx)));
        if (OP == SBIE_OP_S) {
          acc[e] = fma(r[3], ri, acc[e]);
        } else {
          const double dot = fma(r[5], dz, fma(r[4], dy, r[3] * dx));
          acc[e] = fma(dot, ri * ri * ri, acc[e]);
        }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < TPT; ++k) {
    const int i = tid + k * blockDim.x;
    if (i < T) out[(size_t)split * N + (int64_t)t * T + i] = acc[k] * kInv4PiT;
  }
}

// S' and D' through the tree (FP64), grid and lanes as k_tree_eval, with
// d = x - y and the target normal nu_x:
//   proxies (either operator) -qhat (nu_x.d) / r^3,
//   direct S'  -q (nu_x.d) / r^3                           (records x, y, z, W sigma),
//   direct D'  (nu_x.m) / r^3 - 3 (m.d)(nu_x.d) / r^5     (records x, y, z, m = W mu nu_y),
// the kernels of the direct far sums of S' and D'.
template <int OP, int TPT>
__global__ __launch_bounds__(1024) void k_tree_eval_normal(
    const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ z,
    const double* __restrict__ nx, const double* __restrict__ ny, const double* __restrict__ nz,
    const double* __restrict__ src, const double* __restrict__ prox, const int64_t* __restrict__ pptr,
    const int32_t* __restrict__ pidx, const int64_t* __restrict__ dptr, const int32_t* __restrict__ didx, int T,
    int n3p, int nsplit, int64_t N, double* __restrict__ out) {
  constexpr int SW = OP == SBIE_OP_SP ? 4 : 8;
  const int t = blockIdx.x / nsplit, split = blockIdx.x % nsplit, tid = threadIdx.x;
  const int64_t p0 = pptr[t], np = pptr[t + 1] - p0, d0 = dptr[t], nd = dptr[t + 1] - d0;
  double tx[TPT], ty[TPT], tz[TPT], tn[TPT][3], acc[TPT];
#pragma unroll
  for (int k = 0; k < TPT; ++k) {
    const int i = tid + k * blockDim.x;
    const int64_t g = (int64_t)t * T + (i < T ? i : 0);
    tx[k] = x[g];
    ty[k] = y[g];
    tz[k] = z[g];
    tn[k][0] = nx[g];
    tn[k][1] = ny[g];
    tn[k][2] = nz[g];
    acc[k] = 0.0;
  }
  for (int64_t m = p0 + np * split / nsplit; m < p0 + np * (split + 1) / nsplit; ++m) {
    const double* P = prox + (int64_t)pidx[m] * n3p * 4;
    for (int k = 0; k < n3p; k += 4) {
#pragma unroll
      for (int e = 0; e < TPT; ++e) {
        double a[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const double* r = P + 4 * (k + u);
          const double dx = tx[e] - r[0], dy = ty[e] - r[1], dz = tz[e] - r[2];
          const double ri = rsqrt_tree(fma(dz, dz, fma(dy, dy, dx * dx)));
          const double nd_ = fma(tn[e][2], dz, fma(tn[e][1], dy, tn[e][0] * dx));
          a[u] = -r[3] * nd_ * (ri * ri * ri);
        }
        acc[e] += (a[0] + a[1]) + (a[2] + a[3]);
      }
    }
  }
  for (int64_t m = d0 + nd * split / nsplit; m < d0 + nd * (split + 1) / nsplit; ++m) {
    const double* rs = src + (int64_t)didx[m] * T * SW;
    for (int j = 0; j < T; ++j) {
      const double* r = rs + (int64_t)j * SW;
#pragma unroll
      for (int e = 0; e < TPT; ++e) {
        const double dx = tx[e] - r[0], dy = ty[e] - r[1], dz = tz[e] - r[2];
        const double ri = rsqrt_tree(fma(dz, dz, fma(dy, dy, dx * dx)));
        const double ri3 = ri * ri * ri;
        const double nd_ = fma(tn[e][2], dz, fma(tn[e][1], dy, tn[e][0] * dx));
        if (OP == SBIE_OP_SP) {
          acc[e] = fma(-r[3] * nd_, ri3, acc[e]);
        } else {
          const double md = fma(r[5], dz, fma(r[4], dy, r[3] * dx));
          const double nm = fma(tn[e][2], r[5], fma(tn[e][1], r[4], tn[e][0] * r[3]));
          acc[e] = fma(ri3, fma(-3.0 * md * nd_, ri * ri, nm), acc[e]);
        }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < TPT; ++k) {
    const int i = tid + k * blockDim.x;
    if (i < T) out[(size_t)split * N + (int64_t)t * T + i] = acc[k] * kInv4PiT;
  }
}

// The Stokeslet (1/8pi)(q/r + (d.q) d/r^3) and, for C = 4, the pressure
// (1/4pi)(d.q)/r^3 (d = x - y) through the tree in FP64: proxies (s, qhat) and
// direct far particles' records (y, W sigma), both 8 doubles; grid and lanes
// as k_tree_eval; out [nsplit][C][N].
template <int C, int TPT>
__global__ __launch_bounds__(1024) void k_tree_eval_stokes(
    const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ z,
    const double* __restrict__ src, const double* __restrict__ prox, const int64_t* __restrict__ pptr,
    const int32_t* __restrict__ pidx, const int64_t* __restrict__ dptr, const int32_t* __restrict__ didx, int T,
    int n3p, int nsplit, int64_t N, double* __restrict__ out) {
  const int t = blockIdx.x / nsplit, split = blockIdx.x % nsplit, tid = threadIdx.x;
  const int64_t p0 = pptr[t], np = pptr[t + 1] - p0, d0 = dptr[t], nd = dptr[t + 1] - d0;
  double tx[TPT], ty[TPT], tz[TPT], acc[TPT][C];
#pragma unroll
  for (int k = 0; k < TPT; ++k) {
    const int i = tid + k * blockDim.x;
    const int64_t g = (int64_t)t * T + (i < T ? i : 0);
    tx[k] = x[g];
    ty[k] = y[g];
    tz[k] = z[g];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[k][c] = 0.0;
  }
  // one source (r: point and vector charge) into every target of the lane
  auto term = [&](const double* r) {
#pragma unroll
    for (int e = 0; e < TPT; ++e) {
      const double dx = tx[e] - r[0], dy = ty[e] - r[1], dz = tz[e] - r[2];
      const double ri = rsqrt_tree(fma(dz, dz, fma(dy, dy, dx * dx)));
      const double f = fma(dz, r[5], fma(dy, r[4], dx * r[3])) * (ri * ri * ri);
      acc[e][0] = fma(r[3], ri, fma(dx, f, acc[e][0]));
      acc[e][1] = fma(r[4], ri, fma(dy, f, acc[e][1]));
      acc[e][2] = fma(r[5], ri, fma(dz, f, acc[e][2]));
      if constexpr (C == 4) acc[e][3] += f;
    }
  };
  for (int64_t m = p0 + np * split / nsplit; m < p0 + np * (split + 1) / nsplit; ++m) {
    const double* P = prox + (int64_t)pidx[m] * n3p * 8;
    for (int k = 0; k < n3p; ++k) term(P + 8 * k);
  }
  for (int64_t m = d0 + nd * split / nsplit; m < d0 + nd * (split + 1) / nsplit; ++m) {
    const double* rs = src + (int64_t)didx[m] * T * 8;
    for (int j = 0; j < T; ++j) term(rs + 8 * j);
  }
#pragma unroll
  for (int k = 0; k < TPT; ++k) {
    const int i = tid + k * blockDim.x;
    if (i < T)
#pragma unroll
      for (int c = 0; c < C; ++c)
        out[((size_t)split * C + c) * N + (int64_t)t * T + i] = acc[k][c] * (c < 3 ? 0.5 * kInv4PiT : kInv4PiT);
  }
}

// Absolute-coordinate source records (y, W sigma, 0, 0) of the Stokeslet's
// tree from the density [3][N].
__global__ void k_tree_src_stokes(const double* __restrict__ dens, const double* __restrict__ x,
                                  const double* __restrict__ y, const double* __restrict__ z,
                                  const double* __restrict__ w, int64_t N, double* __restrict__ src) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  const double wq = w[g];
  double* r = src + 8 * g;
  r[0] = x[g];
  r[1] = y[g];
  r[2] = z[g];
  r[3] = wq * dens[g];
  r[4] = wq * dens[N + g];
  r[5] = wq * dens[2 * N + g];
  r[6] = 0.0;
  r[7] = 0.0;
}

// Absolute-coordinate source records of the tree for S' (x, y, z, W sigma)
// and D' (x, y, z, W mu nu, 0, 0): the layouts of the single and double
// layers' records, so their proxy charges serve unchanged.
template <int OP>
__global__ void k_tree_src_normal(const double* __restrict__ dens, const double* __restrict__ x,
                                  const double* __restrict__ y, const double* __restrict__ z,
                                  const double* __restrict__ nx, const double* __restrict__ ny,
                                  const double* __restrict__ nz, const double* __restrict__ w, int64_t N,
                                  double* __restrict__ src) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  const double q = w[g] * dens[g];
  if (OP == SBIE_OP_SP) {
    double* r = src + 4 * g;
    r[0] = x[g];
    r[1] = y[g];
    r[2] = z[g];
    r[3] = q;
  } else {
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

inline unsigned cdiv_t(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

template <int OP, int TPT>
void launch_eval(sbie_geom* g, hipStream_t s, int threads) {
  const FarTree& tr = *g->tree;
  const int n3 = (tr.order + 1) * (tr.order + 1) * (tr.order + 1);
  hipLaunchKernelGGL((k_tree_eval<OP, TPT>), dim3(g->M * g->nsplit), dim3(threads), 0, s, g->d_x, g->d_y, g->d_z,
                     g->d_src, tr.d_q, tr.d_pptr, tr.d_pidx, tr.d_dptr, tr.d_didx, g->T, (n3 + 3) & ~3, g->nsplit,
                     g->N, g->d_partial);
}

template <int OP, int TPT>
void launch_eval_normal(sbie_geom* g, hipStream_t s, int threads) {
  const FarTree& tr = *g->tree;
  const int n3 = (tr.order + 1) * (tr.order + 1) * (tr.order + 1);
  hipLaunchKernelGGL((k_tree_eval_normal<OP, TPT>), dim3(g->M * g->nsplit), dim3(threads), 0, s, g->d_x, g->d_y,
                     g->d_z, g->d_nx, g->d_ny, g->d_nz, g->d_src, tr.d_q, tr.d_pptr, tr.d_pidx, tr.d_dptr, tr.d_didx,
                     g->T, (n3 + 3) & ~3, g->nsplit, g->N, g->d_partial);
}

template <int C, int TPT>
void launch_eval_stokes(sbie_geom* g, const double* prox, hipStream_t s, int threads) {
  const FarTree& tr = *g->tree;
  const int n3 = (tr.order + 1) * (tr.order + 1) * (tr.order + 1);
  hipLaunchKernelGGL((k_tree_eval_stokes<C, TPT>), dim3(g->M * g->nsplit), dim3(threads), 0, s, g->d_x, g->d_y,
                     g->d_z, g->d_src, prox, tr.d_pptr, tr.d_pidx, tr.d_dptr, tr.d_didx, g->T, (n3 + 3) & ~3,
                     g->nsplit, g->N, g->d_stk_part);
}

template <bool DIP>
void launch_eval_x3(sbie_geom* g, hipStream_t s) {
  const FarTree& tr = *g->tree;
  const int n3 = (tr.order + 1) * (tr.order + 1) * (tr.order + 1);
  const int T = g->T, T16 = (T + 15) / 16, threads = 64 * std::min(16, (T16 + 3) / 4);
  hipLaunchKernelGGL((k_tree_eval_x3<DIP>), dim3(g->M * g->nsplit), dim3(threads), 24 * T, s, g->d_x, g->d_y,
                     g->d_z, g->d_part, tr.d_box, tr.d_pptr, tr.d_pidx, tr.d_dptr, tr.d_didx,
                     reinterpret_cast<const u4*>(tr.d_prec), tr.d_q32, reinterpret_cast<const u4*>(tr.d_pdrec),
                     reinterpret_cast<const u4*>(tr.d_srec), tr.d_sq32, T, T16, (n3 + 15) / 16, g->nsplit, g->N,
                     g->d_partial);
}

template <int TPT, bool ADD>
void launch_eval32_d(sbie_geom* g, hipStream_t s, int threads) {
  const FarTree& tr = *g->tree;
  const int n3 = (tr.order + 1) * (tr.order + 1) * (tr.order + 1);
  hipLaunchKernelGGL((k_tree_eval32_d<TPT, ADD>), dim3(g->M * g->nsplit), dim3(threads), 0, s, g->d_x, g->d_y,
                     g->d_z, tr.d_src32, g->d_part, tr.d_q, tr.d_pptr, tr.d_pidx, tr.d_dptr, tr.d_didx, g->T,
                     (n3 + 3) & ~3, g->nsplit, g->N, g->d_partial);
}

}  // namespace

void free_tree(sbie_geom* g) {
  if (!g->tree) return;
  if (g->tree->blk && g->tree->blk_owned) (void)hipFree(g->tree->blk);
  delete g->tree;
  g->tree = nullptr;
}

sbie_status build_tree(sbie_geom* g, double theta, int order, int leaf, const TreeAlloc* alloc) {
  const int M = g->M, T = g->T, words = g->excl_words;
  std::vector<uint32_t> excl((size_t)M * words);
  SBIE_HIP(hipSetDevice(g->ctx->device));
  // every copy on the geometry's stream: a copy on the legacy stream would
  // wait for (and, under another thread's graph capture, fail on) other streams
  const hipStream_t cs = g->ctx->stream;
  SBIE_HIP(hipMemcpyAsync(excl.data(), g->d_excl, sizeof(uint32_t) * excl.size(), hipMemcpyDeviceToHost, cs));
  SBIE_HIP(hipStreamSynchronize(cs));
  std::vector<double> centers(3 * (size_t)M), radii(M);
  for (int i = 0; i < M; ++i) {
    for (int d = 0; d < 3; ++d) centers[3 * i + d] = g->h_part[i].c[d];
    radii[i] = 0.5 * g->h_part[i].diam;
  }
  TreePlan plan;
  sbie_status st = plan_tree(M, T, centers.data(), radii.data(), excl.data(), words, theta, order, leaf, &plan);
  if (st != SBIE_OK) return st;
  // only the clusters some target takes through proxies need device data
  std::vector<int> slot(plan.nc, -1), used;
  for (int32_t& c : plan.pidx) {
    if (slot[c] < 0) {
      slot[c] = (int)used.size();
      used.push_back(c);
    }
    c = slot[c];
  }
  const int nu = (int)used.size();
  const int n3 = (order + 1) * (order + 1) * (order + 1);
  std::vector<double> box(6 * (size_t)std::max(nu, 1));
  std::vector<int32_t> piece, cptr(nu + 1, 0);
  for (int u = 0; u < nu; ++u) {
    for (int w = 0; w < 6; ++w) box[6 * (size_t)u + w] = plan.box[6 * (size_t)used[u] + w];
    const int f = plan.first[used[u]], cnt = plan.count[used[u]];
    for (int o = 0; o < cnt; o += kChargeParts) {
      piece.push_back(u);
      piece.push_back(f + o);
      piece.push_back(std::min(kChargeParts, cnt - o));
    }
    cptr[u + 1] = (int32_t)(piece.size() / 3);
  }
  const int npiece = (int)(piece.size() / 3);
  if (piece.empty()) piece.assign(3, 0);
  if (plan.pidx.empty()) plan.pidx.push_back(0);
  if (plan.didx.empty()) plan.didx.push_back(0);
  free_tree(g);
  FarTree* tr = new FarTree();
  g->tree = tr;
  tr->theta = theta;
  tr->nc = plan.nc;
  tr->order = order;
  tr->leaf = leaf;
  tr->nused = nu;
  tr->n_proxy = plan.pptr[M];
  tr->n_direct = plan.dptr[M];
  tr->proxy_evals = tr->n_proxy * (int64_t)n3 * T;
  tr->direct_evals = tr->n_direct * (int64_t)T * T;
  for (int u = 0; u < nu; ++u) tr->charge_evals += (int64_t)plan.count[used[u]] * T * n3;
  tr->npiece = npiece;
  // one device block: boxes, member ranges, the permutation, the lists and
  // the proxy charges
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t sz_box = al(sizeof(double) * box.size()), sz_piece = al(sizeof(int32_t) * piece.size());
  const size_t sz_cptr = al(sizeof(int32_t) * cptr.size());
  const size_t sz_perm = al(sizeof(int32_t) * M), sz_ptr = al(sizeof(int64_t) * (M + 1));
  const size_t sz_pidx = al(sizeof(int32_t) * plan.pidx.size()), sz_didx = al(sizeof(int32_t) * plan.didx.size());
  const size_t sz_q = al(sizeof(double) * 4 * (size_t)std::max(nu, 1) * ((n3 + 3) & ~3));
  const size_t sz_qp = al(sizeof(double) * 3 * (size_t)std::max(npiece, 1) * n3);  // 3: dipole moments
  const int n3b = (n3 + 15) / 16, T16 = (T + 15) / 16;
  const size_t sz_prec = al(sizeof(uint32_t) * 256 * (size_t)std::max(nu, 1) * n3b);
  const size_t sz_srec = al(sizeof(uint32_t) * 256 * (size_t)M * T16);
  const size_t sz_q32 = al(sizeof(float) * 16 * (size_t)std::max(nu, 1) * n3b);
  const size_t sz_sq32 = al(sizeof(float) * 16 * (size_t)M * T16);
  const size_t sz_s32 = al(sizeof(float) * 8 * (size_t)g->N);
  const size_t total = sz_box + sz_piece + sz_cptr + sz_perm + 2 * sz_ptr + sz_pidx + sz_didx + sz_q + sz_qp +
                       2 * sz_prec + sz_srec + sz_q32 + sz_sq32 + sz_s32;
  if (alloc) {
    tr->blk = alloc->fn(alloc->ctx, total);
    tr->blk_owned = false;
    if (!tr->blk) {
      free_tree(g);
      set_error("no device memory for the tree");
      return SBIE_E_BUDGET;
    }
  } else if (hipMalloc(&tr->blk, total) != hipSuccess) {
    (void)hipGetLastError();
    free_tree(g);
    return SBIE_E_NOMEM;
  }
  char* p = tr->blk;
  auto take = [&](size_t sz) {
    char* q = p;
    p += sz;
    return q;
  };
  tr->d_box = reinterpret_cast<double*>(take(sz_box));
  tr->d_piece = reinterpret_cast<int32_t*>(take(sz_piece));
  tr->d_cptr = reinterpret_cast<int32_t*>(take(sz_cptr));
  tr->d_perm = reinterpret_cast<int32_t*>(take(sz_perm));
  tr->d_pptr = reinterpret_cast<int64_t*>(take(sz_ptr));
  tr->d_dptr = reinterpret_cast<int64_t*>(take(sz_ptr));
  tr->d_pidx = reinterpret_cast<int32_t*>(take(sz_pidx));
  tr->d_didx = reinterpret_cast<int32_t*>(take(sz_didx));
  tr->d_q = reinterpret_cast<double*>(take(sz_q));
  tr->d_qpart = reinterpret_cast<double*>(take(sz_qp));
  tr->d_prec = reinterpret_cast<uint32_t*>(take(sz_prec));
  tr->d_pdrec = reinterpret_cast<uint32_t*>(take(sz_prec));
  tr->d_srec = reinterpret_cast<uint32_t*>(take(sz_srec));
  tr->d_q32 = reinterpret_cast<float*>(take(sz_q32));
  tr->d_sq32 = reinterpret_cast<float*>(take(sz_sq32));
  tr->d_src32 = reinterpret_cast<float*>(take(sz_s32));
  tr->bytes = total;
  // the host arrays outlive the copies: the guard, destroyed first, waits for them
  struct StreamGuard {
    hipStream_t s;
    ~StreamGuard() { (void)hipStreamSynchronize(s); }
  } guard{cs};
  SBIE_HIP(hipMemcpyAsync(tr->d_box, box.data(), sizeof(double) * box.size(), hipMemcpyHostToDevice, cs));
  SBIE_HIP(hipMemcpyAsync(tr->d_piece, piece.data(), sizeof(int32_t) * piece.size(), hipMemcpyHostToDevice, cs));
  SBIE_HIP(hipMemcpyAsync(tr->d_cptr, cptr.data(), sizeof(int32_t) * cptr.size(), hipMemcpyHostToDevice, cs));
  SBIE_HIP(hipMemcpyAsync(tr->d_perm, plan.perm.data(), sizeof(int32_t) * M, hipMemcpyHostToDevice, cs));
  SBIE_HIP(hipMemcpyAsync(tr->d_pptr, plan.pptr.data(), sizeof(int64_t) * (M + 1), hipMemcpyHostToDevice, cs));
  SBIE_HIP(hipMemcpyAsync(tr->d_dptr, plan.dptr.data(), sizeof(int64_t) * (M + 1), hipMemcpyHostToDevice, cs));
  SBIE_HIP(hipMemcpyAsync(tr->d_pidx, plan.pidx.data(), sizeof(int32_t) * plan.pidx.size(), hipMemcpyHostToDevice,
                          cs));
  SBIE_HIP(hipMemcpyAsync(tr->d_didx, plan.didx.data(), sizeof(int32_t) * plan.didx.size(), hipMemcpyHostToDevice,
                          cs));
  // the mixed path's geometric records
  const hipStream_t s = g->ctx->stream;
  if (nu > 0)
    hipLaunchKernelGGL(k_tree_proxy_records, dim3(cdiv_t((int64_t)nu * 16 * n3b, 256)), dim3(256), 0, s, tr->d_box,
                       nu, order, n3b, reinterpret_cast<u4*>(tr->d_prec));
  hipLaunchKernelGGL(k_tree_node_records, dim3(cdiv_t((int64_t)M * 16 * T16, 256)), dim3(256), 0, s, g->d_x, g->d_y,
                     g->d_z, g->d_part, M, T, T16, reinterpret_cast<u4*>(tr->d_srec));
  SBIE_HIP(hipGetLastError());
  SBIE_HIP(hipStreamSynchronize(s));
  return SBIE_OK;
}

// Far field of the Stokes single layer (C = 3) or with its pressure (C = 4)
// through the tree into the nsplit partial slices of d_stk_part, in FP64 for
// either precision.  The records overwrite d_src (the Laplace operators'
// records, unused by the Stokes path); the vector-charge table takes the
// memory of the mixed double layer's dipole records (8 doubles per proxy fit
// its 16 words per proxy).
sbie_status far_tree_stokes(sbie_geom* g, int C, const double* d_dens, hipStream_t s) {
  const FarTree& tr = *g->tree;
  const int T = g->T;
  const int n3 = (tr.order + 1) * (tr.order + 1) * (tr.order + 1), n3p = (n3 + 3) & ~3;
  double* prox = reinterpret_cast<double*>(tr.d_pdrec);
  hipLaunchKernelGGL(k_tree_src_stokes, dim3(cdiv_t(g->N, 256)), dim3(256), 0, s, d_dens, g->d_x, g->d_y, g->d_z,
                     g->d_w, g->N, g->d_src);
  SBIE_HIP(hipGetLastError());
  if (tr.nused > 0) {
    hipLaunchKernelGGL(k_tree_charges<kTreeDipoles>, dim3(tr.npiece), dim3(256), 0, s, tr.d_box, tr.d_piece,
                       tr.d_perm, g->d_src, T, tr.order, tr.d_qpart);
    SBIE_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_tree_proxies3, dim3(cdiv_t((int64_t)tr.nused * n3p, 256)), dim3(256), 0, s, tr.d_box,
                       tr.d_cptr, tr.d_qpart, tr.nused, tr.order, n3p, prox);
    SBIE_HIP(hipGetLastError());
  }
  const int tpt = T <= 1024 ? 1 : (T <= 2048 ? 2 : 3);
  const int threads = 64 * (int)cdiv_t(cdiv_t(T, tpt), 64);
  if (C == 4) {
    if (tpt == 1) launch_eval_stokes<4, 1>(g, prox, s, threads);
    else if (tpt == 2) launch_eval_stokes<4, 2>(g, prox, s, threads);
    else launch_eval_stokes<4, 3>(g, prox, s, threads);
  } else {
    if (tpt == 1) launch_eval_stokes<3, 1>(g, prox, s, threads);
    else if (tpt == 2) launch_eval_stokes<3, 2>(g, prox, s, threads);
    else launch_eval_stokes<3, 3>(g, prox, s, threads);
  }
  SBIE_HIP(hipGetLastError());
  return SBIE_OK;
}

// Far field of S' or D' through the tree into the nsplit partial slices, in
// FP64 for either precision.  The density's records overwrite d_src, which
// the direct sums of S' and D' would read but the tree path does not.
sbie_status far_tree_normal(sbie_geom* g, int op, const double* d_dens, hipStream_t s) {
  const FarTree& tr = *g->tree;
  const int T = g->T;
  const int n3 = (tr.order + 1) * (tr.order + 1) * (tr.order + 1), n3p = (n3 + 3) & ~3;
  const bool sp = op == SBIE_OP_SP;
  if (sp)
    hipLaunchKernelGGL(k_tree_src_normal<SBIE_OP_SP>, dim3(cdiv_t(g->N, 256)), dim3(256), 0, s, d_dens, g->d_x,
                       g->d_y, g->d_z, g->d_nx, g->d_ny, g->d_nz, g->d_w, g->N, g->d_src);
  else
    hipLaunchKernelGGL(k_tree_src_normal<SBIE_OP_DP>, dim3(cdiv_t(g->N, 256)), dim3(256), 0, s, d_dens, g->d_x,
                       g->d_y, g->d_z, g->d_nx, g->d_ny, g->d_nz, g->d_w, g->N, g->d_src);
  SBIE_HIP(hipGetLastError());
  if (tr.nused > 0) {
    if (sp)
      hipLaunchKernelGGL(k_tree_charges<SBIE_OP_S>, dim3(tr.npiece), dim3(256), 0, s, tr.d_box, tr.d_piece, tr.d_perm,
                         g->d_src, T, tr.order, tr.d_qpart);
    else
      hipLaunchKernelGGL(k_tree_charges<SBIE_OP_D>, dim3(tr.npiece), dim3(256), 0, s, tr.d_box, tr.d_piece, tr.d_perm,
                         g->d_src, T, tr.order, tr.d_qpart);
    SBIE_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_tree_proxies, dim3(cdiv_t((int64_t)tr.nused * n3p, 256)), dim3(256), 0, s, tr.d_box,
                       tr.d_cptr, tr.d_qpart, tr.nused, tr.order, n3p, n3p, tr.d_q, nullptr);
    SBIE_HIP(hipGetLastError());
  }
  const int tpt = T <= 1024 ? 1 : (T <= 2048 ? 2 : 3);
  const int threads = 64 * (int)cdiv_t(cdiv_t(T, tpt), 64);
  if (sp) {
    if (tpt == 1) launch_eval_normal<SBIE_OP_SP, 1>(g, s, threads);
    else if (tpt == 2) launch_eval_normal<SBIE_OP_SP, 2>(g, s, threads);
    else launch_eval_normal<SBIE_OP_SP, 3>(g, s, threads);
  } else {
    if (tpt == 1) launch_eval_normal<SBIE_OP_DP, 1>(g, s, threads);
    else if (tpt == 2) launch_eval_normal<SBIE_OP_DP, 2>(g, s, threads);
    else launch_eval_normal<SBIE_OP_DP, 3>(g, s, threads);
  }
  SBIE_HIP(hipGetLastError());
  return SBIE_OK;
}

// Far field of S or D through the tree into the nsplit partial slices, the
// sums in FP64 or (mixed) FP32.  The source records d_src (k_prep_f64) must
// be current.
sbie_status far_tree(sbie_geom* g, int op, bool mixed, hipStream_t s) {
  const FarTree& tr = *g->tree;
  const int T = g->T, T16 = (T + 15) / 16;
  const int n3 = (tr.order + 1) * (tr.order + 1) * (tr.order + 1), n3p = (n3 + 3) & ~3, n3b = (n3 + 15) / 16;
  if (mixed) {
    if (op == SBIE_OP_S)
      hipLaunchKernelGGL(k_tree_strengths32, dim3(cdiv_t((int64_t)g->M * 16 * T16, 256)), dim3(256), 0, s, g->d_src,
                         g->M, T, T16, tr.d_sq32);
    else
      hipLaunchKernelGGL(k_tree_src32_d, dim3(cdiv_t(g->N, 256)), dim3(256), 0, s, g->d_src, g->d_part, T, g->N,
                         tr.d_src32);
    SBIE_HIP(hipGetLastError());
  }
  // the mixed double layer's proxies carry dipole moments
  const bool dip = mixed && op == SBIE_OP_D;
  if (tr.nused > 0) {
    if (op == SBIE_OP_S)
      hipLaunchKernelGGL(k_tree_charges<SBIE_OP_S>, dim3(tr.npiece), dim3(256), 0, s, tr.d_box, tr.d_piece, tr.d_perm,
                         g->d_src, T, tr.order, tr.d_qpart);
    else if (dip)
      hipLaunchKernelGGL(k_tree_charges<kTreeDipoles>, dim3(tr.npiece), dim3(256), 0, s, tr.d_box, tr.d_piece,
                         tr.d_perm, g->d_src, T, tr.order, tr.d_qpart);
    else
      hipLaunchKernelGGL(k_tree_charges<SBIE_OP_D>, dim3(tr.npiece), dim3(256), 0, s, tr.d_box, tr.d_piece, tr.d_perm,
                         g->d_src, T, tr.order, tr.d_qpart);
    SBIE_HIP(hipGetLastError());
    if (dip) {
      hipLaunchKernelGGL(k_tree_dipole_records, dim3(cdiv_t((int64_t)tr.nused * 16 * n3b, 256)), dim3(256), 0, s,
                         tr.d_box, tr.d_cptr, tr.d_qpart, tr.nused, tr.order, n3b, reinterpret_cast<u4*>(tr.d_pdrec));
    } else {
      // the mixed single layer also takes FP32 charges in 16-proxy blocks
      const bool q32 = mixed && op == SBIE_OP_S;
      const int nq = q32 ? 16 * n3b : n3p;
      hipLaunchKernelGGL(k_tree_proxies, dim3(cdiv_t((int64_t)tr.nused * nq, 256)), dim3(256), 0, s, tr.d_box,
                         tr.d_cptr, tr.d_qpart, tr.nused, tr.order, n3p, nq, tr.d_q, q32 ? tr.d_q32 : nullptr);
    }
    SBIE_HIP(hipGetLastError());
  }
  // the FP64 sums and the mixed double layer's direct sums: lanes
  // 64 * ceil(T / (64 TPT)) with the smallest TPT that fits 1024
  const int tpt = T <= 1024 ? 1 : (T <= 2048 ? 2 : 3);
  const int threads = 64 * (int)cdiv_t(cdiv_t(T, tpt), 64);
  if (mixed && op == SBIE_OP_S) {
    launch_eval_x3<false>(g, s);
  } else if (mixed) {
    launch_eval_x3<true>(g, s);
    SBIE_HIP(hipGetLastError());
    if (tpt == 1) launch_eval32_d<1, true>(g, s, threads);
    else if (tpt == 2) launch_eval32_d<2, true>(g, s, threads);
    else launch_eval32_d<3, true>(g, s, threads);
  } else if (op == SBIE_OP_S) {
    if (tpt == 1) launch_eval<SBIE_OP_S, 1>(g, s, threads);
    else if (tpt == 2) launch_eval<SBIE_OP_S, 2>(g, s, threads);
    else launch_eval<SBIE_OP_S, 3>(g, s, threads);
  } else {
    if (tpt == 1) launch_eval<SBIE_OP_D, 1>(g, s, threads);
    else if (tpt == 2) launch_eval<SBIE_OP_D, 2>(g, s, threads);
    else launch_eval<SBIE_OP_D, 3>(g, s, threads);
  }
  SBIE_HIP(hipGetLastError());
  return SBIE_OK;
}

}  // namespace sbie

extern "C" {

sbie_status sbie_geom_far_tree(sbie_geom* g, double theta, int32_t order, int32_t leaf) {
  if (!g) {
    sbie::set_error("geometry is NULL");
    return SBIE_E_INVALID;
  }
  return sbie::build_tree(g, theta, order, leaf);
}

sbie_status sbie_geom_far_tree_info(const sbie_geom* g, sbie_tree_info* info) {
  if (!g || !info) {
    sbie::set_error("geometry or info is NULL");
    return SBIE_E_INVALID;
  }
  if (!g->tree) {
    sbie::set_error("the geometry has no tree (sbie_geom_far_tree)");
    return SBIE_E_STATE;
  }
  const sbie::FarTree& t = *g->tree;
  info->clusters = t.nc;
  info->proxy_clusters = t.nused;
  info->proxy_pairs = t.n_proxy;
  info->direct_pairs = t.n_direct;
  info->proxy_evals = t.proxy_evals;
  info->direct_evals = t.direct_evals;
  info->charge_evals = t.charge_evals;
  info->device_bytes = t.bytes;
  return SBIE_OK;
}

sbie_status sbie_far_tree_plan(int32_t M, int32_t T, const double* centers, const double* radii,
                               const uint32_t* excl, int32_t words, double theta, int32_t order, int32_t leaf,
                               int32_t* n_clusters, int64_t* n_proxy, int64_t* n_direct, double* box,
                               int32_t* first, int32_t* count, int32_t* perm, int64_t* proxy_ptr,
                               int32_t* proxy_idx, int64_t* direct_ptr, int32_t* direct_idx) {
  if (!n_clusters || !n_proxy || !n_direct) {
    sbie::set_error("count pointers are NULL");
    return SBIE_E_INVALID;
  }
  sbie::TreePlan plan;
  const sbie_status st = sbie::plan_tree(M, T, centers, radii, excl, words, theta, order, leaf, &plan);
  if (st != SBIE_OK) return st;
  *n_clusters = plan.nc;
  *n_proxy = plan.pptr[M];
  *n_direct = plan.dptr[M];
  if (box) std::copy(plan.box.begin(), plan.box.end(), box);
  if (first) std::copy(plan.first.begin(), plan.first.end(), first);
  if (count) std::copy(plan.count.begin(), plan.count.end(), count);
  if (perm) std::copy(plan.perm.begin(), plan.perm.end(), perm);
  if (proxy_ptr) std::copy(plan.pptr.begin(), plan.pptr.end(), proxy_ptr);
  if (proxy_idx) std::copy(plan.pidx.begin(), plan.pidx.end(), proxy_idx);
  if (direct_ptr) std::copy(plan.dptr.begin(), plan.dptr.end(), direct_ptr);
  if (direct_idx) std::copy(plan.didx.begin(), plan.didx.end(), direct_idx);
  return SBIE_OK;
}

}  // extern "C"
