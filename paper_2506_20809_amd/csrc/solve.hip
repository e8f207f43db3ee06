// Boundary integral equations of Section 5.1 solved with GMRES: the completed
// double-layer Dirichlet problem (sigma/2 + D[sigma] + C[sigma] = f, Eq.
// (testprob), with the point completion of Eq. (completion) or the
// single-layer completion, scaled per particle by the eta table of Section
// 5.2) and the single-layer Neumann problem (-rho/2 + S'[rho] = g for
// u = S+[rho], Eq. (neusol)).  Every vector operation runs in the kernels below
// on the caller's stream; the host keeps only the small Hessenberg
// least-squares problem of GMRES.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "sbie_internal.h"

namespace sbie {

namespace {

constexpr int kBlock = 256;
inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

// Fixed-order block reduction of 256 values in LDS (deterministic).
__device__ inline double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  return sh[0];
}

// q_i = eta_i * int_{Gamma_i} sigma dS (quadrature weights W), one block per particle.
__global__ __launch_bounds__(kBlock) void k_particle_integrals(const double* __restrict__ sigma,
                                                               const double* __restrict__ w,
                                                               const double* __restrict__ eta, int T,
                                                               double* __restrict__ q) {
  __shared__ double sh[kBlock];
  const int i = blockIdx.x;
  double acc = 0.0;
  for (int t = threadIdx.x; t < T; t += kBlock) acc = fma(w[(size_t)i * T + t], sigma[(size_t)i * T + t], acc);
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) q[i] = eta[i] * s;
}

// sigma scaled per particle by eta (input of the single-layer completion).
__global__ void k_scale_particles(const double* __restrict__ sigma, const double* __restrict__ eta, int T,
                                  int64_t N, double* __restrict__ out) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < N) out[g] = eta[g / T] * sigma[g];
}

// out = sigma/2 + dl + C[sigma]: the point completion sums q_i/|x - c_i| over
// particles in ascending order; the single-layer completion adds sl.
__global__ void k_completed(const double* __restrict__ sigma, const double* __restrict__ dl,
                            const double* __restrict__ sl, const double* __restrict__ q,
                            const Particle* __restrict__ part, const double* __restrict__ x,
                            const double* __restrict__ y, const double* __restrict__ z, int M, int64_t N,
                            double* __restrict__ out) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  double c = 0.0;
  if (sl) {
    c = sl[g];
  } else {
    const double xg = x[g], yg = y[g], zg = z[g];
    for (int i = 0; i < M; ++i) {
      const double dx = xg - part[i].c[0], dy = yg - part[i].c[1], dz = zg - part[i].c[2];
      c += q[i] / sqrt(fma(dz, dz, fma(dy, dy, dx * dx)));
    }
  }
  out[g] = 0.5 * sigma[g] + dl[g] + c;
}

// Partial dot products of w with vectors V[0..k-1] (rows of length N): one
// partial per (vector, block), written to part[j][block].
__global__ __launch_bounds__(kBlock) void k_dots_partial(const double* __restrict__ V, const double* __restrict__ w,
                                                         int64_t N, int nblk, double* __restrict__ part) {
  __shared__ double sh[kBlock];
  const int j = blockIdx.y;
  const double* v = V + (size_t)j * N;
  double acc = 0.0;
  for (int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x; g < N; g += (int64_t)nblk * kBlock)
    acc = fma(v[g], w[g], acc);
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) part[(size_t)j * nblk + blockIdx.x] = s;
}

// h[j] = sum over blocks of part[j][*], in block order.
__global__ void k_dots_finish(const double* __restrict__ part, int nblk, int k, double* __restrict__ h) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += part[(size_t)j * nblk + b];
  h[j] = s;
}

// w -= sum_j h[j] V[j] (j ascending).
__global__ void k_sub_combination(const double* __restrict__ V, const double* __restrict__ h, int k, int64_t N,
                                  double* __restrict__ w) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  double s = w[g];
  for (int j = 0; j < k; ++j) s = fma(-h[j], V[(size_t)j * N + g], s);
  w[g] = s;
}

// out = a * v + out
__global__ void k_axpy(const double* __restrict__ v, double a, int64_t N, double* __restrict__ out) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < N) out[g] = fma(a, v[g], out[g]);
}

// out = a * v
__global__ void k_scale(const double* __restrict__ v, double a, int64_t N, double* __restrict__ out) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < N) out[g] = a * v[g];
}

// x = sum_j y[j] V[j] (j ascending)
__global__ void k_combination(const double* __restrict__ V, const double* __restrict__ y, int k, int64_t N,
                              double* __restrict__ x) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  double s = 0.0;
  for (int j = 0; j < k; ++j) s = fma(y[j], V[(size_t)j * N + g], s);
  x[g] = s;
}

struct DevBuf {
  double* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

sbie_status dev_alloc(DevBuf& b, size_t count) {
  if (hipMalloc((void**)&b.p, count * sizeof(double)) != hipSuccess) {
    b.p = nullptr;
    (void)hipGetLastError();
    set_error("device allocation of " + std::to_string(count * sizeof(double)) + " bytes for the solve failed");
    return SBIE_E_NOMEM;
  }
  return SBIE_OK;
}

// Dot products of w with V[0..k-1] into host h (one synchronisation).
sbie_status dots(const double* V, const double* w, int k, int64_t N, double* part, int nblk, double* dh,
                 double* h, hipStream_t s) {
  hipLaunchKernelGGL(k_dots_partial, dim3(nblk, k), dim3(kBlock), 0, s, V, w, N, nblk, part);
  SBIE_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_dots_finish, dim3(cdiv(k, 64)), dim3(64), 0, s, part, nblk, k, dh);
  SBIE_HIP(hipGetLastError());
  SBIE_HIP(hipMemcpyAsync(h, dh, sizeof(double) * k, hipMemcpyDeviceToHost, s));
  SBIE_HIP(hipStreamSynchronize(s));
  return SBIE_OK;
}

}  // namespace

double completion_eta(const Particle& P, int completion) {
  const double R = std::fmax(P.A, P.C) / std::fmin(P.A, P.C);
  const double eps = 1.0 / R;
  const bool prolate = P.C > P.A;
  if (completion == SBIE_COMPLETE_POINT) {
    if (!prolate && R > 3.0) return 0.06;
    double area;
    if (prolate) {
      const double e = std::sqrt(1.0 - (P.A / P.C) * (P.A / P.C));
      area = 2.0 * kPi * P.A * P.A * (1.0 + P.C / (P.A * e) * std::asin(e));
    } else {
      const double e = std::sqrt(1.0 - (P.C / P.A) * (P.C / P.A));
      area = 2.0 * kPi * P.A * P.A * (1.0 + (1.0 - e * e) / e * std::atanh(e));
    }
    return eps / area;
  }
  if (prolate) return R <= 3.0 ? 0.5 : 1.0 / (2.0 * eps * std::log(1.0 / eps));
  return R <= 3.0 ? 1.0 / (4.0 * eps) + 0.25 : 1.0;
}

// K[sigma] into d_out; d_tmp [3][N] work space.
sbie_status apply_completed(sbie_geom* g, int prec, int completion, const double* d_eta, const double* d_sigma,
                            double* d_out, double* d_tmp, hipStream_t s) {
  const int64_t N = g->N;
  double* dl = d_tmp;
  double* scaled = d_tmp + N;
  double* slo = d_tmp + 2 * N;
  sbie_status st = apply_laplace(g, SBIE_OP_D, prec, d_sigma, dl, s, SBIE_PARTS_ALL, false);
  if (st != SBIE_OK) return st;
  const double* sl = nullptr;
  if (completion == SBIE_COMPLETE_SINGLE) {
    hipLaunchKernelGGL(k_scale_particles, dim3(cdiv(N, kBlock)), dim3(kBlock), 0, s, d_sigma, d_eta, g->T, N,
                       scaled);
    SBIE_HIP(hipGetLastError());
    st = apply_laplace(g, SBIE_OP_S, prec, scaled, slo, s, SBIE_PARTS_ALL, false);
    if (st != SBIE_OK) return st;
    sl = slo;
  } else {
    hipLaunchKernelGGL(k_particle_integrals, dim3(g->M), dim3(kBlock), 0, s, d_sigma, g->d_w, d_eta, g->T,
                       g->d_qint);
    SBIE_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_completed, dim3(cdiv(N, kBlock)), dim3(kBlock), 0, s, d_sigma, dl, sl, g->d_qint,
                     g->d_part, g->d_x, g->d_y, g->d_z, g->M, N, d_out);
  SBIE_HIP(hipGetLastError());
  return SBIE_OK;
}

// GMRES without restart from x = 0 for A x = f, A given by matvec(in, out);
// classical Gram-Schmidt applied twice, in the kernels above.
template <typename Matvec>
sbie_status gmres(int64_t N, Matvec&& matvec, const double* d_f, double* d_x, double tol, int maxit, int* iters,
                  double* relres, hipStream_t s) {
  const int nblk = (int)std::min<int64_t>(1024, (N + kBlock - 1) / kBlock);
  DevBuf V, w, part, dh;
  sbie_status st;
  if ((st = dev_alloc(V, (size_t)(maxit + 1) * N)) != SBIE_OK) return st;
  if ((st = dev_alloc(w, N)) != SBIE_OK) return st;
  if ((st = dev_alloc(part, (size_t)(maxit + 1) * nblk)) != SBIE_OK) return st;
  if ((st = dev_alloc(dh, maxit + 1)) != SBIE_OK) return st;
  std::vector<double> H((size_t)(maxit + 1) * maxit, 0.0), cs(maxit), sn(maxit), gv(maxit + 1, 0.0);
  std::vector<double> h1(maxit + 1), h2(maxit + 1);
  auto Hc = [&](int r, int c) -> double& { return H[(size_t)r * maxit + c]; };
  // beta = ||f||, V[0] = f / beta
  double beta2 = 0.0;
  if ((st = dots(d_f, d_f, 1, N, part.p, nblk, dh.p, &beta2, s)) != SBIE_OK) return st;
  const double beta = std::sqrt(beta2);
  *iters = 0;
  *relres = 0.0;
  if (beta == 0.0) {
    hipLaunchKernelGGL(k_scale, dim3(cdiv(N, kBlock)), dim3(kBlock), 0, s, d_f, 0.0, N, d_x);
    SBIE_HIP(hipGetLastError());
    SBIE_HIP(hipStreamSynchronize(s));
    return SBIE_OK;
  }
  hipLaunchKernelGGL(k_scale, dim3(cdiv(N, kBlock)), dim3(kBlock), 0, s, d_f, 1.0 / beta, N, V.p);
  SBIE_HIP(hipGetLastError());
  gv[0] = beta;
  int k = 0;
  double res = 1.0;
  while (k < maxit) {
    // w = A V[k]
    if ((st = matvec(V.p + (size_t)k * N, w.p)) != SBIE_OK) return st;
    // classical Gram-Schmidt, twice
    if ((st = dots(V.p, w.p, k + 1, N, part.p, nblk, dh.p, h1.data(), s)) != SBIE_OK) return st;
    hipLaunchKernelGGL(k_sub_combination, dim3(cdiv(N, kBlock)), dim3(kBlock), 0, s, V.p, dh.p, k + 1, N, w.p);
    SBIE_HIP(hipGetLastError());
    if ((st = dots(V.p, w.p, k + 1, N, part.p, nblk, dh.p, h2.data(), s)) != SBIE_OK) return st;
    hipLaunchKernelGGL(k_sub_combination, dim3(cdiv(N, kBlock)), dim3(kBlock), 0, s, V.p, dh.p, k + 1, N, w.p);
    SBIE_HIP(hipGetLastError());
    for (int j = 0; j <= k; ++j) Hc(j, k) = h1[j] + h2[j];
    double nn = 0.0;
    if ((st = dots(w.p, w.p, 1, N, part.p, nblk, dh.p, &nn, s)) != SBIE_OK) return st;
    const double hn = std::sqrt(nn);
    Hc(k + 1, k) = hn;
    if (hn > 0.0) {
      hipLaunchKernelGGL(k_scale, dim3(cdiv(N, kBlock)), dim3(kBlock), 0, s, w.p, 1.0 / hn, N,
                         V.p + (size_t)(k + 1) * N);
      SBIE_HIP(hipGetLastError());
    }
    // Givens rotations on the new Hessenberg column
    for (int j = 0; j < k; ++j) {
      const double t = cs[j] * Hc(j, k) + sn[j] * Hc(j + 1, k);
      Hc(j + 1, k) = -sn[j] * Hc(j, k) + cs[j] * Hc(j + 1, k);
      Hc(j, k) = t;
    }
    const double r = std::hypot(Hc(k, k), Hc(k + 1, k));
    cs[k] = Hc(k, k) / r;
    sn[k] = Hc(k + 1, k) / r;
    Hc(k, k) = r;
    Hc(k + 1, k) = 0.0;
    gv[k + 1] = -sn[k] * gv[k];
    gv[k] = cs[k] * gv[k];
    ++k;
    res = std::fabs(gv[k]) / beta;
    if (res <= tol || hn == 0.0) break;
  }
  // y from the triangular system, x = V y
  std::vector<double> yv(k);
  for (int i = k - 1; i >= 0; --i) {
    double t = gv[i];
    for (int j = i + 1; j < k; ++j) t -= Hc(i, j) * yv[j];
    yv[i] = t / Hc(i, i);
  }
  SBIE_HIP(hipMemcpyAsync(dh.p, yv.data(), sizeof(double) * k, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_combination, dim3(cdiv(N, kBlock)), dim3(kBlock), 0, s, V.p, dh.p, k, N, d_x);
  SBIE_HIP(hipGetLastError());
  SBIE_HIP(hipStreamSynchronize(s));
  *iters = k;
  *relres = res;
  return SBIE_OK;
}

sbie_status solve_completed(sbie_geom* g, int prec, int completion, const double* d_eta, const double* d_f,
                            double* d_sigma, double tol, int maxit, int* iters, double* relres, hipStream_t s) {
  DevBuf tmp;
  sbie_status st = dev_alloc(tmp, 3 * (size_t)g->N);
  if (st != SBIE_OK) return st;
  auto K = [&](const double* in, double* out) {
    return apply_completed(g, prec, completion, d_eta, in, out, tmp.p, s);
  };
  return gmres(g->N, K, d_f, d_sigma, tol, maxit, iters, relres, s);
}

// -rho/2 + S'[rho]
sbie_status apply_neumann(sbie_geom* g, int prec, const double* d_rho, double* d_out, hipStream_t s) {
  sbie_status st = apply_laplace(g, SBIE_OP_SP, prec, d_rho, d_out, s, SBIE_PARTS_ALL, false);
  if (st != SBIE_OK) return st;
  hipLaunchKernelGGL(k_axpy, dim3(cdiv(g->N, kBlock)), dim3(kBlock), 0, s, d_rho, -0.5, g->N, d_out);
  SBIE_HIP(hipGetLastError());
  return SBIE_OK;
}

sbie_status solve_neumann(sbie_geom* g, int prec, const double* d_g, double* d_rho, double tol, int maxit,
                          int* iters, double* relres, hipStream_t s) {
  auto A = [&](const double* in, double* out) { return apply_neumann(g, prec, in, out, s); };
  return gmres(g->N, A, d_g, d_rho, tol, maxit, iters, relres, s);
}

}  // namespace sbie

using namespace sbie;

namespace {

// Device copy of the per-particle scalings: the table values, or the caller's.
sbie_status upload_eta(sbie_geom* g, int completion, const double* eta, hipStream_t s) {
  std::vector<double> e(g->M);
  for (int i = 0; i < g->M; ++i) e[i] = eta ? eta[i] : completion_eta(g->h_part[i], completion);
  SBIE_HIP(hipMemcpyAsync(g->d_eta, e.data(), sizeof(double) * g->M, hipMemcpyHostToDevice, s));
  SBIE_HIP(hipStreamSynchronize(s));
  return SBIE_OK;
}

sbie_status check_args(sbie_geom* g, sbie_precision prec, sbie_completion c) {
  if (!g) {
    set_error("geometry is NULL");
    return SBIE_E_INVALID;
  }
  if (prec != SBIE_FP64 && prec != SBIE_MIXED) {
    set_error("unknown precision");
    return SBIE_E_INVALID;
  }
  if (c != SBIE_COMPLETE_POINT && c != SBIE_COMPLETE_SINGLE) {
    set_error("unknown completion");
    return SBIE_E_INVALID;
  }
  return SBIE_OK;
}

}  // namespace

extern "C" {

sbie_status sbie_completion_eta(const sbie_geom* g, sbie_completion c, double* eta) {
  if (!g || !eta) {
    set_error("geometry or eta is NULL");
    return SBIE_E_INVALID;
  }
  if (c != SBIE_COMPLETE_POINT && c != SBIE_COMPLETE_SINGLE) {
    set_error("unknown completion");
    return SBIE_E_INVALID;
  }
  for (int i = 0; i < g->M; ++i) eta[i] = completion_eta(g->h_part[i], c);
  return SBIE_OK;
}

sbie_status sbie_apply_completed(sbie_geom* g, sbie_precision prec, sbie_completion c, const double* eta,
                                 const double* sigma, double* out, void* stream, uint32_t flags) {
  sbie_status st = check_args(g, prec, c);
  if (st != SBIE_OK) return st;
  if (!sigma || !out) {
    set_error("sigma or out is NULL");
    return SBIE_E_INVALID;
  }
  SBIE_HIP(hipSetDevice(g->ctx->device));
  hipStream_t s = stream ? (hipStream_t)stream : g->ctx->stream;
  const int64_t N = g->N;
  const bool devptr = (flags & SBIE_DEVICE_PTRS) != 0;
  if ((st = upload_eta(g, c, eta, s)) != SBIE_OK) return st;
  DevBuf tmp, io;
  if ((st = dev_alloc(tmp, 3 * (size_t)N)) != SBIE_OK) return st;
  const double* din = sigma;
  double* dout = out;
  if (!devptr) {
    if ((st = dev_alloc(io, 2 * (size_t)N)) != SBIE_OK) return st;
    SBIE_HIP(hipMemcpyAsync(io.p, sigma, sizeof(double) * N, hipMemcpyHostToDevice, s));
    din = io.p;
    dout = io.p + N;
  }
  if ((st = apply_completed(g, (int)prec, (int)c, g->d_eta, din, dout, tmp.p, s)) != SBIE_OK) return st;
  if (!devptr) SBIE_HIP(hipMemcpyAsync(out, dout, sizeof(double) * N, hipMemcpyDeviceToHost, s));
  // the work buffers are freed on return: wait for the stream first
  SBIE_HIP(hipStreamSynchronize(s));
  return sbie_geom_sync(g, s);
}

sbie_status sbie_solve_completed(sbie_geom* g, sbie_precision prec, sbie_completion c, const double* eta,
                                 const double* f, double* sigma, double tol, int32_t maxit, int32_t* iters,
                                 double* relres, void* stream, uint32_t flags) {
  sbie_status st = check_args(g, prec, c);
  if (st != SBIE_OK) return st;
  if (!f || !sigma || !iters || !relres) {
    set_error("f, sigma, iters or relres is NULL");
    return SBIE_E_INVALID;
  }
  if (maxit < 1 || maxit > 4096 || !(tol > 0.0)) {
    set_error("maxit must be in [1, 4096] and tol > 0");
    return SBIE_E_INVALID;
  }
  SBIE_HIP(hipSetDevice(g->ctx->device));
  hipStream_t s = stream ? (hipStream_t)stream : g->ctx->stream;
  const int64_t N = g->N;
  const bool devptr = (flags & SBIE_DEVICE_PTRS) != 0;
  if ((st = upload_eta(g, c, eta, s)) != SBIE_OK) return st;
  DevBuf io;
  const double* df = f;
  double* ds = sigma;
  if (!devptr) {
    if ((st = dev_alloc(io, 2 * (size_t)N)) != SBIE_OK) return st;
    SBIE_HIP(hipMemcpyAsync(io.p, f, sizeof(double) * N, hipMemcpyHostToDevice, s));
    df = io.p;
    ds = io.p + N;
  }
  int it = 0;
  double res = 0.0;
  if ((st = solve_completed(g, (int)prec, (int)c, g->d_eta, df, ds, tol, maxit, &it, &res, s)) != SBIE_OK)
    return st;
  if (!devptr) SBIE_HIP(hipMemcpyAsync(sigma, ds, sizeof(double) * N, hipMemcpyDeviceToHost, s));
  SBIE_HIP(hipStreamSynchronize(s));
  *iters = it;
  *relres = res;
  return sbie_geom_sync(g, s);
}

sbie_status sbie_solve_neumann(sbie_geom* g, sbie_precision prec, const double* data, double* rho, double tol,
                               int32_t maxit, int32_t* iters, double* relres, void* stream, uint32_t flags) {
  if (!g) {
    set_error("geometry is NULL");
    return SBIE_E_INVALID;
  }
  if (prec != SBIE_FP64 && prec != SBIE_MIXED) {
    set_error("unknown precision");
    return SBIE_E_INVALID;
  }
  if (!data || !rho || !iters || !relres) {
    set_error("data, rho, iters or relres is NULL");
    return SBIE_E_INVALID;
  }
  if (maxit < 1 || maxit > 4096 || !(tol > 0.0)) {
    set_error("maxit must be in [1, 4096] and tol > 0");
    return SBIE_E_INVALID;
  }
  SBIE_HIP(hipSetDevice(g->ctx->device));
  hipStream_t s = stream ? (hipStream_t)stream : g->ctx->stream;
  const int64_t N = g->N;
  const bool devptr = (flags & SBIE_DEVICE_PTRS) != 0;
  DevBuf io;
  const double* dd = data;
  double* dr = rho;
  sbie_status st;
  if (!devptr) {
    if ((st = dev_alloc(io, 2 * (size_t)N)) != SBIE_OK) return st;
    SBIE_HIP(hipMemcpyAsync(io.p, data, sizeof(double) * N, hipMemcpyHostToDevice, s));
    dd = io.p;
    dr = io.p + N;
  }
  int it = 0;
  double res = 0.0;
  if ((st = solve_neumann(g, (int)prec, dd, dr, tol, maxit, &it, &res, s)) != SBIE_OK) return st;
  if (!devptr) SBIE_HIP(hipMemcpyAsync(rho, dr, sizeof(double) * N, hipMemcpyDeviceToHost, s));
  SBIE_HIP(hipStreamSynchronize(s));
  *iters = it;
  *relres = res;
  return sbie_geom_sync(g, s);
}

}  // extern "C"
