// C ABI of include/sbie.h: argument checks, handle lifetime, host/device
// staging and error mapping.  Every entry point returns a status; no C++
// exception crosses the boundary.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "sbie_internal.h"

namespace sbie {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }

sbie_status device_error(hipError_t e, const char* what) {
  g_last_error = std::string("HIP error '") + hipGetErrorString(e) + "' in " + what;
  return SBIE_E_DEVICE;
}

namespace {

sbie_status invalid(const std::string& msg) {
  set_error(msg);
  return SBIE_E_INVALID;
}

void free_geom(sbie_geom* g) {
  if (!g) return;
  sbie::free_tree(g);
  if (g->multi) {
    if (g->multi->blk) (void)hipFree(g->multi->blk);
    delete g->multi;
  }
  if (g->blk && g->blk_owned) (void)hipFree(g->blk);
  if (g->stk_blk) (void)hipFree(g->stk_blk);
  if (g->sdl_blk) (void)hipFree(g->sdl_blk);
  if (g->side) {
    (void)hipStreamSynchronize(g->side);
    (void)hipStreamDestroy(g->side);
  }
  if (g->ev_fork) (void)hipEventDestroy(g->ev_fork);
  if (g->ev_join) (void)hipEventDestroy(g->ev_join);
  for (auto& set : g->timing.sets)
    for (hipEvent_t e : set)
      if (e) (void)hipEventDestroy(e);
  delete g;
}

}  // namespace

sbie_status check_particles(const double* centers, const double* quats, const double* A, const double* C,
                            int32_t M, int32_t p, double eta, std::vector<Particle>* out) {
  if (!centers || !quats || !A || !C) return invalid("particle array is NULL");
  if (M < 1) return invalid("M must be >= 1");
  if (p < 1 || p > kMaxP) return invalid("p must be in [1, 32]");
  if (!(eta >= 0.0) || !std::isfinite(eta)) return invalid("eta must be finite and >= 0");
  out->assign(M, Particle{});
  for (int i = 0; i < M; ++i) {
    const double* c = centers + 3 * i;
    const double* q = quats + 4 * i;
    bool finite = std::isfinite(A[i]) && std::isfinite(C[i]);
    for (int k = 0; k < 3; ++k) finite = finite && std::isfinite(c[k]);
    for (int k = 0; k < 4; ++k) finite = finite && std::isfinite(q[k]);
    if (!finite) return invalid("non-finite particle parameter at particle " + std::to_string(i));
    const double qn = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    if (std::fabs(qn - 1.0) > 1e-6) return invalid("quaternion of particle " + std::to_string(i) + " is not unit");
    const double mx = std::fmax(A[i], C[i]);
    if (!(A[i] > 0.0) || !(C[i] > 0.0) || std::fabs(A[i] - C[i]) <= 1e-6 * mx) {
      set_error("particle " + std::to_string(i) + " is a sphere or has a non-positive semi-axis");
      return SBIE_E_DEGENERATE;
    }
    Particle& P = (*out)[i];
    std::memset(&P, 0, sizeof P);
    for (int k = 0; k < 3; ++k) P.c[k] = c[k];
    const double w = q[0] / qn, x = q[1] / qn, y = q[2] / qn, z = q[3] / qn;
    P.R[0] = 1 - 2 * (y * y + z * z);
    P.R[1] = 2 * (x * y - w * z);
    P.R[2] = 2 * (x * z + w * y);
    P.R[3] = 2 * (x * y + w * z);
    P.R[4] = 1 - 2 * (x * x + z * z);
    P.R[5] = 2 * (y * z - w * x);
    P.R[6] = 2 * (x * z - w * y);
    P.R[7] = 2 * (y * z + w * x);
    P.R[8] = 1 - 2 * (x * x + y * y);
    P.A = A[i];
    P.C = C[i];
    P.oblate = C[i] < A[i];
    P.a = P.oblate ? std::sqrt((A[i] - C[i]) * (A[i] + C[i])) : std::sqrt((C[i] - A[i]) * (C[i] + A[i]));
    P.u0 = C[i] / P.a;
    P.w0 = P.oblate ? (P.u0 * P.u0 + 1.0) : (P.u0 - 1.0) * (P.u0 + 1.0);
    P.diam = 2.0 * mx;
  }
  return SBIE_OK;
}

sbie_status make_geometry(sbie_ctx* ctx, std::vector<Particle>&& parts, int32_t p, double eta, char* blk,
                          size_t blk_bytes, bool fork_near, sbie_geom** out) {
  *out = nullptr;
  SBIE_HIP(hipSetDevice(ctx->device));
  sbie_geom* g = new (std::nothrow) sbie_geom;
  if (!g) return SBIE_E_NOMEM;
  const int M = (int)parts.size();
  g->ctx = ctx;
  g->M = M;
  g->p = p;
  g->Nphi = 2 * p + 2;
  g->T = (p + 1) * g->Nphi;
  g->K = (p + 1) * (p + 1);
  g->Kh = (p + 1) * (p + 2) / 2;
  g->N = (int64_t)M * g->T;
  g->eta = eta;
  g->h_part = std::move(parts);
  g->blk = blk;
  g->blk_bytes = blk_bytes;
  g->blk_owned = false;
  g->fork_near = fork_near;
  sbie_status st = setup_geometry(g, ctx->stream);
  if (st != SBIE_OK) {
    (void)hipStreamSynchronize(ctx->stream);
    free_geom(g);
    return st;
  }
  ++ctx->live_geoms;
  *out = g;
  return SBIE_OK;
}

void destroy_geometry(sbie_geom* g) {
  if (!g) return;
  sbie_ctx* ctx = g->ctx;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  free_geom(g);
  if (--ctx->live_geoms == 0 && ctx->closing) {
    ctx->closing = false;
    sbie_ctx_destroy(ctx);
  }
}

}  // namespace sbie

using namespace sbie;

extern "C" {

const char* sbie_status_str(sbie_status s) {
  switch (s) {
    case SBIE_OK: return "ok";
    case SBIE_E_INVALID: return "invalid argument";
    case SBIE_E_DEGENERATE: return "degenerate spheroid";
    case SBIE_E_OVERLAP: return "particles overlap";
    case SBIE_E_NOMEM: return "out of memory";
    case SBIE_E_BUDGET: return "memory budget exceeded";
    case SBIE_E_DEVICE: return "device error";
    case SBIE_E_TIMEOUT: return "timeout";
    case SBIE_E_NUMERIC: return "continued fraction did not converge";
    case SBIE_E_STATE: return "invalid state";
  }
  return "unknown status";
}

const char* sbie_last_error(void) { return g_last_error.c_str(); }

sbie_status sbie_ctx_create(int device, sbie_ctx** out) {
  if (!out) return invalid("out is NULL");
  *out = nullptr;
  int count = 0;
  SBIE_HIP(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) return invalid("no such HIP device");
  SBIE_HIP(hipSetDevice(device));
  sbie_ctx* c = new (std::nothrow) sbie_ctx;
  if (!c) return SBIE_E_NOMEM;
  c->device = device;
  hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete c;
    return device_error(e, "hipStreamCreateWithFlags");
  }
  *out = c;
  return SBIE_OK;
}

void sbie_ctx_destroy(sbie_ctx* ctx) {
  if (!ctx) return;
  if (ctx->live_geoms > 0) {
    // released with its last geometry
    ctx->closing = true;
    return;
  }
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

sbie_status sbie_geom_create(sbie_ctx* ctx, const double* centers, const double* quats, const double* A,
                             const double* C, int32_t M, int32_t p, double eta, sbie_geom** out) {
  if (!out) return invalid("out is NULL");
  *out = nullptr;
  if (!ctx) return invalid("ctx is NULL");
  std::vector<Particle> parts;
  sbie_status st = check_particles(centers, quats, A, C, M, p, eta, &parts);
  if (st != SBIE_OK) return st;
  return make_geometry(ctx, std::move(parts), p, eta, nullptr, 0, true, out);
}

void sbie_geom_destroy(sbie_geom* g) { destroy_geometry(g); }

int64_t sbie_geom_num_nodes(const sbie_geom* g) { return g ? g->N : 0; }
int64_t sbie_geom_num_near_pairs(const sbie_geom* g) { return g ? g->n_near : 0; }
uint64_t sbie_geom_footprint_bytes(const sbie_geom* g) { return g ? g->footprint : 0; }

sbie_status sbie_geom_nodes(const sbie_geom* g, double* xyz, double* nrm, double* w) {
  if (!g) return invalid("geometry is NULL");
  SBIE_HIP(hipSetDevice(g->ctx->device));
  const int64_t N = g->N;
  hipStream_t s = g->ctx->stream;
  std::string err;
  if (xyz || nrm) {
    double* tmp = new (std::nothrow) double[3 * N];
    if (!tmp) return SBIE_E_NOMEM;
    const double* src[2][3] = {{g->d_x, g->d_y, g->d_z}, {g->d_nx, g->d_ny, g->d_nz}};
    double* dst[2] = {xyz, nrm};
    for (int b = 0; b < 2; ++b) {
      if (!dst[b]) continue;
      for (int k = 0; k < 3; ++k) {
        hipError_t e = hipMemcpyAsync(tmp + k * N, src[b][k], sizeof(double) * N, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
          delete[] tmp;
          return device_error(e, "hipMemcpyAsync(nodes)");
        }
      }
      for (int64_t q = 0; q < N; ++q)
        for (int k = 0; k < 3; ++k) dst[b][3 * q + k] = tmp[k * N + q];
    }
    delete[] tmp;
  }
  if (w) {
    SBIE_HIP(hipMemcpyAsync(w, g->d_w, sizeof(double) * N, hipMemcpyDeviceToHost, s));
    SBIE_HIP(hipStreamSynchronize(s));
  }
  return SBIE_OK;
}

sbie_status sbie_geom_near_pairs(const sbie_geom* g, int32_t* src, int32_t* dst, int64_t cap, int64_t* count) {
  if (!g) return invalid("geometry is NULL");
  if (count) *count = g->n_near;
  int64_t k = 0;
  for (int j = 0; j < g->M; ++j)
    for (int s = g->h_near_ptr[j]; s < g->h_near_ptr[j + 1]; ++s, ++k) {
      if (k >= cap) continue;
      if (src) src[k] = g->h_near_src[s];
      if (dst) dst[k] = j;
    }
  return SBIE_OK;
}

sbie_status sbie_apply(sbie_geom* g, sbie_op op, sbie_precision prec, int32_t nrhs, const double* density,
                       double* potential, void* stream, uint32_t flags) {
  if (!g) return invalid("geometry is NULL");
  if (op != SBIE_OP_S && op != SBIE_OP_D && op != SBIE_OP_STOKES_S && op != SBIE_OP_SP && op != SBIE_OP_DP &&
      op != SBIE_OP_STOKES_SP && op != SBIE_OP_STOKES_D)
    return invalid("unknown operator");
  if (prec != SBIE_FP64 && prec != SBIE_MIXED) return invalid("unknown precision");
  if (nrhs < 1 || nrhs > 16) return invalid("nrhs must be in [1, 16]");
  if ((op == SBIE_OP_STOKES_S || op == SBIE_OP_STOKES_SP || op == SBIE_OP_STOKES_D) && nrhs != 3)
    return invalid("the Stokes operators take nrhs = 3");
  if (!density || !potential) return invalid("density or potential is NULL");
  SBIE_HIP(hipSetDevice(g->ctx->device));
  uint32_t parts = flags & SBIE_PARTS_ALL;
  if (parts == 0) parts = SBIE_PARTS_ALL;
  if (flags & SBIE_FAR_TREE) {
    if (op == SBIE_OP_STOKES_D) return invalid("SBIE_FAR_TREE does not apply to the Stokes double layer");
    if (!g->tree) {
      set_error("SBIE_FAR_TREE without a tree (sbie_geom_far_tree)");
      return SBIE_E_STATE;
    }
    parts |= SBIE_FAR_TREE;
  }
  const bool coef_in = (flags & SBIE_INPUT_COEFFS) != 0;
  if (coef_in) {
    if (op != SBIE_OP_S && op != SBIE_OP_D) return invalid("SBIE_INPUT_COEFFS applies to S and D only");
    parts |= SBIE_INPUT_COEFFS;
  }
  const bool devptr = (flags & SBIE_DEVICE_PTRS) != 0;
  const bool timed = (flags & SBIE_TIMING) != 0;
  hipStream_t s = stream ? (hipStream_t)stream : g->ctx->stream;
  const int64_t N = g->N;
  if (op == SBIE_OP_STOKES_D) {
    const double* din = density;
    double* dout = potential;
    if (!devptr) {
      double* io = nullptr;
      sbie_status st = stokes_dl_staging(g, &io);
      if (st != SBIE_OK) return st;
      SBIE_HIP(hipMemcpyAsync(io, density, sizeof(double) * 3 * N, hipMemcpyHostToDevice, s));
      din = io;
      dout = io + 3 * N;
    }
    sbie_status st = apply_stokes_dl(g, (int)prec, din, dout, s, parts, timed);
    if (st != SBIE_OK) return st;
    if (!devptr) SBIE_HIP(hipMemcpyAsync(potential, dout, sizeof(double) * 3 * N, hipMemcpyDeviceToHost, s));
    if (!stream || !devptr) return sbie_geom_sync(g, s);
    return SBIE_OK;
  }
  if (op == SBIE_OP_STOKES_S || op == SBIE_OP_STOKES_SP) {
    // the three components of the density in, the three velocity components
    // (and the pressure) out
    const int nout = op == SBIE_OP_STOKES_SP ? 4 : 3;
    const double* din = density;
    double* dout = potential;
    if (!devptr) {
      double* io = nullptr;
      sbie_status st = stokes_staging(g, &io);
      if (st != SBIE_OK) return st;
      SBIE_HIP(hipMemcpyAsync(io, density, sizeof(double) * 3 * N, hipMemcpyHostToDevice, s));
      din = io;
      dout = io + 3 * N;
    }
    sbie_status st = apply_stokes(g, (int)prec, din, dout, s, parts, timed, op == SBIE_OP_STOKES_SP);
    if (st != SBIE_OK) return st;
    if (!devptr) SBIE_HIP(hipMemcpyAsync(potential, dout, sizeof(double) * nout * N, hipMemcpyDeviceToHost, s));
    if (!stream || !devptr) return sbie_geom_sync(g, s);
    return SBIE_OK;
  }
  // one input: N nodal values, or M (p+1)^2 coefficients
  const int64_t nin = coef_in ? (int64_t)g->M * g->K : N;
  // several nodal densities: groups of up to four share the far field's pair
  // work (apply_laplace_multi); a last single density takes the plain apply.
  // The mixed double layer keeps one apply per density: its three-piece pair
  // kernel per density is faster than the shared kernel's FP32 products.
  const bool multi = nrhs >= 2 && !coef_in && !(parts & SBIE_FAR_TREE) && !timed && g->T >= 32 &&
                     (op == SBIE_OP_S || prec == SBIE_FP64);
  int r0 = 0;
  if (multi) {
    sbie_status st = sbie::multi_buffers(g);
    if (st != SBIE_OK) return st;
    for (; nrhs - r0 >= 2; r0 += 4) {
      const int nr = nrhs - r0 < 4 ? nrhs - r0 : 4;
      const double* din = density + (size_t)r0 * N;
      double* dout = potential + (size_t)r0 * N;
      if (!devptr) {
        double* io = g->multi->io;
        SBIE_HIP(hipMemcpyAsync(io, din, sizeof(double) * nr * N, hipMemcpyHostToDevice, s));
        din = io;
        dout = io + (size_t)4 * N;
      }
      st = sbie::apply_laplace_multi(g, (int)op, (int)prec, nr, din, dout, s, parts);
      if (st != SBIE_OK) return st;
      if (!devptr)
        SBIE_HIP(hipMemcpyAsync(potential + (size_t)r0 * N, dout, sizeof(double) * nr * N, hipMemcpyDeviceToHost, s));
    }
  }
  for (int r = r0; r < nrhs; ++r) {
    const double* din = density + (size_t)r * nin;
    double* dout = potential + (size_t)r * N;
    if (!devptr) {
      double* stage = coef_in ? g->d_coef : g->d_dens;
      SBIE_HIP(hipMemcpyAsync(stage, din, sizeof(double) * nin, hipMemcpyHostToDevice, s));
      din = stage;
      dout = g->d_out;
    }
    sbie_status st = apply_laplace(g, (int)op, (int)prec, din, dout, s, parts, timed && r == nrhs - 1);
    if (st != SBIE_OK) return st;
    if (!devptr) {
      SBIE_HIP(hipMemcpyAsync(potential + (size_t)r * N, g->d_out, sizeof(double) * N, hipMemcpyDeviceToHost, s));
    }
  }
  if (!stream || !devptr) return sbie_geom_sync(g, s);
  return SBIE_OK;
}

sbie_status sbie_geom_set_depth_cap(sbie_geom* g, int32_t steps) {
  if (!g) return invalid("geometry is NULL");
  if (steps < 8 || steps > kMaxNearDepth) return invalid("depth cap outside [8, 100000]");
  SBIE_HIP(hipSetDevice(g->ctx->device));
  SBIE_HIP(hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(g->d_status + 1), steps, 1, g->ctx->stream));
  SBIE_HIP(hipStreamSynchronize(g->ctx->stream));
  return SBIE_OK;
}

sbie_status sbie_geom_sync(sbie_geom* g, void* stream) {
  if (!g) return invalid("geometry is NULL");
  SBIE_HIP(hipSetDevice(g->ctx->device));
  hipStream_t s = stream ? (hipStream_t)stream : g->ctx->stream;
  unsigned status = 0;
  SBIE_HIP(hipMemcpyAsync(&status, g->d_status, sizeof(unsigned), hipMemcpyDeviceToHost, s));
  SBIE_HIP(hipStreamSynchronize(s));
  if (status) {
    SBIE_HIP(hipMemsetAsync(g->d_status, 0, sizeof(unsigned), s));
    SBIE_HIP(hipStreamSynchronize(s));
  }
  // a target inside its source also breaks the recurrences there: report the cause
  if (status & kStatExterior) {
    set_error("a near-field target lies inside its source spheroid");
    return SBIE_E_OVERLAP;
  }
  if (status & kStatNumeric) {
    set_error("continued fraction for Q_N/Q_{N-1} did not converge at a near-field target");
    return SBIE_E_NUMERIC;
  }
  return SBIE_OK;
}

sbie_status sbie_transform(sbie_geom* g, sbie_op op, int32_t nrhs, const double* density, double* coefs,
                           void* stream, uint32_t flags) {
  if (!g) return invalid("geometry is NULL");
  if (op != SBIE_OP_S && op != SBIE_OP_D) return invalid("transform takes SBIE_OP_S or SBIE_OP_D");
  if (nrhs < 1 || nrhs > 16) return invalid("nrhs must be in [1, 16]");
  if (!density || !coefs) return invalid("density or coefs is NULL");
  SBIE_HIP(hipSetDevice(g->ctx->device));
  const bool devptr = (flags & SBIE_DEVICE_PTRS) != 0;
  hipStream_t s = stream ? (hipStream_t)stream : g->ctx->stream;
  const int64_t N = g->N, MK = (int64_t)g->M * g->K;
  for (int r = 0; r < nrhs; ++r) {
    const double* din = density + (size_t)r * N;
    double* dout = coefs + (size_t)r * MK;
    if (!devptr) {
      SBIE_HIP(hipMemcpyAsync(g->d_dens, din, sizeof(double) * N, hipMemcpyHostToDevice, s));
      din = g->d_dens;
      dout = g->d_coef;
    }
    sbie_status st = transform_only(g, (int)op, din, dout, s);
    if (st != SBIE_OK) return st;
    if (!devptr)
      SBIE_HIP(hipMemcpyAsync(coefs + (size_t)r * MK, g->d_coef, sizeof(double) * MK, hipMemcpyDeviceToHost, s));
  }
  if (!stream || !devptr) SBIE_HIP(hipStreamSynchronize(s));
  return SBIE_OK;
}

sbie_status sbie_geom_spectra(const sbie_geom* g, double* out) {
  if (!g || !out) return invalid("NULL argument");
  SBIE_HIP(hipSetDevice(g->ctx->device));
  SBIE_HIP(hipMemcpyAsync(out, g->d_lam, sizeof(double) * (size_t)g->M * g->Kh * 4, hipMemcpyDeviceToHost,
                          g->ctx->stream));
  SBIE_HIP(hipStreamSynchronize(g->ctx->stream));
  return SBIE_OK;
}

sbie_status sbie_geom_timing(sbie_geom* g, sbie_timing* out) {
  if (!g || !out) return invalid("NULL argument");
  Timing& tm = g->timing;
  if (tm.used == 0) {
    set_error("no timed apply since the previous call");
    return SBIE_E_STATE;
  }
  SBIE_HIP(hipSetDevice(g->ctx->device));
  SBIE_HIP(hipEventSynchronize(tm.sets[tm.used - 1][5]));
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (size_t k = 0; k < tm.used; ++k) {
    hipEvent_t* ev = tm.sets[k].data();
    float ms = 0.0f, ms2 = 0.0f;
    SBIE_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
    acc[0] += ms;
    SBIE_HIP(hipEventElapsedTime(&ms, ev[1], ev[2]));
    acc[1] += ms;
    SBIE_HIP(hipEventElapsedTime(&ms, ev[6], ev[7]));  // near, on the side stream
    acc[2] += ms;
    SBIE_HIP(hipEventElapsedTime(&ms, ev[3], ev[4]));
    acc[3] += ms;
    // assembly: from the later of the far-field and near-field ends
    SBIE_HIP(hipEventElapsedTime(&ms, ev[4], ev[5]));
    SBIE_HIP(hipEventElapsedTime(&ms2, ev[7], ev[5]));
    acc[4] += ms < ms2 ? ms : ms2;
    SBIE_HIP(hipEventElapsedTime(&ms, ev[0], ev[5]));
    acc[5] += ms;
  }
  const double n = (double)tm.used;
  out->prep_ms = acc[0] / n;
  out->transform_ms = acc[1] / n;
  out->near_ms = acc[2] / n;
  out->far_kernel_ms = acc[3] / n;
  out->assemble_ms = acc[4] / n;
  out->total_ms = acc[5] / n;
  out->far_pairs = g->far_pairs;
  {
    const int pmax = (g->M - 1) / 2 + ((g->M & 1) == 0 ? 1 : 0);
    const int ks = g->rev_slots > 0 ? g->rev_slots : 1;
    out->far_launches = g->T >= 32 ? std::max(1, (pmax + ks - 1) / ks) : 0;
  }
  out->near_evals = g->n_near * (int64_t)g->T;
  out->count = (int64_t)tm.used;
  tm.used = 0;
  return SBIE_OK;
}

}  // extern "C"
