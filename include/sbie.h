/*
 * sbie.h -- C ABI of the MI355X spheroidal boundary-integral operator library.
 *
 * The library applies the Laplace single-layer S[sigma] and double-layer D[mu]
 * operators of Crowder, Li, Corona and Veerapaneni (arXiv 2506.20809) to a
 * suspension of prolate and oblate spheroids, following the paper's problem
 * setup (Section 4, "Problem setup": evaluation of u = sum_i K_i[sigma_i] at all
 * particle nodes) and Algorithm 1 (self, near and far split).  Particles are
 * given as the paper's numerical examples give them (Section 5.1): shape,
 * centre and a unit quaternion rotating a reference configuration.
 *
 * Conventions (all arrays are plain C arrays, row-major, contiguous):
 *  - Particle i: centre c_i (3 doubles), unit quaternion q_i = (w,x,y,z)
 *    rotating body coordinates into lab coordinates, equatorial semi-axis A_i
 *    and polar semi-axis C_i along the body z axis.  C > A is prolate, C < A
 *    oblate (Section 2.1, Table 1).
 *  - Order p, grid of (p+1) Gauss-Legendre nodes in v (ascending) times 2p+2
 *    equispaced azimuthal nodes phi_k = 2 pi k / (2p+2) per particle, so
 *    T = (p+1)(2p+2) nodes per particle and N = M*T nodes in all.  Node index
 *    g = i*T + j*(2p+2) + k (particle, v index, phi index).
 *  - Densities and potentials are [nrhs][N] doubles in node order.
 *  - The double-layer value on the surface is the principal value (the average
 *    of the one-sided spectra of Theorem 1); add +-mu/2 for the one-sided limits.
 *  - eta is the near/far parameter of Section 4.1: target particle j is in the
 *    near field of source i iff the surface distance d_ij < eta * diam_i, with
 *    diam_i twice the largest semi-axis of particle i.
 *
 * Ownership: the caller owns every density and potential buffer, on the host or
 * (flag SBIE_DEVICE_PTRS) on the device; the library never frees them.  Handles
 * are released only by their destroy call.  Particle arrays are copied at
 * create time.
 *
 * Errors: every entry point returns an sbie_status; nothing throws across the
 * ABI.  sbie_last_error() returns a thread-local message for the last failure.
 *
 * Threads: one geometry must not be used by concurrent sbie_apply calls; the
 * served-mode calls (sbie_server_*, sbie_session_*, sbie_wait) are thread-safe.
 */
#ifndef SBIE_H
#define SBIE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SBIE_OK = 0,
  SBIE_E_INVALID = -1,    /* bad argument (p out of [1,32], M < 1, non-unit quaternion, ...) */
  SBIE_E_DEGENERATE = -2, /* |A - C| <= 1e-6 max(A,C) or a semi-axis <= 0 (no focal length) */
  SBIE_E_OVERLAP = -3,    /* two particles touch or overlap (d_ij <= 0) */
  SBIE_E_NOMEM = -4,      /* device or host allocation failed */
  SBIE_E_BUDGET = -5,     /* a served session can never fit the memory budget */
  SBIE_E_DEVICE = -6,     /* a HIP call failed; see sbie_last_error() */
  SBIE_E_TIMEOUT = -7,    /* sbie_wait timed out */
  SBIE_E_NUMERIC = -8,    /* continued fraction for Q_N/Q_{N-1} did not converge */
  SBIE_E_STATE = -9       /* call not valid in the current state */
} sbie_status;

typedef enum {
  SBIE_OP_S = 0,       /* Laplace single layer, Eq. (SLP), Theorem 2 */
  SBIE_OP_D = 1,       /* Laplace double layer, Eq. (DLP), Theorem 1 */
  SBIE_OP_STOKES_S = 2, /* Stokes single layer through Laplace potentials, Eq. (stokes); nrhs = 3 */
  SBIE_OP_SP = 3,       /* S': derivative of the single layer along the target's outward normal,
                           principal value on the surface (Section 3.3, Theorem 3) */
  SBIE_OP_DP = 4,       /* D': derivative of the double layer along the target's outward normal
                           (continuous across the surface; Section 3.3) */
  SBIE_OP_STOKES_SP = 5, /* Stokes single layer and its pressure, kernel (1/4pi) r/|r|^3 (Section 4.3):
                           nrhs = 3, potential [4][N], the fourth row the pressure, on the surface
                           its exterior limit */
  SBIE_OP_STOKES_D = 6  /* Stokes double layer 3/(4pi) int (r.mu)(r.nu) r/|r|^5 with the outward normal
                           (a rigid motion gives -mu inside), principal value on the surface, through
                           Laplace double and single layers (Section 4.3); nrhs = 3 */
} sbie_op;

typedef enum {
  SBIE_FP64 = 0, /* every part in double precision */
  SBIE_MIXED = 1 /* far-field sums, transform and near contractions in FP32 (compensated
                    tile accumulation); frame map and Q_n^m recurrence in FP64 */
} sbie_precision;

/* sbie_apply flags */
#define SBIE_DEVICE_PTRS 0x1u  /* density/potential are device pointers */
#define SBIE_TIMING 0x2u       /* record per-part device times (sbie_geom_timing) */
#define SBIE_PARTS_SELF 0x10u  /* include the self interaction (self step of Algorithm 1) */
#define SBIE_PARTS_NEAR 0x20u  /* include the near field (near-field step of Algorithm 1) */
#define SBIE_PARTS_FAR 0x40u   /* include the far field (far-field step of Algorithm 1) */
#define SBIE_PARTS_ALL 0x70u   /* 0 also means all parts */
#define SBIE_FAR_TREE 0x100u   /* S, D, S', D', the Stokes single layer and its pressure: the
                                  far field from the geometry's tree (sbie_geom_far_tree)
                                  instead of the direct sum */
#define SBIE_INPUT_COEFFS 0x200u /* S or D: the input is the coefficients [nrhs][M][(p+1)^2] of
                                  Algorithm 1's forward transform (layout of sbie_transform:
                                  l = n^2 + n + m; for S the modified-basis coefficients of
                                  sqrt(u0^2 -+ v^2) sigma), so the transform step is skipped
                                  ("if not provided").  The far field's nodal density is their
                                  synthesis at the nodes (divided by sqrt(u0^2 -+ v^2) for S). */

typedef struct sbie_ctx sbie_ctx;
typedef struct sbie_geom sbie_geom;

/* Per-part device times, milliseconds, averaged over the timed applies (one
   per right-hand side) since the previous sbie_geom_timing call; measured with
   HIP events.  The near field runs on a second stream of the geometry,
   concurrently with the self interaction and the far field, so the parts
   overlap and do not add up to total_ms.  far_kernel_ms is the far-field
   direct-sum kernel alone. */
typedef struct {
  double prep_ms;
  double transform_ms; /* forward transform, spectra scaling, inverse transform */
  double near_ms;      /* near field, on the geometry's second stream */
  double far_kernel_ms;
  double assemble_ms;  /* from the later of the near and far ends to the end */
  double total_ms;     /* whole apply on the caller's stream */
  int64_t far_pairs;   /* far-field node pairs evaluated per right-hand side */
  int64_t near_evals;  /* near-field (pair, target) evaluations per right-hand side */
  int64_t count;       /* number of timed applies averaged */
  int64_t far_launches; /* launches of the pair-symmetric far-field kernel per apply (it runs over
                           chunks of partner offsets; 0 when the direct pair kernel is not used) */
} sbie_timing;

/* Create a context on HIP device `device` (a stream is created for synchronous
   calls).  *out receives the handle. */
sbie_status sbie_ctx_create(int device, sbie_ctx** out);
/* Release a context.  Geometries created on it stay valid: while any is live
   the context is only marked, and it is released with the last of them. */
void sbie_ctx_destroy(sbie_ctx* ctx);

/* Build a geometry (Algorithm 1 setup: nodes, weights, normals, spectra of
   Theorems 1-2, exact distances and the near/far split of Section 4.1).
   centers [M][3], quats [M][4] (w,x,y,z), A [M], C [M] are host arrays.
   Errors: SBIE_E_INVALID (M < 1, p outside [1,32], eta < 0, non-finite value,
   | |q| - 1 | > 1e-6), SBIE_E_DEGENERATE, SBIE_E_OVERLAP, SBIE_E_NUMERIC,
   SBIE_E_NOMEM, SBIE_E_DEVICE. */
sbie_status sbie_geom_create(sbie_ctx* ctx, const double* centers, const double* quats,
                             const double* A, const double* C, int32_t M, int32_t p,
                             double eta, sbie_geom** out);
void sbie_geom_destroy(sbie_geom* g);

int64_t sbie_geom_num_nodes(const sbie_geom* g);      /* N = M (p+1)(2p+2) */
int64_t sbie_geom_num_near_pairs(const sbie_geom* g); /* directed (source, target) pairs */
uint64_t sbie_geom_footprint_bytes(const sbie_geom* g); /* device memory held by the geometry */

/* Copy nodes [N][3], unit outward normals [N][3] and quadrature weights [N]
   (Gauss-Legendre x trapezoid weights times the area element of Table 2) to
   host arrays; any pointer may be NULL. */
sbie_status sbie_geom_nodes(const sbie_geom* g, double* xyz, double* nrm, double* w);

/* Directed near pairs (source i, target j), sorted by target then source;
   at most cap are written, *count receives the total. */
sbie_status sbie_geom_near_pairs(const sbie_geom* g, int32_t* src, int32_t* dst,
                                 int64_t cap, int64_t* count);

/* Apply S, D, S', D' (or the Stokes single layer) to nrhs densities:
   potential[r][g] = sum over particles of K[density[r]] at node g.  For S'
   and D' the target normal is the outward normal at node g; the near field
   uses the gradient of each neighbour's exterior expansion (Eq.
   (dSLevalformula) and its analogue for D), the far field the differentiated
   kernels.
   S (either precision) and D (FP64) with nrhs >= 2 nodal densities (and at
   least 32 nodes per particle, without SBIE_TIMING, SBIE_FAR_TREE or
   SBIE_INPUT_COEFFS) run in groups of up to four that share the far field's
   pair work: one reciprocal distance per node pair serves every density of
   the group in both directions.  The results agree with one-density applies to rounding (the
   far sums are taken in another order), not bitwise.  Work buffers for this
   are allocated on first use and held with the geometry.
   stream: a hipStream_t, or NULL for the context stream with the call
   returning after completion.  With a non-NULL stream and SBIE_DEVICE_PTRS the
   call is asynchronous on that stream.  flags: SBIE_DEVICE_PTRS, SBIE_TIMING,
   SBIE_PARTS_*, SBIE_FAR_TREE, SBIE_INPUT_COEFFS (S and D: density holds
   coefficients, [nrhs][M][(p+1)^2]).  Errors: SBIE_E_INVALID (op, precision,
   nrhs outside [1,16], Stokes with nrhs != 3, SBIE_INPUT_COEFFS with another
   operator), SBIE_E_NUMERIC, SBIE_E_DEVICE, SBIE_E_NOMEM. */
sbie_status sbie_apply(sbie_geom* g, sbie_op op, sbie_precision prec, int32_t nrhs,
                       const double* density, double* potential, void* stream,
                       uint32_t flags);

/* Wait for `stream` (NULL: the context stream) and return the sticky device
   status of the applies made on this geometry since the last check:
   SBIE_E_OVERLAP if a near-field target was found inside its source (checked
   first: the recurrences fail there too), SBIE_E_NUMERIC if a continued
   fraction did not converge, else SBIE_OK.  Asynchronous
   applies report their numerical failures here. */
sbie_status sbie_geom_sync(sbie_geom* g, void* stream);

/* Test control of the error path of Section 2.3's Legendre algorithm: caps
   the steps of the near-field backward recurrence (the continued fraction for
   Q_N/Q_{N-1}, evaluated bottom-up) past degree p+1 at `steps`, 8 <= steps <=
   100000 (the default and the largest cap).  A near-field evaluation that
   needs more steps runs with the cap and is reported as SBIE_E_NUMERIC by the
   next sbie_geom_sync (or by a synchronous apply); every kernel completes
   normally.  Takes effect for the applies and target evaluations issued after
   it on the geometry's context stream (synchronises that stream).
   SBIE_E_INVALID for a NULL geometry or a cap outside the range. */
sbie_status sbie_geom_set_depth_cap(sbie_geom* g, int32_t steps);

/* Forward transform step of Algorithm 1 alone: the (p+1)^2 real
   spheroidal-harmonic coefficients per particle, index n^2+n+m, of the
   density (op = SBIE_OP_D) or of sqrt(u0^2 -+ v^2) times the density
   (op = SBIE_OP_S, the modified basis of Section 3.2).  density [nrhs][N],
   coefs [nrhs][M][(p+1)^2]; pointers as in sbie_apply (flag SBIE_DEVICE_PTRS). */
sbie_status sbie_transform(sbie_geom* g, sbie_op op, int32_t nrhs, const double* density,
                           double* coefs, void* stream, uint32_t flags);

/* Copy the per-particle spectra to a host array [M][(p+1)(p+2)/2][4] indexed
   by h = n(n+1)/2 + m (m >= 0): D principal value, D exterior limit (Theorem 1),
   S on the surface in the modified basis (Theorem 2), and 1/Q_n^m(z0) (for
   oblates the real function i^{n+1} Q_n^m(i u0)). */
sbie_status sbie_geom_spectra(const sbie_geom* g, double* out);

/* Average per-part times of the applies made with SBIE_TIMING since the
   previous call (waits for them to finish), then starts a new window.
   SBIE_E_STATE if there was no timed apply. */
sbie_status sbie_geom_timing(sbie_geom* g, sbie_timing* out);

/* Particle-to-target evaluation (Section 4, the particle-to-target variant of
   Algorithm 1): S or D (op) of the nodal density at npts points pts [npts][3]
   outside every particle, into val [npts] and, if grad is not NULL, the
   gradient grad [npts][3] (Eq. (dSLevalformula) and its analogue for D).
   Each (point, source particle) pair is near iff the exact distance from the
   point to the source surface is below eta * diam(source): near sources
   contribute their exterior expansion, far ones the smooth quadrature.  With
   SBIE_MIXED only the far sums run in FP32; the transform and the expansions
   are FP64 in both precisions.
   Pointers as in sbie_apply; work buffers are allocated for the call, which
   returns after completion.  SBIE_E_OVERLAP if a point lies inside (or on) a
   particle, SBIE_E_INVALID for other ops or npts outside [0, 2^31]. */
sbie_status sbie_eval_targets(sbie_geom* g, sbie_op op, sbie_precision prec, const double* density,
                              int64_t npts, const double* pts, double* val, double* grad, void* stream,
                              uint32_t flags);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid allocation):
   sbie_eval_targets with its work buffers (target coordinates, near masks,
   near values, far partials, sort keys and order) in a static device array of
   SBIE_TARGETS_SCRATCH_BYTES on each GPU, held until the process ends; the
   call allocates nothing.  density, pts, val and grad are device pointers
   (SBIE_DEVICE_PTRS is required); the results equal sbie_eval_targets's (the
   same kernels in the same order).  The call returns after completion.  Every
   call on one GPU shares that GPU's array: calls that overlap on one GPU (from
   several threads or streams) race.  Errors as sbie_eval_targets, plus
   SBIE_E_INVALID without SBIE_DEVICE_PTRS and SBIE_E_BUDGET when the work
   buffers for npts points on this geometry exceed the array (about
   (64 + 4 ceil(M/32)) bytes per point plus up to 34 MB of far partials). */
#define SBIE_TARGETS_SCRATCH_BYTES (64u << 20)
sbie_status sbie_eval_targets_noalloc(sbie_geom* g, sbie_op op, sbie_precision prec, const double* density,
                                      int64_t npts, const double* pts, double* val, double* grad, void* stream,
                                      uint32_t flags);

/* ---------------------------------------------------------------- completed double-layer solve

   The exterior Dirichlet problem of Section 5.1 in the completed double-layer
   form, K[sigma] = sigma/2 + D[sigma] + C[sigma] = f on the surfaces
   (Eq. (testprob)), with either completion, scaled per particle by eta_i:
     SBIE_COMPLETE_POINT:  C[sigma](x) = sum_i eta_i |x - c_i|^-1 int_{Gamma_i} sigma dS
                           (Eq. (completion), without a 1/(4 pi) factor, as printed);
     SBIE_COMPLETE_SINGLE: C[sigma] = sum_i eta_i S_i[sigma_i].
   eta: host array [M], or NULL for the values of the eta table of Section 5.2
   (elongation eps = minor/major semi-axis; the point completion uses
   eps/area, and 0.06 for oblates of aspect ratio above 3; the single layer
   uses 1/2 or 1/(2 eps log(1/eps)) for prolates, 1/(4 eps) + 1/4 or 1 for
   oblates, split at aspect ratio 3).  Densities and data are [N] doubles in
   node order, host or (SBIE_DEVICE_PTRS) device pointers; the calls return
   after completion. */
typedef enum { SBIE_COMPLETE_POINT = 0, SBIE_COMPLETE_SINGLE = 1 } sbie_completion;

/* The table's eta for every particle of g (host array [M]). */
sbie_status sbie_completion_eta(const sbie_geom* g, sbie_completion c, double* eta);

/* out = K[sigma]. */
sbie_status sbie_apply_completed(sbie_geom* g, sbie_precision prec, sbie_completion c, const double* eta,
                                 const double* sigma, double* out, void* stream, uint32_t flags);

/* GMRES without restart from sigma = 0 until ||f - K sigma|| <= tol ||f|| (the
   Arnoldi residual estimate) or maxit iterations (1..4096); the Krylov
   basis ((maxit+1) N doubles) is allocated for the call and freed on return.
   The geometry's completion scalings are overwritten by each completed apply
   or solve: calls on one geometry must not overlap.  *iters and *relres
   receive the iteration count and the final estimate.  With SBIE_MIXED the
   attainable residual is limited by the operator's ~1e-6 accuracy. */
sbie_status sbie_solve_completed(sbie_geom* g, sbie_precision prec, sbie_completion c, const double* eta,
                                 const double* f, double* sigma, double tol, int32_t maxit, int32_t* iters,
                                 double* relres, void* stream, uint32_t flags);

/* The exterior Neumann problem of Section 5.1 with the single-layer
   representation u = S+[rho] (Eq. (neusol)): GMRES, as sbie_solve_completed,
   for -rho/2 + S'[rho] = data, S' the principal value (Theorem 3) and data the
   outward normal derivative of u on the surfaces. */
sbie_status sbie_solve_neumann(sbie_geom* g, sbie_precision prec, const double* data, double* rho, double tol,
                               int32_t maxit, int32_t* iters, double* relres, void* stream, uint32_t flags);

/* ---------------------------------------------------------------- served mode

   Many independent operator sessions sharing one GPU, for boundary integral
   equation solvers that issue a stream of applies per suspension (the Krylov
   iterations of Section 4 and Section 5.2).  A session is a suspension (geometry, p, eta) with an operator
   and a precision; its applies run in submission order.  The server admits a
   session when one of its lanes is idle and the session's device bytes
   (sbie_session_bytes) fit in the server's HBM arena: first come, first
   served, except that a smaller later session may pass a waiting one at most
   SBIE_MAX_PASS times in a row.  An admitted session keeps its geometry, near
   lists and spectra resident until it is closed; each lane has its own stream,
   so the kernels of concurrent sessions interleave on the device.  With
   SBIE_SERVER_GRAPHS each session's apply is captured once as a HIP graph and
   replayed.  With SBIE_SERVER_BATCH a lane may hold up to four sessions of
   one operator (S or D), precision and order, each of at most 65536 nodes
   with a far field that fits one pair-kernel launch (p >= 3, every partner
   offset within the reverse-sum budget), once no lane is empty, and runs the
   front applies of its sessions
   together: each session's transform and self part, one near-field launch and
   one far-field launch over all of them, each session's assembly.  Results are
   bitwise those of sbie_apply on the same geometry.  With SBIE_SERVER_TREE
   an S or D session of at least 64 particles also builds the tree far field
   of sbie_geom_far_tree (theta 0.6, order 10, leaf 2) in the arena when it
   is admitted, and its applies equal sbie_apply with SBIE_FAR_TREE on that
   tree; when the arena has no room for the tree the session keeps the
   direct far field.  Such sessions do not batch.

   All server calls are thread-safe; the handles of one session must not be
   used after sbie_session_close. */

typedef struct sbie_server sbie_server;
typedef struct sbie_session sbie_session;

#define SBIE_SERVER_GRAPHS 0x100u
#define SBIE_SERVER_BATCH 0x200u
#define SBIE_SERVER_TREE 0x400u
#define SBIE_MAX_PASS 8

typedef struct {
  double open_us;    /* session opened (request arrival), server clock in microseconds */
  double admit_us;   /* session admitted to a lane */
  double ready_us;   /* its geometry built (and graph captured) */
  double submit_us;  /* this apply submitted */
  double start_us;   /* this apply started on its lane */
  double end_us;     /* this apply finished (results in the caller's buffer) */
  int64_t session;   /* session id (1, 2, ... in open order) */
  int32_t lane;
  int32_t status;    /* sbie_status of the apply */
} sbie_apply_stats;

typedef struct {
  uint64_t budget_bytes;    /* arena size */
  uint64_t in_use_bytes;    /* held by admitted sessions now */
  uint64_t peak_bytes;      /* largest in_use_bytes so far */
  int64_t pending;          /* sessions waiting for admission */
  int64_t active;           /* admitted, not yet closed */
  int64_t admitted;         /* sessions admitted so far */
  int64_t passed;           /* admissions that passed a waiting earlier session */
  int64_t waited;           /* sessions that could not be admitted at once */
  int64_t applies;          /* applies completed */
  int32_t lanes;
  int32_t graphs;           /* 1 if applies are replayed as HIP graphs */
  int64_t batched;          /* applies completed inside batched launches */
  int64_t tree_sessions;    /* sessions whose far field runs through a tree */
} sbie_server_info;

/* Device bytes a session of M particles at order p holds while admitted:
   its geometry (setup tables, near lists, work buffers; Stokes buffers for
   SBIE_OP_STOKES_S) plus input and output buffers of nrhs x N doubles (nrhs = 3
   for Stokes, else 1).  0 for invalid sizes. */
uint64_t sbie_session_bytes(int32_t M, int32_t p, sbie_op op);

/* Start a server on ctx's device with max_sessions lanes (1..64), each with a
   stream and a host thread, and an arena of hbm_budget_bytes of device memory
   allocated now.  flags: SBIE_SERVER_GRAPHS, SBIE_SERVER_BATCH, SBIE_SERVER_TREE.  Errors: SBIE_E_INVALID,
   SBIE_E_NOMEM, SBIE_E_DEVICE. */
sbie_status sbie_server_create(sbie_ctx* ctx, int32_t max_sessions, uint64_t hbm_budget_bytes,
                               uint32_t flags, sbie_server** out);

/* Finish every queued apply of the admitted sessions, close all sessions
   (pending ones fail their applies with SBIE_E_STATE), join the lanes and free
   the arena.  Waiting for tickets after this call is invalid. */
void sbie_server_destroy(sbie_server* srv);

/* Open a session (returns at once; admission and the geometry build happen on
   a lane).  Arguments as sbie_geom_create plus op and precision; the particle
   arrays are copied.  Errors now: SBIE_E_INVALID, SBIE_E_DEGENERATE,
   SBIE_E_BUDGET (the session can never fit the arena), SBIE_E_STATE (server
   stopping).  Errors of the build (SBIE_E_OVERLAP, SBIE_E_NUMERIC, ...) are
   reported by each of the session's applies. */
sbie_status sbie_session_open(sbie_server* srv, const double* centers, const double* quats,
                              const double* A, const double* C, int32_t M, int32_t p, double eta,
                              sbie_op op, sbie_precision prec, sbie_session** out);

/* Queue one apply: density and potential are [nrhs][N] (nrhs as in
   sbie_session_bytes), host arrays or, with SBIE_DEVICE_PTRS, device arrays
   whose producing work has completed (the lanes use their own streams); both
   must stay valid until sbie_wait returns for *ticket, when the potential is
   complete on the device.  Errors: SBIE_E_INVALID, SBIE_E_STATE (session
   closing). */
sbie_status sbie_session_apply(sbie_session* s, const double* density, double* potential,
                               uint32_t flags, uint64_t* ticket);

/* Close a session after its queued applies; the handle is invalid afterwards
   and its device bytes return to the arena when the last apply finishes. */
sbie_status sbie_session_close(sbie_session* s);

/* Wait up to timeout_us microseconds (< 0: no limit) for an apply; returns its
   status and, if stats is not NULL, its timeline.  A ticket is consumed by a
   successful wait.  SBIE_E_TIMEOUT if it is still running (the ticket stays
   valid); SBIE_E_INVALID for an unknown ticket. */
sbie_status sbie_wait(sbie_server* srv, uint64_t ticket, int64_t timeout_us, sbie_apply_stats* stats);

sbie_status sbie_server_get_info(sbie_server* srv, sbie_server_info* out);

const char* sbie_status_str(sbie_status s);
const char* sbie_last_error(void);

/* ------------------------------------------------------------------------
   Tree far field.  Section 4.1 sums the far field with a fast multipole
   method; here a barycentric Lagrange treecode (Wang, Krasny and Tlupova,
   2020) takes that role for S and D.  Source particles are clustered by
   recursive bisection of their centres (at most `leaf` particles per leaf).
   A cluster whose box has half-diagonal rho and centre b is taken at target
   particle t (centre c_t, bounding radius r_t = half its diam) through
   proxies, the (order+1)^3 Chebyshev points of the second kind in its box
   with charges from the barycentric Lagrange interpolation of the kernel in
   the source point, when rho + r_t < theta |c_t - b|, the cluster has more
   nodes than proxies and none of its particles is excluded for t (self or
   near, Section 4.1).  Otherwise its children are visited, and at a leaf its
   particles are summed directly unless excluded.  Each far (target, source)
   particle pair is covered exactly once.  S' and D' (Theorem 3) use the same
   proxies, the single layer's charges resp. the double layer's, with the
   kernel's derivative along the target normal; the Stokes single layer (and
   its pressure) takes vector charges, the interpolated W sigma, with the
   Stokeslet (Section 4.3).  These sum in FP64 in either precision.  For S and D the sums follow the apply's
   precision: FP64, or in SBIE_MIXED FP32 terms added four at a time into
   FP64 sums (squared distances on the matrix cores; the double layer's
   proxies then carry its dipole moments, interpolated, since its proxy
   charges cancel within a cluster).  The interpolation error falls geometrically in `order` at a rate
   set by theta.  Measured against the direct FP64 far sum at 512 and 4096
   spheroids (p = 16), relative l2, FP64 sums: theta = 0.5, order = 8: S 2e-8
   to 5e-8, D 3e-7 to 4e-7; theta = 0.6, order = 10: S 7e-9 to 2e-8, D 9e-8 to
   2e-7 at about the same cost; mixed sums at theta = 0.6, order = 10: S 1.2e-7
   to 1.8e-7, D 2.4e-7 to 4.8e-7.
   ------------------------------------------------------------------------ */

/* Build (or rebuild) the tree of a geometry; applies with SBIE_FAR_TREE use
   it.  theta in (0, 1), order in [2, 12], leaf >= 1.  The device memory (boxes,
   lists, proxy charges) is held until the geometry is destroyed or the tree
   rebuilt.  Errors: SBIE_E_INVALID, SBIE_E_NOMEM, SBIE_E_DEVICE. */
sbie_status sbie_geom_far_tree(sbie_geom* g, double theta, int32_t order, int32_t leaf);

typedef struct {
  int32_t clusters;        /* clusters of the tree */
  int32_t proxy_clusters;  /* clusters some target takes through proxies */
  int64_t proxy_pairs;     /* (target particle, cluster) pairs through proxies */
  int64_t direct_pairs;    /* (target particle, source particle) pairs summed directly */
  int64_t proxy_evals;     /* kernel evaluations per apply, targets x proxies */
  int64_t direct_evals;    /* kernel evaluations per apply, targets x direct source nodes */
  int64_t charge_evals;    /* (source node, proxy) terms of the proxy charges per apply */
  uint64_t device_bytes;   /* device memory held by the tree */
} sbie_tree_info;

/* Sizes of the geometry's tree.  SBIE_E_STATE when none was built. */
sbie_status sbie_geom_far_tree_info(const sbie_geom* g, sbie_tree_info* info);

/* The tree plan alone, on the host (no device): M particles with centres
   [M][3] and bounding radii [M], T nodes per particle, exclusion bit rows
   excl [M][words] (bit s of row t set iff source particle s is excluded for
   target t; words >= ceil(M/32)).  Writes the counts; when the array
   pointers are non-NULL also (sized by a first call with NULL arrays):
   box [n_clusters][6] (lo, hi), first/count [n_clusters] (a cluster is
   perm[first .. first+count)), perm [M], proxy_ptr/direct_ptr [M+1] and
   proxy_idx [n_proxy] (cluster ids), direct_idx [n_direct] (particle ids),
   each list by target particle.  Clusters are numbered depth-first, children
   after their parent.  Errors: SBIE_E_INVALID. */
sbie_status sbie_far_tree_plan(int32_t M, int32_t T, const double* centers, const double* radii,
                               const uint32_t* excl, int32_t words, double theta, int32_t order,
                               int32_t leaf, int32_t* n_clusters, int64_t* n_proxy, int64_t* n_direct,
                               double* box, int32_t* first, int32_t* count, int32_t* perm,
                               int64_t* proxy_ptr, int32_t* proxy_idx, int64_t* direct_ptr,
                               int32_t* direct_idx);

#ifdef __cplusplus
}
#endif

#endif /* SBIE_H */
