/*
 * dwsap.h -- C ABI of the MI355X (gfx950) SAP-preconditioned FGMRES-DR
 * solver for the Wilson-Dirac operator.
 *
 * Method: A. Frommer, A. Nobile, P. Zingler, "Deflation and Flexible
 * SAP-Preconditioning of GMRES in Lattice QCD Simulation", arXiv:1204.5463.
 * The library solves D x = b (Section 2) with flexible GMRES with deflated
 * restarts (Section 4, Alg. 4), right-preconditioned by the Schwarz
 * alternating procedure (Section 2, Alg. 2) whose block systems are solved
 * approximately by a fixed number of minimal-residual steps (Sections 3, 5).
 *
 * Operator (eq. 1, mass normalisation, periodic in all four directions):
 *   (D x)(n) = (4 + m0) x(n)
 *      - 1/2 sum_mu [ (1 - g_mu) U_mu(n) x(n+mu) + (1 + g_mu) U_mu(n-mu)^+ x(n-mu) ]
 * The paper's hopping-parameter form corresponds to kappa = 1/(2 (4 + m0)).
 * Gamma matrices: Euclidean chiral basis g_k = [[0, -i s_k], [i s_k, 0]]
 * (k = x, y, z), g_t = [[0, 1], [1, 0]].
 *
 * Conventions for every call:
 *   - Return value: dw_status, DW_OK (0) on success, a negative code on
 *     failure; dw_last_error() gives the calling thread's last message.
 *     No C++ exception crosses this interface.
 *   - Lattice extents L[4] = {Lx, Ly, Lz, Lt}; direction mu = 0..3 is
 *     x, y, z, t. Canonical site index n = x + Lx*(y + Ly*(z + Lz*t)).
 *   - Caller buffers are DEVICE pointers to complex128 numbers stored as
 *     interleaved (re, im) doubles:
 *       spinor fields [rhs][n][spin 4][colour 3]  (12 complex per site),
 *       gauge fields  [mu][n][a 3][b 3]           (U_mu(n)_{ab}).
 *     Caller buffers stay owned by the caller; the library never frees or
 *     retains them after a call returns (server requests excepted).
 *   - Streams: every call enqueues its work on the given HIP stream and is
 *     asynchronous unless stated otherwise. Device memory that the library
 *     needs comes from the context's allocator.
 */
#ifndef DWSAP_H
#define DWSAP_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dw_status;
enum {
  DW_OK = 0,
  DW_EINVAL = -1,    /* invalid argument: geometry, parameters, null pointer */
  DW_ENOMEM = -2,    /* device allocation failed */
  DW_EHIP = -3,      /* a HIP runtime call failed */
  DW_ENOTCONV = -4,  /* solver stopped at max_iter; x holds the last iterate */
  DW_EBUSY = -5,     /* server queue full / request not finished */
  DW_ENOTFOUND = -6  /* unknown server ticket */
};

/* Storage precision of the SAP preconditioner's fields (links and
 * spinors). Arithmetic is FP32 for F32/F16/BF16 storage and FP64 for F64. */
typedef enum { DW_PREC_F64 = 0, DW_PREC_F32 = 1, DW_PREC_F16 = 2, DW_PREC_BF16 = 3 } dw_prec;

/* Device-memory allocator. alloc returns a device pointer of at least
 * `bytes` bytes usable on `stream` (NULL on failure); release frees it. If
 * the context is created with a NULL allocator, hipMalloc/hipFree are used. */
typedef struct dw_allocator {
  void* (*alloc)(size_t bytes, hipStream_t stream, void* user);
  void (*release)(void* ptr, hipStream_t stream, void* user);
  void* user;
} dw_allocator;

typedef struct dw_ctx_s* dw_ctx;
typedef struct dw_field_s* dw_field;
typedef struct dw_server_s* dw_server;

/* SAP preconditioner parameters (Alg. 2; Sections 3 and 5).
 *   block[4]  domain extents; they must divide L and give an even number of
 *             domains per direction (Section 2, red/black colouring); they
 *             must equal the block extents the field was created with.
 *   ncycles   SAP cycles s per application (one cycle = both colours).
 *   nmr       minimal-residual steps per block solve, from y = 0 (with
 *             mr_reduction > 0: the largest number of steps).
 *   storage   dw_prec of the preconditioner's fields.
 *   mr_reduction  0: every block takes nmr steps (Section 5). In (0, 1): an
 *             inexact block solve that stops, block by block, at the first
 *             step whose residual satisfies ||rho|| <= mr_reduction ||r||
 *             (Section 3); r is the block's right-hand side. */
typedef struct sap_params {
  int32_t block[4];
  int32_t ncycles;
  int32_t nmr;
  int32_t storage;
  int32_t reserved;
  double mr_reduction;
} sap_params;

/* FGMRES-DR parameters (Alg. 4; Section 4.7).
 *   m          total basis size per cycle, including the k deflation vectors
 *              (cycles after the first perform m - k Arnoldi steps), 1..48.
 *   k          deflation space dimension, 0 <= k < m (0 = FGMRES(m)).
 *   max_iter   iteration limit; one iteration = one flexible Arnoldi step.
 *   tol        stop when ||b - D x||_2 <= tol ||b||_2 (explicit FP64 residual).
 *   restart_t  clean restart (no deflation) when ||r_explicit|| / ||r_implicit||
 *              exceeds this threshold (the paper suggests 2..10).
 *   sap        preconditioner parameters.
 *   shared_defl  multi-RHS only: 1 = once the batch's first RHS has a
 *              deflation space (D Z_k = V_{k+1} H_k from its last deflated
 *              restart), every other RHS of the lock-step batch projects its
 *              residual onto that space at each restart (minimum residual
 *              over span Z_k) and restarts with a fresh Krylov space, as in
 *              GMRES with projection; 0 = independent FGMRES-DR solves. Not
 *              in the paper; the projection cannot raise the residual.
 *   flags      DW_SOLVE_GRAPHS: capture each restart cycle (its Arnoldi
 *              steps with preconditioner, operator, Gram-Schmidt and small
 *              dense kernels, the cycle end and the restart) as one HIP graph
 *              the first time a cycle of that shape runs, and replay it; the
 *              workspace and the graphs stay with the field, so later solves
 *              with the same m, k, SAP parameters, flags and RHS count
 *              (any mass, tolerance, max_iter, restart_t and b) replay them
 *              too, and such a solve without graphs (flag clear, default
 *              stream, or per-kernel timing on) reuses the workspace.
 *              dw_field_destroy,
 *              dw_field_set_clover or a solve with other parameters frees
 *              them. Used on a non-default stream with per-kernel timing
 *              off, else ignored.
 *              DW_SOLVE_V32: store the Krylov basis V in FP32 (the arithmetic
 *              stays FP64), which halves the Gram-Schmidt traffic; the
 *              Arnoldi relation then holds to FP32 accuracy and the explicit
 *              FP64 residual at every restart (Section 4.7) keeps the solve
 *              exact.
 *              DW_SOLVE_INJECT: at a deflated restart, bring the explicit
 *              FP64 residual r into the new cycle in the two further places
 *              Section 4.7 names: the last column of G_{k+1} is V_{m+1}^H r
 *              instead of the small residual c - H^ eta, and v_{k+1} is r
 *              orthonormalised against the rotated V_k (with the phase of the
 *              rotated v_{k+1}, so that D Z_k = V_{k+1} H^_k keeps holding up
 *              to the difference between the two residuals). In exact
 *              arithmetic nothing changes; it is meant for a low-precision
 *              basis (DW_SOLVE_V32, DW_SOLVE_A32).
 *              DW_SOLVE_A32: the single-precision Arnoldi of Section 4.7:
 *              V and Z stored in FP32, w = D z_j applied in FP32 (FP32 links
 *              and arithmetic) and the Gram-Schmidt sweeps in FP32
 *              arithmetic, so that almost all of the work is low precision;
 *              the iterate, the explicit FP64 residual of every restart (in
 *              c, and with DW_SOLVE_INJECT in G_{k+1} and v_{k+1}), the
 *              small dense problems and the clean-restart test stay FP64.
 *              With a low-precision SAP the column z_j is stored as
 *              sigma M v_j (sigma the input scaling), which leaves the
 *              iterate unchanged. Other bits must be 0. */
enum { DW_SOLVE_GRAPHS = 1, DW_SOLVE_V32 = 2, DW_SOLVE_INJECT = 4, DW_SOLVE_A32 = 8 };

typedef struct fgmresdr_params {
  int32_t m;
  int32_t k;
  int32_t max_iter;
  int32_t shared_defl;
  double tol;
  double restart_t;
  sap_params sap;
  int32_t flags;
  int32_t reserved;
} fgmresdr_params;

/* Per-RHS solver statistics. */
typedef struct dw_solve_stats {
  int32_t converged;       /* 1 if ||b - D x|| <= tol ||b|| */
  int32_t iterations;      /* flexible Arnoldi steps */
  int32_t cycles;          /* restart cycles */
  int32_t clean_restarts;  /* restarts without deflation (Section 4.7) */
  double true_relres;      /* ||b - D x|| / ||b|| in FP64 at exit */
  double implicit_relres;  /* least-squares residual of the last cycle / ||b|| */
  double seconds;          /* wall-clock time of the solve */
} dw_solve_stats;

/* Thread-local text of the last error (never NULL). */
const char* dw_last_error(void);

/* Creates a context on HIP device `device`. `alloc` may be NULL (stream-
 * ordered hipMallocAsync / hipFreeAsync). The allocator struct is copied.
 * dw_ctx_destroy releases the caller's handle; fields created on the
 * context keep it (and call its allocator) until they are destroyed. */
dw_status dw_ctx_create(int32_t device, const dw_allocator* alloc, dw_ctx* out);
dw_status dw_ctx_destroy(dw_ctx ctx);

/* Imports a gauge field (Section 2: U_mu(n) in SU(3), one per site and
 * direction) for lattice L, tiled into SAP domains of extents `block`.
 * U_dev: canonical complex128 gauge array on the device (read during the
 * call's stream work only; the library keeps its own FP64, FP32, FP16 and
 * BF16 copies in a private block-tiled layout). DW_EINVAL if the blocks do
 * not tile L with an even count per direction or exceed 1024 sites. */
dw_status dw_field_create(dw_ctx ctx, const int32_t L[4], const int32_t block[4], const double* U_dev,
                          hipStream_t stream, dw_field* out);
dw_status dw_field_destroy(dw_field field);

/* Adds the clover (Sheikholeslami-Wohlert) term to the field's operator, as
 * in the paper's experiments (Section 5):
 *   D_sw = D + (i c_sw / 2) sum_{mu<nu} sigma_{mu nu} F_{mu nu}(n),
 *   sigma_{mu nu} = (i/2)[g_mu, g_nu], F_{mu nu} = (Q_{mu nu} - Q_{mu nu}^+)/8,
 * Q_{mu nu}(n) the four plaquettes of the (mu, nu) plane around n. The term
 * is site-local, so it is also part of every SAP block operator. It is
 * built on the device from the field's links (asynchronous on `stream`)
 * and used from then on by dw_apply, dw_apply_ex, sap_precondition and
 * fgmresdr_solve. csw = 0 removes it. DW_EINVAL: non-finite csw. */
dw_status dw_field_set_clover(dw_field field, double csw, hipStream_t stream);
/* Lattice sites of the field (convenience for callers sizing buffers). */
int64_t dw_field_volume(dw_field field);

/* y = D x for nrhs right-hand sides, FP64 (eq. 1). x and y: canonical
 * spinor arrays of nrhs * V * 12 complex128 each; they must not overlap.
 * Asynchronous on `stream`: its temporaries come from the context's
 * allocator and go back to it in stream order. */
dw_status dw_apply(dw_field field, double m0, const double* x, double* y, int32_t nrhs, hipStream_t stream);

/* y = D x as dw_apply, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc). It calls no allocator: the internal-layout copies of x and y
 * use a fixed device array of dw_apply_noalloc_max_bytes() bytes (64 MiB)
 * that each GPU holds from the first context created on it until the
 * process ends. Every call on a GPU uses that GPU's one array, so calls
 * that overlap on one GPU (different streams, or threads) race and must be
 * serialised by the caller. Needs 2 * nrhs * V * 192 bytes (plus alignment):
 * DW_EINVAL beyond the limit, before any GPU work. Asynchronous on `stream`. */
dw_status dw_apply_noalloc(dw_field field, double m0, const double* x, double* y, int32_t nrhs, hipStream_t stream);
size_t dw_apply_noalloc_max_bytes(void);

/* Benchmark path: y = D x on buffers already in the library's internal
 * block-tiled layout at storage precision `prec` (complex pairs of that
 * precision, nrhs * V * 12 pairs each; size from dw_internal_bytes). The
 * hopping term uses the field's links at the same precision and FP32
 * arithmetic (FP64 for DW_PREC_F64). dw_pack / dw_unpack convert between
 * the canonical FP64 layout and this one. */
dw_status dw_apply_ex(dw_field field, double m0, int32_t prec, const void* x_int, void* y_int, int32_t nrhs,
                      hipStream_t stream);
size_t dw_internal_bytes(dw_field field, int32_t prec, int32_t nrhs);
dw_status dw_pack(dw_field field, int32_t prec, const double* x, void* x_int, int32_t nrhs, hipStream_t stream);
dw_status dw_unpack(dw_field field, int32_t prec, const void* x_int, double* x, int32_t nrhs, hipStream_t stream);

/* z = M v: `sap.ncycles` SAP cycles (Alg. 2) from z = 0, each block system
 * D^l y^l = r^l (eq. 2) solved by `sap.nmr` minimal-residual steps in the
 * storage precision `sap.storage`. Blocks of colour 0 (even sum of block
 * coordinates, containing the origin) go first; the correction is added,
 * z^l += y^l. v and z: canonical spinor arrays (nrhs each), no overlap.
 * Below FP64 storage each v is scaled to unit RMS entries before the cast
 * (M(a v) = a M(v)), the factor formed on the device. Asynchronous on
 * `stream`, temporaries as for dw_apply. */
dw_status sap_precondition(dw_field field, double m0, const sap_params* sap, const double* v, double* z,
                           int32_t nrhs, hipStream_t stream);

/* SAP as a stand-alone solver for D x = b (Alg. 2 iterated; Section 3 on
 * its divergence as the mass approaches the critical one; Fig. 5):
 *   x_0 = 0,  x_{k+1} = x_k + M (b - D x_k),
 * M being `sap.ncycles` SAP cycles as in sap_precondition. Since a SAP cycle
 * started from z = 0 on the residual continues the sweep on x, x_k equals
 * k * ncycles cycles of Alg. 2 applied to D x = b. The residual b - D x_k
 * and x are FP64 (the preconditioner runs at `sap.storage`, its input
 * scaled per iteration to unit RMS), so low-precision storage does not
 * limit the attainable residual.
 * b, x: canonical spinor arrays (one right-hand side) on the device, no
 * overlap; x receives x_niter. resid: host array of niter + 1 doubles,
 * resid[k] = ||b - D x_k|| / ||b|| (FP64). The call returns when done.
 * An exact solution (zero residual) ends the iteration early, the remaining
 * entries of resid set to 0. DW_EINVAL: niter < 0, b = 0, bad sap_params. */
dw_status sap_solve(dw_field field, double m0, const sap_params* sap, const double* b, double* x, int32_t niter,
                    double* resid, hipStream_t stream);

/* Solves D x = b by SAP-preconditioned FGMRES-DR(m, k) (Alg. 4) from x = 0
 * for nrhs right-hand sides, solved in lock-step (every SAP and stencil
 * launch covering the whole batch): all nrhs in one batch whenever their
 * workspace can be allocated (up to 64), else in batches of as many as
 * 90% of the free device memory holds. Arnoldi, Hessenberg updates, harmonic Ritz
 * deflation and the least-squares problems are FP64; the explicit residual
 * is computed in FP64 once per cycle and enters the least-squares right-hand
 * side (Section 4.7); the preconditioner runs at `params->sap.storage`.
 * b, x: canonical spinor arrays (nrhs each). stats: host array of nrhs
 * entries (may be NULL). The stopping tests (implicit residual, breakdown,
 * iteration limit within a cycle; explicit residual, clean or deflated
 * restart at its end) are taken on the device, so the call synchronises
 * `stream` once per restart cycle (to read each right-hand side's state)
 * and before returning. Returns DW_ENOTCONV if any RHS stopped at max_iter
 * (x then holds its last iterate and stats are filled). */
dw_status fgmresdr_solve(dw_field field, double m0, const fgmresdr_params* params, const double* b, double* x,
                         int32_t nrhs, dw_solve_stats* stats, hipStream_t stream);

/* ---- small dense steps, on host arrays ----------------------------------------
 * The solver runs these one-wavefront FP64 kernels on its own device data;
 * these entry points run the same kernels on host arrays (copied in and out,
 * synchronous on the null stream, temporaries from the context's allocator)
 * so that they can be compared with a reference. Complex numbers are
 * interleaved (re, im) doubles; matrices are column-major.
 *
 * dw_dense_lsq: the least-squares problem of Section 4.2,
 *   eta = argmin ||c - H^ eta||, H^ of (cols + 1) x cols (leading dimension
 *   cols + 1), c of cols + 1 entries; eta receives cols entries, *resid the
 *   residual norm ||c - H^ eta|| (by Householder QR). 1 <= cols <= 48.
 * dw_dense_restart: the deflated restart of Alg. 4 (Lemma 1, Section 4.4)
 *   for a cycle of mm columns: H^ of (mm + 1) x mm (leading dimension mm + 1),
 *   c (mm + 1) and eta (mm). Outputs: ritz (mm entries) all harmonic Ritz
 *   values, eigenvalues of H_m + f h_m^H with H_m^H f = h_m, sorted by
 *   modulus (stable); Q ((mm + 1) x (k + 1), leading dimension mm + 1) the
 *   orthonormal factor of G_{k+1} = [[G_k; 0], c - H^ eta], G_k holding the
 *   unit eigenvectors of the k smallest; Hk ((k + 1) x k, leading dimension
 *   k + 1) = Q^H H^ Q_k. *status: 0 ok, 1 singular H_m, 2 eigenvalue
 *   iteration failed, 3 non-finite value (outputs then undefined).
 *   2 <= mm <= 48, 1 <= k < mm, k <= 23. */
dw_status dw_dense_lsq(dw_ctx ctx, int32_t cols, const double* Hhat, const double* c, double* eta, double* resid);
dw_status dw_dense_restart(dw_ctx ctx, int32_t mm, int32_t k, const double* Hhat, const double* c, const double* eta,
                           double* ritz, double* Q, double* Hk, int32_t* status);

/* ---- serving loop ----------------------------------------------------------
 * A server solves requests of different lattices, masses and RHS counts
 * with continuous batching: requests are queued in arrival order and
 * admitted when a slot is free and their device-memory footprint fits the
 * budget beside the requests already running (a later request may go first
 * only if it leaves room for the oldest waiting one); each slot runs its request
 * on its own HIP stream, so admitted requests overlap on the device, and
 * keeps the request's gauge copies and Krylov / deflation state on the
 * device until the request completes. Server memory comes from the server's
 * own caching allocator (independent of the context's allocator): blocks a
 * slot frees are reused by any slot once that slot's stream has drained, and
 * free cached blocks are returned to the device when an allocation finds it
 * full. A slot keeps the field of its last request (links, workspace and
 * captured restart cycles) while its next request has the same lattice and
 * block; the footprint of the request that made it stays charged until then.
 * Every request runs on restart cycles captured as HIP graphs. */
typedef struct dw_server_params {
  int32_t slots;           /* requests solved concurrently (>= 1) */
  int32_t queue_capacity;  /* queued, not yet admitted requests; solve_submit returns DW_EBUSY beyond */
  double budget_bytes;     /* admission budget; 0 = 80% of the device memory free at creation */
} dw_server_params;

/* A solve request. The pointers are device pointers owned by the caller;
 * they must stay valid and unmodified until solve_poll reports
 * DW_REQ_DONE or DW_REQ_FAILED (the server reads U and b and writes x). */
typedef struct dw_request {
  int32_t L[4];           /* lattice extents */
  int32_t block[4];       /* SAP block extents (params.sap.block must match) */
  double m0;              /* mass */
  double csw;             /* clover coefficient (0: plain Wilson), see dw_field_set_clover */
  const double* U;        /* canonical gauge field, complex128 */
  int32_t nrhs;           /* right-hand sides (solved in lock-step) */
  int32_t reserved;
  const double* b;        /* canonical spinors, nrhs fields */
  double* x;              /* solutions, nrhs fields */
  fgmresdr_params params; /* solver parameters */
} dw_request;

typedef enum { DW_REQ_QUEUED = 0, DW_REQ_RUNNING = 1, DW_REQ_DONE = 2, DW_REQ_FAILED = 3 } dw_req_state;

/* Request timing (seconds on the server's steady clock). */
typedef struct dw_request_times {
  double queued;    /* submit -> admission */
  double running;   /* admission -> completion */
  double latency;   /* submit -> completion */
} dw_request_times;

dw_status dw_server_create(dw_ctx ctx, const dw_server_params* params, dw_server* out);
/* Waits for all admitted and queued requests, then frees the server. */
dw_status dw_server_destroy(dw_server server);
/* Device-memory footprint the server charges for a request (bytes): the
 * field's four link copies, the solver's Krylov bases and work vectors for
 * nrhs right-hand sides, and small per-RHS buffers. 0 if the request is
 * invalid. Host-only arithmetic (no GPU work). */
size_t dw_request_footprint(const dw_request* req);
/* Queues a request (non-blocking). DW_EINVAL: bad geometry or parameters,
 * or footprint above the budget; DW_EBUSY: queue full. */
dw_status solve_submit(dw_server server, const dw_request* req, uint64_t* ticket);
/* Non-blocking status of a ticket. When DONE, stats (nrhs entries, may be
 * NULL) and times (may be NULL) are filled and the ticket is released, so
 * a later poll of it returns DW_ENOTFOUND. A FAILED request's error text is
 * returned by dw_last_error() of the polling thread. */
dw_status solve_poll(dw_server server, uint64_t ticket, dw_req_state* state, dw_solve_stats* stats,
                     dw_request_times* times);

/* ---- autotuner -------------------------------------------------------------
 * The paper fixes the SAP parameters by hardware efficiency and then tunes
 * m and k (Section 5). Because the block shape, the MR step count and the
 * cycle count s change the iteration count as well as the cost per
 * iteration, the tuner's objective is the wall-clock time of the whole
 * solve to the requested tolerance. It searches coordinate-wise from
 * `base`: block shape, then nmr, then s, then (m, k), keeping the best so
 * far each time and repeating the last three `passes` times; a candidate's max_iter is capped at `iter_cap` times the
 * best iteration count so far, so hopeless candidates stop early. */
typedef struct dw_tune_space {
  int32_t nblocks;        /* candidate block shapes in blocks[]; 0 = every shape with extents in
                           * {2, 4, 8}, volume 128..512, longest <= 2 x shortest extent, valid for L */
  int32_t blocks[16][4];
  int32_t nmr_min, nmr_max;  /* MR steps searched (inclusive); nmr_max < nmr_min: keep base */
  int32_t s_min, s_max;      /* SAP cycles searched (inclusive); s_max < s_min: keep base */
  int32_t nmk;               /* (m, k) candidates in mk[] (0: keep base) */
  int32_t mk[8][2];
  int32_t repeats;           /* timed solves per candidate, the fastest counts (>= 1) */
  int32_t passes;            /* sweeps over (nmr, s, (m, k)) after the block search (>= 1) */
  double iter_cap;           /* max_iter of a candidate = iter_cap * best iterations (<= 0: base max_iter) */
} dw_tune_space;

typedef struct dw_tune_trial {
  fgmresdr_params params;  /* the candidate */
  int32_t converged;       /* every RHS reached tol */
  int32_t iterations;      /* largest iteration count over the RHS */
  double seconds;          /* fastest wall-clock time of the whole solve */
} dw_tune_trial;

/* Tunes the solver for lattice L, gauge field U (canonical layout, device),
 * mass m0, clover coefficient csw (0: none) and right-hand sides b (nrhs canonical spinors, device). x is a
 * device work array of the size of b (it holds the last candidate's
 * solution). trials: host array of max_trials entries receiving every
 * candidate in the order tried; *ntrials is set to the count. *best gets
 * the fastest converged candidate (DW_ENOTCONV if none converged). Fields
 * for the candidate block shapes are created and destroyed inside. */
dw_status dw_autotune(dw_ctx ctx, const int32_t L[4], const double* U, double m0, double csw,
                      const fgmresdr_params* base,
                      const dw_tune_space* space, const double* b, double* x, int32_t nrhs, dw_tune_trial* trials,
                      int32_t max_trials, int32_t* ntrials, fgmresdr_params* best, hipStream_t stream);

/* ---- per-kernel-class timing ---------------------------------------------
 * When enabled on a context, every kernel launch made for that context is
 * bracketed by HIP events on the launch stream; elapsed times are resolved
 * at the library's synchronisation points and accumulated per class
 * together with the launch's algorithmic bytes (data the method must move:
 * each operand read once, each result written once) and flops. */
enum {
  DW_K_DSLASH_F64 = 0,  /* FP64 operator of the outer solver (A z, explicit residual) */
  DW_K_DSLASH_LOWP = 1, /* operator at storage precision (dw_apply_ex) */
  DW_K_SAP = 2,         /* one SAP colour sweep (block residual + MR steps) */
  DW_K_DOTS = 3,        /* multi-dot V^H w, first stage */
  DW_K_REDUCE = 4,      /* multi-dot, second stage */
  DW_K_SUBCOLS = 5,     /* w -= V h */
  DW_K_SCALE = 6,       /* y = a x */
  DW_K_COMBINE = 7,     /* x += Z eta */
  DW_K_ROTATE = 8,      /* V <- V Q, Z <- Z Q_k */
  DW_K_CONVERT = 9,     /* precision / layout conversion */
  DW_K_DENSE = 10,      /* small dense FP64 kernels (one workgroup) */
  DW_K_COUNT = 11
};
typedef struct dw_kernel_stats {
  int64_t launches;
  double ms;     /* summed event time */
  double bytes;  /* summed algorithmic bytes */
  double flops;  /* summed algorithmic flops */
} dw_kernel_stats;

/* Turns timing on (1) or off (0) for calls made with this context. */
dw_status dw_profile_enable(dw_ctx ctx, int32_t on);
/* Copies the accumulated statistics of kernel class kclass. */
dw_status dw_profile_get(dw_ctx ctx, int32_t kclass, dw_kernel_stats* out);
/* Clears the accumulated statistics. */
dw_status dw_profile_reset(dw_ctx ctx);

#ifdef __cplusplus
}
#endif

#endif /* DWSAP_H */
