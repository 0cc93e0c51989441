/*
 * lsamg.h -- C-ABI of an MI355X (gfx950) implementation of the solve phase
 * of least-squares AMG-DD for sparse SPD systems A = G^T G.
 *
 * Method: Southworth, Al Daas, Wimmer, Threlfall, "Algebraic Multigrid with
 * Overlapping Schwarz Smoothers and Local Spectral Coarse Grids for Least
 * Squares Problems".  Setup follows Algorithm 1 (sec. 3.2); solve is
 * preconditioned CG (sec. 4.1, relative residual 1e-8) around a V-cycle with
 * one restricted additive Schwarz pre-smoothing (eq:ras, sec. 2.2), the
 * coarse-grid correction eq:cgc with the local-spectral interpolation
 * eq:mg-p (sec. 3.1.1), and one RAS-transpose post-smoothing (eq:ras-t).
 *
 * Conventions shared by every entry point:
 *  - Return value: LSAMG_OK (0) or a negative LSAMG_E* code; the message of
 *    the last error on the calling thread is lsamg_last_error().
 *  - "device" pointers are HIP device (HBM) addresses on the handle's GPU;
 *    "host" pointers are ordinary CPU memory.  The caller owns every buffer
 *    it passes in; the library never frees them and keeps no reference to
 *    them after the call returns.
 *  - Vectors are FP64, indexed in the caller's numbering of the columns of G.
 *  - stream is a hipStream_t passed as void* (NULL = default stream).  Every
 *    entry point that takes a stream enqueues its work on it and returns
 *    after that work completed.
 */
#ifndef LSAMG_H
#define LSAMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LSAMG_OK = 0,
  LSAMG_EINVAL = -1,     /* bad sizes, pointers or parameters               */
  LSAMG_EBADINPUT = -2,  /* non-finite entry in G or in a right-hand side   */
  LSAMG_ENOTSPD = -3,    /* a local or coarsest Cholesky failed (A singular) */
  LSAMG_ENOMEM = -4,     /* host or device allocation failed                */
  LSAMG_EHIP = -5,       /* HIP runtime error                               */
  LSAMG_ENOCONV = -6,    /* maxit reached: x and stats are still written    */
  LSAMG_ENODEV = -7      /* handle has no device copy, or no GPU present    */
};

enum { LSAMG_FP64 = 0, LSAMG_MIXED = 1 };

enum {                    /* operators for lsamg_apply_op (finest level)    */
  LSAMG_OP_A = 0,         /* y = G^T (G x)                 (eq:Ax=b)        */
  LSAMG_OP_RAS = 1,       /* y = sum_i R_i^T D_i A_i^{-1} R_i x   (eq:ras)  */
  LSAMG_OP_RAST = 2,      /* y = sum_i R_i^T A_i^{-1} D_i R_i x   (eq:ras-t)*/
  LSAMG_OP_VCYCLE = 3     /* y = B x, one V-cycle from zero (sec. 3.1.1)    */
};

/* Sparse G in CSR, host memory, FP64.  m rows, n columns; row r holds the
 * entries rowptr[r] .. rowptr[r+1]-1.  Explicit zeros and empty rows are
 * allowed (they are dropped).  Copied by lsamg_setup. */
typedef struct lsamg_csr {
  int64_t m, n, nnz;
  const int64_t* rowptr;
  const int32_t* col;
  const double* val;
} lsamg_csr;

/* Setup parameters (Algorithm 1 inputs, sec. 3.2 and 3.4). */
typedef struct lsamg_params {
  int32_t max_levels;    /* L_max                                   (def 10) */
  int64_t max_coarse;    /* n_coarse: stop once a level is this small (2000) */
  int32_t ndim;          /* lattice dimension of G's columns (2 or 3)        */
  int32_t grid[3];       /* lattice extent per axis, x fastest               */
  int32_t block;         /* lattice block width per axis (4 in 2D, 3 in 3D)  */
  int32_t omega_max;     /* coarse levels shrink the block until every
                            aggregate has at most this many unknowns (800)   */
  int32_t n_eig_fixed;   /* > 0: fixed eigenvector count per aggregate;
                            0: threshold rule of sec. 3.4                    */
  double kappa;          /* target condition number (50, sec. 3.4)           */
  int32_t cmin[8];       /* minimum coarsening ratio per level, the last one
                            repeats (LS_{a,b,...} of sec. 3.4)               */
  int32_t ncmin;
  double tie_rtol;       /* relative width of an eigenvalue cluster (1e-8)   */
  double tie_atol;       /* absolute width of an eigenvalue cluster (1e-12)  */
  double pinv_rtol;      /* pseudo-inverse cutoff in eq:gevp-S: singular
                            values of W^{1/2} G_{nz,Gamma} at or below this
                            times the largest count as null (1e-6, i.e.
                            eigenvalues of A~_GammaGamma at or below 1e-12
                            times the largest)                               */
  double thresh_margin;  /* strict side of the threshold test (1e-10)        */
  double stall_ratio;    /* stop coarsening if n_{l+1} > ratio * n_l (0.9)   */
  int32_t precision;     /* LSAMG_FP64 or LSAMG_MIXED (FP32 V-cycle)         */
  int32_t device;        /* HIP device ordinal; < 0 builds a host-only handle
                            (setup data and lsamg_export_setup only)         */
  int32_t nthreads;      /* host threads for setup (0 = all cores)           */
  int32_t verbose;       /* 1: one progress line per setup phase on stderr   */
  int64_t dense_tail;    /* > 0: the V-cycle from the first level l >= 1 with
                            at most this many unknowns down to the coarsest
                            (a fixed symmetric linear map) is formed once on
                            the GPU and applied as one dense matrix (n_l^2
                            entries per precision); 0: always recurse.
                            Default 16384.                                   */
  int32_t aggregation;   /* LSAMG_AGG_LATTICE (0, default): lattice blocks of
                            `block` points per axis; LSAMG_AGG_STANDARD (1):
                            standard aggregation on the matrix entries of
                            A_l = G_l^T G_l (sec. 3.3), nodes visited in index
                            order, every unaggregated node joining the
                            aggregate of its lowest-numbered aggregated
                            neighbour; needs no lattice (ndim may be 0)      */
  int32_t agg_passes[8]; /* standard aggregation: passes n_agg per level, the
                            last one repeats (Algorithm 1; pass t aggregates
                            the graph of pass t-1's aggregates, T_1 T_2 ...)  */
  int32_t nagg_passes;   /* entries used in agg_passes (default 1: {1})      */
  int32_t cycle;         /* LSAMG_CYCLE_V (0, default): the multiplicative
                            V-cycle (RAS pre-smoother, coarse-grid correction,
                            RAS-T post-smoother, sec. 3.1.1); LSAMG_CYCLE_ADDITIVE
                            (1): the additive method of sec. 3.1.1, the
                            additive Schwarz smoother sum_i R_i^T A_i^{-1} R_i
                            (eq:ras without the partition of unity) plus
                            P (coarse cycle) P^T on every level, exact at the
                            coarsest; setup then also stores the full local
                            inverses A_i^{-1} (|Omega_i|^2 entries each), there
                            is no dense tail, and several right-hand sides are
                            solved one after another                         */
  int32_t setup_device;  /* where the local dense problems of every level
                            (Algorithm 1: the pseudo-inverse Schur complement
                            of eq:gevp-S, the reduced local eigenproblem, the
                            local inverses A_i^{-1}) run.
                            LSAMG_SETUP_HOST (0): on the host's cores;
                            LSAMG_SETUP_DEVICE (1): on the HIP device `device`
                            as batched FP64 factorisations (batched QR,
                            SVD, Cholesky and symmetric eigensolvers of rocSOLVER,
                            batched GEMM and triangular solves of rocBLAS, both
                            loaded when first needed), aggregates of similar
                            size padded into one batch; the integer steps and
                            G_{l+1} = G_l P_l stay on the host.  Needs
                            device >= 0 (else LSAMG_EINVAL);
                            LSAMG_SETUP_AUTO (2, default): on the device when
                            device >= 0 and G has at least 100,000 columns
                            (where the batches fill the GPU), else on the host */
} lsamg_params;

enum {
  LSAMG_SETUP_HOST = 0,
  LSAMG_SETUP_DEVICE = 1,
  LSAMG_SETUP_AUTO = 2
};

enum { LSAMG_AGG_LATTICE = 0, LSAMG_AGG_STANDARD = 1 };
enum { LSAMG_CYCLE_V = 0, LSAMG_CYCLE_ADDITIVE = 1 };

/* Per-solve statistics (host memory, one entry per right-hand side). */
typedef struct lsamg_stats {
  int32_t iters;         /* PCG iterations (applications of A)               */
  int32_t converged;     /* 1 if the recurrence residual and then the true
                            residual b - A x both reached tol ||b||          */
  double rel_res;        /* ||r_k|| / ||b||, recurrence residual             */
  double true_rel_res;   /* ||b - A x|| / ||b||, recomputed in FP64          */
  double rho;            /* average convergence factor (||r_k||/||r_0||)^(1/k)*/
  double seconds;        /* wall time of the whole call                      */
  int32_t restarts;      /* times the recurrence residual passed the test but
                            the true residual did not: r was replaced by
                            b - A x and CG restarted with p = z              */
  int32_t reserved;
} lsamg_stats;

typedef struct lsamg_level_info {
  int64_t n;             /* unknowns                                         */
  int64_t nagg;          /* aggregates (0 on the coarsest level)             */
  int64_t g_rows;        /* stored rows of G_l (after exact row compression) */
  int64_t g_nnz;         /* stored entries of G_l                            */
  int64_t a_nnz;         /* entries of A_l = G_l^T G_l                       */
  int64_t smoother_entries; /* sum_i |omega_i| |Omega_i|                     */
  int64_t p_entries;     /* entries of P_l                                   */
  int32_t block, n_color, n_mult, kmin, kmax;
  double thresh;
  int64_t hazards;       /* aggregates with an eigenvalue at the threshold   */
} lsamg_level_info;

typedef struct lsamg_info {
  int32_t nlevels;
  int64_t n0, m0;
  double setup_seconds;
  size_t device_bytes;
  double op_complexity;      /* sum_l nnz(A_l) / nnz(A_0)                    */
  double smoother_complexity;/* sum_l sum_i |omega_i||Omega_i| / nnz(A_0)    */
  lsamg_level_info level[16];
  int32_t tail_level;        /* level applied as one dense matrix (see
                                dense_tail), -1 if none                      */
} lsamg_info;

/* Integer setup of one level in the canonical numbering: finest-level
 * unknowns are G's columns; a coarse unknown is numbered by (aggregate of the
 * finer level, eigenvector index).  Arrays are owned by the handle and stay
 * valid until the next lsamg_export_setup call or lsamg_destroy. */
typedef struct lsamg_setup_view {
  int64_t n, nagg;
  const int32_t* agg;    /* [n] aggregate of each unknown                    */
  const int64_t* optr;   /* [nagg+1]                                         */
  const int64_t* oidx;   /* Omega_i: omega_i ascending, then Gamma_i ascending */
  const int32_t* k;      /* [nagg] eigenvectors kept                         */
  const int32_t* M;      /* finest level: multiplicity of each kept row of G;
                            NULL on coarser levels                           */
  const double* mu;      /* local eigenvalues mu = 1/lambda, ascending       */
  const int64_t* muptr;  /* [nagg+1]                                         */
  int32_t block, n_color, n_mult;
  double thresh;
} lsamg_setup_view;

/* Per-kernel timing record (see lsamg_profile). */
typedef struct lsamg_kprof {
  char name[80];         /* kernel symbol, e.g. "k_gemv_wide<float, 1, false, 16>" */
  int64_t launches;      /* launches timed since profiling was enabled       */
  double ms;             /* summed HIP-event durations of those launches     */
  double bytes;          /* summed algorithmic bytes of those launches       */
  double flops;          /* summed algorithmic floating-point operations of
                            those launches (matrix-core and dense products:
                            2 x stored matrix entries x columns; else 0)     */
} lsamg_kprof;

typedef struct lsamg_handle lsamg_handle;

/* ---- serving ---------------------------------------------------------- */

/* One solve request.  Requests with equal op_key share one hierarchy: the
 * first builds it (setup, then upload once admitted), later ones find it
 * resident.  When params->setup_device puts the setup's dense local
 * problems on the device, they run on the server's device with 24 GiB of the
 * HBM budget held for them meanwhile; when that cannot be freed, an
 * LSAMG_SETUP_DEVICE request fails with LSAMG_ENOMEM and an LSAMG_SETUP_AUTO
 * one runs its setup on the host.  The device setup's libraries (rocBLAS,
 * rocSOLVER) are opened when the server is created, before its workers
 * launch anything; outside the server they are opened by the first setup on
 * the device, which should not overlap kernel launches of other threads. */
typedef struct lsamg_request {
  uint64_t id;             /* caller's id, returned in lsamg_done                */
  uint64_t op_key;         /* operator identity                                  */
  const lsamg_csr* G;      /* host CSR of G, read on a cache miss only; it and the
                              arrays it points to must stay valid until the
                              request completes                                  */
  const lsamg_params* params; /* setup parameters (params->device is ignored)   */
  const double* b;         /* host, column-major n x nrhs (ld = n); copied at
                              submit                                             */
  double* x;               /* host, column-major n x nrhs; written before the
                              request is reported done                           */
  int32_t nrhs;            /* 1 .. 64                                            */
  int32_t maxit;
  double tol;
} lsamg_request;

typedef struct lsamg_done {
  uint64_t id;
  int32_t status;          /* LSAMG_OK, LSAMG_ENOCONV, or the setup/solve error  */
  int32_t cache_hit;       /* hierarchy resident when the request was taken      */
  int32_t batch_rhs;       /* right-hand sides solved together with this one     */
  int32_t iters_max;       /* most PCG iterations over the request's columns     */
  double true_rel_res_max; /* largest ||b - A x|| / ||b|| over its columns       */
  double t_queue;          /* seconds from submit until taken by a worker        */
  double t_setup;          /* setup + upload (0 on a hit)                        */
  double t_solve;          /* copy-in, solve, copy-out                           */
  double t_total;          /* submit to completion                               */
  int32_t joined_at;       /* PCG iteration of the running solve at which the
                              request's columns entered it (0: it started it)  */
  int32_t reserved;
  char msg[96];            /* error message of a failed request ("" on success) */
} lsamg_done;

typedef struct lsamg_server_stats {
  int64_t submitted, completed, hits, misses, evictions;
  size_t resident_bytes, peak_bytes, budget;
  int32_t queued, active;
  int64_t joins;           /* requests that entered a solve already running      */
  int64_t reserve_misses;  /* solves that added more device memory than their
                              admission reserved (0 unless the bound is wrong)  */
  int64_t iterations;      /* PCG iterations run so far, all solves together     */
} lsamg_server_stats;

typedef struct lsamg_server lsamg_server;

/* Fill p with the defaults listed above (ndim/grid left zero). */
void lsamg_params_default(lsamg_params* p);

/* Build the hierarchy of Algorithm 1 for A = G^T G on the host (FP64) and,
 * if p->device >= 0, upload it to that GPU.  G is host CSR and is copied.
 * On success *out owns all host and device memory of the hierarchy.
 * Errors: EINVAL (sizes, lattice, params), EBADINPUT (non-finite G),
 * ENOTSPD (singular A: a column of G without entries, or a failed local
 * factorisation), ENOMEM, EHIP. */
int lsamg_setup(const lsamg_csr* G, const lsamg_params* p, lsamg_handle** out);

/* Solve A x = b for nrhs right-hand sides with PCG (x0 = 0) preconditioned
 * by one V-cycle per iteration, until ||r_k|| <= tol ||b|| or maxit.
 * b, x: device, FP64, column-major n x nrhs with leading dimension ld >= n.
 * Each column is solved independently (its own CG scalars and stop test).
 * stats: host array of nrhs entries, or NULL.
 * Errors: EINVAL, ENODEV, EBADINPUT (non-finite b), EHIP, ENOCONV. */
int lsamg_solve(lsamg_handle* h, const double* b, double* x, int32_t nrhs,
                int64_t ld, double tol, int32_t maxit, void* stream,
                lsamg_stats* stats);

/* y = op(x) on the finest level (see LSAMG_OP_*), one vector, in the
 * precision selected for the V-cycle.  x, y: device, FP64, length n. */
int lsamg_apply_op(lsamg_handle* h, int32_t op, const double* x, double* y,
                   void* stream);

/* Staging that lsamg_apply_op_noalloc holds on each GPU (32 MiB). */
#define LSAMG_NOALLOC_SCRATCH_BYTES (32ll << 20)

/* Allocation-free variant of lsamg_apply_op, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same operators, arguments and result as
 * lsamg_apply_op, but the call
 *   - allocates nothing: no hipMalloc/hipFree, no library routine that
 *     allocates; its staging (the permuted input and the output before the
 *     permutation, n doubles each, and for LSAMG_OP_A the m rows of G x) lives
 *     in one static array of LSAMG_NOALLOC_SCRATCH_BYTES per GPU, which the
 *     process keeps until it ends; level work vectors are the handle's own,
 *     made at set-up;
 *   - only enqueues its kernels on `stream` (no synchronisation, no HIP
 *     graph, no kernel timing); y is valid once the stream reaches that
 *     point.
 * Every call on a GPU shares that GPU's staging array and the handle's
 * level vectors: calls that overlap on one GPU (another stream, another
 * thread, another handle on the same device) race and must be ordered by the
 * caller.  Errors: EINVAL (null pointer, bad op, single-level hierarchy for
 * RAS/RAS-T, or an operator whose staging exceeds the array: 8 (2n + m)
 * bytes for LSAMG_OP_A, 16 n bytes otherwise; checked before any device
 * work), ENODEV (no device copy), EHIP. */
int lsamg_apply_op_noalloc(lsamg_handle* h, int32_t op, const double* x, double* y,
                           void* stream);

/* Select the V-cycle precision (LSAMG_FP64 or LSAMG_MIXED) for later calls. */
int lsamg_set_precision(lsamg_handle* h, int32_t precision);

enum {
  LSAMG_OPT_BATCHED = 0,  /* 1 (default): nrhs > 1 is solved in batches of up to
                             64 interleaved columns that share every matrix read;
                             0: one column after another                        */
  LSAMG_OPT_MFMA = 1,     /* 1 (default): the FP32 V-cycle of a batch of >= 16
                             columns runs its local solves, transfers and dense
                             coarse operator as matrix-core (MFMA) tiles whose
                             shapes are autotuned on the first such solve;
                             0: plain FMA kernels                               */
  LSAMG_OPT_GRAPH = 2,    /* 1 (default): each V-cycle of a solve is replayed
                             from a HIP graph of kernel nodes built on first use (one per
                             precision and batch width; not while kernel timing
                             is on); 0: kernels launched one by one             */
  LSAMG_OPT_MFMA_TILE = 3, /* 0 (default): the matrix-core tile shapes are
                             autotuned; 100*rt + 10*u + split fixes them for every
                             operator instead: rt in {1,2,4} row tiles of 16 per
                             task, u in {2,8} loop steps loaded together (u = 0
                             with rt = 4: on 64 columns the form that stages the
                             input rows in LDS per 64-row task), split in
                             {1,2,4,8} loop ranges per task (reduced to 1 where
                             the partial-sum buffer is too small).  In FP64 the
                             aggregate-block operators of a batch run on the
                             FP64 matrix cores or on FMA, whichever the
                             autotuner times faster; a fixed shape makes them all
                             FP64 matrix-core tasks with its rt and u (u with
                             rt = 4: 2; u = 0: the LDS-staged form on 64-row
                             tasks), no split                                    */
  LSAMG_OPT_ONEPASS_ATA = 4, /* 1 (default): where the rows of G are short (a
                             finite-difference G), the FP64 A-apply G^T (G P) of
                             the multi-right-hand-side CG recomputes each row of G
                             per unknown instead of storing G P; 0: two passes   */
  LSAMG_OPT_DENSE_SPLIT = 5, /* 0 (default): the FP32 dense level operator of a
                             batch of 64 columns runs as the LDS-staged matrix-core
                             GEMM or as the per-task tiles of the other operators,
                             whichever the autotuner times faster (the latter only
                             while LSAMG_OPT_MFMA_TILE fixes the tiles), and the
                             FP64 one as the FP64 LDS-staged matrix-core GEMM or
                             the FMA kernel, whichever is faster; 1..16: the
                             LDS-staged GEMM with that many loop ranges (fewer
                             where the partial-sum buffer is too small); 17: never
                             the LDS-staged GEMM                                 */
  LSAMG_OPT_ATA_TILES = 6, /* 1 (default): on 64 columns, the finest level's
                             G^T (G X) of the V-cycle residual and of the CG (with
                             LSAMG_OPT_ONEPASS_ATA) runs in one pass over tiles of
                             16 unknowns whose input rows are staged once in LDS,
                             where G's rows are short enough (FP32 forming the
                             tile's rows of G X first, FP64 from each unknown's
                             expanded stencil); 2 or 3: the row form or the
                             expanded form in both precisions; 0: the untiled
                             forms                                              */
  LSAMG_OPT_BGROUP = 7,   /* 0 (default): on 64 columns in FP32, each coarse
                             level's residual runs as the row-group pass (R_g^T R_g
                             per group, staged) or as two CSR passes, whichever the
                             autotuner times faster; 1: the row-group pass where
                             built; 2: the CSR passes                           */
  LSAMG_OPT_KRYLOV = 8    /* LSAMG_KRYLOV_CG (default): the outer iteration is
                             preconditioned CG, beta = rho_new / rho_old;
                             LSAMG_KRYLOV_FCG: flexible CG with one stored
                             direction (Notay 2000), beta = -(z . A p) / (p . A p),
                             which keeps consecutive directions A-orthogonal when
                             the V-cycle is a slightly varying or unsymmetric
                             operator (its FP32 form); the same in exact
                             arithmetic with a fixed symmetric preconditioner.
                             Applies to single and batched solves.
                             LSAMG_KRYLOV_BLOCK: several right-hand sides run as
                             block CG (O'Leary 1980) in batches of up to 64
                             columns: one iterate per column minimising its
                             error over all columns' Krylov spaces, directions
                             A-orthogonalised per block through the 64 x 64
                             Gram matrix P^T A P (pseudo-inverse: dependent
                             directions drop out); all columns of a batch
                             iterate until every one has converged.  A single
                             right-hand side runs as CG                      */
};

enum { LSAMG_KRYLOV_CG = 0, LSAMG_KRYLOV_FCG = 1, LSAMG_KRYLOV_BLOCK = 2 };

/* Set a solve-path option (LSAMG_OPT_*) for later calls.  Values are 0 or 1
 * except for LSAMG_OPT_MFMA_TILE, LSAMG_OPT_DENSE_SPLIT, LSAMG_OPT_BGROUP,
 * LSAMG_OPT_ATA_TILES and LSAMG_OPT_KRYLOV.
 * EINVAL on an unknown option or value. */
int lsamg_set_option(lsamg_handle* h, int32_t opt, int64_t value);

/* Y = B X: one V-cycle from zero (the preconditioner of lsamg_solve, sec.
 * 3.1.1) applied to nrhs <= 64 columns at once by the multi-right-hand-side
 * path, in the selected precision.  X, Y: device, FP64, column-major
 * n x nrhs with leading dimension ld >= n.  Errors: EINVAL, ENODEV, EHIP. */
int lsamg_apply_vcycle_batch(lsamg_handle* h, const double* X, double* Y,
                             int32_t nrhs, int64_t ld, void* stream);

/* Kernel timing.  mode 1: bracket every kernel launch of later solve /
 * apply calls with a pair of HIP events recorded on the launch stream; if
 * only != NULL, only launches of that kernel symbol are bracketed (the others
 * run undisturbed).  mode 2: as mode 1, with the V-cycle kernels reported per
 * hierarchy level (name suffix " @L<level>").  mode 0: stop.  Recording is bounded (65536 launches).
 * Each record also carries the launch's algorithmic bytes: the bytes the
 * kernel must move at least (matrix entries, index lists, every distinct
 * vector entry read once, outputs). */
int lsamg_profile(lsamg_handle* h, int32_t mode, const char* only);

/* Synchronize the recorded events and write per-kernel totals (host array
 * out of cap entries; *count = number written).  Resets the totals. */
int lsamg_profile_read(lsamg_handle* h, lsamg_kprof* out, int32_t cap, int32_t* count);

int lsamg_info_get(const lsamg_handle* h, lsamg_info* out);
int lsamg_export_setup(lsamg_handle* h, int32_t level, lsamg_setup_view* out);
size_t lsamg_device_bytes(const lsamg_handle* h);
void lsamg_destroy(lsamg_handle* h);
const char* lsamg_last_error(void);

/* Continuous-batching request server on one GPU.  max_slots worker threads,
 * each with its own HIP stream, run solves: a worker takes a queued request
 * whose hierarchy is resident and idle (or new) and starts a multi-right-
 * hand-side PCG on that operator, 8 to 64 columns wide, with the queued
 * requests for it that fit.  At every PCG iteration boundary requests for the
 * operator that arrived meanwhile enter free columns and start their own CG
 * there (their own tolerance and iteration limit), first come first served
 * (a request waiting for columns is not overtaken by a narrower later one),
 * and a request is reported as soon as its last column converges, freeing
 * its columns; the solve ends when no column is active and no queued request
 * for the operator fits.  When the columns waiting for the operator amount
 * to a full batch of the running width, that solve takes no more requests
 * and drains, so the next one starts wider (up to 64 columns).  A
 * request for a new operator builds its hierarchy on the host while the
 * other slots keep the GPU busy, and is admitted when its exact device
 * footprint fits hbm_budget; each solve is then admitted with an upper bound
 * of the device memory it can add (multi-right-hand-side buffers, autotuning,
 * request staging), narrowed to fewer columns if needed.  Idle hierarchies
 * are evicted least-recently-used first; memory that cannot fit fails the
 * request with ENOMEM.  Solves of different operators run concurrently on
 * their slots' streams.  Errors: EINVAL, ENODEV, ENOMEM. */
int lsamg_server_create(int32_t device, size_t hbm_budget, int32_t max_slots,
                        lsamg_server** out);

/* Queue a request (non-blocking; b is copied).  EINVAL on bad fields. */
int lsamg_server_submit(lsamg_server* s, const lsamg_request* req);

/* Up to cap completed requests into out (host array); waits up to wait_ms
 * milliseconds for the first one.  *count = number written. */
int lsamg_server_poll(lsamg_server* s, lsamg_done* out, int32_t cap, int32_t* count,
                      int32_t wait_ms);

int lsamg_server_stats_get(lsamg_server* s, lsamg_server_stats* out);

/* Finish every queued request, stop the workers, free all hierarchies. */
void lsamg_server_destroy(lsamg_server* s);

#ifdef __cplusplus
}
#endif
#endif /* LSAMG_H */
