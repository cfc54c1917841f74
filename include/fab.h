/*
 * fab.h -- C ABI of the MI355X sketched-Krylov f(A)b library (libfab.so).
 *
 * Method: Cortinovis, Kressner & Nakatsukasa, "Speeding up Krylov subspace
 * methods for computing f(A)b via randomization".  Given A (accessed only
 * through matrix-vector products, Section 1 / Table 1 "matrix access"), b,
 * a function f analytic near the spectrum of A (Section 1), a Krylov
 * dimension m, a truncation parameter k (Algorithm 2) and a sketch size s
 * (Section 2.1.1), the library returns
 *
 *      out = ||b||_2 V_m f(H_hat) e_1,   H_hat = H_m + h_{m+1,m} y e_m^T
 *
 * (Algorithm 4, last line; eq. (6) for H_hat) where (V_{m+1}, Hbar_m) is the
 * Arnoldi-like decomposition of eq. (3) built by k-truncated orthogonalisation
 * (Algorithm 2) and y approximates the least-squares solution of eq. (7): by
 * sketch-and-solve (Remark 3), by sketch-preconditioned LSQR refinement
 * (Blendenpik, Section 3.1.1) or y = 0 (Algorithm 5, eq. (8)).
 *
 * All of the method's arithmetic runs in HIP kernels on one gfx950 GPU.
 * Precision: the basis is stored in FP32 (or FP64), matrix-vector products,
 * dots, norms and sketches accumulate in FP64; the sketched QR / least
 * squares, f(H_hat) and the final combination are FP64.
 *
 * Conventions common to every entry point:
 *  - Every function returns an int status (enum fab_status); nothing is
 *    thrown across the ABI.  fab_strerror() names a status.
 *  - Vectors b and out are FP64 DEVICE pointers with nrhs right-hand sides
 *    interleaved row-major, layout [n][nrhs] (element (i, r) at i*nrhs + r).
 *  - Caller memory is never freed or retained by the library beyond the
 *    documented lifetime (until the call returns for fab_solve, until
 *    fab_poll/fab_wait reports completion for fab_submit).
 *  - A context is bound to one device and one HIP stream.  Calls on one
 *    context are serialised internally (thread-safe); distinct contexts are
 *    independent.
 */
#ifndef FAB_H
#define FAB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fab_ctx_s* fab_ctx;
typedef struct fab_matrix_s* fab_matrix;
typedef uint64_t fab_request;

enum fab_status {
  FAB_OK = 0,
  FAB_EINVAL = 1,     /* bad shape, parameter or pointer                         */
  FAB_ENOMEM = 2,     /* the request can never fit the arena                      */
  FAB_EDEVICE = 3,    /* a HIP runtime call failed                                */
  FAB_ENUMERIC = 4,   /* NaN/Inf in b, in the basis or in f(H_hat)                */
  FAB_EBUSY = 5,      /* matrix still referenced by in-flight requests            */
  FAB_ENOTFOUND = 6,  /* unknown request handle                                   */
  FAB_ESCRATCH = 7    /* fab_solve_noalloc: the request's workspace exceeds
                         FAB_NOALLOC_SCRATCH_BYTES                               */
};

/* The function f (Section 1: analytic on a domain containing the spectrum). */
enum fab_func_kind {
  FAB_F_EXP = 1,      /* f(z) = exp(alpha z); the solve returns FAB_ENUMERIC when
                         ||alpha H_hat||_1 > 16384 (work bound of the Taylor action) */
  FAB_F_POW = 2,      /* f(z) = (z + sigma)^p, p = +1/2 or -1/2 (principal branch) */
  FAB_F_POLY = 3,     /* f(z) = sum_j coef[j] z^j (test hook: exact for deg <= m-1) */
  FAB_F_SIGN = 4      /* f(z) = sign(Re z), computed as (A^2)^{-1/2} (A b) (Section 5.1.3):
                         the basis is built for the operator A^2, applied in every step
                         as two products with A (FP64 arithmetic, the intermediate A u
                         kept in FP64; A^2 is never formed), from the start vector A b,
                         with f(z) = z^{-1/2}; m, k, s, ... apply to that solve;
                         info.beta is ||A b||.  alpha, sigma, p are ignored.          */
};
typedef struct {
  int kind;
  double alpha, sigma, p;
  const double* coef; /* host pointer, ncoef <= 64; read during the call only   */
  int ncoef;
} fab_func;

/* Sketch Theta in R^{s x n} (Section 2.1.1). */
enum fab_sketch_kind {
  FAB_SKETCH_SRHT = 1,        /* s rows of the Walsh-Hadamard transform times random signs */
  FAB_SKETCH_SPARSE_SIGN = 2  /* zeta nonzeros +-1/sqrt(zeta) per column                    */
};
/* Basis storage precision. */
enum fab_prec {
  FAB_PREC_FP32 = 1,          /* FP32 basis, FP64 accumulation                            */
  FAB_PREC_FP64 = 2,          /* FP64 basis                                                */
  FAB_PREC_AUTO = 3           /* FP32, re-run in FP64 if the a-posteriori estimate fails   */
};
/* Least-squares policy for y in eq. (7). */
enum fab_ls_mode {
  FAB_LS_AUTO = 0,            /* sketch-and-solve, then LSQR refinement if the gate fails  */
  FAB_LS_SKETCH = 1,          /* sketch-and-solve only (Remark 3; equivalent to sFOM)      */
  FAB_LS_NONE = 2,            /* y = 0: Algorithm 5                                        */
  FAB_LS_LSQR = 3,            /* always refine with sketch-preconditioned LSQR (Algorithm 4
                                 with Blendenpik, Section 3.1.1); LSQR stops when
                                 ||M^T r|| <= (tol/10) ||M||_F ||r|| (Paige & Saunders'
                                 test, M = V_m R^{-1}) or at ls_maxit (info.ls_limit = 1) */
  FAB_LS_GRAM = 4             /* the exact least squares through the Gram matrix of
                                 V_{m+1} (one pass over the basis, Cholesky of the normal
                                 equations; error ~ kappa(V)^2 u, for the well-conditioned
                                 sketched-GS and whitened bases).  Blocking calls with one
                                 right-hand side and m <= 127; otherwise, or when R's
                                 diagonal spreads by more than 1e4, a pivot fails or the
                                 estimated kappa_1(R) exceeds min(1e4, sqrt(tol/(10 u)))
                                 (u = 2^-53, so that kappa^2 u <= tol/10), LSQR as
                                 FAB_LS_LSQR.  Not in the paper, which uses LSQR.           */
};

/* Construction of the basis. */
enum fab_basis {
  FAB_BASIS_TRUNCATED = 0,    /* k-truncated orthogonalisation (Algorithm 2)              */
  FAB_BASIS_SKETCHED_GS = 1,  /* Gram-Schmidt on the sketch (Algorithm 1): Theta V_{m+1} is
                                 orthonormal, v_i = (A v_{i-1} - V_{i-1} r_i) / r_ii; with
                                 FAB_LS_AUTO the least squares are always refined by LSQR,
                                 which gives Algorithm 3                                    */
  FAB_BASIS_SKETCHED_GS2 = 2, /* as FAB_BASIS_SKETCHED_GS with the Gram-Schmidt step on the
                                 sketch repeated once on its residual (r_i = r' + r''; not in
                                 the paper): same long-vector work, Theta V stays orthonormal
                                 to rounding when s is close to m                         */
  FAB_BASIS_WHITENED = 3      /* truncated orthogonalisation with whitening (Section 2.1.2):
                                 every 5 steps kappa_1(R) of Theta V_i = Q R is tested; above
                                 1000 (Section 5.1.3) the basis becomes V_i R^{-1}, Hbar
                                 R Hbar R^{-1}, the sketch Q, and the remaining steps follow
                                 Algorithm 1, with LSQR for the least squares (FAB_LS_AUTO).
                                 All right-hand sides of a call whiten together when one
                                 triggers.  Blocking calls only (fab_submit: FAB_EINVAL)   */
};

typedef struct {
  int m;              /* Krylov dimension, 1 <= m < n (m <= 500)                  */
  int k;              /* truncation window, 1 <= k <= 8 (Algorithm 2; ignored by
                         FAB_BASIS_SKETCHED_GS)                                    */
  int s;              /* sketch rows, m < s <= min(8192, padded n)                */
  int sketch;         /* enum fab_sketch_kind                                     */
  int zeta;           /* sparse-sign nonzeros per column, 1 <= zeta <= min(s,16)  */
  uint64_t seed;      /* fully determines Theta                                   */
  int prec;           /* enum fab_prec                                            */
  int ls_mode;        /* enum fab_ls_mode                                         */
  double tol;         /* target relative accuracy for AUTO policies (e.g. 1e-6)    */
  int basis;          /* enum fab_basis; 0 (a zero-initialised struct) = truncated  */
  int ls_maxit;       /* LSQR iteration limit, 0..1024; 0 = default: 32 for the
                         truncated basis (Blendenpik-preconditioned), 128 for the
                         sketched Gram-Schmidt bases and a whitened basis (whose
                         sketch is already orthonormal)                          */
} fab_params;

/* Per right-hand side diagnostics. */
typedef struct {
  double err_est;     /* max(ls_gate, round_est): a-posteriori error estimate; after an
                         LSQR refinement max(Paige-Saunders measure, round_est)    */
  double ls_gate;     /* ||R (c_y - c_0)|| / ||R c_y||: sensitivity to the last column */
  double round_est;   /* basis-rounding amplification estimate                      */
  double conv_est;    /* ||R (c_m - [c_{m-d}; 0])|| / ||R c_m||, d = max(5, m/10)     */
  double kappa_R;     /* condition estimate of the R factor of Theta V_m            */
  double h_last;      /* h_{m+1,m}                                                   */
  double beta;        /* ||b||_2 as used (norm of the stored first basis vector)      */
  int m_used;         /* dimension actually used (< m after a lucky breakdown)       */
  int breakdown;      /* 1 if an invariant subspace was found                        */
  int fell_back;      /* 1 if an FP32 result was recomputed with an FP64 basis       */
  int ls_iters;       /* LSQR iterations performed                                   */
  int prec_used;      /* FAB_PREC_FP32 or FAB_PREC_FP64                              */
  int whitened_at;    /* FAB_BASIS_WHITENED: step at which the basis was whitened
                         (0: never)                                                  */
  int ls_limit;       /* 1: the LSQR refinement stopped at its iteration limit before
                         meeting its stopping test (err_est then exceeds tol/10)     */
  int block_rhs;      /* served requests: right-hand sides of the block solve this
                         request ran in (1: on its own; see fab_set_block_limit)     */
  double latency_us;  /* submit-to-completion wall time                              */
} fab_info;

/* Create a context on `device` (HIP ordinal).  `arena_dev_ptr` (device memory,
 * e.g. a torch uint8 tensor's data) of `arena_bytes` bytes is sub-allocated for
 * matrices and per-request workspaces; pass NULL to let the library allocate
 * an arena of `arena_bytes` itself (freed by fab_finalize).  `hip_stream` is
 * the hipStream_t the blocking calls run on (NULL = the library's own stream);
 * served requests run on library-owned streams of the same device, one
 * admitted request per stream at a time: 12 of them, or FAB_SERVING_STREAMS
 * (1..16) from the environment.  They run concurrently only on as many HIP
 * hardware queues (GPU_MAX_HW_QUEUES, read when HIP starts: give one per
 * stream, plus the caller's own streams).
 * Errors: FAB_EINVAL (null ctx, arena_bytes < 1 MiB), FAB_EDEVICE.           */
int fab_init(fab_ctx* ctx, int device, void* arena_dev_ptr, size_t arena_bytes, void* hip_stream);

/* A constant-coefficient stencil operator (no device memory needed):
 * dim = 2 (nz must be 1) or 3; grid nx*ny*nz, row = x + nx*(y + ny*z);
 * coeff = (centre, x-1, x+1, y-1, y+1, z-1, z+1), each multiplying the value at
 * that neighbour; neighbours outside the grid are zero (Dirichlet).
 * Errors: FAB_EINVAL (dims < 1, n >= 2^31, dim mismatch).                     */
int fab_create_matrix_stencil(fab_ctx ctx, int dim, int nx, int ny, int nz,
                              const double coeff[7], fab_matrix* A);

/* A general sparse operator in CSR: rowptr int32[n+1], col int32[nnz],
 * val float32[nnz] (columns sorted or not).  The arrays are copied into the
 * arena (from host memory, or device memory if ptr_is_device != 0) and stay
 * resident until fab_destroy_matrix.
 * Errors: FAB_EINVAL (n < 1, nnz < 0, rowptr inconsistent), FAB_ENOMEM.        */
int fab_create_matrix_csr(fab_ctx ctx, int64_t n, int64_t nnz, const int32_t* rowptr,
                          const int32_t* col, const float* val, int ptr_is_device,
                          fab_matrix* A);

/* Release a matrix.  FAB_EBUSY while submitted requests still use it.         */
int fab_destroy_matrix(fab_matrix A);

/* Blocking solve: out = ||b|| V_m f(H_hat) e_1 per right-hand side.
 * nrhs in {1, 2, 4, 8, 16, 32}; b and out are FP64 device arrays [n][nrhs]
 * (out may not alias b).  info (nullable) is an array of nrhs records.
 * A lucky breakdown is not an error: the exact result is returned with
 * info.m_used < m.  Errors: FAB_EINVAL, FAB_ENOMEM (the workspace can never
 * fit the arena), FAB_ENUMERIC (non-finite b or result), FAB_EDEVICE.         */
int fab_solve(fab_ctx ctx, fab_matrix A, const double* b, int nrhs, fab_func f,
              const fab_params* p, double* out, fab_info* info);

/* Intermediate results of one solve, copied to HOST buffers the caller owns
 * (each pointer nullable; sizes per right-hand side, rhs-major):
 *   hbar  (m+1) x m  column-major: Hbar_m of eq. (3) (zero outside the band)
 *   sv    s x (m+1)  column-major: Theta V_{m+1}, the sketched normalised basis
 *   y     m          least-squares solution used for the last column (eq. (6))
 *   c     m          f(H_hat) e_1
 *   eta   m+1        norms of the stored (unnormalised) basis vectors          */
typedef struct {
  double* hbar;
  double* sv;
  double* y;
  double* c;
  double* eta;
} fab_diag;

/* fab_solve plus a copy of the intermediates into `diag` (for diagnostics and
 * stage-by-stage verification).  Same arguments, errors and semantics.       */
int fab_solve_diag(fab_ctx ctx, fab_matrix A, const double* b, int nrhs, fab_func f,
                   const fab_params* p, double* out, fab_info* info, const fab_diag* diag);

/* Size of the static device scratch that fab_solve_noalloc works in (per GPU). */
#define FAB_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* Allocation-free fab_solve, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  Same arguments, semantics and results as fab_solve (the same
 * kernels, launched directly), but the per-request workspace and the sampled
 * SRHT rows live in a static device array of FAB_NOALLOC_SCRATCH_BYTES that
 * the library holds on every GPU it runs on until the process ends, instead
 * of the context's arena; the call allocates nothing (no hipMalloc, no graph).
 * The caller still passes b and out (FP64 device arrays [n][nrhs]).
 * The array is shared by every call on that GPU and keeps the last call's
 * contents (every region the solve reads first is cleared by the solve
 * itself).  Calls on one GPU are serialised by the library (blocking, one at
 * a time per device); work of other kinds that a caller enqueues on the same
 * memory by other means would race with them.
 * Errors: as fab_solve; FAB_ESCRATCH when the workspace of the request (the
 * basis, (m+1) n nrhs elements of 4 or 8 bytes, plus small per-request
 * regions) exceeds FAB_NOALLOC_SCRATCH_BYTES, checked before any launch; with
 * FAB_PREC_AUTO an FP64 rerun that does not fit also returns FAB_ESCRATCH.  */
int fab_solve_noalloc(fab_ctx ctx, fab_matrix A, const double* b, int nrhs, fab_func f,
                      const fab_params* p, double* out, fab_info* info);

/* Non-blocking submit to the context's serving loop.  The request is admitted
 * when its workspace fits the arena next to the requests already running
 * (continuous batching: admitted requests run concurrently on separate
 * streams); until then it waits in FIFO order.  Single-rhs requests queued
 * together on the same matrix with the same function and fab_params (the
 * sketch seed included) are merged into one block solve of up to
 * fab_set_block_limit right-hand sides (a power of two): the operator is
 * applied to the whole block in each step (Algorithm 2 on a block of vectors;
 * Table 1 "matrix access" once per step for all of them).  Each column's
 * result equals the request's result alone to the basis precision (the
 * reductions group differently).  b and out must stay valid until completion
 * is reported.  Errors as fab_solve, reported at submit for argument checks
 * and at fab_poll/fab_wait for execution.                                    */
int fab_submit(fab_ctx ctx, fab_matrix A, const double* b, int nrhs, fab_func f,
               const fab_params* p, double* out, fab_request* req);

/* Never blocks.  *done = 1 once the request finished; then info (nullable,
 * nrhs records) is filled and the request's status is returned, and the
 * handle is released.  While running: *done = 0 and FAB_OK.
 * FAB_ENOTFOUND for an unknown or already-released handle.                   */
int fab_poll(fab_ctx ctx, fab_request req, int* done, fab_info* info);

/* Blocks until the request finishes; then as fab_poll with done = 1.          */
int fab_wait(fab_ctx ctx, fab_request req, fab_info* info);

/* Largest number of single-rhs served requests merged into one block solve
 * (1..32; 1 disables merging; default 32).  Errors: FAB_EINVAL.               */
int fab_set_block_limit(fab_ctx ctx, int max_rhs);

/* hold != 0: the serving loop admits no queued request until fab_hold(ctx, 0),
 * so that a burst submitted meanwhile is admitted (and merged) together;
 * running requests continue.  Blocking calls are not affected.
 * Errors: FAB_EINVAL (null ctx).                                              */
int fab_hold(fab_ctx ctx, int hold);

/* Kernel timing for measurement.  For the classes selected by a bit mask,
 * blocking solves on this context record a HIP event pair on the context's
 * stream around every launch and accumulate the elapsed times per class:      */
enum fab_kernel_class {
  FAB_K_DOTS = 0,     /* matvec + window dots + reductions (one per Krylov step);
                         sketched-GS basis: matvec + sketch partials              */
  FAB_K_UPDATE = 1,   /* Gram-Schmidt update + norm + fused sketch (one per step);
                         sketched-GS basis: u_i = w - V_{i-1} r_i                  */
  FAB_K_COMBINE = 2,  /* out = beta V_m c                                          */
  FAB_K_DENSE = 3,    /* sketched QR / least squares, f(H_hat) e_1, weights         */
  FAB_K_OTHER = 4,    /* first vector, final reduction; sketched-GS basis: sketch
                         reduction and the Gram-Schmidt step on the sketch        */
  FAB_K_NCLASS = 5
};
/* Time the classes whose bit (1 << class) is set in class_mask; 0 disables.
 * Errors: FAB_EINVAL (null ctx, mask out of range).                          */
int fab_profile_enable(fab_ctx ctx, int class_mask);
/* Launch count and summed duration in ms of class `cls` since the last reset;
 * reset != 0 clears that class.  Errors: FAB_EINVAL (bad ctx or class).        */
int fab_profile_read(fab_ctx ctx, int cls, long long* launches, double* total_ms, int reset);

/* Wait for all requests, release every matrix and the context.               */
int fab_finalize(fab_ctx ctx);

/* Static string naming a status code.                                         */
const char* fab_strerror(int code);

/* Library version string.                                                     */
const char* fab_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FAB_H */
