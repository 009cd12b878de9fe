/*
 * rid.h -- C ABI of the MI355X (gfx950) rid-preconditioned Davidson library.
 *
 * The library solves the linear-response TDDFT problems of Zhou & Parker,
 * "Converging TDDFT calculations in 5 iterations with minimal auxiliary
 * preconditioning":
 *   - the k lowest excitation energies of the TDA problem A X = Omega X
 *     (Eq. TDA) or of the full problem (Eq. Casida), by a Davidson method
 *     (Sec. 2.1, Fig. 1);
 *   - the dynamic polarizability alpha_uv(omega) (Eq. TDDFT_polar) by a
 *     Krylov linear solve;
 * with either the diagonal preconditioner or the minimal-auxiliary ris model
 * T applied through an inner Krylov solve (Eq. precondition, Sec. 3).
 *
 * Operators.  With orbital energies eps (occupied i, j; virtual a, b), a
 * three-index tensor B^P_pq with (pq|rs) = sum_P B^P_pq B^P_rs (Eq.
 * pqrs_approx, metric folded in) and exchange fraction a_x (c_x of
 * Eq. hessian), the XC kernel dropped:
 *   A   = diag(de) + 2K - a_x W,           B = 2K - a_x W',
 *   A+B = diag(de) + 4K - a_x (W + W'),    A-B = diag(de) - a_x (W - W'),
 * de_ia = eps_a - eps_i, K_{ia,jb} = (ia|jb), W_{ia,jb} = (ij|ab),
 * W'_{ia,jb} = (ib|ja).  The ris model T has the same form built from the ris
 * tensor: Coulomb from all naux_ris rows, exchange from the leading
 * naux_ris_k rows (the (d, s) split of Sec. 3.2) and only over orbitals inside
 * the energy window of Sec. 3.1 (virtuals with eps_a <= eps_HOMO + t_cut,
 * occupieds with eps_i >= eps_LUMO - t_cut).
 *
 * Layouts.  Response vectors have length N = no*nv, index ia = i*nv + a; a
 * block of n vectors is n contiguous vectors (row-major n x N).  Tensors are
 * row-major: b_ia (naux, no, nv), b_ij (naux, no, no), b_ab (naux, nv, nv);
 * the ij and ab slices must be symmetric.  Orbital energies are sorted
 * ascending within the occupied and within the virtual set.
 *
 * Memory.  Every pointer named *_dev is device memory on the context's
 * device; *_host is host memory.  Device tensors handed to
 * rid_problem_create are borrowed: the caller keeps them alive until
 * rid_problem_destroy and the library never frees or writes them.  All device
 * memory the library needs comes from the context's allocator.
 *
 * Streams.  All work is enqueued on the context's stream.  Solve calls are
 * synchronous: host outputs are valid on return, device outputs are written
 * in stream order.
 *
 * Errors.  Every call returns a rid_status.  Negative values are errors; the
 * message of the last error on a context is returned by rid_last_error.  No
 * call writes outputs after returning an error other than
 * RID_WARN_NOT_CONVERGED.  Handles are not thread-safe: use one context per
 * host thread (the server is internally threaded).
 */
#ifndef RID_H_
#define RID_H_

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define RID_API __attribute__((visibility("default")))
#else
#define RID_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rid_status;

#define RID_OK 0
#define RID_WARN_NOT_CONVERGED 1   /* outputs written with the last Ritz values */
#define RID_ERR_INVALID_ARG (-1)   /* null pointer, bad enum, bad option */
#define RID_ERR_SHAPE (-2)         /* inconsistent or out-of-range dimensions */
#define RID_ERR_DTYPE (-3)         /* unsupported tensor dtype */
#define RID_ERR_NO_MEMORY (-4)     /* allocator failed or budget exceeded */
#define RID_ERR_HIP (-5)           /* a HIP runtime call failed */
#define RID_ERR_INDEFINITE (-6)    /* A-B (or its projection) not positive definite */
#define RID_ERR_BREAKDOWN (-7)     /* every new direction dropped before convergence */
#define RID_ERR_NEAR_SINGULAR (-8) /* frequency within the guard of a pole */
#define RID_ERR_NO_DEVICE (-9)     /* no usable gfx950 device */
#define RID_ERR_INTERNAL (-10)
#define RID_ERR_CANCELLED (-11)    /* server request cancelled */
#define RID_ERR_TIMEOUT (-12)      /* server wait timed out */
#define RID_ERR_PENDING (-13)      /* server request not finished yet */

typedef enum { RID_F64 = 0, RID_F32 = 1, RID_BF16 = 2 } rid_dtype;
typedef enum { RID_PRECOND_DIAG = 0, RID_PRECOND_RIS = 1 } rid_precond;
/* RID_PRECISION_FP64: every product in FP64.  RID_PRECISION_MIXED: outer
 * products with FP32 operands (FP64 reduction of partial sums), ris products
 * with BF16 operands and FP32 accumulation; subspace orthonormalisation and
 * all projected (small dense) problems stay FP64. */
typedef enum { RID_PRECISION_FP64 = 0, RID_PRECISION_MIXED = 1 } rid_precision;
typedef enum { RID_TDA = 0, RID_RPA = 1 } rid_mode;
/* Operators for rid_apply_operator. */
typedef enum {
  RID_OP_A = 0,     /* y = A x */
  RID_OP_APB_AMB = 1, /* y = (A+B) x, y2 = (A-B) x */
  RID_OP_T = 2,     /* y = T x (ris model of A) */
  RID_OP_TPM = 3    /* y = T+ x, y2 = T- x (ris models of A+B, A-B) */
} rid_operator;

typedef struct rid_context rid_context;
typedef struct rid_problem rid_problem;
typedef struct rid_server rid_server;

/* Device memory provider (required by rid_context_create).  alloc returns a
 * device pointer with at least 256-byte alignment or NULL; free releases it.
 * Either may be called from any thread of the library -- the caller's, the
 * solve threads of rid_batch_solve and of the server, and their product
 * threads -- but never two at once: the library serialises the calls. */
typedef struct {
  void* user;
  void* (*alloc)(void* user, size_t bytes);
  void (*free)(void* user, void* ptr);
} rid_allocator;

typedef struct {
  int32_t no, nv;            /* occupied and virtual orbital counts, >= 1 */
  int32_t naux;              /* rows of the full tensor, >= 1 */
  int32_t naux_ris;          /* rows of the ris tensor, 0 = no ris tensor */
  int32_t naux_ris_k;        /* leading ris rows used for exchange, 0..naux_ris */
  double a_x;                /* exact-exchange fraction (c_x of Eq. hessian) */
  double t_cut_ha;           /* exchange energy window of Sec. 3.1, Hartree; <= 0 or inf = none */
  const double* eps_occ_host;  /* [no], ascending */
  const double* eps_vir_host;  /* [nv], ascending */
  const void* b_ia_dev;      /* (naux, no, nv) */
  const void* b_ij_dev;      /* (naux, no, no) symmetric slices */
  const void* b_ab_dev;      /* (naux, nv, nv) symmetric slices */
  int32_t b_dtype;           /* RID_F64, or RID_F32: then only MIXED-precision solves (FP32 outer
                                products) are possible and no FP32 copy is made */
  const void* bris_ia_dev;   /* (naux_ris, no, nv) or NULL */
  const void* bris_ij_dev;
  const void* bris_ab_dev;
  int32_t bris_dtype;        /* RID_F64, or RID_F32: then the ris model runs in BF16 only */
  /* Range-separated hybrid (optional; the paper's wB97X, Sec. 4): the
   * exchange integrals are a_x (pq|rs) + b_x (pq|rs)^LR with the long-range
   * integrals factored through a second tensor, (pq|rs)^LR = sum_Q C^Q_pq
   * C^Q_rs, so W -> a_x W + b_x W^LR and W' likewise (Coulomb unchanged).
   * C is borrowed like B, in b_dtype; the ris model uses every row of its own
   * long-range tensor (bris_dtype) inside the Sec. 3.1 window.  naux_lr = 0:
   * a global hybrid. */
  double b_x;
  int32_t naux_lr;
  const void* blr_ia_dev;    /* (naux_lr, no, nv) */
  const void* blr_ij_dev;    /* (naux_lr, no, no) symmetric slices */
  const void* blr_ab_dev;    /* (naux_lr, nv, nv) symmetric slices */
  int32_t naux_ris_lr;       /* rows of the ris model's long-range tensor */
  const void* brislr_ia_dev;
  const void* brislr_ij_dev;
  const void* brislr_ab_dev;
} rid_problem_desc;

typedef struct {
  int32_t precond;       /* rid_precond */
  int32_t precision;     /* rid_precision */
  double tol;            /* outer residual threshold (1e-5, Sec. 3) */
  int32_t max_iter;      /* outer iterations, >= 1 */
  int32_t n_extra_init;  /* -1: min(k,3) for ris, 8 for diag (Sec. 3.2) */
  double inner_tol;      /* inner relative threshold (1e-2, Sec. 3.1) */
  int32_t inner_max_iter;/* inner iterations (20, Sec. 3.1) */
  double init_tol;       /* ris initial-guess threshold (1e-3, Sec. 3.1) */
  int32_t init_max_iter; /* ris initial-guess iterations (20) */
  int32_t m_max;         /* subspace cap before restart, 0 = max(200, 40 k) */
  /* Warm start (eigen-solves): n_guess device vectors (n_guess x N, FP64,
   * row-major, caller-owned, read during the call) that span a start
   * subspace, e.g. the X (and Y) of a solve on a related problem.  When
   * given they replace the Sec. 3.2 initial guess (no ris guess solve); the
   * N_init unit vectors of the smallest de are appended and the set is
   * orthonormalised (dependent directions dropped).  NULL / 0: none. */
  const double* guess_dev;
  int32_t n_guess;
  /* 1: a solve that has the device to itself (not batched, not served, no
   * profiling) runs each operator-product shape (block width) once
   * directly and then as a captured HIP graph, replayed whenever that shape
   * recurs on the problem -- in this solve and in later solves on the same
   * problem.  The graph reads and writes staging copies of the vectors (two
   * or three device copies per product), and is captured again when the
   * problem's scratch has moved.  Results are bit-identical to 0. */
  int32_t graphs;
} rid_solve_opts;

#define RID_MAX_HISTORY 128

typedef struct {
  int32_t n_iter;        /* outer block products, the first included */
  int32_t n_mv;          /* vectors multiplied by the outer operator */
  int32_t n_inner_mv;    /* vectors multiplied by T (preconditioner + guess) */
  int32_t n_inner_iter;  /* inner block products */
  int32_t n_history;
  double history[RID_MAX_HISTORY]; /* max residual norm per outer iteration */
  double t_matvec_ms;    /* outer operator products (device time; submission time when sharing a batch) */
  double t_precond_ms;   /* preconditioner and ris initial guess */
  double t_other_ms;     /* projection, small dense, residuals, orthonormalisation */
  double t_total_ms;
  uint64_t bytes_resident; /* device bytes held by the solve at its peak */
  int32_t n_blocks_cholqr; /* new-direction blocks orthonormalised by two Cholesky-QR passes */
  int32_t n_blocks_mgs;    /* blocks that took modified Gram-Schmidt (near dependence, drops) */
} rid_stats;

/* ---- errors ---------------------------------------------------------- */
RID_API const char* rid_status_string(rid_status s);
/* Message of the last failing call on ctx (or of rid_context_create when
 * ctx is NULL).  Valid until the next call on the same context. */
RID_API const char* rid_last_error(const rid_context* ctx);

/* ---- context ----------------------------------------------------------
 * device: HIP device ordinal; hip_stream: a hipStream_t (NULL = the null
 * stream); alloc: required -- every device buffer the library uses comes
 * from alloc->alloc and goes back through alloc->free (the library never
 * calls hipMalloc); NULL, or a NULL callback, gives RID_ERR_INVALID_ARG. */
RID_API rid_status rid_context_create(int32_t device, void* hip_stream, const rid_allocator* alloc,
                              rid_context** out);
RID_API rid_status rid_context_destroy(rid_context* ctx);

/* ---- problem ----------------------------------------------------------
 * Validates the descriptor, copies the orbital energies, computes the
 * exchange window of Sec. 3.1 and makes the reduced-precision copies of the
 * tensors that MIXED solves use (FP32 full tensor, BF16 ris tensor), charged
 * to the allocator.  Borrowed tensors are never written. */
RID_API rid_status rid_problem_create(rid_context* ctx, const rid_problem_desc* desc, rid_problem** out);
RID_API rid_status rid_problem_destroy(rid_problem* prob);
/* Bytes the problem holds on the device (cast copies and constants). */
RID_API rid_status rid_problem_footprint(const rid_problem* prob, uint64_t* bytes);
/* Active exchange window: occupied i >= *i0, virtual a < *nv_act. */
RID_API rid_status rid_problem_window(const rid_problem* prob, int32_t* i0, int32_t* nv_act);

RID_API void rid_solve_opts_default(rid_solve_opts* opts);

/* ---- operator products (Eq. hessian; ris model of Sec. 2.2.2) --------
 * y_dev (and y2_dev for the pair operators) = op applied to the nvec vectors
 * x_dev (nvec x N, FP64).  precision: RID_F64 computes in FP64; RID_F32
 * reads FP32 copies of tensor and vectors (FP64 reduction of partial sums);
 * RID_BF16 (ris operators only) reads BF16 copies with FP32 accumulation.
 * Outputs are FP64.  Synchronous. */
RID_API rid_status rid_apply_operator(rid_problem* prob, int32_t op, int32_t precision, int32_t nvec,
                              const double* x_dev, double* y_dev, double* y2_dev);

/* ---- operator products without allocation ------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  Same
 * operation, arguments and layouts as rid_apply_operator, but:
 *   - every intermediate of the product (vector layouts in the compute type,
 *     Coulomb partial sums, exchange chunks S^P / Q^P, split partial sums)
 *     lives in one fixed device region of RID_NOALLOC_SCRATCH_BYTES per GPU,
 *     a static array of the library whose device address is looked up once
 *     per device by rid_context_create; the region is held until the
 *     process ends;
 *   - no allocator call, hipMalloc/hipFree, event creation or autotuning
 *     run (the tile shape follows the untuned default rule, at most 16
 *     partial sums per reduction, exchange chunks of at most one eighth of
 *     the region), and no profiling events are recorded; results agree with
 *     rid_apply_operator up to the rounding of the partial sums;
 *   - the problem's tensor copies for this operator and precision must exist
 *     already: a first rid_apply_operator or solve in that precision makes
 *     them (RID_ERR_INVALID_ARG otherwise);
 *   - a product whose intermediates do not fit the region returns
 *     RID_ERR_SHAPE before any kernel runs (roughly: nvec * N * 40 bytes of
 *     vector layouts plus the Coulomb and exchange partials must stay under
 *     128 MiB; the no=20, nv=80 problems fit with dozens of vectors);
 *   - the work is enqueued on the context's stream and the call returns
 *     without waiting: outputs are valid in stream order.
 * Every call on a GPU uses that GPU's one region and leaves the last call's
 * contents in it; the kernels overwrite every element of the region they
 * read, so nothing has to start at zero.  Calls whose work overlaps on one
 * GPU (other streams, other contexts, other host threads) race on the
 * region: order them on one stream. */
#define RID_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
RID_API rid_status rid_apply_operator_noalloc(rid_problem* prob, int32_t op, int32_t precision, int32_t nvec,
                                              const double* x_dev, double* y_dev, double* y2_dev);

/* ---- auxiliary-basis tensors from a molecule (Sec. 2.2.2) ---------------
 * The RI tensor of Eq. TDDFT-ris_approx, K^P_pq = (pq|P), J = (P|Q)^-1,
 * factored as B = sqrt(kappa) L^-1 K with (P|Q) = L L^T, so that
 * sum_P B^P_pq B^P_rs = kappa sum_PQ (pq|P) [(P|Q)^-1]_PQ (Q|rs); the three
 * blocks of B are what rid_problem_desc takes.  Molecular orbitals
 * p = sum_mu C_mu,p chi_mu over normalised s-type Gaussian atomic orbitals
 * chi_mu (exponents per atom, centred on the atoms).  The auxiliary basis is
 * either the list of shells given (nshell > 0: atom, angular momentum l <= 2,
 * exponent), or the minimal basis of the ris model (nshell = 0): one shell
 * of each l <= lmax on every atom with exponent theta / R_A^2 (the paper's
 * rid preconditioner: lmax = 2, theta = 0.6).  Functions are ordered s
 * shells first, then p (x, y, z), then d (real solid harmonics xy, xz, yz,
 * x^2 - y^2, 2 z^2 - x^2 - y^2), shells in the order given (minimal basis:
 * by atom); the leading naux_s rows of B are then the tensor of the s
 * functions alone -- pass naux_s as rid_problem_desc.naux_ris_k for the
 * (d, s) design of Sec. 3.2.  Lengths in bohr.  At most 1024 auxiliary
 * functions; RID_ERR_INDEFINITE when (P|Q) is not positive definite. */
typedef struct {
  int32_t natom;
  const double* coords_host;      /* natom x 3 */
  const double* radius_host;      /* natom: R_A of the exponent rule (minimal basis) */
  const int32_t* ao_count_host;   /* natom: s-type atomic orbitals on each atom */
  const double* ao_exp_host;      /* nao exponents, atom by atom */
  int32_t nao;
  const double* mo_dev;           /* nao x (no + nv), row-major, device, FP64 */
  int32_t no, nv;                 /* occupied orbitals first */
  double kappa;                   /* scale of the Coulomb operator (> 0) */
  int32_t nshell;                 /* > 0: the explicit shells below; 0: the minimal basis */
  const int32_t* shell_atom_host;
  const int32_t* shell_l_host;
  const double* shell_exp_host;
  double theta;                   /* minimal basis: exponent theta / R_A^2 */
  int32_t lmax;                   /* minimal basis: highest angular momentum, 0..2 */
} rid_aux_basis_desc;

/* Number of auxiliary functions (naux) and of s functions (naux_s). */
RID_API rid_status rid_aux_basis_size(const rid_aux_basis_desc* desc, int32_t* naux, int32_t* naux_s);
/* Build b_ia (naux, no, nv), b_ij (naux, no, no), b_ab (naux, nv, nv) into
 * the caller's FP64 device buffers, on the context stream; synchronous.
 * Scratch (the integrals over atomic orbitals, naux * nao^2 doubles, and
 * the transformed tensor) comes from the context's allocator. */
RID_API rid_status rid_aux_tensor_build(rid_context* ctx, const rid_aux_basis_desc* desc, double* b_ia_dev,
                                        double* b_ij_dev, double* b_ab_dev);

/* ---- eigen-solve (Sec. 2.1; Eqs. TDA, Casida) ---------------------------
 * The k lowest roots in ascending order into omega_host[k].  TDA: x_dev
 * (k x N, optional) gets unit-norm eigenvectors.  RPA: x_dev and y_dev
 * (optional) get X and Y with X^T X - Y^T Y = 1.  resid_host (optional, k)
 * gets the final residual norms.  Returns RID_WARN_NOT_CONVERGED when
 * max_iter is reached (outputs written), RID_ERR_INDEFINITE when the
 * projected A-B is not positive definite, RID_ERR_BREAKDOWN when every new
 * direction is dropped. */
RID_API rid_status rid_eigen_solve(rid_problem* prob, const rid_solve_opts* opts, int32_t k, int32_t mode,
                           double* omega_host, double* x_dev, double* y_dev, double* resid_host,
                           rid_stats* stats);

/* ---- polarizability (Eq. TDDFT_polar) -----------------------------------
 * alpha_uv(w_f) = -2 P_u^T U_v(w_f), (A+B) U - w U' = -P, (A-B) U' - w U = 0,
 * for p_dev (nrhs x N) and the nfreq frequencies omega_host (Hartree, >= 0).
 * alpha_host: nfreq x nrhs x nrhs; u_dev (optional): nfreq x nrhs x N;
 * resid_host (optional): nfreq x nrhs relative residuals.  Frequencies at or
 * above 0.999 times the lowest diagonal element de_min give
 * RID_ERR_NEAR_SINGULAR before any work is done. */
RID_API rid_status rid_response_solve(rid_problem* prob, const rid_solve_opts* opts, int32_t nrhs,
                              const double* p_dev, int32_t nfreq, const double* omega_host,
                              double* alpha_host, double* u_dev, double* resid_host,
                              rid_stats* stats);

/* ---- persistent tuning ----------------------------------------------------
 * The first product of every GEMM launch shape on a context times the tile
 * configurations and keeps the fastest.  rid_tune_save writes those
 * decisions to a text file, rid_tune_load adds a file's decisions to a
 * context (replacing its own decision for a shape listed in both), so that a new process
 * skips the timing runs.  The file records the library build and the device
 * architecture; a file from another build or device, or a malformed one, is
 * refused with RID_ERR_INVALID_ARG and changes nothing.  count (optional)
 * receives the number of decisions written or read.  Tuning never changes a
 * result: every tile configuration sums in the same order. */
RID_API rid_status rid_tune_save(rid_context* ctx, const char* path, int32_t* count);
RID_API rid_status rid_tune_load(rid_context* ctx, const char* path, int32_t* count);

/* ---- kernel profiling ---------------------------------------------------
 * While enabled, every launch of the library's main kernel families is
 * bracketed by HIP events on the stream it runs on (the recording costs a
 * few percent of a solve's time; rid_profile_only limits it to one family).
 * rid_profile_read waits for the context stream and returns per-family
 * totals (launch count, summed event time, algorithmic FLOPs and bytes) of
 * the launches that have completed, then resets them; launches still running
 * on other streams (batched or served solves) count at a later read.  Both
 * calls are safe while solves run on other threads.
 * Families: "exch_s" (S^P = B_ij X), "exch_w" (sum_P S^P B_ab), "exch_q"
 * (Q^P = B_ia X^T), "exch_wp" (sum_P Q^P B_ja), "coul_fwd", "coul_bwd",
 * "combine", "ris_*" (the same families of the ris model), "gram", "combo",
 * "small_dense". */
typedef struct {
  char name[32];
  int64_t launches;
  double total_ms;
  double flops;  /* algorithmic floating-point operations, summed */
  double bytes;  /* algorithmic HBM bytes, summed */
} rid_kernel_stat;

RID_API rid_status rid_profile_enable(rid_context* ctx, int32_t on);
/* Record only the launches of one family (for example "exch_w"), so that
 * the timing of one kernel costs a fraction of the events; NULL: every
 * family again.  Takes effect for launches enqueued after the call. */
RID_API rid_status rid_profile_only(rid_context* ctx, const char* family);
RID_API rid_status rid_profile_read(rid_context* ctx, rid_kernel_stat* out, int32_t cap, int32_t* n);

/* ---- batched solves (many molecules per launch) -------------------------
 * A request is an eigen-solve (kind 0: k, mode) or a polarizability solve
 * (kind 1: nrhs, p_dev, nfreq, omega_host).  Results are written into the
 * caller-owned rid_result of each request.  rid_batch_solve runs up to 16
 * solves at once (largest first, while their estimated footprints fit 80% of
 * the device memory free at the call), each on a stream of its own; the
 * operator products of all
 * solves waiting at the same time go out together, one persistent grouped
 * GEMM launch per contraction stage and tile shape.  Each result equals
 * that of the same request solved alone.  Returns the worst status. */
typedef struct {
  int32_t kind;            /* 0 = eigen, 1 = polarizability */
  int32_t k, mode;         /* eigen */
  int32_t nrhs, nfreq;     /* polarizability */
  const double* p_dev;     /* nrhs x N */
  const double* omega_host;/* nfreq */
  rid_solve_opts opts;
  double* x_dev;           /* eigen: optional output X (k x N, device, caller-owned) or NULL */
  double* y_dev;           /* eigen RPA: optional output Y (k x N) or NULL */
} rid_request;

typedef struct {
  rid_status status;
  double* omega_host;      /* caller buffer: k (eigen) */
  double* alpha_host;      /* caller buffer: nfreq*nrhs*nrhs (polarizability) */
  double* resid_host;      /* caller buffer or NULL */
  rid_stats stats;
  double t_arrival_ms, t_admit_ms, t_done_ms; /* server timestamps; rid_batch_solve: 0, start, end of
                                                 the request from the start of the batch */
} rid_result;

RID_API rid_status rid_batch_solve(rid_context* ctx, int32_t n, rid_problem* const* probs,
                           const rid_request* reqs, rid_result* results);

/* Estimated device bytes a request needs while it runs (subspace, products,
 * inner-solve blocks, operator scratch); the server and rid_batch_solve
 * admit by it.  The problem's own tensor copies (FP32 casts and transposes,
 * BF16 ris copies) are made when a request is submitted or a batch starts,
 * and count in rid_problem_footprint instead. */
RID_API rid_status rid_request_footprint(const rid_problem* prob, const rid_request* req, uint64_t* bytes);

/* ---- continuous-batching server -----------------------------------------
 * Requests are admitted in arrival order while their estimated device
 * footprint fits hbm_budget_bytes and one of max_slots (1..64) slots is free.
 * Admitted requests run at the same time, each keeping its subspace in device
 * memory; their operator products are grouped as in rid_batch_solve, and a
 * request admitted while others run joins their grouped launches at once.
 * States: queued -> running -> done / failed / cancelled. */
typedef struct {
  uint64_t hbm_budget_bytes;
  int32_t max_slots;
} rid_server_opts;

RID_API rid_status rid_server_create(rid_context* ctx, const rid_server_opts* opts, rid_server** out);
RID_API rid_status rid_server_submit(rid_server* srv, rid_problem* prob, const rid_request* req,
                             rid_result* result, uint64_t* ticket);
/* RID_OK when done (result written), RID_ERR_PENDING otherwise. */
RID_API rid_status rid_server_poll(rid_server* srv, uint64_t ticket);
RID_API rid_status rid_server_wait(rid_server* srv, uint64_t ticket, int32_t timeout_ms);
RID_API rid_status rid_server_cancel(rid_server* srv, uint64_t ticket);
RID_API rid_status rid_server_destroy(rid_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* RID_H_ */
