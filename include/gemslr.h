/*
 * gemslr.h -- C ABI of the MI355X GeMSLR preconditioner library (libgemslr.so)
 *
 * GeMSLR is the multilevel Schur-complement low-rank preconditioner of
 * Xu, Kalantzis, Li and Saad, "parGeMSLR: A Parallel Multilevel Schur
 * Complement Low-Rank Preconditioning and Solution Package for General Sparse
 * Matrices" (arXiv 2205.03224).  The library builds the preconditioner on the
 * host and one GPU (Alg. 1), applies M^{-1} on the GPU (Alg. 2) and runs
 * right-preconditioned flexible GMRES around it (Sec. 4.1, Sec. 5).
 *
 * Conventions for every entry point:
 *  - Return value: GS_OK (0) on success, > 0 for a usable but incomplete
 *    result, < 0 for an error.  No C++ exception crosses this boundary; the
 *    message of the last error of a context is available from gs_last_error.
 *  - Pointers documented as "host" are read during the call only and stay
 *    owned by the caller.  Pointers documented as "device" are caller-owned
 *    device memory (e.g. torch tensors) on the context's device; the library
 *    never frees them.
 *  - Values of type GS_C128 are interleaved (re, im) float64 pairs.
 *  - Sparse matrices are CSR: rowptr (int64, n+1, rowptr[0] = 0),
 *    col (int32, sorted strictly ascending inside each row), values.
 *  - Device work is queued on the context's HIP stream; functions that hand
 *    a result to the host (solve, the setup routines) synchronise it.
 */
#ifndef GEMSLR_H
#define GEMSLR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- codes */
enum {
  GS_OK = 0,
  GS_NOT_CONVERGED = 1, /* solve stopped at maxit; best iterate returned      */
  GS_EINVAL = -1,       /* invalid argument or malformed CSR                    */
  GS_EZEROPIVOT = -2,   /* zero or non-finite pivot in an incomplete LU          */
  GS_ESINGULAR = -3,    /* |1 - theta| < 1e-12 for a Ritz value: I - R singular  */
  GS_EDEVICE = -4,      /* HIP runtime error                                     */
  GS_ESTATE = -5,       /* call out of order (e.g. apply before setup)           */
  GS_ENOMEM = -6        /* device or host allocation failed                      */
};

enum { GS_F64 = 0, GS_C128 = 1 };                  /* value type of A, b, x  */
enum { GS_PREC_F64 = 0, GS_PREC_F32 = 1, GS_PREC_BF16 = 2 }; /* apply storage */
enum { GS_ILUT = 0, GS_ILU0 = 1 };

/* ---------------------------------------------------------------- options */
typedef struct {
  int ilu_kind;           /* GS_ILUT (dual threshold, Saad 1994) or GS_ILU0   */
  int lfil;               /* ILUT: max entries kept per row in L and in U,
                             diagonal excluded                        [10]    */
  int fgmres_restart;     /* FGMRES cycle length m (Sec. 5)           [50]    */
  int maxit;              /* total FGMRES iteration cap (Sec. 5)      [1000]  */
  double arnoldi_tol;     /* Ritz residual / |theta| accepted: two digits
                             of accuracy (Sec. 5)                     [1e-2]  */
  int arnoldi_max_cycles; /* thick-restart cycles per level           [20]    */
  int lowrank_last_level; /* 1: low-rank term also at level L-1       [1]     */
  int precision;          /* GS_PREC_*: storage of L, U, E, F, W in the apply;
                             F32/BF16 solve in float32           [GS_PREC_F64] */
  int grid_ndim;          /* >0: A is a grid operator with lexicographic
                             numbering x + N0*y + N0*N1*z (geometric
                             separator); 0: nested dissection of the graph
                             of A (gs_partition_graph)                   [0]  */
  int32_t grid_dims[3];   /* points per axis for the geometric separator     */
  uint64_t seed;          /* Arnoldi start vectors (SplitMix64)        [0]    */
  int nthreads;           /* host threads for the factorisation (0 = all)     */
  int defer_lowrank;      /* 1: gs_setup stops after the factorisation; the
                             rank-k terms are built later by gs_lowrank  [0]  */
  int block_max_iters;    /* gs_lowrank: the block iteration from a starting
                             basis may use block_max_iters * k products of
                             G_l before falling back to Arnoldi          [8]  */
  int inner_gmres_its;    /* steps of right-preconditioned GMRES on
                             S_hat_0 = C_0 - E_0 U_0^{-1} L_0^{-1} F_0 inside
                             every apply (Alg. 2, l = 0), preconditioned by
                             the l > 0 branch; 0 = none, at most 16, float64
                             and complex128 forms only.  Nonzero makes M^{-1}
                             vary with its input (FGMRES handles that)   [0]  */
  double ilu_shift;       /* s: every on-diagonal block (B_l and the blocks of
                             C_last) is factored as B + i s mean|a_ii| I, the
                             mean over A's diagonal (Sec. 5, Helmholtz: the
                             paper uses s = 0.05); complex A only; E, F and
                             the Schur products keep A unshifted         [0]  */
  int warm_start;         /* gs_lowrank with starting bases Y_l: 0 = block
                             Rayleigh-Ritz iteration from span(Y_l); 1 =
                             the thick-restart Arnoldi of Sec. 2.3 started
                             from v_0 = Y_l Y_l^T r (r the seeded start
                             vector), a vector of the predicted subspace
                                                                         [0]  */
  /* Optional partition given by the caller (host arrays, read during
   * gs_setup; all NULL: the library partitions A itself, Alg. 3).  Same
   * format as gs_partition_grid writes: part_perm[new] = old (n entries),
   * part_level_start (part_nlevels + 2 entries: starts of B_0 .. B_{L-1},
   * C_last, then n), and optionally part_block_ptr / part_block_count (the
   * diagonal blocks of every segment).  Without block lists each segment's
   * blocks are the connected components of its rows in the graph of A,
   * which must each be contiguous in part_perm.  gs_setup's levels and
   * nparts are then not used.  Checked as gs_partition_check does.   [NULL] */
  const int64_t* part_perm;
  const int64_t* part_level_start;
  int part_nlevels;
  const int64_t* part_block_ptr;
  const int64_t* part_block_count;
} gs_opts;

/* Fill *opts with the defaults shown in brackets above. */
void gs_opts_default(gs_opts* opts);

/* ---------------------------------------------------------------- info */
#define GS_MAX_LEVELS 8
typedef struct {
  int its;                  /* FGMRES iterations of the last solve           */
  double relres;            /* true ||b - A x|| / ||b|| at exit (float64)     */
  int converged;            /* 1 if relres <= tol                             */
  int nlevels;              /* L: levels with a Schur complement              */
  int64_t d[GS_MAX_LEVELS + 1];      /* rows of B_l (index L: C_last)          */
  int64_t s[GS_MAX_LEVELS + 1];      /* rows of C_l                           */
  int64_t nblocks[GS_MAX_LEVELS + 1];
  int32_t k[GS_MAX_LEVELS + 1];      /* rank kept at level l                  */
  int32_t depth_l[GS_MAX_LEVELS + 1];/* max wavefront depth of L over blocks  */
  int32_t depth_u[GS_MAX_LEVELS + 1];/* same for U                            */
  int32_t arnoldi_cycles[GS_MAX_LEVELS + 1];
  int32_t arnoldi_matvecs[GS_MAX_LEVELS + 1];
  int32_t arnoldi_converged[GS_MAX_LEVELS + 1];
  int32_t lowrank_method[GS_MAX_LEVELS + 1]; /* 0 Arnoldi, 1 block iteration
                                                from a given basis, 2 block
                                                iteration then Arnoldi fallback,
                                                3 Arnoldi started in the span
                                                of a given basis */
  int64_t nnz_lu;           /* sum of nnz(L)+nnz(U) incl. diagonals, all levels */
  int64_t nnz_ef;           /* sum of nnz(E_l)+nnz(F_l)                       */
  int64_t nnz_a;            /* nnz(A)                                         */
  double fill;              /* nnz_lu / nnz_a (Sec. 5 "fill")                 */
  double fill_lowrank;      /* (nnz_lu + sum s_l k_l + k_l^2) / nnz_a         */
  double apply_bytes;       /* compulsory HBM bytes of one apply: every
                               factor, E/F/W entry and index read once, every
                               vector entry read or written once per launch */
  double t_partition, t_factor, t_layout, t_lowrank, t_solve; /* seconds     */
} gs_info;

/* ---------------------------------------------------------------- context */
typedef struct gs_ctx gs_ctx;

/* Create a context on HIP device `device` that queues its work on `stream`
 * (a hipStream_t, e.g. torch.cuda.current_stream().cuda_stream; NULL = the
 * device's null stream).  device < 0 creates a host-only context that can
 * run the host stages (partition, factorisation) but not apply/solve.
 * Errors: GS_EINVAL (ctx NULL), GS_EDEVICE. */
int gs_create(gs_ctx** ctx, int device, void* stream);

/* Release every resource the context owns.  NULL is ignored. */
void gs_destroy(gs_ctx* ctx);

/* Message of the context's last error ("" if none); valid until the next
 * call on the context.  ctx NULL returns the last error of a call without a
 * context (gs_create and the host stages gs_partition_*, gs_ilu). */
const char* gs_last_error(const gs_ctx* ctx);

/* ---------------------------------------------------------------- setup */
/* Build M^{-1} for the n x n matrix A (Alg. 1, Sec. 4.2):
 *  - reorder A with a multilevel p-way vertex separator (Alg. 3, Sec. 3)
 *    into `levels` levels of `nparts` parts (fewer when the separator is too
 *    small to split, Sec. 3.2): the geometric separator when
 *    opts->grid_ndim > 0, else nested dissection of A's graph (nparts a
 *    power of two);
 *  - incomplete LU of every diagonal block of B_l (ILUT(drop_tol, lfil) or
 *    ILU(0)), and block-Jacobi ILU of the last separator (Sec. 4.3);
 *  - rank-`rank` Schur-complement correction W_l, R_l at every level,
 *    bottom-up, by thick-restart Arnoldi on G_l = E_l U_l^{-1} L_l^{-1} F_l
 *    C_l^{-1} with cycle length 2*rank (Sec. 2.3, Sec. 4.2), run on the GPU.
 * A (host CSR, dtype GS_F64 or GS_C128) is copied; the caller keeps it.
 * Errors: GS_EINVAL (malformed CSR, missing diagonal, n <= 0, rank < 0,
 * nparts not a dim-th power, no grid), GS_EZEROPIVOT, GS_ESINGULAR,
 * GS_EDEVICE, GS_ENOMEM.  A previous setup of the context is released. */
int gs_setup(gs_ctx* ctx, int64_t n, const int64_t* rowptr,
             const int32_t* col, const void* val, int dtype, int levels,
             int nparts, int rank, double drop_tol, const gs_opts* opts);

/* One level of an explicitly given preconditioner, in permuted numbering.
 * Level l acts on the index range [start_l, n) of the permuted vector:
 * B_l = [start_l, start_l + d) and C_l = [start_l + d, n), s = n - start_l - d
 * (Sec. 2.4; the per-level permutations compose into one).  The final entry
 * (C_last, Sec. 4.3) has s = 0 and no E, F, W, H.  All pointers are host,
 * values of the context's dtype. */
typedef struct {
  int64_t d;                    /* rows of B_l                                  */
  int64_t nblocks;              /* diagonal blocks of B_l                       */
  const int64_t* block_ptr;     /* nblocks+1 row offsets in [0, d]              */
  const int64_t* l_rowptr; const int32_t* l_col; const void* l_val;
                                /* strictly lower ILU factor (unit diagonal
                                   implied), d x d, level-local columns         */
  const int64_t* u_rowptr; const int32_t* u_col; const void* u_val;
                                /* upper ILU factor with diagonal, d x d        */
  const int64_t* e_rowptr; const int32_t* e_col; const void* e_val;
                                /* E_l: s x d (rows in C_l, columns in B_l)     */
  const int64_t* f_rowptr; const int32_t* f_col; const void* f_val;
                                /* F_l: d x s (rows in B_l, columns in C_l)     */
  int32_t k;                    /* rank of the correction, 0 <= k <= min(s, 1024) */
  const void* w;                /* W_l: s x k, column-major                     */
  const void* h;                /* H_l = (I - R_l)^{-1} - I: k x k, column-major */
} gs_level_data;

/* Install an explicitly given preconditioner (same M^{-1} as an external
 * setup, e.g. for checking the apply against an independent
 * implementation).  A is the unpermuted matrix (used by gs_solve); perm[i]
 * is the original index of permuted position i; levels has nlevels+1
 * entries whose d sum to n.  Copies everything.  Errors: GS_EINVAL (also
 * for a malformed block: NULL or non-monotone rowptr, rowptr[0] != 0, a
 * column out of range, NULL col/val of a block with entries, NULL w or h
 * with k > 0), GS_EDEVICE, GS_ENOMEM. */
int gs_setup_explicit(gs_ctx* ctx, int64_t n, const int64_t* rowptr,
                      const int32_t* col, const void* val, int dtype,
                      const int64_t* perm, int nlevels,
                      const gs_level_data* levels, const gs_opts* opts);
/* On a host-only context (gs_create with device < 0) gs_setup_explicit keeps
 * the host copy only: gs_export, gs_get_level*, gs_get_perm and gs_get_info
 * work; apply, solve and precision changes return GS_ESTATE. */

/* Write the installed preconditioner -- the setup product of Alg. 1: A, the
 * permutation and, per level, the block partition, the ILU factors L_l and
 * U_l, E_l, F_l, W_l and H_l -- to the host file `path` (created or
 * truncated).  Layout, little endian ("value": 8 bytes for GS_F64, 16 for
 * GS_C128 as interleaved re, im; a CSR block is int64 nnz, int64
 * rowptr[rows + 1], int32 col[nnz], value val[nnz]; all numbering as in
 * gs_level_data):
 *   char[8] "GEMSLR01", int32 dtype, int32 nlevels L, int64 n,
 *   CSR A (n rows, original numbering), int64 perm[n],
 *   for l = 0 .. L: int64 d, int64 nblocks, int64 block_ptr[nblocks + 1],
 *     CSR L_l (d rows), CSR U_l (d rows), then for l < L (s = n - start_l
 *     - d): CSR E_l (s rows), CSR F_l (d rows), int32 k, int32 0,
 *     value W_l[s*k], value H_l[k*k] (both column-major),
 *   char[8] "GEMSLREN".
 * Works on device and host-only contexts.  Errors: GS_ESTATE (no setup),
 * GS_EINVAL (NULL path, file not writable or a write failed). */
int gs_export(const gs_ctx* ctx, const char* path);

/* Install the preconditioner of a file written by gs_export, exactly as
 * gs_setup_explicit of its contents (so applies equal those of the exporting
 * context bit for bit in the same storage precision); opts as for
 * gs_setup_explicit (NULL: keep the context's options).  A previous setup is
 * released.  Errors: GS_EINVAL (unreadable file, bad magic or end marker,
 * truncated or inconsistent contents -- every array is validated as in
 * gs_setup_explicit), GS_EDEVICE, GS_ENOMEM. */
int gs_import(gs_ctx* ctx, const char* path, const gs_opts* opts);

/* Change the storage precision of the installed preconditioner (GS_PREC_*):
 * the factors, E, F and W are re-uploaded from the host copy.  FGMRES,
 * residuals and orthogonalisation stay float64.  Real dtype only for
 * F32/BF16.  Errors: GS_ESTATE, GS_EINVAL, GS_EDEVICE. */
int gs_set_precision(gs_ctx* ctx, int precision);

/* ---------------------------------------------------------------- apply */
/* y = M^{-1} x (Alg. 2; opts.inner_gmres_its inner steps at level 0, none by
 * default, in which case M^{-1} is a fixed linear operator).  x, y: device,
 * n values of the context's dtype, original (unpermuted) ordering; they must
 * not alias.  Asynchronous on the context's stream.
 * Errors: GS_ESTATE (no setup), GS_EINVAL (NULL or aliasing), GS_EDEVICE. */
int gs_apply(gs_ctx* ctx, const void* x, void* y);

/* Same as gs_apply for `nrhs` vectors stored one after another
 * (x + j*n, y + j*n), device memory, x and y not overlapping.  With two or
 * more vectors every launch of a level covers all of them (several
 * right-hand sides per factor pass, named as future work in Sec. 6).  In a
 * triangular sweep a workgroup may sweep a group of up to 8 vectors over
 * the same staged chunks of factor entries, which then cross HBM once for
 * the group; the group size per level follows from how many workgroups LDS
 * lets share a CU: groups pay where one vector's workgroups already fill
 * every CU (level 0: three vectors per workgroup at the 3,375 - 4,096-row
 * blocks of the 128^3 workloads), single-vector workgroups where one vector
 * leaves CUs idle.  With inner GMRES steps the vectors go one at a time.
 * Every column equals gs_apply of that column.  nrhs = 0 is an empty batch:
 * nothing is read or written, and x and y may be NULL.  Errors as gs_apply,
 * and GS_EINVAL for nrhs < 0. */
int gs_apply_many(gs_ctx* ctx, int nrhs, const void* x, void* y);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): gs_apply
 * with every scratch buffer of the apply (the permuted working vector, the
 * partial sums of W_l^H z_2, staging vectors) cut from a static device
 * region of 64 MiB (67,108,864 bytes) that the library holds on each GPU
 * until the process ends.  The call allocates nothing; the preconditioner's
 * own data stay where the setup put them.  x, y as for gs_apply.  Every call
 * on one GPU uses the same region: calls that overlap in time on one GPU
 * (several streams, several host threads) race and must be ordered by the
 * caller.  No region content has to start at zero (each apply writes every
 * scratch entry before reading it).
 * Errors: GS_ESTATE (no setup), GS_EINVAL (NULL or aliasing vectors; scratch
 * needed above 64 MiB -- e.g. n above ~4.1M float64 unknowns; inner GMRES
 * steps switched on), GS_EDEVICE. */
int gs_apply_noalloc(gs_ctx* ctx, const void* x, void* y);

/* ---------------------------------------------------------------- learned start */
/* Per-node features of the interface unknowns C_l of level l (0 <= l < L), for
 * a network that predicts starting bases of the low-rank terms.  Host only
 * (after a setup).  X: host, s_l x ncols row-major float32 (cols_cap >= 38);
 * *ncols receives the feature count.  Features of node j (grid operators):
 * normalised coordinates (3), sin/cos(m pi coordinate), m = 1..4, per axis
 * (24), per-axis "coordinate on a cut" flags (3), log(|a_jj| / mean |a_ii|)
 * and its mean over grid neighbours (2), per-axis convection proxy
 * (a_{j,+axis} - a_{j,-axis}) / |a_jj| (3), sum |E_l(j,:)| / |a_jj| and
 * sum |F_l(:,j)| / |a_jj| (2), level / L (1).
 * Errors: GS_ESTATE, GS_EINVAL. */
int gs_features(const gs_ctx* ctx, int level, float* X, int64_t rows_cap, int cols_cap,
                int* ncols);

/* Build (or rebuild) the rank-`rank` terms of every level bottom-up on the
 * GPU (Sec. 4.2).  warm: NULL, or L device pointers (entries may be NULL);
 * warm[l] is a float32 s_l x rank row-major starting basis for level l (the
 * future-work "block" setup of Sec. 6): the level then runs a block
 * Rayleigh-Ritz iteration -- Ritz pairs of the search space V (starting as
 * orth(warm[l]), at most 3k columns), expansion by the residuals of the
 * wanted pairs not yet accepted, thick restart to the leading wanted Ritz
 * vectors when full -- accepted when every wanted Ritz pair meets
 * opts.arnoldi_tol; after opts.block_max_iters * k products it falls back to
 * thick-restart Arnoldi.  Levels without a basis use Arnoldi.  Per-level
 * product counts (both methods together) and the method used go to gs_info.
 * Errors: GS_ESTATE, GS_EINVAL, GS_ESINGULAR, GS_EDEVICE. */
int gs_lowrank(gs_ctx* ctx, int rank, const float* const* warm);

/* The network of the learned start (not in the paper): a 3-layer perceptron
 * in -> hidden -> hidden -> out with tanh after the first two layers, all
 * float32 on the GPU, trained with the rotation-invariant subspace loss
 * ||Y^T Y||_F^2 - 2 ||W^T Y||_F^2 + k_w against bases W from the library's own
 * Arnoldi.  Parameters are packed W1 (in x hidden, row-major), b1, W2, b2, W3,
 * b3.  Layer widths <= 64.  Errors: GS_EINVAL, GS_EDEVICE. */
typedef struct gs_mlp gs_mlp;
/* The weights start Glorot-uniform, biases at zero: packed parameter j (a
 * weight of the layer a -> b) is sqrt(6 / (a + b)) * v_j with v the SplitMix64
 * start vector of `seed` (2 u_j - 1, u_j the top 53 bits of its j-th output;
 * the generator of the Arnoldi start vectors), so a seed fixes the network
 * before training; gs_mlp_set_params overwrites it. */
int gs_mlp_create(gs_mlp** mlp, int in_dim, int hidden, int out_dim, uint64_t seed, int device,
                  void* stream);
void gs_mlp_destroy(gs_mlp* mlp);
int gs_mlp_nparams(const gs_mlp* mlp);
const char* gs_mlp_last_error(const gs_mlp* mlp);
/* host arrays of gs_mlp_nparams floats; set_params also resets Adam state */
int gs_mlp_set_params(gs_mlp* mlp, const float* params);
int gs_mlp_get_params(const gs_mlp* mlp, float* params);
int gs_mlp_get_grads(const gs_mlp* mlp, float* grads);
int gs_mlp_zero_grad(gs_mlp* mlp);
/* Y = network(X): device, X rows x in, Y rows x out, row-major float32 */
int gs_mlp_forward(gs_mlp* mlp, const float* X, int64_t rows, float* Y);
/* Forward on X, loss against the target basis W (device, rows x kw
 * row-major), gradients added to the accumulated ones; *loss on the host. */
int gs_mlp_loss_backward(gs_mlp* mlp, const float* X, const float* W, int64_t rows, int kw,
                         double* loss);
/* One Adam update (bias-corrected) of the parameters with the accumulated
 * gradients. */
int gs_mlp_adam_step(gs_mlp* mlp, float lr, float beta1, float beta2, float eps);

/* ---------------------------------------------------------------- measurement */
/* Run `reps` applies of x (as gs_apply) with a HIP event pair recorded on the
 * context's stream around every kernel launch.  On return *nsteps holds the
 * launches per apply (<= cap) and, for launch i in launch order, step_ms[i] is
 * its mean duration in ms and step_bytes[i] its compulsory HBM bytes (every
 * stored array read once, every vector entry read or written once per touch).
 * Labels: gs_apply_step_label.  For measurement only; synchronises.
 * Errors: GS_ESTATE, GS_EINVAL (also cap too small), GS_EDEVICE. */
int gs_apply_profile(gs_ctx* ctx, const void* x, void* y, int reps, double* step_ms,
                     double* step_bytes, int cap, int* nsteps);
/* Label of launch i of the last gs_apply_profile ("" if out of range). */
const char* gs_apply_step_label(const gs_ctx* ctx, int i);

/* Event probe: after this call every launch of kernel class `kind`
 * (0 = block triangular solves of level 0, 1 = those of the other levels,
 * 2 = interface step, 3 = low-rank update, 4 = permutations; -1 = off) made by
 * later gs_apply / gs_solve calls is bracketed by a HIP event pair on the
 * context's stream, up to max_launches launches.  gs_probe_read synchronises
 * and returns the probed launch count, their summed duration (ms) and summed
 * compulsory bytes since the previous read.  Errors: GS_ESTATE, GS_EINVAL. */
int gs_probe_enable(gs_ctx* ctx, int kind, int max_launches);
int gs_probe_read(gs_ctx* ctx, int64_t* launches, double* total_ms, double* total_bytes);

/* ---------------------------------------------------------------- solve */
/* Solve A x = b by right-preconditioned FGMRES(m) with M^{-1} applied every
 * iteration (Sec. 4.1, Sec. 5).  b, x: device, n values, original ordering;
 * x holds the initial guess on entry and the iterate on exit.  Stops when the
 * float64 true residual ||b - A x|| / ||b|| <= tol.  Synchronises the stream.
 * Returns GS_OK, or GS_NOT_CONVERGED after opts.maxit iterations with the
 * best iterate in x.  info may be NULL.  Errors: GS_ESTATE, GS_EINVAL,
 * GS_EDEVICE. */
int gs_solve(gs_ctx* ctx, const void* b, void* x, double tol, gs_info* info);

/* Copy the setup statistics (sizes, ranks, depths, fill, timings). */
int gs_get_info(const gs_ctx* ctx, gs_info* info);

/* ---------------------------------------------------------------- host stages */
/* Check a partition given by the caller against the pattern of A and
 * complete its block lists (host only; usable without a device).
 *  perm, level_start, nlevels: as gs_partition_grid writes them (perm[new] =
 *              old; level_start: starts of B_0 .. B_{L-1}, C_last, then n)
 *  block_ptr, block_count: the segments' diagonal blocks in the same format,
 *              or NULL: each segment's blocks are the connected components
 *              of its rows in the symmetrised graph of A
 *  block_ptr_out, block_count_out: out (may be NULL), the blocks used;
 *              block_cap: capacity of block_ptr_out (n + nlevels + 2 always
 *              suffices)
 * Rejected (GS_EINVAL): perm not a permutation of 0..n-1, level_start not
 * rising from 0 to n, an empty segment, blocks that do not tile their
 * segment, a component that is not contiguous in perm, and two blocks of one
 * B_l (l < L) coupled by an entry of A (B_l must be block diagonal, Sec. 2;
 * C_last's blocks are cut on purpose, Sec. 4.3). */
int gs_partition_check(int64_t n, const int64_t* rowptr, const int32_t* col, const int64_t* perm,
                       const int64_t* level_start, int nlevels, const int64_t* block_ptr,
                       const int64_t* block_count, int64_t* block_ptr_out,
                       int64_t* block_count_out, int64_t block_cap);

/* Multilevel geometric vertex-separator reordering of a grid operator
 * (Alg. 3, Sec. 3.2).  Host only; usable without a device.
 *  perm:       out, n entries, perm[new] = old
 *  level_start:out, levels+2 entries: start of B_0..B_{L-1}, C_last, n
 *  nlevels:    out, L
 *  block_ptr:  out, global block boundaries of all L+1 segments, each
 *              segment's list [b_0, ..., b_nb] stored one after another
 *  block_count:out, L+1 entries: blocks per segment
 *  block_cap:  capacity of block_ptr (n + levels + 2 always suffices)
 * Errors: GS_EINVAL. */
int gs_partition_grid(int ndim, const int32_t* dims, int nparts, int levels,
                      int64_t n, const int64_t* rowptr, const int32_t* col,
                      int64_t* perm, int64_t* level_start, int* nlevels,
                      int64_t* block_ptr, int64_t* block_count,
                      int64_t block_cap);

/* The same level structure for a matrix without grid coordinates (the paper
 * partitions with ParMETIS, Sec. 3.2; here: nested dissection by
 * breadth-first level structures).  nparts must be a power of two.  One
 * bisection of a vertex set P: if P's subgraph is disconnected, its
 * components (largest first, ties by smallest vertex) go to the lighter half
 * with no separator; otherwise the breadth-first levels from a
 * pseudo-peripheral vertex (start at the smallest vertex, move to the
 * smallest vertex of the last level while the eccentricity grows, at most
 * 10 moves) are split at the level m of the median vertex in (level, index)
 * order (the last level is replaced by the one before it): the separator is
 * the level-m vertices with a neighbour in level m+1.  log2(nparts) rounds of
 * bisection give a p-way separator; the separator is partitioned again at
 * the next level (Alg. 3); vertex classes, the stop rule, block order and
 * outputs are those of gs_partition_grid, with at most as many levels as
 * separator classes.  gs_setup uses it when opts.grid_ndim is 0.  Host only.
 * Errors: GS_EINVAL. */
int gs_partition_graph(int nparts, int levels, int64_t n, const int64_t* rowptr,
                       const int32_t* col, int64_t* perm, int64_t* level_start, int* nlevels,
                       int64_t* block_ptr, int64_t* block_count, int64_t block_cap);

/* Incomplete LU of one square host CSR matrix (ILUT(tau, lfil) or ILU(0),
 * row-wise IKJ).  Host only.  L (strictly lower, unit diagonal implied) and U
 * (upper with diagonal) are written to caller arrays of capacity l_cap and
 * u_cap entries (rowptr arrays need n+1).  Errors: GS_EINVAL (also when a
 * capacity is too small), GS_EZEROPIVOT. */
int gs_ilu(int64_t n, const int64_t* rowptr, const int32_t* col,
           const void* val, int dtype, int kind, double tau, int lfil,
           int64_t* l_rowptr, int32_t* l_col, void* l_val, int64_t l_cap,
           int64_t* u_rowptr, int32_t* u_col, void* u_val, int64_t u_cap);

/* Copy out the installed preconditioner's level `l` (0..L) as host arrays
 * (the format of gs_level_data; caller supplies arrays of the sizes
 * reported by gs_get_level_sizes).  For checkpointing and inspection.
 * sizes[0..7] = d, s, nblocks, nnz(L), nnz(U), nnz(E), nnz(F), k. */
int gs_get_level_sizes(const gs_ctx* ctx, int l, int64_t* sizes);
int gs_get_level(const gs_ctx* ctx, int l, int64_t* block_ptr,
                 int64_t* l_rowptr, int32_t* l_col, void* l_val,
                 int64_t* u_rowptr, int32_t* u_col, void* u_val,
                 int64_t* e_rowptr, int32_t* e_col, void* e_val,
                 int64_t* f_rowptr, int32_t* f_col, void* f_val,
                 void* w, void* h);
/* perm: n entries (perm[new] = old). */
int gs_get_perm(const gs_ctx* ctx, int64_t* perm);

#ifdef __cplusplus
}
#endif
#endif /* GEMSLR_H */
