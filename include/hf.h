/*
 * hf.h -- C ABI of the hybrid mixed-precision sparse LDL^T factorization
 * (Suzuki, "A Hybrid Factorization Algorithm for Sparse Matrix with Mixed
 * Precision Arithmetic", arXiv 2208.01907) for AMD Instinct MI355X (gfx950).
 *
 * The problem (Sec. 2): a sparse symmetric matrix Kbar of order L, given in CSR
 * form with the full pattern (both triangles).  The library scales it to
 * K = Q Kbar Q with unit / zero diagonal, splits the indices into a moderate part
 * Lambda_1 and a hard part Lambda_2 by a low-precision LDL^T with symmetric
 * pivoting and threshold postponing (Sec. 2.1-2.2, Algorithm 1 step 1), builds
 * the Schur complement S22 = K22 - K21 K11^{-1} K12 with preconditioned block GCR
 * (Algorithm 5, Algorithm 1 steps 3-4) and factorizes S22 in FP64 with a
 * rank-revealing symmetric pivoting (Algorithm 1 step 5).  Solves follow
 * Algorithm 2.
 *
 * Conventions
 *   - Host pointers are marked _host, device pointers _dev.  Device buffers are
 *     plain hipMalloc'ed memory; streams are hipStream_t passed as void*.
 *     NULL stream means the default stream.
 *   - Every call returns HF_OK (0) or a negative HF_ERR_* code.  On error the
 *     outputs are left untouched and the context stays usable: a failed
 *     hf_factorize leaves the context in the "analysed" state.
 *   - A context is not thread-safe; different contexts may be used concurrently.
 *   - The library copies what it needs from its inputs; it keeps no pointer to
 *     caller memory after a call returns.
 */
#ifndef HF_H_
#define HF_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
enum {
  HF_OK = 0,
  HF_ERR_ARG = -1,             /* invalid argument (NULL, sizes, options) */
  HF_ERR_PATTERN = -2,         /* CSR not square/sorted/symmetric, diagonal missing,
                                  or the tree is not a valid nested dissection */
  HF_ERR_VALUE = -3,           /* NaN or Inf among the values */
  HF_ERR_STATE = -4,           /* call order violated (e.g. solve before factorize) */
  HF_ERR_NO_CONVERGENCE = -5,  /* block GCR did not reach the tolerance */
  HF_ERR_BREAKDOWN = -6,       /* block GCR Gram matrix lost all directions */
  HF_ERR_OOM = -7,             /* device or host allocation failed */
  HF_ERR_HIP = -8,             /* a HIP runtime call failed */
  HF_ERR_NOT_IMPLEMENTED = -9
};

/* precision of the step-1 factorization (the preconditioner).  HF_PREC_FP16 and
   HF_PREC_FP16_PAIR: FP32 fronts and factor, with the two front updates (the
   trailing update of the pivot block after each panel and the contribution
   block) multiplied on the FP16 matrix cores: each 64 x 16 operand tile is
   scaled by a power of two that brings its largest magnitude just below 2^14,
   and the products are accumulated and unscaled in FP32.  HF_PREC_FP16 casts
   every scaled operand to FP16 (11 significant bits); HF_PREC_FP16_PAIR carries
   it as a pair of FP16 numbers (hi + lo, about 22 bits) and forms three products
   per tile (hi*hi, hi*lo, lo*hi) */
enum { HF_PREC_FP16 = 16, HF_PREC_FP16_PAIR = 17, HF_PREC_FP32 = 32, HF_PREC_FP64 = 64 };

typedef struct hf_ctx hf_ctx;

typedef struct hf_options {
  double tau;               /* postponing threshold of Sec. 2.2 (default 1e-2) */
  int32_t low_precision;    /* HF_PREC_FP32 (mixed, default), HF_PREC_FP16,
                               HF_PREC_FP16_PAIR or HF_PREC_FP64 */
  int32_t first_pivot_unit; /* 1 (default): the first pivot of a node is compared
                               with 1, the unit diagonal of the scaled matrix;
                               0: it is accepted whenever nonzero */
  int32_t n_enlarge;        /* enlargement count n of Sec. 2.2 (default 4) */
  int32_t gcr_block;        /* block width of the Schur-complement block GCR;
                               0 (default) = all postponed columns in one block,
                               as in Sec. 3.5 (blocks of at most 64) */
  double gcr_tol;           /* per-column relative residual (default 1e-15) */
  int32_t gcr_maxit;        /* iteration cap of block GCR (default 50) */
  double ker_tol;           /* kernel pivots of S22: magnitude <= ker_tol in the
                               units of the scaled matrix (default 1e-10) */
  int32_t refine_steps;     /* hf_solve: residual-correction passes of
                               Algorithm 2 after the first one, the residual
                               taken in the caller's variables (default 1) */
  double refine_tol;        /* block-GCR tolerance inside a correction pass
                               (default 1e-3): a correction only has to be
                               accurate relative to the residual it corrects */
  int32_t nd_leaf_max;      /* hf_analyse without ordering and tree: largest
                               leaf of the nested dissection it computes
                               (default 512; see hf_order) */
  int32_t sweep_front_min;  /* FP32 preconditioner sweeps: a tree level with at
                               least this many fronts, each of at most 512
                               pivots, runs every front in one workgroup
                               (default 256; 0 = never).  Same arithmetic
                               either way up to the order of the sums. */
  int32_t sweep_wide_min;   /* sweeps with more than 16 right-hand sides: a
                               launch of at least this many 64-row tiles uses
                               the LDS-staged 64x64 tile products, smaller ones
                               the 16-row register-fed ones (default 256) */
  int32_t sweep_node_inverse; /* the L11 of every node of more than 512 pivots
                               also gets one explicit inverse, formed after step 1
                               by recursive doubling of its 512-column step
                               inverses, and each sweep direction can take such a
                               level in one diagonal product instead of a chain of
                               512-column steps.  1 (default): with an FP32
                               factor, only for the nodes whose L11 has no
                               positive entry below the diagonal (the factor of
                               an M-matrix, such as a diffusion operator: its
                               inverse has no negative entry, so the products
                               add terms of one sign), since a product with an
                               inverse of mixed signs loses accuracy to
                               cancellation that substitution does not; a level
                               takes the one product when all its nodes of more
                               than one step pass (FP64 factors: always).
                               2: always; 0: never */
} hf_options;

typedef struct hf_info_t {
  int64_t n;                /* order L */
  int64_t nnz;
  int32_t n_nodes;          /* nested-dissection tree nodes */
  int32_t n_levels;         /* levels of the factorization schedule */
  int32_t max_front;        /* largest frontal matrix order */
  int32_t max_pivots;       /* largest node */
  int64_t factor_entries;   /* E: stored low-precision factor entries (symbolic) */
  double factor_flops;      /* F: step-1 flops of the symbolic structure */
  double factor_flops_done; /* step-1 flops actually performed (after postponing) */
  int64_t front_bytes;      /* device arena of the frontal matrices */
  int32_t M;                /* size of the hard part Lambda_2 */
  int32_t kernel_dim;       /* k */
  int32_t gcr_blocks;       /* Schur-complement block GCR runs */
  int32_t gcr_iters_max;    /* largest iteration count of those runs */
  int32_t gcr_iters_total;
  int32_t solve_gcr_iters;  /* iterations of the last hf_solve */
  double rank_gap;          /* smallest non-kernel / largest kernel candidate pivot */
  int32_t rank_candidates;  /* postponed set of the second stage after enlargement */
  int32_t state;            /* 0 empty, 1 analysed, 2 factorized */
  double t_analyse_ms;
  double t_step1_ms;        /* scale + low-precision factorization + split */
  double t_gcr_ms;          /* block GCR for X12 */
  double t_s22_ms;          /* S22, its LDL^T, kernel */
  double t_solve_ms;        /* last hf_solve */
} hf_info_t;

/* Fill *opt with the defaults listed above.  Always succeeds for non-NULL opt. */
void hf_default_options(hf_options* opt);

/*
 * Nested-dissection ordering of a pattern (host only; Sec. 2.2: the indices
 * are bisected recursively by separators into the sets of a tree, each set
 * eliminated after its subtree).  For patterns without coordinates: in every
 * connected part a level structure is grown from a pseudo-peripheral vertex and
 * the level of its median vertex (less the vertices with no neighbour in the
 * next level) separates the levels before it from those after it; parts of at
 * most leaf_max indices, or of fewer than three levels, are leaves; connected
 * parts that a separator leaves become sibling subtrees (a forest at the top);
 * a separator or leaf of more than 4096 indices (the largest node hf_analyse
 * takes) becomes a chain of nodes of at most 4096, each the parent of the one
 * before.
 *   n, indptr_host, indices_host   pattern as for hf_analyse (validated)
 *   leaf_max        largest leaf (>= 1)
 *   perm_host       int32 [n], out: perm[k] = original index eliminated k-th
 *   n_nodes_host    out: number of tree nodes
 *   node_ptr_host   int32 [n + 1] (room for the largest possible tree), out:
 *                   node j owns positions node_ptr[j] .. node_ptr[j+1]-1
 *   parent_host     int32 [n], out: parent node or -1; postorder, subtrees
 *                   contiguous; every off-diagonal entry couples a node with
 *                   itself, an ancestor or a descendant
 * The outputs are what hf_analyse takes.  Host arrays owned by the caller.
 * Errors: HF_ERR_ARG, HF_ERR_PATTERN, HF_ERR_NOT_IMPLEMENTED (n >= 2^31 - 1),
 * HF_ERR_OOM.
 */
int hf_order(int64_t n, const int64_t* indptr_host, const int32_t* indices_host, int32_t leaf_max,
             int32_t* perm_host, int32_t* n_nodes_host, int32_t* node_ptr_host, int32_t* parent_host);

/*
 * Symbolic analysis (host only; Sec. 2.2 nested dissection).
 *   n                 order L (>= 0)
 *   indptr_host       int64 [n+1], CSR row pointers, indptr[0] = 0
 *   indices_host      int32 [indptr[n]], column indices, sorted and unique in
 *                     every row, full symmetric pattern, diagonal present
 *   perm_host         int32 [n] or NULL: perm[k] = original index eliminated
 *                     k-th (nested-dissection order); NULL = identity
 *   n_nodes           number of tree nodes (>= 1 when n > 0)
 *   node_ptr_host     int32 [n_nodes+1]: node j owns positions
 *                     node_ptr[j] .. node_ptr[j+1]-1 of the permuted order
 *   parent_host       int32 [n_nodes]: parent node, -1 for roots; nodes are in
 *                     postorder (children before parents, subtrees contiguous)
 *   opt               options or NULL for defaults
 *   out               receives the new context
 * With node_ptr_host == NULL and parent_host == NULL: if perm_host is NULL too
 * and n exceeds opt->nd_leaf_max, the ordering and the tree are those hf_order
 * computes from the pattern; otherwise the whole matrix is one node (a dense
 * front, usable only for small n) in the order perm_host gives.
 * Errors: HF_ERR_ARG, HF_ERR_PATTERN (includes couplings between sibling
 * subtrees), HF_ERR_NOT_IMPLEMENTED (a node of more than 4096 indices, a front
 * of 2^31 or more entries, or more than 2^31 border entries in total),
 * HF_ERR_OOM, HF_ERR_HIP.
 */
int hf_analyse(int64_t n, const int64_t* indptr_host, const int32_t* indices_host,
               const int32_t* perm_host, int32_t n_nodes, const int32_t* node_ptr_host,
               const int32_t* parent_host, const hf_options* opt, hf_ctx** out);

/*
 * Numerical factorization, Algorithm 1 (Sec. 3).
 *   values_dev   float64 [nnz] on the device, the values of Kbar on the analysed
 *                pattern (same order as indices_host)
 *   stream       hipStream_t (void*); all work is ordered on it.  The call returns
 *                after the small device-to-host reads it needs (the hard part,
 *                convergence flags, the kernel dimension).
 * May be called again with new values on the same pattern.
 * Errors: HF_ERR_STATE (not analysed), HF_ERR_VALUE, HF_ERR_NO_CONVERGENCE,
 * HF_ERR_BREAKDOWN, HF_ERR_OOM, HF_ERR_HIP.
 */
int hf_factorize(hf_ctx* ctx, const double* values_dev, void* stream);

/*
 * Solve Kbar X = B, Algorithm 2 (Sec. 3).
 *   r         number of right-hand sides (>= 0)
 *   B_dev     float64, column-major n x r, leading dimension ldb >= n
 *   X_dev     float64, column-major n x r, leading dimension ldx >= n; must not
 *             alias B_dev
 * For singular Kbar the returned solution is orthogonal (Euclidean, original
 * variables) to the detected kernel, i.e. the minimum-norm solution of a
 * consistent system.
 * Errors: HF_ERR_STATE (not factorized), HF_ERR_ARG, HF_ERR_NO_CONVERGENCE,
 * HF_ERR_OOM, HF_ERR_HIP.
 */
int hf_solve(hf_ctx* ctx, int32_t r, const double* B_dev, int64_t ldb, double* X_dev, int64_t ldx,
             void* stream);

/*
 * Adjoint of hf_solve on the current factors.  An extension, not a step of the
 * paper: one more solve with Algorithm 2 (Sec. 3) on the factors of the last
 * hf_factorize gives the derivatives of a loss l(X) through X = Kbar^+ B.
 *   X_dev     float64 n x r, leading dimension ldx >= n: the solution hf_solve
 *             returned for B
 *   G_dev     float64 n x r, leading dimension ldg >= n: dl/dX
 *   Lam_dev   float64 n x r, leading dimension ldl >= n, output:
 *             Lambda = Kbar^+ P G, with P the orthogonal projector onto the range
 *             of Kbar (orthogonal to the detected kernel); Lambda is dl/dB for
 *             right-hand sides in the range
 *   GV_dev    float64 [nnz] or NULL, output: dl/dvalues on the analysed pattern,
 *             in the order of indices_host: the entry (i, j) receives
 *             -sum_c Lambda[i, c] X[j, c]
 * P is formed with the kernel basis of hf_kernel_basis, so P G is consistent only
 * to the accuracy of that basis, which bounds the backward error of Lambda (about
 * 1e-12 for a 1e6 coefficient contrast at 2.6e5 unknowns, where the basis is
 * 4.5e-8 from the exact kernel).
 * The value gradient is exact along perturbations of Kbar that keep its kernel
 * (for example coefficient changes of a pure-Neumann operator); along others the
 * pseudo-inverse is not differentiable.  Lam_dev may alias neither G_dev nor
 * X_dev, GV_dev none of the other three.  With r == 0, GV_dev (if given) is set
 * to zero.
 * Errors: HF_ERR_STATE (not factorized), HF_ERR_ARG, HF_ERR_NO_CONVERGENCE,
 * HF_ERR_OOM, HF_ERR_HIP.
 */
int hf_adjoint(hf_ctx* ctx, int32_t r, const double* X_dev, int64_t ldx, const double* G_dev, int64_t ldg,
               double* Lam_dev, int64_t ldl, double* GV_dev, void* stream);

/*
 * Autotuning of the launch shapes of the preconditioner sweeps (Sec. 3.2) for
 * the current factors: applies Q^{-1} to r columns (1 <= r <= 64) with every
 * combination of sweep_front_min in {0, 128, 256, 512} and sweep_wide_min in
 * {128, 256, 512, 1024}, timed with events after one untimed application each,
 * and keeps the fastest in the context's options (later factorizations and
 * solves use them).  The choices change which kernels run, not what they
 * compute (up to the order of the FP32 sums).  Either output may be NULL.
 *   front_min_host, wide_min_host   out: the chosen values
 *   ms_host                         out: the chosen combination's time per application
 * Errors: HF_ERR_STATE (not factorized), HF_ERR_ARG, HF_ERR_OOM, HF_ERR_HIP.
 */
int hf_tune(hf_ctx* ctx, int32_t r, int32_t* front_min_host, int32_t* wide_min_host, double* ms_host,
            void* stream);

/*
 * The preconditioner Q^{-1} of Sec. 3.2 on the current factors: forward and
 * backward substitution with the low-precision LDL^T of K11 (step 1 of
 * Algorithm 1), the operator block GCR applies in every iteration.  Works in
 * the library's own variables, not the caller's: rows in elimination order
 * (position i is original index perm[i]) of the symmetrically scaled matrix.
 *   r      number of columns, 0 <= r <= 64
 *   R_dev  float64, row-major n x r (leading dimension r); the rows of the hard
 *          part Lambda_2 are not read
 *   Y_dev  float64, row-major n x r, output (leading dimension r); zero on the
 *          rows of the hard part; must not alias R_dev
 * Errors: HF_ERR_STATE (not factorized), HF_ERR_ARG, HF_ERR_OOM, HF_ERR_HIP.
 */
int hf_precond(hf_ctx* ctx, int32_t r, const double* R_dev, double* Y_dev, void* stream);

/* Kernel dimension k found by the rank-revealing LDL^T of S22 (Sec. 2.2, Algorithm 1 step 5).
 * Errors: HF_ERR_ARG, HF_ERR_STATE. */
int hf_kernel_dim(const hf_ctx* ctx, int32_t* k_host);

/*
 * Orthonormal kernel basis of Kbar in original variables, float64 column-major
 * n x k (leading dimension ldn >= n), lifted from the null vectors of S22.
 * Errors: HF_ERR_ARG, HF_ERR_STATE, HF_ERR_HIP.
 */
int hf_kernel_basis(const hf_ctx* ctx, double* N_dev, int64_t ldn, void* stream);

/*
 * Schur complement of the hard part, Algorithm 1 step 4.
 *   m_host          receives M = #Lambda_2
 *   lambda2_host    int32 [M] or NULL: the hard-part indices in original
 *                   numbering, ascending
 *   S22_dev         float64 [M x M] column-major (leading dimension lds >= M) or
 *                   NULL: S22 of the scaled matrix K = Q Kbar Q, rows and
 *                   columns in the order of lambda2_host
 * Call with NULL buffers to query M.  Errors: HF_ERR_ARG, HF_ERR_STATE, HF_ERR_HIP.
 */
int hf_schur(const hf_ctx* ctx, int32_t* m_host, int32_t* lambda2_host, double* S22_dev, int64_t lds,
             void* stream);

/*
 * hf_schur without any allocation, for callers that cannot allocate memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid it).
 * Same arguments, outputs and errors as hf_schur; lambda2_host is sorted in
 * place and the permutation of S22 is staged in a fixed device array of the
 * library (one per GPU, kept until the process ends) instead of memory
 * allocated per call.  The hard part may hold at most 16384 indices:
 * HF_ERR_NOT_IMPLEMENTED beyond (the size query with NULL buffers still
 * succeeds).  Calls on one GPU share that array, so calls that overlap on one
 * GPU (different streams or threads) race; calls in sequence do not.
 */
int hf_schur_noalloc(const hf_ctx* ctx, int32_t* m_host, int32_t* lambda2_host, double* S22_dev, int64_t lds,
                     void* stream);

/*
 * Diagonal scaling Q (Sec. 2) as float64 [n] on the device: K = Q Kbar Q.
 * Errors: HF_ERR_ARG, HF_ERR_STATE, HF_ERR_HIP.
 */
int hf_scaling(const hf_ctx* ctx, double* q_dev, void* stream);

/* Diagnostics.  Errors: HF_ERR_ARG. */
int hf_info(const hf_ctx* ctx, hf_info_t* info_host);

/*
 * Per-kernel-class timing (measurement support).  Every class but
 * HF_K_SOLVE_GATHER and HF_K_OTHER holds the launches of one kernel.  When
 * enabled, every launch of an instrumented kernel is bracketed by HIP events on
 * the caller's stream; the
 * elapsed times are accumulated at the end of each hf_factorize / hf_solve /
 * hf_adjoint,
 * together with the algorithmic bytes and flops of each launch (computed on the
 * host from the sizes of the fronts involved).  Enabling resets the counters.
 */
enum {
  HF_K_PANEL = 0,         /* k_panel: pivot search + panel of F11 (serial pivot chain) */
  HF_K_PERMUTE_L11 = 1,   /* k_l11_gather + k_l11_back: L11 columns put in pivot order */
  HF_K_F11_UPDATE = 2,    /* k_syrk: trailing update of F11 after each panel */
  HF_K_GATHER_BORDER = 3, /* k_gather_border: F21 in pivot order before the TRSM */
  HF_K_TRSM = 4,          /* k_trsm: L21 = F21 L11^{-T} D^{-1} */
  HF_K_SYRK = 5,          /* k_syrk: contribution block F22 -= L21 D L21^T */
  HF_K_EXTEND_ADD = 6,    /* k_extend_add: the children's contribution blocks */
  HF_K_FWD_DIAG = 7,      /* k_fwd_diag: diagonal steps of the forward sweep */
  HF_K_FWD_UPDATE = 8,    /* k_fwd_upd: off-diagonal products of the forward sweep */
  HF_K_BWD_BORDER = 9,    /* k_bwd_border_part: border products of the backward sweep */
  HF_K_BWD_DIAG = 10,     /* k_bwd_diag: diagonal steps of the backward sweep */
  HF_K_BWD_UPDATE = 11,   /* k_bwd_upd: off-diagonal products of the backward sweep */
  HF_K_SOLVE_GATHER = 12, /* gathers / extend-adds / border sums of the sweeps */
  HF_K_SPMM = 13,         /* k_spmm_k11: FP64 CSR products with K */
  HF_K_GRAM = 14,         /* k_gram_partial: FP64 Gram products of block GCR */
  HF_K_COMBINE = 15,      /* k_combine: FP64 block updates X += P C of block GCR */
  HF_K_OTHER = 16,        /* everything else */
  HF_K_VALUE_GRAD = 17,   /* k_value_grad: value gradient of hf_adjoint */
  HF_K_FWD_FRONT = 18,    /* k_fwd_front: whole forward step of a small front (one workgroup) */
  HF_K_BWD_FRONT = 19,    /* k_bwd_front: whole backward step of a small front (one workgroup) */
  HF_K_NCLASS = 20
};

typedef struct hf_kstat_t {
  double ms;             /* summed event time */
  int64_t launches;
  double bytes;          /* summed algorithmic bytes */
  double flops;          /* summed algorithmic flops */
} hf_kstat_t;

/* Enable (1) or disable (0) the timing; enabling clears the counters.
 * Errors: HF_ERR_ARG. */
int hf_timing_enable(hf_ctx* ctx, int32_t on);

/* Counters of one class (0 <= cls < HF_K_NCLASS).  Errors: HF_ERR_ARG. */
int hf_timing_get(const hf_ctx* ctx, int32_t cls, hf_kstat_t* out_host);

/*
 * Record of the step-1 pivoting of the last hf_factorize (diagnostics of the
 * threshold postponing of Sec. 2.2).  Every output may be NULL.
 *   npiv_host    int32 [n_nodes]: accepted pivots of every tree node; the
 *                node's other indices were postponed (they form Lambda_2)
 *   d_host       float64 [n]: the accepted pivots d (factor precision, widened),
 *                node j's at positions node_ptr[j] .. node_ptr[j]+npiv[j]-1 in
 *                the order they were taken; 0 at the postponed positions
 *   dstop_host   float64 [n_nodes]: diagonal value of the candidate whose ratio
 *                test stopped the node; NaN when every index was accepted
 *   margin_host  float64 [n_nodes]: min over the node's ratio tests of
 *                |log10(|d| / (tau |d_ref|))| in decades, d_ref the previous
 *                accepted pivot (1 for the first one when first_pivot_unit);
 *                a zero candidate is no test; +inf when the node made none
 * Errors: HF_ERR_ARG, HF_ERR_STATE (not factorized), HF_ERR_HIP.
 */
int hf_pivots(const hf_ctx* ctx, int32_t* npiv_host, double* d_host, double* dstop_host, double* margin_host);

/*
 * Pivot magnitudes of the FP64 LDL^T of S22 (Algorithm 1 step 5), float64 [M]
 * on the host, in elimination order: |d| of a 1x1 pivot, the smaller |eigenvalue|
 * of a 2x2 block for both of its positions.  Errors: HF_ERR_ARG, HF_ERR_STATE,
 * HF_ERR_HIP.
 */
int hf_s22_pivots(const hf_ctx* ctx, double* mags_host);

/*
 * Residual histories of the block-GCR runs (Algorithm 5): for every run the max
 * over the active columns of ||r_k||_2 / ||b_k||_2 (recurrence residual) after
 * the initial guess and after each iteration.  The runs of the last
 * hf_factorize (the column blocks of K11 X12 = K12) come first, then those of
 * the last hf_solve or hf_adjoint (per 64-column chunk: the first pass, then
 * each residual-correction pass).
 *   nruns_host    receives the number of runs (required)
 *   nfactor_host  receives how many of them belong to hf_factorize (or NULL)
 *   run_ptr_host  int32 [nruns+1] or NULL: run r owns hist[run_ptr[r] ..
 *                 run_ptr[r+1]-1]
 *   hist_host     float64 [run_ptr[nruns]] or NULL
 * Call with NULL arrays to query the sizes.  Errors: HF_ERR_ARG.
 */
int hf_gcr_history(const hf_ctx* ctx, int32_t* nruns_host, int32_t* nfactor_host, int32_t* run_ptr_host,
                   double* hist_host);

/* Static message for a status code (never NULL). */
const char* hf_strerror(int status);

/* Release the context and all device memory it owns.  NULL is ignored. */
void hf_destroy(hf_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* HF_H_ */
