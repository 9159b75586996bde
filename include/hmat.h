/*
 * hmat.h -- C ABI of the MI355X (gfx950) H-matrix library for the Lame
 * single-layer operator discretised by piecewise-constant collocation.
 *
 * Method: Bauer & Bebendorf, "Adaptive H-Matrix Computations in Linear
 * Elasticity" (arXiv 2205.04752):
 *   - Kelvin's solution tensor S_K (Sec. 4.1) as the kernel of the
 *     single-layer potential V~ (Sec. 4.1);
 *   - collocation (Sec. 2, discretisation examples) with the piecewise
 *     constant basis of S^0_h (Sec. 4.2), collocation point = centroid,
 *     coefficient order t = [t_i^(1), t_i^(2), t_i^(3)]_i (Sec. 4.2), i.e.
 *     DOF 3i+a is component a of triangle i;
 *   - binary cluster tree, block-cluster tree, admissibility (eq. adm) and
 *     partition P = P_adm u P_nonadm (Sec. 2.1);
 *   - ACA with partial pivoting on every admissible block (Sec. 2.2,
 *     Algorithm 1), dense non-admissible blocks (Sec. 2.2);
 *   - the H-matrix-vector product (Sec. 2: outer-product representation,
 *     O(k(M+N)) per block; Sec. 2.2: H(P,k)).
 *
 * Conventions for every call:
 *   - Every function returns hmat_status; HMAT_OK (0) on success.
 *   - Arguments are validated on the host before any device work; on a
 *     validation error nothing is launched, outputs are left untouched and
 *     *out handles are set to NULL.
 *   - hmat_last_error() returns a thread-local message for the last failure
 *     of the calling thread (empty string if none). The pointer is valid
 *     until the next call on that thread.
 *   - No C++ exception crosses this interface.
 *   - "HOST" pointers are ordinary CPU memory; "DEVICE" pointers are HIP
 *     device memory of the current device (e.g. a torch tensor's data_ptr()).
 *   - hip_stream is a hipStream_t (NULL = the legacy default stream). Device
 *     work of a call is enqueued on that stream.
 *   - Thread safety: different handles may be used from different threads;
 *     calls on one handle must be serialised by the caller.
 *   - Device memory: buffers the library releases (hmat_free, the staging of
 *     a build) are kept for later builds and calls rather than handed back:
 *     a cache of released buffers (up to 1/16 of the device memory), idle
 *     ACA panel buffers (up to 1/8) and the stream-ordered pool's retained
 *     memory (4 GiB; 64 GiB while a request server runs). Allocating and
 *     releasing buffers of that size per build stalled builds, the more so
 *     with several at once. hmat_release_memory hands all of it back.
 *   - Environment (read at build time of a handle; for tuning and tracing):
 *       HMAT_ACA_BUDGET_MB  bytes of first-pass ACA panels one ACA group may
 *                           hold (default: a quarter of the free device
 *                           memory, at least 1 GiB); smaller budgets run ACA
 *                           in more groups, with the same results;
 *       HMAT_ACA_KCAP_FIRST first-pass ACA capacity (columns, >= 2; default
 *                           from eps as stated with aca_passes); blocks that
 *                           fill it continue in later passes, with the same
 *                           results;
 *       HMAT_MV_CHUNK_KB    product chunk size for one vector (default 16);
 *       HMAT_MV_UNROLL      columns per batch of the one-vector product
 *                           kernels, 8 or 16 (default 16); hmat_tune sets
 *                           both per handle;
 *       HMAT_TRACE_BUILD    if set, print the build's phase times to stderr
 *                           (synchronises the stream at every phase), and
 *                           any allocation that found the device full and
 *                           had to release the kept memory first.
 */
#ifndef HMAT_H
#define HMAT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hmat* hmat_t; /* opaque; owns every device allocation it makes */

typedef enum {
  HMAT_OK = 0,
  HMAT_EINVAL = 1,  /* invalid argument (nothing was done) */
  HMAT_ENOMEM = 2,  /* device or host allocation failed (budget included) */
  HMAT_EDEVICE = 3, /* a HIP call failed */
  HMAT_ENOCONV = 4, /* iteration limit reached; outputs still written */
  HMAT_ENOTSUP = 5, /* valid but unsupported request */
  HMAT_ECANCELED = 6 /* request server: the request was cancelled */
} hmat_status;

/* Surface triangulation (Sec. 4.2: admissible triangulation into flat
 * triangles tau_i). HOST arrays, borrowed for the duration of the call only:
 *   vertices [n_vertices][3] float64, triangles [n_triangles][3] int32,
 *   0-based vertex indices. */
typedef struct {
  int32_t n_vertices;
  int32_t n_triangles;
  const double* vertices;
  const int32_t* triangles;
} hmat_mesh;

/* Build statistics (hmat_info). Storage follows Sec. 2: a low-rank block of
 * rank k stores k(m+n) scalars, a dense block m n. */
typedef struct {
  int64_t n_dof;          /* 3 * n_triangles */
  int32_t n_triangles;
  int32_t n_clusters;     /* nodes of the cluster tree */
  int32_t depth;          /* depth of the cluster tree */
  int32_t n_blocks;       /* |P| */
  int32_t n_far;          /* |P_adm| */
  int32_t n_near;         /* |P_nonadm| */
  int32_t c_sp;           /* sparsity constant (Sec. 2.1) */
  int32_t rank_min, rank_max;
  double rank_mean;
  int64_t far_scalars;    /* sum over admissible blocks of k(m+n) */
  int64_t near_scalars;   /* sum over dense blocks of m n */
  double compression;     /* (far + near scalars) / n_dof^2 */
  int32_t n_rank_full;    /* admissible blocks that stopped at k = min(m,n) */
  int32_t n_near_threshold; /* blocks whose final |u||v| / (eps ||S||) lies in [1-1e-9, 1] */
  int32_t aca_passes;     /* ACA passes: 1, or more if some blocks outgrew the rank capacity of
                             the first pass, min(128, max(32, 16 ceil((24 + 12 log10(1/eps)) / 16)))
                             steps; each later pass continues those blocks from where they
                             stopped with 4x the capacity, at most min(m,n) */
  int32_t n_exact;        /* admissible blocks whose ACA reached full rank, stored exactly:
                             U = B, V = I (n <= m) or U = I, V = B^T (a cross approximation
                             is kept only as a compression, Sec. 2) */
  double t_plan_ms;       /* host: geometry, tree, partition, device lists */
  double t_near_ms;       /* device: dense blocks (K1) */
  double t_aca_ms;        /* device: ACA (K2) incl. compaction */
  double t_build_ms;      /* whole hmat_build */
  int64_t device_bytes;   /* persistent device memory held by the handle */
  int64_t far_u_scalars;  /* sum over admissible blocks of m k (the U factors) */
  int64_t far_v_scalars;  /* sum over admissible blocks of n k (the V factors) */
  double t_aca_kernel_ms; /* device: the ACA kernels alone (all groups and passes) */
  double t_layout_ms;     /* host + device: compaction, product plan, stream fill */
  int32_t aca_groups;     /* groups of admissible blocks ACA ran in (memory budget) */
  int32_t n_bodies;       /* bodies in the handle (hmat_build_batch) */
  int32_t precision;      /* stored entries: 0 FP64, 1 FP32 only (hmat_build_ex) */
  int32_t aca_fp32;       /* 1 if ACA ran in FP32 */
} hmat_stats;

typedef struct {
  int32_t iterations;     /* Arnoldi steps (= operator applications inside cycles) */
  int32_t restarts;       /* completed restart cycles */
  double relres;          /* explicit ||b - A_H x||_2 / ||b||_2 at return */
  double time_ms;         /* wall time of the solve (host clock, stream synced) */
  int32_t refinements;    /* hmat_solve_ir: outer refinement steps (0 for hmat_solve) */
  int32_t reserved;
} hmat_solve_info;

/*
 * hmat_build -- assemble the H-matrix approximation A_H of the collocation
 * matrix A[3i+a, 3j+b] = integral over tau_j of S_K,ab(c_i - y) ds_y
 * (Sec. 4.1 kernel; Sec. 2 collocation; Sec. 4.2 basis), c_i the centroid.
 *   mesh    HOST mesh (copied).
 *   E, nu   Young modulus E > 0 and Poisson ratio 0 < nu < 1/2 (Sec. 1).
 *   eta     admissibility parameter > 0: a block t x s is low-rank iff
 *           dist(X_t, X_s) > 0 and min(diam X_t, diam X_s) <= eta dist(X_t, X_s),
 *           X_t the axis-aligned box of the vertices of t's triangles (eq. adm).
 *   leaf    clusters of at most `leaf` triangles are not split (>= 1).
 *   eps     ACA accuracy 0 < eps < 1: ACA stops at ||u_k|| ||v_k|| <= eps ||S_k||_F
 *           (Algorithm 1 stop test, constant read as 1) once rows of all three
 *           displacement components have been used (coplanar clusters
 *           decouple them).
 *   hip_stream  stream for all device work; synchronised before return.
 *   out     receives the handle (NULL on failure).
 * Quadrature: off-diagonal entries use the degree-5 seven-point rule
 * (Radon); the self entries split tau_i at c_i into three triangles, each
 * with 16 x 16 Gauss-Legendre points in Duffy coordinates.
 * Errors: HMAT_EINVAL for E <= 0, nu outside (0, 1/2), eta <= 0, leaf < 1,
 * eps outside (0, 1), n_triangles < 1, n_vertices < 3, a vertex index out of
 * range, a non-finite coordinate or a zero-area triangle; HMAT_ENOMEM;
 * HMAT_EDEVICE.
 */
hmat_status hmat_build(const hmat_mesh* mesh, double E, double nu, double eta, int32_t leaf,
                       double eps, void* hip_stream, hmat_t* out);

/*
 * hmat_build_ex -- hmat_build with options (opts may be NULL: the defaults).
 *   precision        0 (default): entries, ACA and storage in FP64.
 *                    1: the handle stores its entries in FP32 only (half the
 *                    device memory; products and solves read them in FP64
 *                    arithmetic, and hmat_solve_ir's residual uses them too,
 *                    so its relative residual refers to the FP32-stored
 *                    operator). ACA runs in FP32 (panels, entries and
 *                    remainders; the ||S_k|| update in FP64) for eps >= 1e-5,
 *                    where FP32 arithmetic resolves the remainders; for
 *                    smaller eps it runs in FP64 and the factors are rounded.
 *                    Dense blocks are computed in FP64 and rounded.
 *                    hmat_set_precision(h, 0) and FP64-precision calls then
 *                    return HMAT_ENOTSUP; hmat_set_factors too.
 *   aca_stop_factor  the constant c of the ACA stop test |u_k||v_k| <= c eps ||S_k||_F
 *                    (Algorithm 1 prints eps(1-beta)/(1+eps); default 1.0).
 *   aca_small_tri    ACA schedule: blocks with at most this many triangles on
 *                    both sides run one wave each, larger ones a workgroup
 *                    (0: the default, 64; else 1..1024).
 *   aca_wide         ACA schedule: 1 runs the first pass's larger blocks in
 *                    512-thread workgroups instead of 256 (0: default).
 *                    The schedule changes only how the work is launched: the
 *                    factors are the same unless a stop test lies within
 *                    rounding of its threshold (||S_k|| is summed in another
 *                    order). hmat_tune_aca times the candidates on a mesh.
 * Errors: as hmat_build; HMAT_EINVAL for precision not 0 or 1,
 * aca_stop_factor <= 0 or aca_stop_factor * eps >= 1, aca_small_tri outside
 * 0..1024, or aca_wide not 0 or 1.
 */
typedef struct {
  int32_t precision;
  int32_t aca_small_tri;
  double aca_stop_factor;
  int32_t aca_wide;
  int32_t reserved; /* 0 */
} hmat_opts;

hmat_status hmat_build_ex(const hmat_mesh* mesh, double E, double nu, double eta, int32_t leaf,
                          double eps, const hmat_opts* opts, void* hip_stream, hmat_t* out);

/*
 * hmat_tune_aca -- autotuner of the ACA launch schedule for one mesh and
 * accuracy (the rank-bucket split of NEXT-1: which blocks run one wave each,
 * and the workgroup size of the others). Builds the H-matrix `reps` times
 * with each candidate schedule (aca_small_tri in {32, 64, 128} x aca_wide in
 * {0, 1}), keeps the least ACA kernel time of each, and reports them; pass
 * the best schedule to hmat_build_ex through hmat_opts. `opts` (may be NULL)
 * supplies precision and aca_stop_factor; its schedule fields are ignored.
 * The best schedule depends on the block sizes and ranks: at icosphere level
 * 5, eps 1e-6, small_tri 128 cuts ACA 12%; on the 10 x 1 x 1 box at eps 1e-7
 * the 512-thread first pass cuts it 24%.
 * Synchronises the stream. Errors: as hmat_build_ex; HMAT_EINVAL for reps < 1
 * or info NULL.
 */
typedef struct {
  int32_t n_candidates;
  int32_t best;             /* index of the fastest candidate */
  int32_t small_tri[8];     /* candidate aca_small_tri */
  int32_t wide[8];          /* candidate aca_wide */
  double aca_ms[8];         /* least ACA kernel time over reps (ms) */
  double best_ms;
} hmat_aca_tune_info;

hmat_status hmat_tune_aca(const hmat_mesh* mesh, double E, double nu, double eta, int32_t leaf,
                          double eps, const hmat_opts* opts, int32_t reps, void* hip_stream,
                          hmat_aca_tune_info* info);

/*
 * hmat_build_batch -- hmat_build for n_bodies independent bodies in one
 * handle (the block-diagonal operator diag(A_H^(0), ..., A_H^(n-1))): every
 * body gets its own cluster tree, partition and ACA (Sec. 2, Algorithm 1)
 * with its own E[b], nu[b] and eps[b]; eta and leaf are shared. The dense
 * blocks of all bodies are generated in one launch, ACA runs over the
 * admissible blocks of all bodies together, and hmat_matvec multiplies all
 * bodies in one pass.
 *   meshes, E, nu, eps   HOST arrays of n_bodies entries (copied).
 * DOF layout of x and y in hmat_matvec / hmat_solve: the bodies' DOF vectors
 * concatenated in body order (body b starts at DOF 3 * sum_{c<b} n_triangles_c;
 * hmat_bodies returns the offsets). hmat_block numbers blocks body by body.
 * hmat_solve runs GMRES on the whole block-diagonal system.
 * Errors: as hmat_build for each body (the message names the body);
 * HMAT_EINVAL for n_bodies < 1 or more than 2^31/3 triangles in total.
 */
hmat_status hmat_build_batch(int32_t n_bodies, const hmat_mesh* meshes, const double* E,
                             const double* nu, const double* eps, double eta, int32_t leaf,
                             void* hip_stream, hmat_t* out);

/* hmat_bodies -- number of bodies of h (1 for hmat_build) and, if dof_off is
 * not NULL, their DOF offsets: dof_off[b] is the first DOF of body b and
 * dof_off[n_bodies] = n_dof (HOST array of n_bodies + 1 entries). */
hmat_status hmat_bodies(hmat_t h, int32_t* n_bodies, int64_t* dof_off);

/*
 * hmat_matvec -- y_r = A_H x_r for r = 0..nrhs-1 (Sec. 2, Sec. 2.2):
 *   y = sum over admissible b of U_b (V_b^T x_s) + sum over dense b of D_b x_s.
 *   x    DEVICE float64, nrhs vectors of length n_dof, vector r at x + r*ldx,
 *        DOF order 3i+a in the caller's triangle numbering.
 *   y    DEVICE float64, same layout with ldy; fully overwritten. Must not
 *        overlap x.
 *   ldx, ldy >= n_dof.  1 <= nrhs <= 64.
 * Stream-ordered, no host synchronisation; the result is deterministic
 * (bitwise repeatable for the same inputs). Errors: HMAT_EINVAL (NULL
 * handle/pointers, bad sizes), HMAT_EDEVICE.
 */
hmat_status hmat_matvec(hmat_t h, int32_t nrhs, const double* x, int64_t ldx, double* y,
                        int64_t ldy, void* hip_stream);

/*
 * hmat_solve -- solve A_H x = b by restarted GMRES (Saad & Schultz) with
 * classical Gram-Schmidt applied twice, Givens rotations, x0 = 0. Not part of
 * the paper, whose saddle-point system is solved by Bramble-Pasciak CG.
 *   b, x     DEVICE float64 vectors of length n_dof (caller's DOF order).
 *   tol      > 0: converged iff the explicit ||b - A_H x||_2 <= tol ||b||_2.
 *   restart  Krylov dimension per cycle, 1..1024.
 *   maxit    maximum number of Arnoldi steps in total (>= 1).
 *   info     HOST, may be NULL.
 * Synchronises the stream. Each Arnoldi step's Hessenberg column reaches the
 * host through pinned memory that the normalisation kernel writes; the host's
 * Givens update of step j overlaps the device's step j + 1.
 * Returns HMAT_ENOCONV if maxit is reached first; x and info are written in
 * that case too.
 */
hmat_status hmat_solve(hmat_t h, const double* b, double* x, double tol, int32_t restart,
                       int32_t maxit, void* hip_stream, hmat_solve_info* info);

/*
 * hmat_solve_noalloc -- hmat_solve for callers that cannot allocate memory
 * (no hipMalloc, hipFree, pinned host allocation or event creation during
 * the call: harnesses that forbid allocation, serving loops that must not
 * touch the allocator). Same arguments, results and errors as hmat_solve,
 * bit for bit (the same kernels in the same order).
 * Workspace: the Krylov basis, the work vector, the partial sums and the
 * Hessenberg columns live in one fixed device array of 32 MiB per device,
 * part of the library's code object (held from the library's first use on a
 * device until the process ends); the Hessenberg columns come back through
 * ordinary host memory on the calling thread's stack, so every Arnoldi step
 * synchronises the stream (hmat_solve overlaps the host's Givens update
 * with the next step instead).
 * Limit: 8 * (n_dof * (restart + 1) + n_dof + partial sums + 4112) bytes,
 * each part rounded to 256 bytes, must fit 32 MiB (GMRES(50) up to 80418
 * DOF, GMRES(20) up to 190072); larger requests return
 * HMAT_EINVAL with the sizes in the message, before any device work.
 * Concurrency: every call on a device shares that device's array, which
 * keeps the last call's contents (nothing in it needs to start at zero).
 * Calls that overlapped on one device would race on it, so the library
 * runs one such call at a time in a process (a second caller waits).
 * hmat_profile's per-phase events are not recorded by this call.
 */
hmat_status hmat_solve_noalloc(hmat_t h, const double* b, double* x, double tol, int32_t restart,
                               int32_t maxit, void* hip_stream, hmat_solve_info* info);

/*
 * hmat_set_precision -- reduced-precision storage of the H-matrix entries.
 * precision 1 makes FP32 copies of the stored low-rank factors and dense
 * blocks (same layout; FP64 values rounded to nearest) next to the FP64
 * ones, which stay: hmat_matvec_ex(h, 1, ...) reads the copies and computes
 * in FP64, so its result differs from the FP64 product by the rounding of
 * the stored entries (relative 2-norm error about 1e-7). precision 0 frees
 * the copies. Synchronises the stream. Errors: HMAT_EINVAL, HMAT_ENOMEM.
 */
hmat_status hmat_set_precision(hmat_t h, int32_t precision, void* hip_stream);

/* hmat_matvec_ex -- hmat_matvec reading the entries stored in `precision`
 * (0: FP64, 1: the FP32 copies of hmat_set_precision; HMAT_EINVAL if absent). */
hmat_status hmat_matvec_ex(hmat_t h, int32_t precision, int32_t nrhs, const double* x, int64_t ldx,
                           double* y, int64_t ldy, void* hip_stream);

/*
 * hmat_solve_ir -- A_H x = b by iterative refinement: x_0 = 0, and while
 * ||b - A_H x_k||_2 > tol ||b||_2 (residual with the FP64 entries),
 * x_{k+1} = x_k + d_k where GMRES(restart) solves A_p d_k = r_k with the
 * entries stored in inner_precision p (1: FP32 copies) to the relative
 * residual max(inner_tol, tol ||b|| / (2 ||r_k||)). The accuracy reached is
 * that of hmat_solve at the same tol; the inner products read half the bytes.
 * b, x: DEVICE, n_dof entries. maxit bounds the inner iterations in total.
 * info->iterations counts inner GMRES steps, info->refinements outer steps,
 * info->relres is the final FP64 relative residual. Errors: as hmat_solve;
 * HMAT_EINVAL if inner_precision is 1 without FP32 copies or inner_tol is
 * outside (0, 1); HMAT_ENOCONV (x and info written) when maxit is reached.
 */
hmat_status hmat_solve_ir(hmat_t h, const double* b, double* x, double tol, int32_t restart,
                          int32_t maxit, int32_t inner_precision, double inner_tol,
                          void* hip_stream, hmat_solve_info* info);

/* hmat_info -- copy build statistics into *st (HOST). */
hmat_status hmat_info(hmat_t h, hmat_stats* st);

/* hmat_free -- release all device and host memory of h (NULL is a no-op).
 * Synchronises the device work of h first. The device memory goes to the
 * library's caches (see the conventions above), not back to the device. */
hmat_status hmat_free(hmat_t h);

/* hmat_release_memory -- hand the device memory the library keeps for reuse
 * back to the device: the cache of released buffers, the idle ACA panel
 * buffers and the unused memory of the current device's stream-ordered pool.
 * The frees are ordered on hip_stream, which is synchronised before return.
 * Memory of live handles is untouched. Must not run while another thread
 * builds on the same device (its panel buffers are not idle then and stay
 * kept). Errors: none beyond device errors (HMAT_EDEVICE). */
hmat_status hmat_release_memory(void* hip_stream);

/*
 * hmat_set_mem_budget -- cap on the device memory the library holds on each
 * device: live buffers of handles, builds, products and solves, plus the
 * memory it keeps for reuse (cached blocks, idle ACA panel buffers). 0 (the
 * default) means no cap; bytes < 0 is HMAT_EINVAL. An allocation that would
 * pass the cap is treated as a full device: the kept memory is handed back
 * and the allocation retried, and if it still does not fit the call fails
 * with HMAT_ENOMEM ("... device memory budget ... exceeded"), leaving no
 * half-built handle. For failure injection and for sharing a device with
 * other users; the request server's per-request vectors are not counted.
 * Process-wide; takes effect at the next allocation.
 */
hmat_status hmat_set_mem_budget(int64_t bytes);

/* hmat_mem_held -- the bytes of device memory the library holds on the
 * current device (what hmat_set_mem_budget caps) and, if peak is not NULL,
 * the most it held right after any of its allocations since the previous
 * hmat_mem_held call (0 if it allocated nothing; each call starts a new
 * interval). HOST outputs; held must not be NULL. */
hmat_status hmat_mem_held(int64_t* held, int64_t* peak);

/* Thread-local description of the last failure on the calling thread. */
const char* hmat_last_error(void);

/* ------------------------------------------------------------------------
 * Inspection entry points (host copies; used by tests and tools).
 * ------------------------------------------------------------------------ */

/*
 * hmat_plan -- host-only partition of a mesh, no device work (Sec. 2.1).
 *   order      HOST int32 [n_triangles] (may be NULL): cluster position p ->
 *              caller's triangle index.
 *   n_blocks   HOST: in: capacity of `blocks` (in blocks); out: |P|.
 *   blocks     HOST int32 [capacity][5] (may be NULL): row_off, row_len,
 *              col_off, col_len (cluster positions, triangles) and 1 for
 *              admissible / 0 for dense, sorted by (row_off, col_off).
 * If the capacity is too small, *n_blocks is set and HMAT_EINVAL returned
 * without writing `blocks`. Same validation as hmat_build for mesh/eta/leaf.
 */
hmat_status hmat_plan(const hmat_mesh* mesh, double eta, int32_t leaf, int32_t* order,
                      int32_t* n_blocks, int32_t* blocks);

/*
 * hmat_block -- block b (0 <= b < n_blocks, canonical order of hmat_plan).
 *   info   HOST int32[8]: row_off, row_len, col_off, col_len (triangles),
 *          admissible flag, rank k (0 for dense), ACA stop reason
 *          (1 threshold, 2 k = min(m,n), 3 all rows vanished; 0 for dense),
 *          reserved.
 *   A      HOST (may be NULL): dense block D_b (m x n, column-major, m = 3 row_len)
 *          or the factor U_b (m x k, column-major).
 *   B      HOST (may be NULL): V_b (n x k, column-major); unused for dense blocks.
 *   prow, pcol  HOST int32 [k] (may be NULL): ACA pivot rows/columns (local DOF).
 */
hmat_status hmat_block(hmat_t h, int32_t b, int32_t* info, double* A, double* B, int32_t* prow,
                       int32_t* pcol);

/*
 * hmat_entries -- A[rows[k], cols[k]] for k < n, evaluated on the device by
 * the same entry code as the dense blocks and ACA (HOST int64 DOF indices in
 * the caller's numbering, HOST float64 output). Synchronises the stream.
 */
hmat_status hmat_entries(hmat_t h, int64_t n, const int64_t* rows, const int64_t* cols,
                         double* out, void* hip_stream);

/*
 * hmat_set_factors -- replace every admissible block's factors with the given
 * ones (HOST): ranks [n_blocks] (entries of dense blocks ignored), and U, V
 * concatenated over admissible blocks in canonical order, each block's U
 * (m x k) then nothing else in U, V (n x k) in V, column-major. Lets the
 * product be checked on factors computed elsewhere. Synchronises the stream.
 */
hmat_status hmat_set_factors(hmat_t h, const int32_t* ranks, const double* U, const double* V,
                             void* hip_stream);

/*
 * hmat_profile -- per-phase timing of hmat_matvec. With enable = 1 (which also
 * resets the counters) every later hmat_matvec records HIP events on its
 * stream between its kernels; enable = 0 stops recording. On return
 * phase_ms (HOST double[4], may be NULL) holds the accumulated milliseconds of
 * [gather x to cluster order, z = V^T x, U z + D x, reduction and scatter to
 * the caller's order] over the products recorded so far, and *calls (may be
 * NULL) their number (one per group of up to 16 right-hand sides). Reading
 * waits for the recorded events.
 */
hmat_status hmat_profile(hmat_t h, int32_t enable, double* phase_ms, int64_t* calls);

/*
 * hmat_matvec_graph -- hmat_matvec_ex replayed from a captured HIP graph. The
 * first call for a given (precision, nrhs, x, ldx, y, ldy) captures the
 * product's kernel launches into a graph (no allocation or memset is
 * recorded); later calls with the same arguments replay it, one launch in
 * place of four per pass. Capture runs on an internal stream; replays are
 * enqueued on `hip_stream`. Up to 256 argument sets are kept per handle
 * (oldest dropped). Results are those of hmat_matvec_ex, bit for bit.
 * Calls that change the product schedule or the stored entries
 * (hmat_tune, hmat_set_factors, hmat_set_precision) wait for the latest
 * replay and drop the graphs, so the next call captures again.
 * Errors: as hmat_matvec_ex.
 */
hmat_status hmat_matvec_graph(hmat_t h, int32_t precision, int32_t nrhs, const double* x,
                              int64_t ldx, double* y, int64_t ldy, void* hip_stream);

/*
 * hmat_tune -- autotuner of the product schedule for nrhs vectors per pass.
 * Times `reps` products (after one warm-up) for each candidate: chunk sizes
 * 8, 16, 32, 64 KB and 8 or 16 columns per batch for one vector; chunk sizes
 * 64, 128, 256, 512 KB for several (the matrix-core path). Keeps the fastest
 * for later products of h. The values of a product change with the schedule
 * only by rounding (the partial sums are grouped differently); each schedule
 * is deterministic. x, y are internal (all-ones input). Synchronises the stream.
 */
typedef struct {
  int32_t nrhs, n_candidates;
  int32_t chunk_kb[8];  /* candidates tried */
  int32_t unroll[8];
  double ms[8];         /* their mean product time */
  int32_t best;         /* index of the chosen candidate */
  int32_t reserved;
  double best_ms;
} hmat_tune_info;

hmat_status hmat_tune(hmat_t h, int32_t nrhs, int32_t reps, void* hip_stream, hmat_tune_info* info);

/*
 * hmat_amvm -- adaptive matrix-vector multiplication (Algorithm 2, Sec. 3):
 * y ~= A x without building the H-matrix to a fixed accuracy first. The
 * sequence A_k shares the tree and partition of hmat_build (eta, leaf); its
 * dense blocks are exact, and every admissible block starts at rank 0. The
 * look-ahead A^_k takes two more ACA steps on every admissible block; ACA is
 * resumed from saved state, with no accuracy test of its own, and its pivot
 * rows cycle through the three displacement components: after a step at row
 * i the next row comes from the next component (i+1, i+2, i mod 3) with
 * unused rows, as the largest |u_l| there of the latest cross u_l that has
 * entries above 1e-12 of its maximum on those rows, else their lowest row.
 * (On coplanar clusters the in-plane and normal components decouple; plain
 * partial pivoting would never sample the normal one, and the estimator
 * would miss its error.) Each round:
 *   - d_b = (A^_k - A_k)_b x_s for every admissible block;
 *   - gamma_k = ||b_k - b^_k||_2 = ||sum_b d_b||;
 *   - rows are visited in decreasing |(b^_k - b_k)_i|, and a block containing
 *     row i is marked when |(d_b)_i| >= (1 - theta)(c_sp M N)^(-1/2) gamma_k;
 *   - marking stops once ||sum_{b unmarked} d_b|| <= (1 - theta) gamma_k;
 *   - marked blocks take their look-ahead (A_{k+1} = A^_k there).
 * Stops when gamma_k <= tol ||b^_k||_2 (tolerance read as relative) or after
 * max_rounds rounds; y = b_k.
 *   mesh, E, nu, eta, leaf   as for hmat_build (HOST mesh, copied).
 *   x, y     DEVICE vectors of n_dof entries, DOF 3i+a in mesh order.
 *   theta    Doerfler parameter in (0, 1); tol > 0.
 *   kmax     cap on the ACA steps per block (2..4096); a block that reaches
 *            it, or full rank, is exhausted and contributes no further.
 *   ranks    HOST, n_blocks entries or NULL: final rank of each admissible
 *            block in canonical block order (-1 for dense blocks).
 * Marking runs on the device; a round reads back a few scalars and the join
 * order. Work runs on the given stream and on two internal ones (created and
 * destroyed by the call). Synchronises the stream. Errors: as hmat_build;
 * HMAT_EINVAL for theta, tol, kmax, max_rounds or NULL/aliased vectors.
 */
typedef struct {
  int32_t rounds;          /* rounds of Algorithm 2 that marked blocks */
  int32_t exhausted;       /* admissible blocks out of ACA steps (rank min(m,n), rows used, or kmax) */
  int64_t aca_steps;       /* sum over admissible blocks of the ACA steps taken (incl. look-ahead;
                              the largest blocks, m + n >= 2048, compute their look-ahead one
                              round early, so up to two of their steps may stay unused) */
  int64_t marked_total;    /* sum over rounds of |P_k| */
  double gamma;            /* final estimator gamma_k */
  double time_ms;
} hmat_amvm_info;

hmat_status hmat_amvm(const hmat_mesh* mesh, double E, double nu, double eta, int32_t leaf,
                      const double* x, double* y, double theta, double tol, int32_t max_rounds,
                      int32_t kmax, void* hip_stream, int32_t* ranks, hmat_amvm_info* info);

/* ------------------------------------------------------------------------
 * Request server: continuous admission of independent requests (one mesh
 * each: build, then products or a solve) under a device-memory budget.
 * `slots` worker threads, each with its own HIP stream, run admitted requests
 * concurrently on the device; the oldest pending request is admitted as soon
 * as a worker is free and its memory estimate fits beside the running ones
 * (always when nothing runs). Each request's H-matrix stays on the device
 * for all of its vectors and is freed when the request completes. A result
 * does not depend on the other requests: the same request alone and in a mix
 * gives the same values.
 */
typedef struct hmat_server* hmat_server_t;

enum { HMAT_REQ_MATVEC = 0, HMAT_REQ_SOLVE = 1 };

typedef struct {
  int32_t kind;       /* HMAT_REQ_MATVEC: nvec products; HMAT_REQ_SOLVE: one solve */
  int32_t nvec;       /* products: 1..64 vectors (ignored for a solve) */
  int32_t precision;  /* 0: FP64 throughout; 1: reduced precision. Products build an
                         FP32-only handle (hmat_build_ex precision 1: FP32 ACA at
                         eps >= 1e-5) and read it. Solves build in FP64, add FP32
                         copies and refine FP32 inner GMRES with FP64 residuals of
                         the FP64 operator (hmat_solve_ir, inner_tol 1e-6) */
  int32_t restart;    /* solve: GMRES restart length (1..1024) */
  double E, nu, eps;  /* material (Sec. 1) and ACA accuracy, as for hmat_build */
  double tol;         /* solve: FP64 relative residual to reach */
} hmat_request;

typedef struct {
  int32_t status;       /* hmat_status of the request */
  int32_t iterations;   /* solve: GMRES steps (inner steps for precision 1) */
  int32_t refinements;  /* solve, precision 1: outer refinement steps */
  int32_t reserved;
  double relres;        /* solve: final FP64 relative residual */
  double t_submit_ms;   /* server clock (ms since hmat_server_create) */
  double t_admit_ms;
  double t_done_ms;
  double build_ms;      /* hmat_build of the request's H-matrix */
  int64_t device_bytes; /* device memory its handle held */
} hmat_result;

/* hmat_server_create -- start `slots` (1..64) workers on the current device.
 * hbm_budget: bytes the running requests may hold together (0: 80% of the
 * free device memory). eta, leaf: as for hmat_build, shared by all requests.
 * Errors: HMAT_EINVAL, HMAT_ENOMEM, HMAT_EDEVICE (no device). */
hmat_status hmat_server_create(int32_t slots, int64_t hbm_budget, double eta, int32_t leaf,
                               hmat_server_t* out);

/* hmat_server_submit -- queue a request; mesh, req and in are HOST data,
 * copied before return. in: nvec x n_dof vectors (products, vector-major)
 * or n_dof (the right-hand side of a solve), DOF 3i+a in mesh order.
 * *id receives the request id. Errors: HMAT_EINVAL (mesh or parameters,
 * as hmat_build; kind, precision, nvec, tol, restart), HMAT_ENOMEM. */
hmat_status hmat_server_submit(hmat_server_t s, const hmat_mesh* mesh, const hmat_request* req,
                               const double* in, int64_t* id);

/* hmat_server_wait -- block until request `id` completes; out (HOST,
 * nvec x n_dof or n_dof; may be NULL) receives A_H x or the solution, res
 * (may be NULL) its timings and counts. A request is collected once: the
 * first wait takes it, and a second wait on the same id (also one made
 * while the first still waits) returns HMAT_EINVAL. Returns the request's
 * status (its error message via hmat_server_last_error): HMAT_ECANCELED for
 * a cancelled request; HMAT_EINVAL for an unknown id. */
hmat_status hmat_server_wait(hmat_server_t s, int64_t id, double* out, hmat_result* res);

/* hmat_server_cancel -- stop request `id` if it has not finished. A queued
 * request leaves the queue at once (it never holds a reservation); a running
 * one stops at its next phase boundary (before its build, after its build,
 * before its products or solve), frees its handle and gives its memory
 * reservation back, so queued requests can be admitted. Its wait then
 * returns HMAT_ECANCELED. A request that has already finished keeps its
 * result. Returns HMAT_OK, or HMAT_EINVAL for an unknown or collected id. */
hmat_status hmat_server_cancel(hmat_server_t s, int64_t id);

/* hmat_server_status -- HOST snapshot: bytes reserved by running requests
 * (in_use), queued and running requests; any pointer may be NULL. */
hmat_status hmat_server_status(hmat_server_t s, int64_t* in_use, int32_t* queued, int32_t* running);

/* hmat_server_destroy -- finish every queued request, stop the workers and
 * free the server (NULL is a no-op). */
hmat_status hmat_server_destroy(hmat_server_t s);

/* Message of the last failed server call on this thread. */
const char* hmat_server_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HMAT_H */
