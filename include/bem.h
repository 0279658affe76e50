/*
 * bem.h - C ABI of libbem: Galerkin boundary-element weak-form entries on an
 * AMD Instinct MI355X (gfx950), the adaptive cross approximation (ACA) that
 * consumes them, and the H-matrix assembly built on both.
 *
 * What is computed (Vater, Betcke, Dilba, "Simple and efficient GPU
 * parallelization of existing H-Matrix accelerated BEM code", Section 2):
 *
 *   single layer, Eq. (slp):  A_ij = int_Gi int_Gj psi_i(x) g(x,y)     phi_j(y)
 *   double layer, Eq. (dlp):  A_ij = int_Gi int_Gj psi_i(x) dg/dn_y    phi_j(y)
 *   adjoint double layer, Eq. (adlp):
 *                             A_ij = int_Gi int_Gj psi_i(x) dg/dn_x    phi_j(y)
 *   hypersingular, Eq. (hypsHelmholtz), P1 only:
 *                             A_ij = int_Gi int_Gj g(x,y) [curl psi_i(x) . curl phi_j(y)
 *                                                    - k^2 psi_i(x) phi_j(y) n_x . n_y]
 *   g(x,y) = exp(i k |x-y|) / (4 pi |x-y|)   (Helmholtz; Laplace is k = 0)
 *
 * Row i is the test function psi_i (variable x), column j the trial function
 * phi_j (variable y); n_y is the unit normal of the trial triangle, n_x that
 * of the test triangle.  With the same space and rule on both sides the
 * adjoint double layer is the transposed double layer, A'_ij = K_ji, and is
 * evaluated that way (the same kernels with test and trial exchanged).  For
 * the hypersingular operator curl u = n x grad_Gamma u is constant on each
 * triangle for the hat functions; P0 requests fail with BEM_E_ARG.  Its far
 * entries cancel like (h/r)^2 (the curls of a triangle's three hat functions
 * sum to zero), so FP32 loses about that factor in relative accuracy.  Basis
 * functions: P0 (one dof per triangle, the indicator of the triangle) or P1
 * (one dof per vertex, the continuous piecewise-linear hat function).
 * Both integrals use the same symmetric Gauss rule per triangle (Section
 * 3.2.1: the 6-point rule of degree 4; the 4-point rule of degree 3 is the
 * other choice), tensorised over each pair of triangles.  Only regular pairs
 * are integrated: triangles that share no vertex (Section 3.2.3 leaves
 * identical, edge- and vertex-adjacent pairs to a singular scheme).  A pair
 * that shares a vertex either contributes zero (BEM_NEAR_SKIP) or fails the
 * whole call (BEM_NEAR_ERROR).
 *
 * Conventions for every call
 *   - Indices are 0-based int32 dof ids: triangle ids for P0, vertex ids for
 *     P1, 3 t + a for DP1.  Duplicated indices are allowed.
 *   - Outputs are row-major nrows x ncols.  Element type by (operator,
 *     precision): Laplace FP64 -> double, Laplace FP32 -> float, Helmholtz
 *     FP64 -> complex double, Helmholtz FP32 -> complex float; complex values
 *     are interleaved (re, im).
 *   - k must be 0 for Laplace and real, finite and > 0 for Helmholtz.
 *   - Meshes must be welded (shared vertices share an index) and
 *     outward-oriented: the normal of triangle (a,b,c) points along
 *     (b-a) x (c-a); the double-layer sign depends on it.
 *   - The caller owns every buffer passed in; the library copies what it
 *     keeps.  Outputs are written only when the call returns BEM_OK.
 *   - Every entry point is thread-safe; many host threads may call
 *     concurrently (that is how ACA workers use the library).
 *   - On failure a negative status is returned and bem_last_error() gives a
 *     message (per calling thread).
 *   - The library runs on the HIP device that is current when the first
 *     mesh is created (device 0 by default).
 */
#ifndef BEM_H
#define BEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define BEM_OK 0
#define BEM_E_ARG (-1)        /* invalid argument (index out of range, bad k, ...) */
#define BEM_E_OOM (-2)        /* host or device allocation failed / request too large */
#define BEM_E_DEVICE (-3)     /* HIP runtime error */
#define BEM_E_NEARFIELD (-4)  /* a contributing pair shares a vertex under BEM_NEAR_ERROR */
#define BEM_E_BUSY (-5)       /* object still in use by requests in flight */
#define BEM_E_CANCELLED (-6)  /* request cancelled (server shut down) */
#define BEM_E_TIMEOUT (-7)    /* wait timed out; the request is still pending */
#define BEM_E_INTERNAL (-8)   /* internal inconsistency */

typedef enum {
    BEM_LAPLACE_SLP = 0,
    BEM_LAPLACE_DLP = 1,
    BEM_HELMHOLTZ_SLP = 2,
    BEM_HELMHOLTZ_DLP = 3,
    BEM_LAPLACE_ADLP = 4,
    BEM_HELMHOLTZ_ADLP = 5,
    BEM_LAPLACE_HYPS = 6,     /* P1 only */
    BEM_HELMHOLTZ_HYPS = 7    /* P1 only */
} bem_op;
/* Trial and test spaces (the same on both sides): BEM_P0, one dof per
 * triangle (its indicator); BEM_P1, one dof per vertex (the continuous hat
 * function); BEM_DP1, three dofs per triangle, dof 3 t + a the barycentric
 * function of local vertex a on triangle t alone (discontinuous piecewise
 * linear: the space whose single layer gives the hypersingular operator by
 * sparse transformations, Eq. hyp_via_slp). */
typedef enum { BEM_P0 = 0, BEM_P1 = 1, BEM_DP1 = 2 } bem_space;
/* BEM_FP64: plain FP64 quadrature.  BEM_FP32: FP32 quadrature with
 * compensated (TwoSum) accumulation, centroid-relative geometry and, for
 * Helmholtz, the phase k r reduced to a turn in FP64. */
typedef enum { BEM_FP64 = 0, BEM_FP32 = 1 } bem_prec;
/* Vertex-sharing (identical, edge- or vertex-adjacent) triangle pairs:
 * BEM_NEAR_ERROR fails the call, BEM_NEAR_SKIP lets them contribute zero,
 * BEM_NEAR_SINGULAR integrates them on the device with a singular scheme
 * (Section 3.2.3 leaves them to one; here: coordinates around the pair's
 * singular set with the radial integral in closed form and composite
 * Gauss-Legendre rules for the rest, ~1e-12 relative, FP64, added to the
 * regular part; Helmholtz: the radial integral of e^{ikr} as a 48-term
 * power series in omega = k |c| (x - y = rho c), accurate to ~5e-10 up to
 * omega = 12: a Helmholtz request whose vertex-sharing pairs reach beyond
 * that (about one element per wavelength or coarser) fails with BEM_E_ARG;
 * P1: each pair's 3 x 3 local matrix, then a fixed-order sum per entry; the
 * hypersingular operators: the hat functions' constant curls times each
 * pair's P0 single-layer integral, minus k^2 n_x . n_y times its P1
 * single-layer local matrix).  BEM_NEAR_SINGULAR is available for every
 * operator and space (the hypersingular operator: P1 only, as everywhere). */
typedef enum { BEM_NEAR_ERROR = 0, BEM_NEAR_SKIP = 1, BEM_NEAR_SINGULAR = 2 } bem_near;

typedef struct bem_mesh bem_mesh;
typedef struct bem_ticket bem_ticket;
typedef struct bem_hmat bem_hmat;

/* Returns a message describing the last failure on the calling thread. */
const char *bem_last_error(void);

/* ---- meshes ------------------------------------------------------------ */
/* Upload a triangle mesh and precompute its geometry on the device
 * (Section 3.2.1: the grid is copied to the device whole, normals,
 * Jacobians and quadrature points are computed there and kept resident).
 *   xyz: nv x 3 vertex coordinates (host, row-major); tri: nt x 3 vertex ids
 *   (host, row-major, counter-clockwise seen from outside);
 *   quad_points: 6 (degree-4 rule) or 4 (degree-3 rule).
 * Errors: BEM_E_ARG (index out of range, degenerate triangle, bad
 * quad_points), BEM_E_OOM, BEM_E_DEVICE.  *out receives the handle. */
int bem_mesh_create(const double *xyz, int64_t nv, const int32_t *tri, int64_t nt,
                    int quad_points, bem_mesh **out);

/* Release a mesh.  BEM_E_BUSY while requests on it are in flight. */
int bem_mesh_destroy(bem_mesh *mesh);

typedef struct {
    int64_t nv, nt;
    int32_t quad_points;
    int32_t max_star;          /* largest number of triangles around a vertex */
    double mean_jacobian;      /* mean of |(b-a) x (c-a)| */
    double mean_edge;          /* mean edge length */
    size_t device_bytes;       /* resident device memory of the mesh */
} bem_mesh_info_t;
int bem_mesh_info(const bem_mesh *mesh, bem_mesh_info_t *info);

/* ---- weak-form entries ------------------------------------------------- */
/* A[rows, cols] of operator op on space `space` (test and trial spaces are
 * the same), evaluated on the device; blocks until the result is in `out`
 * (host memory, nrows*ncols elements of the type given above).
 * nrows == 0 or ncols == 0 returns BEM_OK and writes nothing.
 * Errors: BEM_E_ARG (index out of range, bad k/op/space/prec),
 * BEM_E_NEARFIELD (BEM_NEAR_ERROR and a contributing pair shares a vertex;
 * out untouched), BEM_E_OOM (request larger than the server arena),
 * BEM_E_DEVICE. */
int bem_eval_entries(bem_mesh *mesh, bem_op op, bem_space space, double k,
                     const int32_t *rows, int64_t nrows, const int32_t *cols, int64_t ncols,
                     bem_prec prec, bem_near near, void *out);

/* Same request, submitted to the device request server without waiting.
 * rows/cols are copied before the call returns; `out` (host memory) must
 * stay valid until the ticket completes.  Requests submitted by any thread
 * are admitted by memory, fused into shared kernel launches and overlap on
 * the device.  The ticket must be released with bem_ticket_free. */
int bem_submit(bem_mesh *mesh, bem_op op, bem_space space, double k,
               const int32_t *rows, int64_t nrows, const int32_t *cols, int64_t ncols,
               bem_prec prec, bem_near near, void *out, bem_ticket **ticket);

/* Wait up to timeout_s seconds (negative: forever).  Returns the request's
 * status (BEM_OK, BEM_E_NEARFIELD, ...) or BEM_E_TIMEOUT if still pending. */
int bem_ticket_wait(bem_ticket *ticket, double timeout_s);

/* Submit/complete timestamps of a finished request, seconds on the
 * library's monotonic clock. */
int bem_ticket_times(const bem_ticket *ticket, double *t_submit, double *t_done);

/* Release a ticket; waits for the request first if it is still pending. */
int bem_ticket_free(bem_ticket *ticket);

/* Same request with the result written to device memory `dev_out` on the
 * caller's HIP stream `stream` (hipStream_t; NULL = null stream), without
 * host synchronisation.  rows/cols are host arrays, expanded and staged
 * through pinned memory by the library; the call returns once the work is
 * enqueued, and dev_out is complete when the stream reaches that point.
 * Workspace comes from the stream-ordered allocator on the same stream.
 * Under BEM_NEAR_ERROR the adjacency check runs on the host before anything
 * is enqueued (BEM_E_NEARFIELD, nothing enqueued). */
int bem_eval_entries_async(bem_mesh *mesh, bem_op op, bem_space space, double k,
                           const int32_t *rows, int64_t nrows, const int32_t *cols, int64_t ncols,
                           bem_prec prec, bem_near near, void *dev_out, void *stream);

/* For callers that cannot allocate device memory (code that runs under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same request as bem_eval_entries_async, computed by the same kernels, with
 * its workspace (descriptor, block table, singular-pair records, staged
 * inputs, status word) in a fixed 32 MiB static device array instead of the
 * stream-ordered allocator, and its host image in a per-thread pageable
 * buffer instead of pinned staging.  The call makes no device or pinned
 * allocation.  Differences from bem_eval_entries_async:
 *   - a request whose workspace exceeds 32 MiB fails with BEM_E_OOM
 *     (nothing enqueued); a P1 row or column of 4,096 entries needs well
 *     under 1 MiB;
 *   - the copy of the workspace from pageable host memory is synchronous
 *     with the host, so the call returns once the stream has reached it;
 *   - every call on one device uses the same workspace: calls that overlap on
 *     a device race (two streams, or two host threads) and must be ordered
 *     by the caller, for instance by issuing them on one stream from one
 *     thread.  The workspace keeps the last call's contents; everything a
 *     call reads is rewritten by that call.
 * dev_out (device, nrows x ncols, types as bem_eval_entries) is complete
 * when `stream` reaches the end of the work this call enqueued.  Arguments
 * and errors otherwise as bem_eval_entries_async. */
int bem_eval_entries_async_noalloc(bem_mesh *mesh, bem_op op, bem_space space, double k,
                                   const int32_t *rows, int64_t nrows, const int32_t *cols, int64_t ncols,
                                   bem_prec prec, bem_near near, void *dev_out, void *stream);

/* ---- pair-based dense blocks ------------------------------------------- */
typedef struct {
    int64_t pairs;               /* triangle pairs integrated (row-star x column-star triangles, all panels) */
    int64_t panels;              /* row panels */
    double seconds;              /* wall time of the call */
    int64_t first_pairs;         /* pairs of the first panel */
    double first_local_seconds;  /* its local-matrix kernel, HIP events on the compute stream */
    double first_gather_seconds; /* its gather kernel */
} bem_dense_stats;

/* A[rows, cols] of a P1 block by triangle pairs (Section 3's dense
 * assembly: kernel values at all pairs of Gauss points of a triangle pair,
 * weighted with the basis functions of every local dof pair): each regular
 * pair of star(rows) x star(cols) is integrated once into its 3 x 3 local
 * matrix on the device (144 kernel evaluations per entry of a full matrix,
 * where row requests integrate a pair once per test vertex), then every
 * entry adds its pairs' values in a fixed order (row star outer, column star
 * inner; compensated in FP32).  Rows go in panels whose local matrices fit
 * BEM_DENSE_BUDGET_MB (environment, default 1024) MiB of device memory; a
 * panel's assembly overlaps the transfer of the previous panel's entries.
 * out: host, nrows x ncols row-major (types as bem_eval_entries).  Single
 * and double layer (Laplace, Helmholtz), P1, BEM_NEAR_ERROR (checked on the
 * host before anything runs) or BEM_NEAR_SKIP; stats may be NULL.  The
 * call allocates its device workspace and pinned staging and frees them
 * before it returns.  Errors as bem_eval_entries. */
int bem_eval_dense(bem_mesh *mesh, bem_op op, bem_space space, double k, const int32_t *rows, int64_t nrows,
                   const int32_t *cols, int64_t ncols, bem_prec prec, bem_near near, void *out,
                   bem_dense_stats *stats);

/* ---- request server ---------------------------------------------------- */
/* Size the request server (Section 4's block threads are replaced by it):
 * arena_bytes of device memory (and the same amount of pinned host staging),
 * split into up to 16 batch slots (one per MiB of arena, at least 2), hold
 * the batches in flight, so a batch admits
 * requests while their inputs, outputs and tables fit one slot (admission by
 * memory; a single request larger than a slot fails with BEM_E_OOM);
 * max_batch_requests bounds how many requests one fused launch takes.
 * Defaults: 1 GiB, 16384.  arena_bytes >= 4 MiB, else BEM_E_ARG.  A running
 * server is drained and restarted with the new sizes at the next submission;
 * it must be idle (no request pending or in flight, no borrowed result
 * outstanding), else BEM_E_BUSY and nothing changes.  A submission racing
 * with the drain fails with BEM_E_BUSY. */
int bem_server_config(size_t arena_bytes, int max_batch_requests);

typedef struct {
    int64_t requests;        /* completed requests */
    int64_t entries;         /* completed entries */
    int64_t batches;         /* fused launches */
    int64_t kernel_evals;    /* pair-quadrature kernel evaluations (Q^2 per regular pair) */
    double latency_p50;      /* seconds, submit -> completion, over the window */
    double latency_p99;
    double latency_max;
    double busy_seconds;     /* wall time with at least one batch on the device */
    double kernel_seconds;   /* entry-kernel execution times (device clock), summed over the timed
                                batches and scaled to all batches */
    int64_t kernel_launches; /* launches timed: every launch of one batch in eight carries start/stop
                                HIP events, so kernel_seconds covers that sample */
    double dispatch_seconds; /* host time spent staging and enqueueing batches */
    double complete_seconds; /* host time spent completing batches (after their event) */
    double wait_seconds;     /* completion-thread time spent waiting for batch events */
    double dispatch_hip_seconds; /* part of dispatch_seconds spent inside HIP enqueue calls */
    /* request-weighted means of the four legs of submit -> completion */
    double mean_queue_seconds;    /* submitted -> taken into a batch */
    double mean_stage_seconds;    /* taken -> batch enqueued on its stream */
    double mean_device_seconds;   /* enqueued -> batch event observed complete */
    double mean_complete_seconds; /* event observed -> request completed (callbacks included) */
} bem_server_stats_t;

/* Statistics since the last reset; reset != 0 clears them afterwards. */
int bem_server_stats(bem_server_stats_t *stats, int reset);

/* Per kernel variant, over the launches of one batch in eight: launches,
 * durations and the work those timed launches covered.  `seconds` is the
 * kernels' own execution time (earliest wavefront start to latest wavefront
 * end on the device's constant-rate clock); `seconds_events` is the time
 * between HIP events recorded around each launch on its stream, which also
 * holds whatever separates the start event from the kernel's start (host
 * submission of the launch, other work of the same hardware queue).  One
 * entry launch serves row and column requests alike.
 * Records with persistent = 1 would be resident launches serving the
 * server's batches of ACA rows and columns one after another (every such
 * launch ended since the last reset, with all the work of its batches, both
 * times its whole residency); those launches are switched off in this build
 * (BEM_SERVER_PERSIST=1 makes the server refuse to start), so none appear. */
typedef struct {
    int32_t op, space, prec, quad_points;
    int32_t persistent;        /* 1: resident launches serving batch after batch */
    int32_t reserved;
    int64_t launches;
    int64_t workgroups;        /* 256-thread workgroups of these launches */
    int64_t entries;           /* entries of the requests these launches served */
    int64_t pair_evals;        /* Q^2 x (fixed, lane) triangle pairs; vertex-sharing pairs, which are
                                  skipped, are included (there are none in admissible blocks) */
    int64_t triangle_loads;    /* lane-triangle geometry records gathered (one per lane per workgroup) */
    double seconds;            /* summed kernel execution times (device clock) */
    double seconds_events;     /* summed HIP-event launch brackets */
    int64_t blocks;            /* blocks of entry work served (one per workgroup of a launch of its own) */
} bem_kernel_stats_t;

/* Copies up to max_entries variant records into out, sets *count to the
 * number of variants recorded; reset != 0 clears them afterwards. */
int bem_server_kernel_stats(bem_kernel_stats_t *out, int max_entries, int *count, int reset);

/* ---- adaptive cross approximation --------------------------------------- */
typedef struct {
    double tol;          /* relative stopping tolerance: ||u_k|| ||v_k|| <= tol ||S_k||_F */
    int32_t max_rank;    /* upper bound on the rank */
    double zero_abs;     /* a residual row with max |entry| <= zero_abs vanishes; < 0: derived
                            from the block geometry */
} bem_aca_params;

/* ACA on the block A[rows, cols] (Algorithm "ACA", Section 2.1): rows and
 * columns of the block are evaluated on the device through the request
 * server (precision `prec`), pivots and residual updates run in FP64 on the
 * host.  Output A ~= U V^T with U column-major m x max_rank and V
 * column-major n x max_rank (double, or complex double for Helmholtz);
 * columns >= *rank are left untouched.  *entries_evaluated counts the
 * entries requested from the device.  Every pair must be regular
 * (BEM_E_NEARFIELD otherwise). */
int bem_aca_block(bem_mesh *mesh, bem_op op, bem_space space, double k,
                  const int32_t *rows, int64_t m, const int32_t *cols, int64_t n,
                  const bem_aca_params *params, bem_prec prec,
                  void *U, void *V, int32_t *rank, int64_t *entries_evaluated);

/* ACA on caller-supplied entries (no device involved): get_row(ctx, i, out)
 * writes block row i (n values), get_col(ctx, j, out) block column j (m
 * values), as double or interleaved complex double (is_complex != 0).  Same
 * algorithm and outputs as bem_aca_block. */
typedef void (*bem_row_fn)(void *ctx, int64_t i, double *out);
typedef void (*bem_col_fn)(void *ctx, int64_t j, double *out);
int bem_aca_callback(int64_t m, int64_t n, int is_complex, bem_row_fn get_row, bem_col_fn get_col,
                     void *ctx, const bem_aca_params *params, void *U, void *V, int32_t *rank);

/* ---- cluster tree, block tree, H-matrix --------------------------------- */
/* Geometric partition (Section 2.1): a cluster tree over the dof points,
 * split at the midpoint of the longest bounding-box side (median split when
 * one side would be empty), and the block tree from (root, root) whose
 * leaves are admissible when dist > 0 and min(diam) <= eta dist on the
 * clusters' support boxes and, with max_block > 0, neither cluster holds
 * more than max_block dofs (0: no bound); dense when either cluster is a
 * leaf.
 * Host-only.  Writes up to max_blocks leaves as (row cluster, col cluster,
 * admissible) triples and the dof ranges of every cluster: cluster c holds
 * dofs perm[cl_begin[c] .. cl_end[c]); perm holds one entry per dof of the
 * space (nt, nv or 3 nt).  Sizes are returned in *nblocks and
 * *nclusters; when a capacity is too small nothing else is written and
 * BEM_E_ARG is returned with the needed sizes. */
int bem_partition(const double *xyz, int64_t nv, const int32_t *tri, int64_t nt, bem_space space,
                  int32_t leaf_size, double eta, int32_t max_block,
                  int32_t *perm, int32_t *cl_begin, int32_t *cl_end, int64_t max_clusters,
                  int32_t *blocks /* 3 x max_blocks */, int64_t max_blocks,
                  int64_t *nclusters, int64_t *nblocks);

typedef struct {
    int32_t leaf_size;      /* 100 */
    double eta;             /* 1.0 */
    double aca_tol;         /* 1e-5 */
    int32_t max_rank;       /* 200 */
    int32_t n_workers;      /* host ACA worker threads */
    int32_t blocks_per_worker; /* ACA blocks each worker keeps in flight */
    bem_prec prec;          /* precision of the device entries */
    int32_t dense_mode;     /* 0: dense leaves left empty; 1: their regular part (BEM_NEAR_SKIP);
                               2: complete, singular pairs included (BEM_NEAR_SINGULAR) */
    int32_t max_block;      /* largest dimension of an admissible block (0: no bound); larger
                               cluster pairs are split further */
    int32_t hyps_via_slp;   /* hypersingular operators: 1 = assemble the single layer on DP1 (same
                               parameters) and apply D = sum_j Q_j^T S Q_j - k^2 sum_j P_j^T S P_j
                               with the sparse curl (Q_j) and normal (P_j) factors, Eq. hyp_via_slp
                               (its entries are sums of positive-kernel integrals, so FP32 ACA keeps
                               its accuracy); 0 = assemble D's entries directly */
} bem_hmat_params;

/* Fill every admissible leaf of the block tree by ACA (all rows and columns
 * on the device) and, if dense_mode is 1 or 2, every dense leaf (its regular
 * part, or all of it).  The caller gets an H-matrix handle.  With
 * hyps_via_slp the handle applies D through the DP1 single layer: its
 * matvec takes P1 vectors, its statistics, block info and dense blocks are
 * those of the DP1 single layer. */
int bem_hmat_assemble(bem_mesh *mesh, bem_op op, bem_space space, double k,
                      const bem_hmat_params *params, bem_hmat **out);

/* y = H x (host vectors of length ndof, double or interleaved complex
 * double). */
int bem_hmat_matvec(const bem_hmat *h, const void *x, void *y);

typedef struct {
    int64_t ndof;
    int64_t admissible_blocks, dense_blocks;
    int64_t aca_entries;       /* entries requested by ACA */
    int64_t dense_entries;     /* entries of dense leaves evaluated */
    int64_t aca_requests;      /* row and column requests */
    int64_t rank_sum;
    int32_t rank_max;
    size_t bytes;              /* storage of U, V and dense leaves */
    double seconds;            /* wall time of the assembly */
    double partition_seconds;  /* cluster and block tree */
    double setup_seconds;      /* lane sets of the clusters (host expansion + upload), leaf lists */
    double aca_seconds;        /* worker phase: ACA and dense leaves */
    double worker_busy_seconds;/* summed over workers: time spent outside waits */
} bem_hmat_stats;
int bem_hmat_stats_get(const bem_hmat *h, bem_hmat_stats *stats);

/* Dense reconstruction of block b (leaf order as bem_hmat_block_info):
 * out is rows x cols row-major in the block's local dof order. */
int bem_hmat_block_info(const bem_hmat *h, int64_t b, int32_t *admissible, int64_t *m, int64_t *n,
                        int32_t *rank, const int32_t **rows, const int32_t **cols);
int bem_hmat_block_dense(const bem_hmat *h, int64_t b, void *out);
int bem_hmat_destroy(bem_hmat *h);

/* ---- served ACA block streams ------------------------------------------- */
/* An ACA plan is the set-up of bem_hmat_assemble kept for repeated use: the
 * partition (leaf_size, eta, max_block of params) and, on the device, the
 * lane sets of every cluster of an admissible block.  bem_aca_plan_run then
 * approximates any list of the plan's admissible blocks by ACA (Algorithm
 * "ACA", Section 2.1), every block row and column evaluated on the device
 * through the request server, as a served stream: block i starts no earlier
 * than arrival[i] seconds after the call, params->n_workers host threads
 * keep up to params->blocks_per_worker blocks each in flight (Section 4
 * gives every block its own CPU thread; here each thread holds many blocks
 * as resumable state machines).  Plan block ids run 0 .. n_blocks-1 over
 * the admissible leaves in block-tree order.  aca_tol, max_rank come from
 * params; the precision is chosen per run.  Errors: BEM_E_ARG (bad
 * arguments, a block id out of range, arrival times not finite or
 * decreasing), BEM_E_OOM, BEM_E_DEVICE. */
typedef struct bem_aca_plan bem_aca_plan;
int bem_aca_plan_create(bem_mesh *mesh, bem_op op, bem_space space, double k, const bem_hmat_params *params,
                        bem_aca_plan **out);
/* n_blocks: admissible blocks; ndof: dofs of the space; setup_seconds:
 * partition and lane sets. */
int bem_aca_plan_info(const bem_aca_plan *plan, int64_t *n_blocks, int64_t *ndof, double *setup_seconds);
/* Dimensions and dof lists of plan block b (pointers owned by the plan). */
int bem_aca_plan_block(const bem_aca_plan *plan, int64_t b, int64_t *m, int64_t *n, const int32_t **rows,
                       const int32_t **cols);

typedef struct {
    int64_t blocks;             /* blocks approximated */
    int64_t entries;            /* entries requested from the device */
    int64_t requests;           /* row and column requests */
    int64_t rank_sum;
    int32_t rank_max;
    double seconds;             /* call -> last block finished */
    double mean_start_delay;    /* arrival -> first request of a block, mean over blocks */
    double mean_block_seconds;  /* first request -> factors stored, mean over blocks */
} bem_aca_run_stats;

/* Approximates plan blocks blocks[0 .. n) with entries of precision prec;
 * arrival (seconds after the call, non-decreasing) may be NULL: every block
 * is available at once.  The factors replace those of the previous run. */
int bem_aca_plan_run(bem_aca_plan *plan, const int64_t *blocks, const double *arrival, int64_t n, bem_prec prec,
                     bem_aca_run_stats *stats);
/* One served stream over the blocks of several plans (several meshes,
 * operators or wavenumbers in one device queue): block i is block
 * blocks[i] of plans[plan_index[i]], available arrival[i] seconds after the
 * call (NULL: at once; non-decreasing); n_workers host threads, each with up
 * to blocks_per_worker blocks in flight, take the blocks in arrival order
 * whatever plan they belong to, so one pool of ACA workers serves every plan
 * (the plans' own n_workers and blocks_per_worker are not used).  Each
 * block is approximated with its plan's operator, mesh, wavenumber,
 * tolerance and rank bound, entries of precision prec; its factors replace
 * those of the plan's previous run (a plan's blocks not in this run have
 * none afterwards).  The plans must share the value type (all Laplace or all
 * Helmholtz) and no other run may use them meanwhile.  stats: totals over
 * all blocks.  Errors: BEM_E_ARG (bad arguments, an index out of range,
 * mixed value types), BEM_E_OOM, BEM_E_DEVICE. */
int bem_aca_plans_run(bem_aca_plan *const *plans, int64_t nplans, const int64_t *plan_index, const int64_t *blocks,
                      const double *arrival, int64_t n, bem_prec prec, int32_t n_workers, int32_t blocks_per_worker,
                      bem_aca_run_stats *stats);
/* Factors of plan block b from the last run: *rank, and when U, V are not
 * NULL, U column-major m x rank and V column-major n x rank (double or
 * complex double), block ~= U V^T.  BEM_E_ARG if b was not in the last run. */
int bem_aca_plan_factors(const bem_aca_plan *plan, int64_t b, int32_t *rank, void *U, void *V);
int bem_aca_plan_destroy(bem_aca_plan *plan);

#ifdef __cplusplus
}
#endif

#endif /* BEM_H */
