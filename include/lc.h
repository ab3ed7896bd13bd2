/*
 * lc.h -- C ABI of the MI355X (gfx950) linear-construction covariance path.
 *
 * The path follows the paper's problem statement (Sect. 2.1-2.3, 4.3):
 *   mocks D, each with two random catalogues R1 and R2 of about the data
 *   size; pair counts DD, DR_i and RR_i in (r, mu) bins; the split
 *   Landy-Szalay estimate for (D,R1), (D,R2) and (D, R1 u R2); its Legendre
 *   multipoles l = 0, 2, 4; the sample covariances C^a, C^b over the mocks;
 *   and the linear construction C^LC = A + B/M with A = 2C^b - C^a,
 *   B = 2 M_a (C^a - C^b).
 *
 * Conventions for every call:
 *   - Return value is an lc_status: 0 = LC_OK, negative on error.  No call
 *     aborts or exits.  lc_last_error() gives a message for the calling
 *     thread's last failed call.
 *   - "DEVICE" pointers are HIP device memory on the current device, owned
 *     by the caller; "HOST" arrays are read before the call returns and are
 *     not retained.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Calls are
 *     asynchronous on that stream unless stated otherwise.
 *   - Every error that can be detected on the host is reported before any
 *     work is enqueued.  An asynchronous HIP fault surfaces as LC_ERR_HIP.
 *   - Coordinates are int32 in units of 2^-12 Mpc/h.  Periodic boxes:
 *     0 <= x < box_units <= 2^24.  Open geometry: |x| < 2^24.
 */
#ifndef LC_H
#define LC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lc_status;

#define LC_OK            0
#define LC_ERR_INVALID  -1  /* NULL pointer, bad size, bad edges, bad ids, bad mode */
#define LC_ERR_RANGE    -2  /* coordinate outside the geometry; r_max too large for the box */
#define LC_ERR_OVERFLOW -3  /* a size or index exceeds what the layout supports */
#define LC_ERR_HIP      -4  /* HIP runtime error (message holds hipGetErrorString) */
#define LC_ERR_NOMEM    -5  /* device or pinned allocation failed */

#define LC_LOS_Z    0       /* plane-parallel, line of sight = z axis (Sect. 4.1) */
#define LC_LOS_MID  1       /* line of sight = pair midpoint seen from the origin (open geometry) */
#define LC_LOS_RPPI 2       /* plane-parallel along z, bins in (r_p, pi) instead of (r, mu): the
                               binning of the projected correlation function (Sect. 2.3) */

#define LC_MAX_BINS 32768   /* n_r * n_mu (the block histogram lives in LDS) */
#define LC_MAX_NMU  1024

/* Thread-local message of the last failed call; valid until the next lc_* call. */
const char* lc_last_error(void);

/*
 * Separation binning (Sect. 4.3: 2D correlation function in r and mu).
 *   r bin k:  r_edges[k] <= r < r_edges[k+1]; pairs outside [r_edges[0],
 *             r_edges[n_r]) are not counted.
 *   mu bin m: m = floor(n_mu * |mu|), the last bin closed at |mu| = 1;
 *             mu is the cosine between the line of sight and the pair
 *             separation; a pair at zero separation goes to mu bin 0.
 * Every comparison is exact: it equals the integer rule
 *   r_edges[k]^2 <= d^2 < r_edges[k+1]^2 and the largest m < n_mu with
 *   m^2 d^2 <= n_mu^2 s_z^2 (midpoint: m^2 d^2 |l|^2 <= n_mu^2 (s.l)^2, l = x_i + x_j).
 * LC_LOS_RPPI bins r_p = |(s_x, s_y)| by the r edges
 *   (r_edges[k]^2 <= s_x^2 + s_y^2 < r_edges[k+1]^2) and pi = |s_z| in n_mu
 *   uniform bins of [0, pi_max): m = floor(n_mu |s_z| / pi_max); pairs with
 *   |s_z| >= pi_max are not counted.  The projected correlation function
 *   w_p(r_p) = 2 sum_m xi(r_p, pi_m) (pi_max / n_mu) is then a linear map of
 *   the estimate (lc_map_vectors); the multipole part of lc_xi_multipoles'
 *   output has no meaning for this binning.
 */
typedef struct {
    int32_t periodic;         /* 1: periodic cube [0, box_units)^3, minimal image; 0: open */
    int32_t box_units;        /* periodic side, even, <= 2^24; ignored when open */
    int32_t los;              /* LC_LOS_Z, LC_LOS_MID (requires periodic = 0) or LC_LOS_RPPI */
    int32_t n_r;              /* >= 1 */
    const int32_t* r_edges;   /* HOST, n_r + 1 strictly increasing values >= 0;
                                 periodic: r_edges[n_r] < box_units / 2; open: < 2^25 */
    int32_t n_mu;             /* 1 .. LC_MAX_NMU, n_r * n_mu <= LC_MAX_BINS (LC_LOS_RPPI: pi bins) */
    int32_t pi_max;           /* LC_LOS_RPPI only: 1 <= pi_max < 2^24 units (periodic: < box_units / 2);
                                 ignored otherwise */
} lc_binning;

/*
 * Chaining mesh of many catalogues (counting sort by cell, one grid shared
 * by all catalogues).  Opaque; owned by the library; immutable once built.
 */
typedef struct lc_cells lc_cells;

/* Mesh options; NULL or 0 fields = library defaults. */
typedef struct {
    int32_t cell_units;       /* coarse cell side in coordinate units (default: about
                                 96 points per cell of a mean catalogue, kept within
                                 [r_max / 3, r_max]); rounded so cells tile the box */
    int32_t sub;              /* sub-cells per axis inside a coarse cell: 1, 2 or 4
                                 (default 2); pair counting skips the sub-cells that
                                 lie beyond r_max of each group of 64 points */
    int32_t arrival_order;    /* 0 (default): the points of a sub-cell are stored in
                                 (x, y, z) order, so the mesh, and the candidate tests
                                 counted in stats, depend only on the catalogues (a
                                 pass quadratic in each sub-cell's size and a 16-byte
                                 staging record per point during the build); 1: in
                                 the order the build's atomic counters hand out, which
                                 can change from run to run.  Counts are exact either
                                 way */
    int32_t reserved;
} lc_mesh_opts;

/*
 * lc_build_cells: sort every catalogue into a shared chaining mesh.
 *   xyz          DEVICE int32 SoA [3][n_total]: x[0..n), y[0..n), z[0..n);
 *                catalogues stored back to back.  Not retained.
 *   cat_offsets  HOST int64 [n_cat + 1]; [0] = 0, non-decreasing,
 *                [n_cat] = n_total.  Catalogue c = points [off[c], off[c+1]).
 *   b            binning the mesh will be used with (geometry, r_max).
 *   opts         HOST or NULL (defaults).
 *   out          receives the mesh; free with lc_free_cells.
 * Synchronises `stream` (once for a periodic box, twice for open geometry:
 * the bounding box, then the device range-check word).  A point outside the
 * geometry returns LC_ERR_RANGE and no mesh.  Every catalogue must hold
 * fewer than 2^28 points (else LC_ERR_OVERFLOW).  Any mesh of open geometry
 * serves every line of sight (the midpoint one recovers absolute coordinates
 * from the cell origins, exactly, since open geometry keeps |x| < 2^24).
 */
lc_status lc_build_cells(const int32_t* xyz, int64_t n_total, const int64_t* cat_offsets,
                         int32_t n_cat, const lc_binning* b, const lc_mesh_opts* opts,
                         void* stream, lc_cells** out);
/* Free a mesh once no queued work uses it; also drops the pair-count graphs
 * (LC_GRAPH) captured on it.  NULL is ignored. */
void lc_free_cells(lc_cells* cells);

/* Mesh facts (HOST): grid cells per axis, cell side in units, points. */
typedef struct {
    int32_t n_cat;
    int32_t grid[3];          /* coarse cells per axis */
    double cell_side[3];
    int32_t sub;              /* sub-cells per axis in a coarse cell */
    int32_t reserved;
    int64_t n_total;
    int64_t bytes;            /* device memory held by the mesh */
} lc_cells_info;
lc_status lc_cells_get_info(const lc_cells* cells, lc_cells_info* info);

/*
 * A counting task: catalogues a and b.  a == b: unordered pairs i < j of
 * one catalogue (DD, and RR of one random sub-catalogue -- pairs between
 * different sub-catalogues are never formed, Sect. 2.1 "split");
 * a != b: every pair (i in a, j in b) (DR).
 */
typedef struct { int32_t cat_a, cat_b; } lc_task;

/* lc_pair_count_batch modes */
#define LC_PERSISTENT   0   /* one persistent launch over a work queue of (task, cell) tiles */
#define LC_PER_TASK     1   /* baseline: one launch per task, sized to that task */
#define LC_GRAPH        2   /* flag: capture the launch sequence in a hipGraph, cache, replay.
                                 Replays of one cached configuration share its work-queue
                                 counters: they must not overlap (one stream, or ordered) */
#define LC_FORCE_EXACT  4   /* flag (testing): bin every pair with the integer rule only */

/* Tuning knobs; NULL or 0 fields = library defaults. */
typedef struct {
    int32_t cells_per_item;   /* cells of one catalogue per work item */
    int32_t waves_per_block;  /* 1, 2, 4, 8, 12, 16: waves sharing a work item and a histogram.
                                 Default: batched, the shape with the most resident waves per CU,
                                 the smallest on a tie (4, unless a large histogram leaves LDS for
                                 fewer blocks; 12 is tried with 16-bit bins and for the midpoint
                                 line of sight); LC_PER_TASK, 16 (a single task's few items finish
                                 sooner with more waves each) */
    int32_t blocks_per_cu;    /* persistent grid = CUs * blocks_per_cu (<= occupancy) */
    int32_t chunk;            /* i points tested together against each gathered j set:
                                 a multiple of 4 in [4, 256];
                                 default the maximum */
    int32_t flush_limit;      /* testing: candidate tests a wave may register before it moves
                                 the block histogram out to counts (the overflow guard).
                                 0 = the largest safe value, 2^32 / waves_per_block, which keeps
                                 every uint32 bin from wrapping; a small value forces the guard */
    int32_t queue_order;      /* order of the work queue of a persistent launch (tasks are taken
                                 largest first, by n_a n_b, halved for auto pairs):
                                 LC_QUEUE_XCD_RANGES (0, default): eight contiguous ranges of
                                 equal cost, one per XCD, so an XCD's L2 serves neighbouring
                                 tasks; LC_QUEUE_XCD_DEALT: the cost order dealt to the eight
                                 XCD queues in turn; LC_QUEUE_SHARED: one queue for every block.
                                 A block whose queue is empty takes work from the next one */
    int32_t hist_bits;        /* block histogram bins: 0 = library choice (32-bit, or two 16-bit
                                 bins per word where the 32-bit histogram keeps waves off the CU,
                                 as with 200 x 100 bins), 16 or 32.  A 16-bit bin that wraps is
                                 corrected in the counts at once, so counts stay exact */
    int32_t wrap_test;        /* testing: with 16-bit bins, every bin starts 16 counts below its
                                 wrap (the start values are taken off again), so the wrap
                                 corrections run all the time */
} lc_tuning;

#define LC_QUEUE_XCD_RANGES 0
#define LC_QUEUE_XCD_DEALT  1
#define LC_QUEUE_SHARED     2

/*
 * lc_pair_count_batch: add the (r, mu) pair counts of every task.
 *   cells    mesh from lc_build_cells (built with the same geometry and
 *            an r_max >= this binning's last edge).
 *   tasks    HOST [n_tasks]; catalogue ids < n_cat.
 *   b        binning; n_r * n_mu bins.
 *   counts   DEVICE uint64 [n_tasks][n_r][n_mu], ADDED INTO (zero it first).
 *   mode     LC_PERSISTENT or LC_PER_TASK, optionally | LC_GRAPH | LC_FORCE_EXACT.
 *   tune     NULL for defaults.
 *   stats    DEVICE uint64 [4] or NULL, ADDED INTO: [0] candidate pair
 *            tests, [1] overflow-guard flushes (a wave moved the block
 *            histogram out before its task ended; see flush_limit), [2] pairs
 *            decided by the integer rule (their float estimate was within its
 *            error bound of an edge), [3] block flushes (task changes and the
 *            end of each block's work).  Binned pairs = the sum of counts.
 * Asynchronous.  Counts are exact; the result does not depend on mode,
 * tuning, or the order in which tiles run.
 */
lc_status lc_pair_count_batch(const lc_cells* cells, const lc_task* tasks, int32_t n_tasks,
                              const lc_binning* b, uint64_t* counts, int32_t mode,
                              const lc_tuning* tune, uint64_t* stats, void* stream);

/*
 * lc_pair_count_batch_noalloc: lc_pair_count_batch for callers that cannot
 * allocate device memory (code being captured into a graph, tight serving
 * loops, harnesses that forbid hipMalloc).  It allocates nothing: the launch
 * plan (task order, stencil, squared edges, cell origins, work-queue
 * counters) is written by small kernels, from their arguments, into a static
 * device array of LC_NOALLOC_PLAN_BYTES that the library holds on every
 * device it runs on until the process ends; the caller passes the mesh,
 * tasks, counts and stats as for lc_pair_count_batch.
 *   Arguments, layouts, results and errors as for lc_pair_count_batch, except:
 *   mode      LC_PERSISTENT or LC_PER_TASK, optionally | LC_FORCE_EXACT;
 *             LC_GRAPH returns LC_ERR_INVALID (the graph cache allocates).
 *   A plan larger than LC_NOALLOC_PLAN_BYTES (about 12 bytes per task plus
 *   16 per stencil offset; LC_PER_TASK adds 32 bytes per task) returns
 *   LC_ERR_OVERFLOW before anything is enqueued.
 * Every call on one device shares that device's plan array and rewrites it
 * (the queue counters included) before its launch: calls on one stream run
 * in order, but calls that overlap on one device (other streams, other
 * threads) race.  Asynchronous.
 */
#define LC_NOALLOC_PLAN_BYTES (1 << 20)
lc_status lc_pair_count_batch_noalloc(const lc_cells* cells, const lc_task* tasks, int32_t n_tasks,
                                      const lc_binning* b, uint64_t* counts, int32_t mode,
                                      const lc_tuning* tune, uint64_t* stats, void* stream);

/*
 * lc_xi_multipoles: split Landy-Szalay estimates and their multipoles
 * (Sect. 2.1, 2.3, 4.3), float64.
 *   counts     DEVICE uint64 [n_tasks][n_r][n_mu] from lc_pair_count_batch.
 *   tasks      HOST [n_tasks], as counted.
 *   cat_sizes  HOST int64 [n_cat]: points per catalogue.
 *   est        HOST int32 [n_mock][5]: task ids of DD, DR1, DR2, RR1, RR2 of
 *              each mock; DD = (D,D), DR_i = (D,R_i), RR_i = (R_i,R_i).
 *   xi         DEVICE double [n_mock][3][P], P = n_r*n_mu + 3*n_r, written.
 *              Estimate 0 = (D,R1) with M = 1, 1 = (D,R2) with M = 1,
 *              2 = (D, R1 u R2) split with M = 2.  Vector layout:
 *              [xi(r,mu) r-major | xi_0(r) | xi_2(r) | xi_4(r)].
 *   Normalisation: dd = DD/(N_d(N_d-1)/2), dr_i = DR_i/(N_d N_r,i),
 *   rr_i = RR_i/(N_r,i(N_r,i-1)/2); xi = (dd - (2/M) sum dr_i)/((1/M) sum rr_i) + 1;
 *   a bin with rr = 0 gives NaN.  Multipoles integrate P_l exactly over
 *   every |mu| bin: xi_l(r) = sum_m (2l+1) [int_{mu_m}^{mu_m+1} P_l] xi(r, mu_m).
 */
lc_status lc_xi_multipoles(const uint64_t* counts, const lc_task* tasks, int32_t n_tasks,
                           const int64_t* cat_sizes, int32_t n_cat, const int32_t* est,
                           int32_t n_mock, int32_t n_r, int32_t n_mu, double* xi,
                           void* stream);

/* lc_covariance precision */
#define LC_FP64               0  /* float64 covariance products */
#define LC_FP32_MFMA          1  /* float32 MFMA products, float64 mean/combination/check */
#define LC_FP32_MFMA_CHECKED  2  /* as LC_FP32_MFMA and also the float64 path, for the report */
#define LC_ACC32              8  /* flag for the two float32 modes: accumulate the MFMA products in
                                    float32 over all mocks; without it the float32 accumulators are
                                    added into float64 every 256 mocks */

/* Positive-definiteness report (Sect. 3: C^LC is not guaranteed to be
 * positive definite; check its spectrum).  Block 0 = the (r, mu) part
 * [0, n_r*n_mu), block 1 = the multipole part; the full vector is singular
 * (multipoles are linear in xi(r, mu)), so blocks are checked separately. */
typedef struct {
    int32_t chol_ok[2];       /* 1: Cholesky succeeded (all pivots > 0) */
    int32_t n_neg_eig[2];     /* eigenvalues < 0 (Sturm count at 0); -1 if NaN present */
    double min_eig[2];
    double max_eig[2];
    double rel_frob_vs_fp64[3]; /* ||X32 - X64||_F / ||X64||_F for C, A, B; -1 unless CHECKED */
} lc_cov_report;

/*
 * lc_covariance: sample covariances over mocks and the linear construction.
 *   xi        DEVICE double [n_mock][3][P] from lc_xi_multipoles, P = n_r*n_mu + 3*n_r.
 *   n_mock    >= 2.
 *   m_a       random/data size ratio of R1 and R2 (1 in the paper, Sect. 4.3).
 *   M         target ratio; INFINITY gives A (the infinite-random limit).
 *   A, B, C   DEVICE double [P][P] full symmetric, written; A and B may be NULL.
 *             C^a = (Cov x + Cov x')/2, C^b = Cov y, Cov = sum (v - mean)(v - mean)^T / (N - 1).
 *   rep       HOST or NULL.  Non-NULL runs the float64 Cholesky and
 *             eigenvalue check of C on the device and synchronises `stream`.
 * NaN entries of xi propagate to the affected rows and columns.
 */
lc_status lc_covariance(const double* xi, int32_t n_mock, int32_t n_r, int32_t n_mu,
                        int32_t m_a, double M, int32_t precision,
                        double* A, double* B, double* C, lc_cov_report* rep, void* stream);

/*
 * lc_xi_split: one split Landy-Szalay estimate per mock with M = n_sub random
 * sub-catalogues (the estimator whose sample covariance the linear
 * construction predicts, Sect. 2.1-2.3), with its multipoles; float64.
 *   counts, tasks, cat_sizes  as for lc_xi_multipoles.
 *   est     HOST int32 [n_mock][1 + 2 n_sub]: task ids of DD, DR_1 .. DR_M,
 *           RR_1 .. RR_M; DD = (D,D), DR_i = (D,R_i), RR_i = (R_i,R_i), R_i != D.
 *   xi      DEVICE double, row n (P = n_r*n_mu + 3*n_r values, laid out as one
 *           estimate of lc_xi_multipoles) at xi + n * ld_xi, written.
 *   ld_xi   row stride in doubles, >= P; 0 means P.  ld_xi = 3P with xi
 *           offset by e*P writes estimate e of the [n_mock][3][P] layout
 *           that lc_covariance and lc_covariance_general read.
 * Same normalisation and estimator as lc_xi_multipoles, the sums over
 * subsets taken in the order given; with n_sub = 2 it reproduces that call's
 * third estimate.  Errors: LC_ERR_INVALID for inconsistent task ids or
 * n_sub outside [1, 4096].  Asynchronous.
 */
lc_status lc_xi_split(const uint64_t* counts, const lc_task* tasks, int32_t n_tasks,
                      const int64_t* cat_sizes, int32_t n_cat, const int32_t* est, int32_t n_sub,
                      int32_t n_mock, int32_t n_r, int32_t n_mu, double* xi, int64_t ld_xi, void* stream);

/*
 * lc_covariance_general: the construction from covariances at two general
 * random/data ratios M_a < M_b (Sect. 2.3, Eq. CovAB):
 *   A = (M_b C^b - M_a C^a)/(M_b - M_a),  B = M_a M_b (C^a - C^b)/(M_b - M_a),
 *   C = A + B/M  (M = INFINITY gives A),
 * with C^a = (Cov x + Cov x')/2 and C^b = Cov y over the mocks.
 *   xi        DEVICE double [n_mock][3][P]: per mock two estimates x, x' with
 *             ratio M_a and one estimate y with ratio M_b (lc_xi_split with
 *             ld_xi = 3P fills it); any data vector, e.g. after lc_map_vectors.
 *   n_split   the check treats [0, n_split) and [n_split, P) as two blocks
 *             (0 <= n_split <= P; an empty block reports chol_ok = 1,
 *             n_neg_eig = 0 and NaN extremes).
 *   m_a, m_b  0 < m_a < m_b < infinity.
 *   precision, A, B, C, rep as for lc_covariance, which is this call with
 *             P = n_r*n_mu + 3*n_r, n_split = n_r*n_mu and M_b = 2 M_a.
 * Errors: LC_ERR_INVALID for NULL xi or C, n_mock < 2, P or n_split out of
 * range, bad ratios or precision.  Asynchronous unless rep is given.
 */
lc_status lc_covariance_general(const double* xi, int32_t n_mock, int32_t P, int32_t n_split, double m_a,
                                double m_b, double M, int32_t precision, double* A, double* B, double* C,
                                lc_cov_report* rep, void* stream);

/*
 * lc_rebin_counts: co-added pair counts (Sect. 4.3: the one-dimensional
 * correlation function co-adds the counts over mu; wider r bins co-add
 * adjacent r bins).  Exact uint64 sums.
 *   counts  DEVICE uint64 [n_tasks][n_r][n_mu], read.
 *   w_r     r bins per output bin, 1 <= w_r <= n_r; the last output bin takes
 *           the n_r mod w_r bins that are left (edges e_0, e_{w_r}, ..., e_{n_r}).
 *   w_mu    mu bins per output bin; must divide n_mu (the output mu bins stay
 *           uniform; w_mu = n_mu gives one bin, the 1D count).
 *   out     DEVICE uint64 [n_tasks][ceil(n_r/w_r)][n_mu/w_mu], written; must
 *           not alias counts.  It feeds lc_xi_multipoles / lc_xi_split with
 *           the output n_r and n_mu.
 * Errors: LC_ERR_INVALID for bad sizes or NULL buffers.  Asynchronous.
 */
lc_status lc_rebin_counts(const uint64_t* counts, int32_t n_tasks, int32_t n_r, int32_t n_mu, int32_t w_r,
                          int32_t w_mu, uint64_t* out, void* stream);

/*
 * lc_map_vectors / lc_map_matrix: a linear map T of data vectors in which
 * input element i goes, with weight weight[i], to output element group[i]
 * (group[i] = -1 drops it).  Re-binning (weights 1/w over w adjacent bins)
 * and selecting (e.g. the multipoles over a range of r) are such maps; the
 * construction is linear, so it commutes with them (Sect. 2.3), and the
 * covariances can be re-binned after the fact (Sect. 5.3).
 *   group, weight  HOST [P_in], read before the call returns; every group
 *                  id in [-1, P_out), weights finite.
 *   lc_map_vectors: y_n = T x_n for n_vec rows; x DEVICE double, row n at
 *                  x + n ld_x; y DEVICE double, row n at y + n ld_y, written
 *                  (ld 0 = dense).  Each output sums w_i x_i over its members
 *                  in increasing i.  The [n_mock][3][P] layout maps as
 *                  n_vec = 3 n_mock rows.
 *   lc_map_matrix: Y = T X T^T; X DEVICE double [P_in][P_in], Y DEVICE double
 *                  [P_out][P_out], written.  Y_gh = sum_a w_a (sum_b w_b X_ab)
 *                  over a in g, b in h, increasing.
 * Outputs with no member are 0.  y / Y must not alias the input.  Errors:
 * LC_ERR_INVALID for bad sizes, ids, weights or NULL buffers.  Asynchronous.
 */
lc_status lc_map_vectors(const double* x, int64_t n_vec, int32_t P_in, int64_t ld_x, const int32_t* group,
                         const double* weight, int32_t P_out, double* y, int64_t ld_y, void* stream);
lc_status lc_map_matrix(const double* X, int32_t P_in, const int32_t* group, const double* weight, int32_t P_out,
                        double* Y, void* stream);

/*
 * Maps for lc_map_vectors / lc_map_matrix (HOST calls: they fill host arrays
 * and touch no device).  group and weight are HOST arrays of P_in entries,
 * written; *P_out receives the mapped length.  LC_ERR_INVALID for NULL
 * pointers or sizes out of range.
 *
 * lc_map_multipoles: from the data vector [xi(r, mu) | xi_0 | xi_2 | xi_4]
 *   (P_in = n_r n_mu + 3 n_r) to the multipoles selected by ell_mask (bit 0:
 *   l = 0, bit 1: l = 2, bit 2: l = 4; output blocks in increasing l) over
 *   the r bins [r_lo, r_hi), each output the mean of w adjacent r bins, the
 *   last group narrower when w does not divide r_hi - r_lo.  w = 1 selects:
 *   the 540-element vector of Sect. 5.3 (xi_0, xi_2, xi_4 of the 1 Mpc/h
 *   bins between 20 and 200 Mpc/h); w > 1 re-bins to wider r bins, with the
 *   wide bin's multipole the mean of its narrow bins' (Table 3).
 * lc_map_projected: from the data vector of a (r_p, pi) binning (LC_LOS_RPPI,
 *   n_rp r_p bins x n_pi pi bins, P_in = n_rp n_pi + 3 n_rp) to the projected
 *   correlation function w_p(r_p) = 2 sum_m xi(r_p, pi_m) (pi_max / n_pi)
 *   (Sect. 2.3), in the unit of pi_max; P_out = n_rp.
 * lc_map_rebin_blocks: P_in = n_blocks n; the mean of w adjacent elements
 *   within each block of n (e.g. the r bins of each multipole), the last
 *   group of a block narrower when w does not divide n.
 */
lc_status lc_map_multipoles(int32_t n_r, int32_t n_mu, int32_t w, int32_t r_lo, int32_t r_hi, int32_t ell_mask,
                            int32_t* group, double* weight, int32_t* P_out);
lc_status lc_map_projected(int32_t n_rp, int32_t n_pi, double pi_max, int32_t* group, double* weight,
                           int32_t* P_out);
lc_status lc_map_rebin_blocks(int32_t n_blocks, int32_t n, int32_t w, int32_t* group, double* weight,
                              int32_t* P_out);

/*
 * lc_sample_covariance: the sample covariance over mocks of one estimate
 * (Sect. 2.2): C = sum_n (x_n - mean)(x_n - mean)^T / (N - 1), two-pass.
 *   x          DEVICE double [n_mock][P] (e.g. from lc_xi_split); n_mock >= 2.
 *   precision  LC_FP64, or LC_FP32_MFMA (float32 deviations, MFMA products
 *              accumulated in float32 over blocks of 256 mocks and summed in
 *              float64), optionally | LC_ACC32 (float32 over all mocks).
 *   C          DEVICE double [P][P], written (full symmetric).
 * Asynchronous; NaN entries propagate to their rows and columns.
 */
lc_status lc_sample_covariance(const double* x, int32_t n_mock, int32_t P, int32_t precision, double* C,
                               void* stream);

/* Summary of lc_covcov (Sect. 5.3, Table 3). */
typedef struct {
    double chi2_2_lc, chi2_2_smp;   /* <chi^2_2> of the LC and of the sample covariance */
    double cost_lc, cost_smp;       /* pair-count cost per realisation in units of the pairs of
                                       one data catalogue, N_d^2 / 2 (Sect. 2.3): LC counts DD
                                       once and two split estimates with ratio M_a, 1 + 6 M_a;
                                       the split sample covariance at ratio M, 1 + 3M */
    double ifom_lc, ifom_smp;       /* inverse figures of merit, cost x chi^2_2 */
    double gain;                    /* ifom_smp / ifom_lc */
} lc_covcov_report;

/*
 * lc_covcov: the error of the covariance estimates for Gaussian data vectors
 * (covariance of covariance, Sect. 3.2 and 3.3), from A and B of lc_covariance
 * standing in for their ensemble values:
 *   sample covariance at ratio M:  Var C_ij = (C_ii C_jj + C_ij^2)/(N-1), C = A + B/M;
 *   LC covariance at ratio M:      Var C_ij = (D_ii D_jj + D_ij^2
 *                                   + (1/(2M_a) - 1/M)^2 (B_ii B_jj + B_ij^2))/(N-1),
 *   with D = A + B/(2 M_a), the ensemble covariance at M = 2 M_a.  (The
 *   paper prints D = A + B/M_a; only A + B/(2 M_a) reproduces the formula's
 *   derivation from the two estimates.)
 *   A, B     DEVICE double [P][P].
 *   Cref     DEVICE double [P][P] normalising chi^2_2 (its diagonal), or NULL
 *            for C = A + B/M.
 *   n_mock   N for the standard deviations (>= 2 when sd_lc or sd_smp is given).
 *   sd_lc, sd_smp  DEVICE double [P][P] or NULL: element standard deviations.
 *   rep      HOST or NULL; non-NULL synchronises `stream`.  chi^2_2 averages
 *            the N = 2 variances over all P^2 elements, each divided by
 *            Cref_ii Cref_jj (Eq. chi2, Sect. 5.3).
 * M = INFINITY is allowed (the sample covariance's cost is then infinite).
 */
lc_status lc_covcov(const double* A, const double* B, int32_t P, int32_t m_a, double M, const double* Cref,
                    int32_t n_mock, double* sd_lc, double* sd_smp, lc_covcov_report* rep, void* stream);

/* Result of lc_autotune: the mesh options and launch tuning to use. */
typedef struct {
    int32_t cell_units;       /* for lc_mesh_opts.cell_units */
    int32_t sub;              /* for lc_mesh_opts.sub */
    lc_tuning tune;           /* for lc_pair_count_batch */
    double sample_ms;         /* time of one launch over the sampled tasks */
    int32_t n_tried;          /* configurations timed */
    int32_t sample_tasks;     /* tasks in the sample */
    int32_t cached;           /* 1: returned from the cache, nothing was timed */
    int32_t reserved;
} lc_autotune_result;

/*
 * lc_autotune: choose the mesh (cell side, sub-cell split) and the launch
 * shape (i points per gather) for a batch of tasks by timing them.
 * Pair counts do not depend on these choices (they are exact); only the time
 * does, through the number of candidate tests and the cost of gathering
 * neighbour cells.  Candidates: cell sides r_max / k (k = 1, 1.5, 2, 3, 4) and
 * the default, each with sub-cell splits 1, 2 and 4; then chunks of i points
 * for the best mesh.  The library default is timed first, and a candidate
 * replaces the incumbent only when it is more than 2% faster on the sample
 * (waves per block keep the default: a sample of the tasks predicts small
 * differences poorly for the whole batch).  Each is timed with HIP events over `sample_tasks` tasks
 * spread evenly over the list (one untimed launch, then two timed).  Last, the three
 * queue orders (lc_tuning.queue_order) are timed on the whole batch, one launch each, on the
 * chosen mesh (an order changes the launch's tail, which a sample does not show); skipped when
 * the sample is the whole batch.
 *   xyz, n_total, cat_offsets, n_cat, b   as for lc_build_cells.
 *   tasks     HOST [n_tasks], as for lc_pair_count_batch.
 *   sample_tasks  tasks to time (<= 0: 64).
 *   out       HOST, written.
 * Synchronises `stream` (blocking call).  The result is cached per device
 * and configuration (binning, catalogue sizes, task list, sample size) until
 * lc_release_caches; a cached call times nothing.
 */
lc_status lc_autotune(const int32_t* xyz, int64_t n_total, const int64_t* cat_offsets, int32_t n_cat,
                      const lc_binning* b, const lc_task* tasks, int32_t n_tasks, int32_t sample_tasks,
                      void* stream, lc_autotune_result* out);

/* Release cached device buffers, graphs, autotuning results and pinned
 * staging memory of the current device (they are otherwise kept until the
 * process ends). */
void lc_release_caches(void);

#ifdef __cplusplus
}
#endif
#endif /* LC_H */
