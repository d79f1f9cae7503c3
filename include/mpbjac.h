/*
 * mpbjac -- mixed-precision block-Jacobi preconditioned conjugate gradient
 * for one AMD Instinct MI355X (gfx950).
 *
 * C ABI of the library libmpbjac.so. Every entry point takes plain pointers
 * and sizes; "device" pointers are HIP device memory (the caller may obtain it
 * from any allocator), "host" pointers are ordinary host memory. No entry
 * point allocates device memory: the caller passes workspaces whose sizes the
 * *_query calls report. Work is enqueued on the caller's HIP stream (passed
 * as void*, NULL = the default stream); calls return after it is enqueued
 * unless stated otherwise. No C++ exception crosses this boundary.
 * Threads: one handle must not be used by two threads at once (a solve
 * caches its captured iteration graph and capture stream in the handle);
 * distinct handles, each with its own workspaces, may be used from distinct
 * threads at the same time. The library's only shared state is a cache of
 * per-(kernel, device) occupancy figures, filled under a lock.
 *
 * Method (arXiv 2407.15973, "Mixed Precision Block-Jacobi Preconditioner"):
 *   Sec. 3.1, eq. 3-1 with one outer step: M^-1 = D_b^-1, the inverse of the
 *     block-diagonal part of A on a partition into contiguous row blocks;
 *   Sec. 3.2, Algorithm 3.1 (fMP): each block inverse is formed in FP64 and
 *     stored in a lower precision; r is converted to FP32, multiplied in the
 *     low format with FP32 accumulation, the result widened to FP64;
 *   Algorithms 3.2 / 3.3 (aMP hl / lh): per application, the all-FP64 or the
 *     low map is chosen by comparing the recursive relative residual with
 *     adp_tol; the first application sees relres = +infinity;
 *   PCG (Sec. 3.2, Hestenes-Stiefel) runs entirely in FP64 with x0 = 0 and
 *     stops when ||r_j|| / ||r_0|| <= tol (Sec. 4.2).
 * Per-block precision maps beyond the paper: a condition/dominance rule and a
 * learned selector (16 block features -> MLP 16-64-64-3).
 */
#ifndef MPBJAC_H
#define MPBJAC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPBJAC_ABI_VERSION 4
#define BJAC_MAX_BLOCK 64        /* largest diagonal block (rows) */
#define BJAC_NFEAT 16            /* block features per block */
#define BJAC_MLP_NPARAM 5443     /* W1[64,16] b1[64] W2[64,64] b2[64] W3[3,64] b3[3] */
#define BJAC_MLP_NBLOB (BJAC_MLP_NPARAM + 2 * BJAC_NFEAT)  /* + feature mean, std */

/* ---- return codes ---------------------------------------------------- */
enum {
  BJAC_OK = 0,
  BJAC_NOT_CONVERGED = 1,   /* maxit reached; x holds the last iterate      */
  BJAC_EINVAL = -1,         /* bad argument (null pointer, size, partition) */
  BJAC_ENOTSPD = -2,        /* a diagonal block had a non-positive pivot    */
  BJAC_EBREAKDOWN = -3,     /* p^T A p <= 0, (r, z) <= 0, or non-finite     */
  BJAC_EHIP = -4,           /* a HIP runtime call failed                    */
  BJAC_ENOMEM = -5          /* workspace smaller than the query reported    */
};

/* ---- storage precisions of a block inverse ---------------------------- */
typedef enum { BJAC_FP64 = 0, BJAC_FP32 = 1, BJAC_BF16 = 2, BJAC_FP16 = 3 } bjac_prec;

/* ---- how the per-block precision map is chosen ------------------------ */
typedef enum {
  BJAC_UNIFORM = 0,   /* every block FP64 (uniform-BJAC of Sec. 4.2)          */
  BJAC_FIXED = 1,     /* every block in policy.low (fMP-BJAC, Algorithm 3.1)  */
  BJAC_RULE = 2,      /* lowest of FP16/FP32/FP64 with kappa_1(A_ii) u <= theta,
                         FP16 also needing row dominance >= d16               */
  BJAC_LEARNED = 3,   /* argmax of the selector MLP on the block features     */
  BJAC_EXPLICIT = 4   /* policy.explicit_tags                                 */
} bjac_mode;

/* ---- temporal switch between the all-FP64 map and the chosen map ------ */
typedef enum {
  BJAC_TEMPORAL_NONE = 0,
  BJAC_TEMPORAL_HL = 1,   /* Algorithm 3.2: FP64 while relres >= adp_tol */
  BJAC_TEMPORAL_LH = 2    /* Algorithm 3.3: low map while relres >= adp_tol */
} bjac_temporal;

/* ---- storage of the block inverses ------------------------------------
 * FULL: every stored block keeps all b^2 entries of its inverse (Sec. 3.2's
 * M^-1(p_l): the inverse rounded to the block's format).
 * BAND: a cheaper storage of the same inverses (not in the paper). Block k
 * keeps the diagonals |i - j| <= w_k of its inverse H, with the smallest w_k
 * such that sum_{|i-j| > w_k} H_ij^2 <= tau^2 sum_ij H_ij^2, where tau is
 * policy.band_rtol, or, when band_rtol <= 0, the unit roundoff of the block's
 * format (2^-53, 2^-24, 2^-8, 2^-11 for FP64, FP32, BF16, FP16): the dropped
 * part is then no larger than the rounding the format already makes. The kept
 * band is symmetric, taken from H's upper triangle, with the same scale and
 * rounding as FULL. The inverse of a diagonally dominant banded block decays
 * away from its diagonal, so w_k is usually far below b_k: the application
 * reads (w_k + 1) / bpad_k of FULL's bytes. Band handles serve every entry
 * point that takes a handle (bjac_apply, bjac_apply_multi, pcg_solve,
 * pcg_solve_batched); the multi-column products then run on the vector units
 * instead of the matrix cores.
 * SYM: the same inverses as FULL in fewer bytes (not in the paper). The
 * inverse H of an SPD block is symmetric, so of its 16 x 16 quarters H_IJ
 * only those with I <= J are stored, with FULL's scale and rounding, and the
 * application uses the transpose of H_JI for H_IJ below the diagonal. A block
 * of padded size 32, 48, 64 keeps 3/4, 2/3, 5/8 of FULL's bytes; blocks of 16
 * are stored as FULL. The computed FP64 inverse is symmetric up to its own
 * rounding (about one unit in the last place of FP64, far below every storage
 * format's rounding), so the application matches FULL's to within the
 * accumulation's rounding.
 * SYM handles serve bjac_apply, bjac_get_block (which returns the mirrored
 * block) and pcg_solve; bjac_apply_multi and pcg_solve_batched return
 * BJAC_EINVAL for them. */
typedef enum {
  BJAC_STORE_FULL = 0,
  BJAC_STORE_BAND = 1,
  BJAC_STORE_SYM = 2
} bjac_storage;

/* Square CSR matrix, all arrays device memory, caller-owned, read-only.
 * row_ptr[n+1] (row_ptr[0] = 0, non-decreasing), col_idx[nnz] in [0, n),
 * val[nnz] FP64. Columns need not be sorted. A must be symmetric positive
 * definite for PCG; the setup only needs SPD diagonal blocks. */
typedef struct {
  int64_t n;
  int64_t nnz;
  const int32_t *row_ptr;
  const int32_t *col_idx;
  const double *val;
} bjac_csr;

typedef struct {
  int32_t mode;                  /* bjac_mode                                  */
  int32_t low;                   /* bjac_prec used by BJAC_FIXED               */
  int32_t temporal;              /* bjac_temporal                              */
  int32_t storage;               /* bjac_storage                               */
  double adp_tol;                /* threshold of the temporal switch           */
  double theta;                  /* RULE: kappa_1 * u <= theta (default 1e-2)  */
  double d16;                    /* RULE: min row dominance for FP16 (1.0)     */
  const float *mlp_blob;         /* LEARNED: device, BJAC_MLP_NBLOB floats     */
  const uint8_t *explicit_tags;  /* EXPLICIT: host, nb entries of bjac_prec    */
  double band_rtol;              /* BAND: tolerance tau of the dropped part
                                    (<= 0: each block's unit roundoff)         */
} bjac_policy;

typedef struct bjac_handle bjac_handle;

typedef struct {
  int64_t n;
  int32_t nb;
  int32_t max_block;
  int32_t blocks_per_prec[4];    /* low map histogram, indexed by bjac_prec    */
  int64_t low_bytes;             /* bytes of the stored low map                */
  int64_t high_bytes;            /* bytes of the all-FP64 map (temporal only)  */
  int32_t temporal;
  int32_t mode;
  int32_t ntiles;                /* apply wave tiles (whole blocks, <= 64 padded rows) */
  int32_t reserved;
} bjac_info;

typedef struct {
  double tol;                    /* stop when ||r|| / ||b|| <= tol             */
  int32_t maxit;
  int32_t chunk;                 /* iterations per captured graph launch (0 = 16) */
  double *relres_hist;           /* optional device buffer [maxit]: relres after
                                    each x update                              */
  uint8_t *high_hist;            /* optional device buffer [maxit + 1]: 1 where
                                    the application used the FP64 map          */
  int32_t profile;               /* 1: launch without graphs, time every kernel
                                    with HIP events on the stream (stats.*_ms) */
  int32_t verify;                /* > 0: when the recursive relres reaches tol,
                                    recompute ||b - A x|| / ||b|| in FP64; if it
                                    exceeds tol, replace r by b - A x and
                                    restart CG (p = z), at most `verify` times
                                    (then BJAC_NOT_CONVERGED). Graph mode only. */
  int32_t variant;               /* bjac_pcg_variant                           */
  int32_t cache_hints;           /* bjac_cache_hints (0 = AUTO)                */
} bjac_solve_opts;

/* PCG recurrences (both produce the same iterates in exact arithmetic):
 * TEXTBOOK: Hestenes-Stiefel as the paper uses it (Sec. 3.2): per iteration
 *   q = A p with (p, q), then x, r updated, z = M^-1 r with (r, r), (r, z):
 *   two reduction phases.
 * SINGLE_REDUCTION: the Chronopoulos-Gear recurrence (not in the paper):
 *   x, r, p and s = A p updated from the last dots, u = M^-1 r, then w = A u
 *   with (r, r), (r, u), (w, u) taken together: one reduction phase, and the
 *   product gathers only u at the neighbouring rows. The convergence test
 *   and the iteration count are the textbook ones. Serves stored-inverse
 *   handles without the adaptive switch (temporal or paper-mode handles:
 *   BJAC_EINVAL). */
typedef enum {
  BJAC_PCG_TEXTBOOK = 0,
  BJAC_PCG_SINGLE_REDUCTION = 1
} bjac_pcg_variant;

/* Cache hints of the launches of a PCG iteration: the product and the update
 * + application, in both recurrences and with the adaptive switch (they never
 * change a result, only which kernel variant runs):
 * PLAIN: ordinary loads and stores. STREAM: non-temporal loads and stores of
 * everything one launch touches once (the matrix is always read
 * non-temporally), for solves whose iteration moves far more bytes than the
 * last-level cache holds. AUTO: STREAM when one iteration reads more than
 * twice the 256 MiB last-level cache of the MI355X (matrix at 9 bytes per
 * entry, row pointers, the stored low map, 88 bytes per row of vectors),
 * else PLAIN. Other values: BJAC_EINVAL. Band-stored and paper-mode
 * applications use plain accesses throughout. */
typedef enum {
  BJAC_HINTS_AUTO = 0,
  BJAC_HINTS_PLAIN = 1,
  BJAC_HINTS_STREAM = 2
} bjac_cache_hints;

typedef struct {
  int32_t iters;                 /* x updates performed                        */
  int32_t status;                /* BJAC_OK, BJAC_NOT_CONVERGED, BJAC_EBREAKDOWN */
  double relres;                 /* recursive ||r|| / ||b|| at exit            */
  double rnorm0;                 /* ||b||                                      */
  int32_t high_applications;     /* applications that used the FP64 map       */
  int32_t graph_launches;
  double solve_ms;               /* wall time of the solve on the stream       */
  /* profile mode only: summed kernel durations over the iterations that ran.
     apply_ms covers the application (with the x / r update when fused);
     update_ms the separate update launch of adaptive and paper-mode handles */
  double spmv_ms, apply_ms, update_ms;
  int32_t n_spmv, n_apply, n_update;
  int32_t restarts;              /* verify: residual replacements performed    */
  double true_relres;            /* verify: last FP64 ||b - A x|| / ||b||, else -1 */
} bjac_stats;

/* ---- library ------------------------------------------------------------ */
int bjac_abi_version(void);
const char *bjac_strerror(int code);

/* ---- block-Jacobi setup (Sec. 3.1 D_b, Algorithm 3.1 storage) -----------
 * block_ptr: HOST array of nb+1 row offsets, block_ptr[0] = 0,
 * block_ptr[nb] = n, 1 <= block size <= BJAC_MAX_BLOCK.
 * bjac_setup_query reports the workspace the setup needs (an upper bound
 * valid for any precision map the policy can produce).
 * bjac_setup extracts every diagonal block from the CSR rows, inverts it in
 * FP64 (Gauss-Jordan without pivoting, valid for SPD blocks), computes the 16
 * block features, selects the block precisions, scales and rounds (correctly
 * rounded from FP64, ties to even) and stores them in *workspace, which must
 * stay alive and untouched until bjac_destroy. It synchronises the stream
 * once when the policy's map depends on the data (RULE, LEARNED) and once at
 * its end. A is only read during the call. On error no handle is returned. */
int bjac_setup_query(const bjac_csr *A, const int32_t *block_ptr, int32_t nb,
                     const bjac_policy *policy, size_t *workspace_bytes);
int bjac_setup(const bjac_csr *A, const int32_t *block_ptr, int32_t nb,
               const bjac_policy *policy, void *workspace, size_t workspace_bytes,
               void *stream, bjac_handle **out);
void bjac_destroy(bjac_handle *h);
int bjac_get_info(const bjac_handle *h, bjac_info *info);
/* Copies to HOST memory: tags[nb] (bjac_prec of the low map),
 * features[nb * 16] (FP32, row-major), synchronising the handle's stream. */
int bjac_get_tags(const bjac_handle *h, uint8_t *tags);
int bjac_get_features(const bjac_handle *h, float *features);
/* Copies one stored block to HOST memory as FP64 values of the stored
 * numbers (b x b, row-major) and its scale s (the block represents s * out).
 * which = 0: low map, 1: all-FP64 map (temporal handles only). */
int bjac_get_block(const bjac_handle *h, int32_t which, int32_t block, double *out, double *scale);
/* BAND handles: copies the half-bandwidth w_k of every block of map `which`
 * (0 low, 1 all-FP64 map of temporal handles) to HOST memory w[nb]. FULL and
 * paper-mode handles: BJAC_EINVAL. */
int bjac_get_band(const bjac_handle *h, int32_t which, uint8_t *w);

/* ---- paper-mode BJAC(k, t) (Sec. 3.1 eq. 3-1 to 3-3; Sec. 3.2) ----------
 * The preconditioner as the paper defines it for large blocks (one per
 * process there): k outer steps z_1 = Dhat^-1 r, z_{j+1} = z_j + Dhat^-1
 * (r - A z_j), where Dhat^-1 applies t point-Jacobi sweeps y <- y + D^-1 (v -
 * D_b y) from y = 0 inside every diagonal block (D_b: the entries of A whose
 * row and column lie in the same block; D: its diagonal). Nothing is
 * inverted; blocks are contiguous row ranges of any size (block_ptr as for
 * bjac_setup, no size limit). low != 0: every operation of the application
 * in FP32 (FP32 copy of A's values and of 1/a_ii, r rounded to FP32 on entry,
 * z widened on exit; Algorithm 3.1's fMP); low = 0: FP64. temporal/adp_tol:
 * Algorithms 3.2 / 3.3 between the FP64 and FP32 applications.
 * The handle keeps A's device pointers: A must stay alive and unchanged while
 * the handle is used (bjac_apply, pcg_solve with the same A). bjac_apply's
 * `which` selects the low (0) or FP64 (1) application. bjac_get_features and
 * bjac_get_block return BJAC_EINVAL for these handles. A non-positive
 * diagonal entry gives BJAC_ENOTSPD. */
typedef struct {
  int32_t k;             /* outer steps (1..64)                            */
  int32_t t;             /* Jacobi sweeps per block solve (1..64)          */
  int32_t low;           /* 1: FP32 application, 0: FP64                   */
  int32_t temporal;      /* bjac_temporal                                  */
  double adp_tol;        /* threshold of the temporal switch               */
} bjac_poly_params;

int bjac_poly_setup_query(const bjac_csr *A, const int32_t *block_ptr, int32_t nb,
                          const bjac_poly_params *params, size_t *workspace_bytes);
int bjac_poly_setup(const bjac_csr *A, const int32_t *block_ptr, int32_t nb,
                    const bjac_poly_params *params, void *workspace, size_t workspace_bytes,
                    void *stream, bjac_handle **out);

/* ---- z = M^-1 r (eq. 3-1, k = 1; Algorithm 3.1) --------------------------
 * r, z: device FP64 vectors of length n (distinct). which = 0 applies the
 * low map, 1 the all-FP64 map (temporal handles; for others both are the
 * low map). Reduced blocks use the FP32 copy of r and FP32 accumulation. */
int bjac_apply(const bjac_handle *h, int32_t which, const double *r, double *z, void *stream);

/* ---- Z = M^-1 R for up to 8 columns (Algorithm 3.1 on a block of columns)
 * R, Z: device FP64, row-major [n][m] (the m values of one row contiguous),
 * distinct, 1 <= m <= 8. Applies the low map only. Each block product runs on
 * the 16x16x4 matrix-core instructions: FP32 for FP32/BF16/FP16 blocks (the
 * FP32 copy of R, FP32 accumulation, then times the block scale in FP64),
 * FP64 for FP64 blocks. Returns BJAC_EINVAL for a handle with symmetric
 * storage (BJAC_STORE_SYM). */
int bjac_apply_multi(const bjac_handle *h, const double *R, double *Z, int32_t m, void *stream);

/* ---- q = A p, the FP64 CSR product used by PCG ------------------------- */
int bjac_spmv(const bjac_csr *A, const double *p, double *q, void *stream);

/* ---- correctly rounded conversion (the storage step of Algorithm 3.1) ---
 * out[i] = RNE_prec(in[i] / scale), with scale a power of two; out is FP32,
 * BF16 or FP16 bits (2 or 4 bytes per element), device memory. */
int bjac_round(const double *in, void *out, int64_t count, int32_t prec, double scale, void *stream);

/* ---- PCG (Sec. 3.2; Sec. 4.2 stopping test, x0 = 0) ---------------------
 * pcg_workspace_query: bytes of the solver workspace for n rows.
 * pcg_workspace_query_csr: the same plus room for a compact copy of A
 * (2 bytes per non-zero, 32 bytes and two 256-entry dictionaries more).
 * Given a workspace that large, pcg_solve encodes A at the start of the
 * call and its matrix-vector products read the compact copy: with at most
 * 256 distinct offsets col - row, a 1-byte code per column, and then with at
 * most 256 distinct values (bitwise) a 1-byte code per value as well (CSR-VI
 * value indexing); else the 2-byte offsets col - row when every entry lies
 * within 32767 rows of its row; else the 4-byte indices and 8-byte values.
 * The iterates are the same either way.
 * pcg_solve: solves A x = b; b, x device FP64 [n] (x is overwritten). The
 * iterations run as captured HIP graphs of opts->chunk iterations with all
 * scalars on the device; the host reads one status word per graph launch.
 * Returns BJAC_OK, BJAC_NOT_CONVERGED, BJAC_EBREAKDOWN or an error; stats may
 * be NULL. The call synchronises the stream before it returns. */
int pcg_workspace_query(int64_t n, size_t *workspace_bytes);
int pcg_workspace_query_csr(const bjac_csr *A, size_t *workspace_bytes);
int pcg_solve(const bjac_csr *A, const bjac_handle *M, const double *b, double *x,
              const bjac_solve_opts *opts, void *workspace, size_t workspace_bytes,
              bjac_stats *stats, void *stream);

/* ---- streaming probe (a measurement aid, not a step of the method) ------
 * The HBM rate a plain streaming kernel reaches for a mix of n_in read and
 * n_out write streams (0..8, 0..2, at least one), the practical ceiling the
 * hot kernels' roofline fractions are read against: the SpMV reads about six
 * bytes for each one it writes, the fused update + application about four.
 * in[n_in], out[n_out]: HOST arrays of device pointers to `count` doubles
 * each (16-byte aligned, count even); out[j][i] = sum_k in[k][i] + j, with
 * non-temporal loads and stores, `unroll` (1, 2 or 4) 16-byte accesses per
 * lane and stream in flight, grid-stride over `grid` workgroups of 256
 * (0 = 8192). The read-only mix (n_out = 0) writes one double per thread to
 * sink (device, grid * 256 doubles). */
int bjac_stream_probe(const double *const *in, int32_t n_in, double *const *out, int32_t n_out,
                      int64_t count, int32_t grid, int32_t unroll, double *sink, void *stream);

/* ---- PCG without allocation --------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): pcg_solve
 * with the solver workspace in a static device array of the library
 * (5 n + 8192 doubles and the device state, for n up to 1,048,576 rows:
 * about 40 MiB per GPU, held until the process ends). Arguments as
 * pcg_solve without the workspace; A, M, b and x remain the caller's. The
 * call allocates nothing: no hipMalloc or hipFree, no graph and no event;
 * each chunk of opts->chunk iterations is launched directly (the same
 * kernels in the same order as pcg_solve, so the same iterates) and
 * stats->solve_ms is host time. The products read the 4-byte column indices.
 * Returns BJAC_ENOMEM for n > 1,048,576 and BJAC_EINVAL for opts->profile.
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind (each call re-initialises what it reads): calls that overlap on one
 * GPU, from several threads or streams, race and must not be made. */
int pcg_solve_noalloc(const bjac_csr *A, const bjac_handle *M, const double *b, double *x,
                      const bjac_solve_opts *opts, bjac_stats *stats, void *stream);

/* ---- batched multi-RHS PCG (Sec. 3.2 per system and column) -------------
 * nsys independent SPD systems stacked as one block-diagonal CSR A (system s
 * owns rows sys_row[s] .. sys_row[s+1]-1 and only couples inside them) with
 * sys_m[s] in 1..8 right-hand sides each. M is a handle set up on the same
 * stacked A whose block partition has every sys_row[s] as a block boundary;
 * only its low map is used (no temporal switch). Every (system, column) pair
 * runs its own CG with x0 = 0 and its own scalars and stops on its own
 * ||r|| / ||r_0|| <= tol (Sec. 4.2); the z = M^-1 R products of a block with
 * up to 8 columns run on the 16x16x4 matrix-core instructions (FP32 for
 * FP32/BF16/FP16 blocks with the FP32 copy of R, FP64 for FP64 blocks).
 * sys_row[nsys+1], sys_m[nsys]: HOST arrays. b, x: device FP64, system s's
 * block at offset sum_{t<s} rows_t * m_t, row-major [rows_s][m_s] (the m_s
 * values of one row are contiguous). col_iters, col_status, col_relres: HOST
 * arrays of sum_s m_s entries (may be NULL), column order = system order,
 * then column. opts: tol, maxit, chunk (iterations per captured graph) are
 * used, and profile (eager launches, kernel times in stats->spmv_ms,
 * apply_ms and update_ms = the per-system reductions); relres_hist and
 * high_hist are ignored; variant must be BJAC_PCG_TEXTBOOK; cache_hints is
 * ignored (the batched kernels always store non-temporally what only the
 * next launch reads). */
/* Launch shape. The matrix-vector product cuts every system into chunks of
 * floor(64 / m) rows (at most 64 (row, column) elements, one wave pass); the
 * chunks are split into 8 runs of about equal cost, one per XCD, whose waves
 * take them in increasing order from a counter of that run. The update +
 * apply cuts every system into chunks of whole blocks (at most apply_rows
 * padded rows) and deals them round-robin over all waves of its grid. */
typedef struct {
  int32_t spmv_grab;       /* matrix-vector chunks a wave takes per counter
                              grab (1..64; 0 = 4)                             */
  int32_t wg_per_cu;       /* workgroups of 256 threads per compute unit in
                              the update + apply launch (1..32; 0 = 32); at
                              most 8192 workgroups                            */
  int32_t spmv_wg_per_cu;  /* the same for the matrix-vector launch, at most
                              what is resident at once (1..32; 0 = 32)        */
  int32_t apply_rows;      /* padded rows per apply chunk (>= 64; 0 = 256).
                              Chunks never cross systems.                     */
} bjac_batch_cfg;

int pcg_batched_workspace_query(const bjac_csr *A, const bjac_handle *M, int32_t nsys,
                                const int32_t *sys_row, const int32_t *sys_m,
                                const bjac_batch_cfg *cfg, size_t *workspace_bytes);
/* Returns BJAC_OK when every column converged, else BJAC_EBREAKDOWN if any
 * column broke down, else BJAC_NOT_CONVERGED. stats: iters = the largest
 * column count, relres = the largest column relres. Synchronises the stream.
 * Both calls return BJAC_EINVAL for a handle with symmetric storage
 * (BJAC_STORE_SYM). */
int pcg_solve_batched(const bjac_csr *A, const bjac_handle *M, int32_t nsys, const int32_t *sys_row,
                      const int32_t *sys_m, const double *b, double *x, const bjac_solve_opts *opts,
                      const bjac_batch_cfg *cfg, void *workspace, size_t workspace_bytes,
                      int32_t *col_iters, int32_t *col_status, double *col_relres,
                      bjac_stats *stats, void *stream);
/* Autotuner: times `iters` PCG iterations of the batch (x is overwritten)
 * under each of the ncand configurations and returns the fastest in *best;
 * ms_per_iter (HOST, ncand entries, may be NULL) receives every timing. The
 * workspace must hold the largest query over the candidates. Synchronises
 * the stream. */
int pcg_batched_tune(const bjac_csr *A, const bjac_handle *M, int32_t nsys, const int32_t *sys_row,
                     const int32_t *sys_m, const double *b, double *x, const bjac_batch_cfg *cands,
                     int32_t ncand, int32_t iters, void *workspace, size_t workspace_bytes,
                     float *ms_per_iter, int32_t *best, void *stream);

/* ---- learned per-block precision selector -------------------------------
 * Network: standardised 16 block features -> 64 ReLU -> 64 ReLU -> 3 logits
 * (class 0 = FP64, 1 = FP32, 2 = FP16), FP32 throughout. blob: device
 * BJAC_MLP_NBLOB floats = the 5443 parameters (layout in BJAC_MLP_NPARAM's
 * comment, row-major out x in) followed by the feature mean[16] and std[16].
 * feat: device [n * 16] FP32. Block features correlate with the mixed-
 * precision convergence delay (Sec. 4.5: multiscale strength, eq. 4-5, and
 * diagonal dominance); the network learns that relation from labels
 * produced by the solver's own runs. */
/* logits: device [n * 3] (may be NULL); tags: device [n] bjac_prec of the
 * argmax class, ties to the higher precision (may be NULL). */
int bjac_mlp_forward(const float *blob, const float *feat, int32_t n, float *logits, uint8_t *tags, void *stream);
int bjac_mlp_workspace_query(int32_t n, size_t *workspace_bytes);
/* grad: device [BJAC_MLP_NPARAM], overwritten with the gradient of the mean
 * softmax cross-entropy over the n samples (labels: device int32 classes);
 * loss: device scalar or NULL. Deterministic for a given n. */
int bjac_mlp_backward(const float *blob, const float *feat, const int32_t *labels, int32_t n, float *grad,
                      float *loss, void *workspace, size_t workspace_bytes, void *stream);
/* One Adam step on the parameter part of blob (m, v: device moment buffers
 * [BJAC_MLP_NPARAM]; t >= 1 the step number for bias correction). */
int bjac_mlp_adam(float *blob, const float *grad, float *m, float *v, int32_t t, float lr, float beta1,
                  float beta2, float eps, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* MPBJAC_H */
