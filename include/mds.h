/*
 * mds.h - C ABI of libmds, interpolation MDS on one AMD MI355X (gfx950).
 *
 * The method is interpolation MDS from Delicado and Pachon-Garcia,
 * "Multidimensional scaling for big data", Section 3.1:
 *   fit   - classical MDS (Section 2) on l landmark rows drawn at random:
 *           Delta1 = squared distances, Q1 = -1/2 P Delta1 P, the r largest
 *           eigenpairs (V, Lambda), X1 = V Lambda^{1/2};
 *   embed - Gower's interpolation formula, eq. (2), for any set of rows:
 *           y = 1/2 Lambda^{-1/2} V' (q1 - d), d_j = |x - m_j|^2, which is
 *           eq. (2) after the cancellation (1/l) X1 S1^{-1} = V Lambda^{-1/2}
 *           shown in Section 3.1.
 * Dissimilarities are squared Euclidean distances between data rows
 * (Section 4.1 uses Euclidean distances between rows).
 *
 * Conventions common to every entry point:
 *   - Pointers named X / Y are DEVICE pointers; every other array argument
 *     is a HOST pointer.  Matrices are row-major with the given leading
 *     dimension (elements, not bytes).
 *   - The caller owns X, Y and streams; the library owns the model and
 *     server memory it allocates (hipMalloc) and frees it in mds_free /
 *     mds_serve_destroy.
 *   - "stream" is a hipStream_t passed as void*; NULL means the default
 *     stream.
 *   - Every call returns an mds_status; no C++ exception crosses the ABI.
 *     mds_last_error() returns a thread-local message for the last failure
 *     on the calling thread.  Errors of asynchronous kernels surface at the
 *     caller's next synchronisation or at the next library call.
 */
#ifndef MDS_H
#define MDS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mds_status;
enum {
  MDS_OK = 0,
  MDS_ERR_INVALID_ARG = 1,   /* null pointer, bad size, bad index, non-finite landmark */
  MDS_ERR_OOM = 2,           /* device or host allocation failed */
  MDS_ERR_BUDGET = 3,        /* serving: would exceed the server's byte budget */
  MDS_ERR_DEGENERATE = 4,    /* lambda_1 <= 0: all landmarks coincide */
  MDS_ERR_HIP = 5,           /* HIP runtime/launch error (see mds_last_hip_error) */
  MDS_ERR_NOT_CONVERGED = 6, /* eigensolver hit its iteration limit */
  MDS_ERR_NOT_FOUND = 7,     /* serving: unknown model id or ticket */
  MDS_ERR_STATE = 8          /* serving: call not valid in the current state */
};

/* element type of X */
enum { MDS_F32 = 0, MDS_F64 = 1 };

/* arithmetic of the distance block and projection in mds_embed */
enum {
  MDS_PREC_FP64 = 0,        /* FP64 MFMA; Y is double */
  MDS_PREC_FP32 = 1,        /* FP32 MFMA; Y is float */
  MDS_PREC_SPLIT_BF16 = 2,  /* x.m from hi/lo BF16 operands, FP32 accumulate;
                               epilogue and projection FP32; Y is float */
  MDS_PREC_SPLIT_FP16 = 3   /* as above with FP16 hi/lo operands, scaled by
                               a power of two fixed at fit time */
};

/* Rank handling: eigen-direction k is live when lambda_k > MDS_TAU *
 * lambda_1 (Section 2 keeps only the r greatest non-negative eigenvalues).
 * Dead directions get exactly zero W, X1 and output coordinates. */
#define MDS_TAU 1e-9
#define MDS_MAX_R 64

typedef struct mds_model mds_model;

/* ---- landmark sampling (host only, no GPU needed) ---------------------
 * Section 3.1 draws the landmark subset at random.  The draw is defined as:
 * SplitMix64 (Steele-Lea-Flood 2014) seeded with `seed`, Lemire's bounded
 * integer method, and a partial Fisher-Yates shuffle over 0..n-1 whose first
 * l slots are the landmarks; idx_out (host, l entries, caller-owned) gets
 * them in ascending order.
 * Errors: INVALID_ARG if idx_out is NULL or not 1 <= l <= n. */
mds_status mds_sample_landmarks(int64_t n, int64_t l, uint64_t seed, int64_t* idx_out);

/* ---- fit: classical MDS on the landmarks (Section 2, Section 3.1) ------
 * X:     device, n x p rows, leading dimension ldx >= p, element type dt
 *        (MDS_F32 or MDS_F64).  Only the l landmark rows are read.
 * l, r:  landmark count (2 <= l <= n) and output dimension
 *        (1 <= r <= min(l - 1, MDS_MAX_R)).
 * seed / idx_or_null: landmarks come from mds_sample_landmarks(n, l, seed)
 *        unless idx_or_null (host, l distinct indices in [0, n)) is given;
 *        those are used as given, sorted ascending.
 * The fit always computes in FP64: gather, Delta1 by direct differences,
 * double centring, top-r eigenpairs by Lanczos with full
 * reorthogonalisation, eigenvector sign convention (largest-|.| component
 * positive, smallest index on ties), then X1, W = 1/2 V Lambda^{-1/2},
 * c = q1 - |m|^2 and the FP32 / BF16 / FP16 copies used by mds_embed.
 * It runs on `stream` and returns when the model is complete (it must read
 * Lambda to decide which directions are live).
 * *out is written only on success; release it with mds_free.
 * Errors: INVALID_ARG (sizes, pointers, duplicate / out-of-range idx,
 * non-finite landmark values), DEGENERATE, NOT_CONVERGED, OOM, HIP. */
mds_status mds_fit_landmarks(const void* X, int32_t dt, int64_t n, int64_t p,
                             int64_t ldx, int64_t l, int32_t r, uint64_t seed,
                             const int64_t* idx_or_null, void* stream,
                             mds_model** out);

/* ---- embed: Gower's interpolation, eq. (2), for n_new rows -------------
 * X:   device, n_new x p rows (p of the model), leading dimension ldx >= p.
 *      dt must be MDS_F32 for FP32 / split precisions; MDS_PREC_FP64 takes
 *      MDS_F32 or MDS_F64.
 * Y:   device, n_new x r, leading dimension ldy >= r; double for
 *      MDS_PREC_FP64, float otherwise.  Row i of Y is the embedding of row
 *      i of X (landmark rows are interpolated like any other row).
 * Asynchronous on `stream`.  The model is read-only, so concurrent calls on
 * different streams are safe.  The result of a row does not depend on the
 * other rows passed with it (fixed per-row reduction order).
 * n_new == 0 is a no-op returning MDS_OK.
 * Errors: INVALID_ARG (null model/pointers, ldx < p, ldy < r, dt/prec
 * mismatch), HIP. */
mds_status mds_embed(const mds_model* m, const void* X, int32_t dt, int64_t n_new,
                     int64_t ldx, int32_t prec, void* Y, int64_t ldy, void* stream);

/* ---- dissimilarity input (Section 2 starts from a matrix of squared
 * dissimilarities; they need not be squared Euclidean distances) ----------
 * D1:  device, l x l FP64, row-major with ldd >= l: squared dissimilarities
 *      among the l landmark points.  Symmetric (|d_ij - d_ji| <= 1e-12
 *      (|d_ij| + |d_ji|)) and finite, else INVALID_ARG; it is symmetrised
 *      exactly before use.  Negative eigenvalues of Q1 are allowed: only the
 *      r largest are kept and non-positive ones are dead directions.
 * The fit runs from the double centring on, exactly as in
 * mds_fit_landmarks.  The model holds no landmark vectors: mds_embed on it
 * returns INVALID_ARG; use mds_embed_from_sqdist.  It reports n_fit = l
 * and p = 0, and its landmarks are 0..l-1.  Synchronous; errors as mds_fit_landmarks. */
mds_status mds_fit_from_sqdist(const double* D1, int64_t l, int64_t ldd, int32_t r, void* stream,
                               mds_model** out);

/* Eq. (2) for n_new points given their squared dissimilarities to the l
 * landmarks:  y = 1/2 Lambda^{-1/2} V' (q1 - a).
 * A2:  device, n_new x l, leading dimension lda >= l, element type dt.
 * prec MDS_PREC_FP64 (Y double; A2 F32 or F64) or MDS_PREC_FP32 (Y float;
 *      A2 F32).  Works with models from either fit (for a model fitted on
 *      vectors, a = squared distances to the landmarks gives mds_embed's
 *      result).  Asynchronous on `stream`; a memory-bound streaming kernel.
 * Errors: INVALID_ARG (null pointers, lda < l, ldy < r, dt/prec mismatch),
 * HIP. */
mds_status mds_embed_from_sqdist(const mds_model* m, const void* A2, int32_t dt, int64_t n_new,
                                 int64_t lda, int32_t prec, void* Y, int64_t ldy, void* stream);

/* ---- MaxMin landmark selection (the landmark choice of LMDS, Section 3.1)
 * From row `first`, repeatedly add the row whose smallest squared
 * Euclidean distance to the rows chosen so far is largest (smallest row
 * index on ties).  Each squared distance is summed in FP64 over the columns
 * in order, one rounded product and one rounded sum per column, so the
 * choices do not depend on the launch shape.  One pass over X per landmark.
 * X: device, n x p rows, leading dimension ldx >= p, element type dt.
 * idx_out: host, l int64 (caller-owned), in selection order.  The result
 * can be passed to mds_fit_landmarks (LMDS = this choice of landmarks plus
 * Gower's formula, by Proposition 1) or mds_pivot_mds.  Synchronous.
 * Errors: INVALID_ARG (pointers, sizes, first outside [0, n)), DEGENERATE
 * (fewer than l distinct rows), OOM, HIP. */
mds_status mds_maxmin_landmarks(const void* X, int32_t dt, int64_t n, int64_t p, int64_t ldx,
                                int64_t l, int64_t first, int64_t* idx_out, void* stream);

/* ---- MaxMin without allocation ---------------------------------------------
 * For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * selection as mds_maxmin_landmarks, with the same arguments and the same
 * result, computed with the row-major steps only, on a static device array
 * of MDS_NOALLOC_SCRATCH_BYTES bytes that the library holds on each GPU it
 * runs on until the process ends (its address is looked up once per
 * device, on the first call there).  Calls no allocating routine.  Every
 * call on a GPU shares that GPU's array, which keeps the last call's
 * contents: calls that overlap on one GPU (other streams or threads) race,
 * and the caller must serialise them.  Synchronous, like
 * mds_maxmin_landmarks.
 * Errors: as mds_maxmin_landmarks, plus INVALID_ARG when
 * n > MDS_NOALLOC_MAX_N or l > MDS_NOALLOC_MAX_L (no work is done). */
#define MDS_NOALLOC_MAX_N 1048576
#define MDS_NOALLOC_MAX_L 16384
#define MDS_NOALLOC_SCRATCH_BYTES 8585472
mds_status mds_maxmin_landmarks_noalloc(const void* X, int32_t dt, int64_t n, int64_t p, int64_t ldx,
                                        int64_t l, int64_t first, int64_t* idx_out, void* stream);

/* ---- pivot MDS (Section 3.1) ---------------------------------------------
 * With l pivot rows, C is the double-centred n x l block of squared
 * distances between all rows and the pivots, and its singular value
 * decomposition C = U Sigma W' stands in for the eigendecomposition of Q:
 * lambda_k = sigma_k sqrt(n / l) estimates Q's eigenvalues (exact when the
 * pivots are all the rows) and Y = U_r Lambda_r^{1/2}.  The sign of column
 * k follows W's column k (largest-|.| entry positive, first pivot on ties);
 * direction k is live when sigma_k^2 > MDS_TAU * sigma_1^2: the rule of
 * Section 2 (keep eigenvalues above MDS_TAU times the largest) applied to
 * the matrix pivot MDS decomposes, C'C, whose eigenvalues are sigma^2 (so
 * lambda_k > sqrt(MDS_TAU) lambda_1); dead columns are zero and report
 * lambda = 0.  Dissimilarities
 * are squared Euclidean distances, for which C = Xc Mc' (rows and pivots
 * centred on their means); the work is computed through that identity in
 * FP64 (means, p x p cross-product, l x l eigenproblem, one streaming pass).
 * Pivots: idx_or_null (host, l distinct rows, e.g. from
 * mds_maxmin_landmarks), else mds_sample_landmarks(n, l, seed).  The scale
 * estimate assumes pivots representative of the data, as random ones are.
 * X as for mds_maxmin_landmarks; 2 <= l <= min(n, MDS_DC_MAX_L),
 * 1 <= r <= min(l - 1, MDS_MAX_R), p <= 4096.  Y: device, n x r doubles,
 * ldy >= r.  lam: host, r doubles (may be NULL); r_eff: host (may be NULL).
 * Synchronous.  Errors: INVALID_ARG (pointers, sizes, bad pivots, non-finite
 * X), DEGENERATE (lambda_1 <= 0), OOM, HIP. */
mds_status mds_pivot_mds(const void* X, int32_t dt, int64_t n, int64_t p, int64_t ldx, int64_t l,
                         int32_t r, uint64_t seed, const int64_t* idx_or_null, double* Y,
                         int64_t ldy, double* lam, int32_t* r_eff, void* stream);

/* ---- affine form of eq. (2) for squared Euclidean distances ------------
 * Eq. (2) reads y = W'(c - |x|^2 1 + 2 M x) with W = 1/2 V Lambda^{-1/2}
 * and c = q1 - |m|^2; the columns of V sum to zero (Q1 1 = 0, Section 2),
 * so y = A x + b with A = 2 W' M and b = W' c, formed in FP64 at fit time.
 * This is the same map as mds_embed in exact arithmetic (the landmark
 * principal-component projection, since classical MDS of Euclidean
 * vectors is their PCA), at 2 p r flops per row instead of 2 l (p + r).
 * It is a separate mode: it does not evaluate the distances of eq. (2).
 * Arguments as mds_embed; prec is MDS_PREC_FP64 (Y double, X F32 or F64)
 * or MDS_PREC_FP32 (Y float, X F32).  Asynchronous on `stream`; a
 * memory-bound streaming kernel.  n_new == 0 is a no-op.
 * Errors: INVALID_ARG (null pointers, model fitted on dissimilarities,
 * ldx < p, ldy < r, dt/prec mismatch), HIP. */
mds_status mds_embed_affine(const mds_model* m, const void* X, int32_t dt, int64_t n_new,
                            int64_t ldx, int32_t prec, void* Y, int64_t ldy, void* stream);

/* ---- divide-and-conquer MDS (Section 3.2) ------------------------------
 * The rows are split at random into parts that share c connecting points;
 * classical MDS (Section 2) runs on every part and each part's
 * configuration is mapped onto the first one by the Procrustes rotation and
 * shift fitted on the connecting rows.
 * Partition: row i gets the key SplitMix64(seed) output number i+1 (the
 * finaliser of seed + (i+1) * 0x9E3779B97F4A7C15); rows are ordered by
 * (key, index).  The first c rows of that order are the connecting points,
 * the rest are cut in order into pieces of l - c; part j is the connecting
 * rows followed by piece j, so there are ceil(1 + (n - l) / (l - c)) parts
 * (one part holding every row when n <= l), all of l rows but perhaps the
 * last.  Dissimilarities are squared Euclidean distances between rows.
 * X:      device, n x p rows, leading dimension ldx >= p, element type dt.
 * l, c, r: part size, connecting points, output dimension:
 *         1 <= r <= MDS_MAX_R, c >= r + 1, c < l <= MDS_DC_MAX_L, c < n.
 * Y:      device, n x r doubles, leading dimension ldy >= r; row i is the
 *         configuration of row i of X.  The sign of each column of the first
 *         part's configuration follows the fit's convention (largest-|.|
 *         entry positive, first row in part order on ties); columns whose
 *         eigenvalue in the first part is <= MDS_TAU * lambda_1 are zero.
 *         The Procrustes fit is orthogonal with a shift and no dilation,
 *         over the live columns.
 * lam_bar: host, r doubles (may be NULL): (1/parts) sum_j lambda^j / n_j,
 *         the column-variance estimates of Section 3.2.
 * r_eff:  host (may be NULL): live columns.
 * order_out: device, n int64 (may be NULL): the row order (position ->
 *         row) that defines the parts.
 * Everything runs in FP64 on `stream`; the call returns when Y is complete.
 * Errors: INVALID_ARG (pointers, sizes, non-finite X), DEGENERATE (a part
 * whose rows all coincide, or connecting rows that do not fix the rotation:
 * smallest singular value of the cross-product matrix <= 1e-9 of the
 * largest), OOM, HIP. */
#define MDS_DC_MAX_L 2048
mds_status mds_divide_conquer(const void* X, int32_t dt, int64_t n, int64_t p, int64_t ldx,
                              int64_t l, int64_t c, int32_t r, uint64_t seed, double* Y,
                              int64_t ldy, double* lam_bar, int32_t* r_eff, int64_t* order_out,
                              void* stream);

/* Release every device and host buffer of the model.  NULL is a no-op.
 * The caller must ensure no embed on any stream still uses m. */
void mds_free(mds_model* m);

/* ---- model getters (synchronous; host output buffers owned by caller) ----
 * info: any output pointer may be NULL.  r_eff = number of live directions. */
mds_status mds_model_info(const mds_model* m, int64_t* n_fit, int64_t* p, int64_t* l,
                          int32_t* r, int32_t* r_eff);
/* idx: l int64, ascending landmark indices (Section 3.1 random subset). */
mds_status mds_get_landmarks(const mds_model* m, int64_t* idx);
/* lam: r doubles, Lambda in decreasing order (not divided by l; lambda/l
 * estimates the variance of each output column, Section 3.1 and eq. (1)). */
mds_status mds_get_eigenvalues(const mds_model* m, double* lam);
/* X1: l x r doubles row-major, V Lambda^{1/2} of the landmarks (Section 2,
 * step 4), dead columns zero. */
mds_status mds_get_landmark_coords(const mds_model* m, double* X1);
/* q: l doubles, diag(Q1) (Section 3.1). */
mds_status mds_get_q(const mds_model* m, double* q);
/* bytes of device memory the model holds. */
int64_t mds_model_bytes(const mds_model* m);
/* eigensolver statistics: Lanczos steps taken and restarts after an
 * invariant subspace was found; either pointer may be NULL. */
mds_status mds_fit_stats(const mds_model* m, int32_t* lanczos_steps, int32_t* restarts);

const char* mds_last_error(void);
int32_t mds_last_hip_error(void);

/* ---- serving: continuous batching over resident models ------------------
 * A server keeps fitted models resident, admits embed requests against a
 * byte budget and a slot limit, and runs every admitted request's row
 * tiles through one persistent fused launch per step (replayed from a
 * captured HIP graph), admitting new requests between steps while earlier
 * steps are still on the device.  Each row is computed by exactly the
 * code path of mds_embed, so a request's result is the same alone and in
 * any mix.  Calls that overlap in time must come from one thread, except
 * mds_serve_poll / mds_serve_wait / mds_serve_stats, which are thread-safe.
 */
typedef struct mds_server mds_server;

typedef struct {
  int64_t submitted, admitted, completed;
  int64_t queued;            /* waiting for admission */
  int64_t in_flight;         /* admitted, not yet complete */
  int64_t steps;             /* persistent launches issued */
  int64_t tiles;             /* row tiles processed */
  int64_t points;            /* rows embedded */
  int64_t bytes_in_use;      /* models + admitted requests */
  int64_t budget_bytes;
} mds_serve_stats_t;

/* budget_bytes: device bytes models plus in-flight requests may occupy
 * (models charge mds_model_bytes; a request charges 4*n_pts*(p + r)).
 * max_slots: admitted requests at once (1..65536).
 * tiles_per_step: row tiles per persistent launch (0 = default). */
mds_status mds_serve_create(int64_t budget_bytes, int32_t max_slots, int32_t tiles_per_step,
                            mds_server** out);
/* Make a fitted model resident.  The server does not take ownership: keep
 * m alive until mds_serve_destroy.  Errors: BUDGET if it does not fit. */
mds_status mds_serve_add_model(mds_server* s, const mds_model* m, int32_t* model_id);
/* Queue an embed request (non-blocking).  X, Y as for mds_embed (device,
 * caller-owned, must stay valid until the ticket completes): X holds n_pts
 * rows of the model's p values, dt must be MDS_F32; Y holds n_pts rows of
 * at least r floats.  prec is MDS_PREC_FP32 or MDS_PREC_SPLIT_BF16 / _FP16.
 * Errors: INVALID_ARG (dt other than MDS_F32, prec, NULL pointers,
 * ldx < p, ldy < r), NOT_FOUND (model id), BUDGET if the request alone
 * exceeds the budget left after the models. */
mds_status mds_serve_submit(mds_server* s, int32_t model_id, const void* X, int32_t dt,
                            int64_t n_pts, int64_t ldx, int32_t prec, void* Y, int64_t ldy,
                            int64_t* ticket);
/* Ticket state: 0 queued, 1 admitted, 2 done.  Times are seconds on the
 * server's monotonic clock; any output pointer may be NULL. */
mds_status mds_serve_poll(mds_server* s, int64_t ticket, int32_t* state, double* t_submit,
                          double* t_admit, double* t_done);
/* Block until the ticket is done (timeout_s < 0 waits forever).
 * Errors: STATE on timeout. */
mds_status mds_serve_wait(mds_server* s, int64_t ticket, double timeout_s);
/* Counters of the server (thread-safe snapshot). */
mds_status mds_serve_stats(mds_server* s, mds_serve_stats_t* out);
/* seconds on the server's clock (for stamping arrivals). */
double mds_serve_now(mds_server* s);
/* Finish every submitted request, stop the worker, free server memory. */
void mds_serve_destroy(mds_server* s);

/* ---- test hook (host only) -----------------------------------------------
 * The first `draws` values of the landmark sampler's bounded draw below k
 * from SplitMix64(seed), written to out (host, caller-owned); returns draws.
 * Lets the sampler's building blocks be checked without a GPU. */
uint64_t mds_debug_bounded(uint64_t seed, uint64_t k, int32_t draws, uint64_t* out);

#ifdef __cplusplus
}
#endif
#endif /* MDS_H */
