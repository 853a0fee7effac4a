/*
 * rbd.h -- C ABI of the MI355X (gfx950) Reduced Basis Decomposition library.
 *
 * Reduced Basis Decomposition (Y. Chen, "Reduced Basis Decomposition: a
 * Certified and Fast Lossy Data Compression Algorithm") approximates a data
 * matrix X (m x n, one sample per column, eq. (1)) by Y T, where Y (m x d) has
 * orthonormal columns built greedily and T = Y'X (d x n).  Algorithm 1 of
 * section 3.1 adds, at each step, the column of X whose projection error onto
 * span(Y) is largest, after Gram-Schmidt orthonormalisation against Y.  With
 * the identity weight (A = I in eq. (3)) the squared error of column j is
 * ||x_j||^2 - ||T(:, j)||^2.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All array arguments are DEVICE pointers to caller-owned memory.  The
 *    library never allocates or frees device memory and never synchronises
 *    the stream; every call is stream-ordered on `stream` (a hipStream_t,
 *    NULL for the legacy default stream).
 *  - Matrices are row-major with an explicit leading dimension (elements
 *    between consecutive rows).  Indices are 0-based.
 *  - The synchronous return value reports argument validation and launch
 *    errors only.  Conditions found on the device (non-finite data) are
 *    written to the `status` word in device memory; read it after the stream
 *    has completed.
 *  - Calls on different streams are independent as long as they use
 *    different workspaces and outputs.  Results are bitwise reproducible
 *    for identical inputs on the same device (all reductions run in a fixed
 *    order; no floating-point atomics).
 */
#ifndef RBD_H_
#define RBD_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* In C++ the enumerations below have int as their fixed underlying type, so
 * every int a C caller passes is a value of the type (and is then validated:
 * an unknown value gives RBD_EINVAL). */
#ifdef __cplusplus
#define RBD_ENUM_BASE : int
#else
#define RBD_ENUM_BASE
#endif

/* Storage type of X (and V).  Arithmetic is always FP64: stored values are
 * widened exactly, products and sums are formed in FP64. */
typedef enum RBD_ENUM_BASE {
    RBD_F32 = 0,
    RBD_BF16 = 1, /* bfloat16 bit patterns (uint16) */
    RBD_F16 = 2,  /* IEEE binary16 */
    RBD_F64 = 3
} rbd_dtype;

/* Storage of the basis while a fit runs (rbd_fit_basis).  RBD_BASIS_F64 is
 * rbd_fit's.  RBD_BASIS_F32 keeps Y in FP32 in the workspace once the fit
 * passes 128 columns (half the bytes of the pass over Y each step), with all
 * arithmetic still FP64, and writes its FP64 copy to the output Y at the end. */
typedef enum RBD_ENUM_BASE { RBD_BASIS_F64 = 0, RBD_BASIS_F32 = 1 } rbd_basis;

/* How `tol` is read: RBD_TOL_ABS uses tau = tol, RBD_TOL_REL uses
 * tau = tol * max_j ||x_j|| (the largest error before the first step). */
typedef enum RBD_ENUM_BASE { RBD_TOL_ABS = 0, RBD_TOL_REL = 1 } rbd_tol_mode;

/* Return / status codes. */
enum {
    RBD_OK = 0,
    RBD_EINVAL = -1,      /* bad pointer, size, leading dimension or option      */
    RBD_ENONFINITE = -2,  /* X holds NaN or Inf (device status only)              */
    RBD_EWORKSPACE = -3,  /* workspace smaller than the size query returned       */
    RBD_EDEVICE = -4,     /* a HIP launch or runtime call failed                  */
    RBD_EMATRIX = -5,     /* sparse A: an index outside its rows (device status)  */
    RBD_ETOOLARGE = -6    /* rbd_fit_noalloc: the fit needs more than its scratch */
};

/* Why the greedy loop ended (written to stop_reason when non-NULL). */
enum {
    RBD_STOP_TOL = 1,     /* step 2.4: largest error <= tau                      */
    RBD_STOP_DMAX = 2,    /* d reached min(d_max, m, n)                           */
    RBD_STOP_BREAK = 3    /* step 2.2: ||v|| < tau (or ||v|| = 0) after GS        */
};

/* Largest basis size supported by rbd_fit (registers hold one row of Y). */
#define RBD_MAX_D 1024

/*
 * rbd_fit_workspace_size -- bytes of device workspace rbd_fit needs.
 * Arguments as for rbd_fit.  Returns RBD_OK and sets *bytes, or RBD_EINVAL.
 */
int rbd_fit_workspace_size(int64_t m, int64_t n, int32_t d_max, rbd_dtype xt, size_t* bytes);

/*
 * rbd_fit -- Algorithm 1, (Y, T) = RBD(X, eps_R, d_max), with A = I
 * (section 3.1; error evaluation of section 3.2, eq. (3)).
 *
 *   X        m x n, row-major, leading dimension ldx >= n, storage type xt.
 *   tol      eps_R >= 0, read according to `mode`.
 *   d_max    1 <= d_max; the loop runs at most D = min(d_max, m, n) steps,
 *            and D must not exceed RBD_MAX_D.
 *   start    first column (step 1); start < 0 takes the lowest index of
 *            max_j ||x_j|| (the first step of column-pivoted QR).
 *
 * Outputs (device memory, caller-owned, written in full):
 *   Y        m x d_max row-major (ld = d_max), FP64.  Columns 0..d-1 hold
 *            the orthonormal basis xi_1..xi_d; columns >= d are zeroed.
 *   T        d_max x n row-major (ld = n), FP64; T(k, :) = xi_k' X; rows >= d
 *            are zeroed.
 *   pivots   d_max int64; pivots[k] = column used at step k+1; -1 after d.
 *   col_err  n FP64; ||x_j - Y T(:, j)|| for the final d (0 for pivots).
 *            Certified: the downdated value ||x_j||^2 - sum_k T(k,j)^2 is
 *            replaced by an exact evaluation of the residual whenever it has
 *            fallen below 2^-20 of the last exact value, so cancellation
 *            never decides a step.
 *   err_hist d_max+1 FP64; err_hist[0] = max_j ||x_j||, err_hist[k] = the
 *            largest error after step k (E_cur of step 2.3); 0 after d.
 *   d_out    one int32: d, the number of basis vectors kept.
 *   status   one int32: RBD_OK or RBD_ENONFINITE.
 *   stop_reason  one int32 (may be NULL): an RBD_STOP_* value, 0 if d = 0
 *            because of a non-finite input.
 *   workspace    at least rbd_fit_workspace_size() bytes, 256-byte aligned.
 *   stream       hipStream_t (as void*).
 *
 * Returns RBD_OK, RBD_EINVAL, RBD_EWORKSPACE or RBD_EDEVICE.
 */
int rbd_fit(const void* X, rbd_dtype xt, int64_t m, int64_t n, int64_t ldx,
            double tol, rbd_tol_mode mode, int32_t d_max, int64_t start,
            double* Y, double* T, int64_t* pivots, double* col_err, double* err_hist,
            int32_t* d_out, int32_t* status, int32_t* stop_reason,
            void* workspace, size_t workspace_bytes, void* stream);

/*
 * rbd_fit_basis -- rbd_fit with a choice of how the basis is stored while
 * the loop runs (rbd_fit_basis(..., RBD_BASIS_F64, ...) is rbd_fit).  With
 * RBD_BASIS_F32 inputs small enough for rbd_fit's single-launch loop (X of at
 * most 64 MB, whose passes read the caches, not HBM) run exactly as rbd_fit;
 * otherwise the first 128 steps run exactly as rbd_fit's (a fit that ends
 * within 128 columns gives rbd_fit's results); when the fit passes 128
 * columns the basis is rounded to FP32, and every later basis vector xi_k is
 * formed in FP64 as by rbd_fit and stored rounded to FP32.  From then on the
 * Gram-Schmidt passes and the exact refreshes read the stored (rounded)
 * vectors, while the row T(k, :) is formed from the FP64 vector before
 * rounding.  The output Y holds the stored values (for fits past 128
 * columns, orthonormal to about 1e-7 instead of 1e-15).  The
 * downdated errors then carry, between exact refreshes, an absolute error of
 * order 2^-24 ||x_j||^2 / e_j in e_j (the rounded basis is orthonormal only
 * to FP32 precision), so the mode is meant for data whose errors stay well
 * above 2^-12 ||x_j||: BF16 storage (unit roundoff 2^-9), whose fits it
 * speeds up by halving the bytes of the pass over Y.  The exact refreshes and
 * their trigger are those of rbd_fit.
 *   basis       RBD_BASIS_F64 or RBD_BASIS_F32; other arguments as for rbd_fit.
 *   workspace   at least rbd_fit_basis_workspace_size() bytes.
 * Returns what rbd_fit returns; RBD_EINVAL for an unknown `basis`.
 */
int rbd_fit_basis_workspace_size(int64_t m, int64_t n, int32_t d_max, rbd_dtype xt, rbd_basis basis,
                                 size_t* bytes);
int rbd_fit_basis(const void* X, rbd_dtype xt, int64_t m, int64_t n, int64_t ldx,
                  double tol, rbd_tol_mode mode, int32_t d_max, int64_t start, rbd_basis basis,
                  double* Y, double* T, int64_t* pivots, double* col_err, double* err_hist,
                  int32_t* d_out, int32_t* status, int32_t* stop_reason,
                  void* workspace, size_t workspace_bytes, void* stream);

/*
 * rbd_fit_noalloc -- rbd_fit for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same computation, kernels and results as rbd_fit with
 * the same arguments, but no workspace argument.  The workspace is a fixed
 * scratch array of RBD_NOALLOC_MAX_BYTES in the library's device code, one
 * per GPU, held until the process ends; its device address is looked up once
 * per device (on the first call with that device current).  The call
 * allocates and frees nothing and never synchronises.
 *   All arguments and outputs are those of rbd_fit; `stream` must belong to
 *   the current device.
 * Every call on one GPU shares that GPU's scratch: calls whose execution
 * overlaps on one GPU (other streams, other host threads) race and give
 * undefined results; serialise them (one stream, or events).  The scratch
 * keeps the last call's contents; every call initialises what it reads.
 * Returns RBD_ETOOLARGE (before any device call) when
 * rbd_fit_workspace_size() exceeds RBD_NOALLOC_MAX_BYTES, else what rbd_fit
 * returns; RBD_EDEVICE if the scratch address cannot be obtained.
 */
#define RBD_NOALLOC_MAX_BYTES ((size_t)64 << 20)
int rbd_fit_noalloc(const void* X, rbd_dtype xt, int64_t m, int64_t n, int64_t ldx,
                    double tol, rbd_tol_mode mode, int32_t d_max, int64_t start,
                    double* Y, double* T, int64_t* pivots, double* col_err, double* err_hist,
                    int32_t* d_out, int32_t* status, int32_t* stop_reason, void* stream);

/*
 * rbd_fit_weighted -- Algorithm 1 with the A-norm of section 3.2 for a general
 * diagonal A = diag(weights), which weights some entries of every column
 * more than others: the basis Y and T = Y'X are built exactly as by rbd_fit, but
 * every error of step 2.3 (hence E_0, the relative tolerance, the pivot
 * choice, col_err and err_hist) is ||x_j - Y T(:, j)||_A, eq. (3).
 *   weights  m FP64 device values, all > 0 (not checked on the device); the
 *            other arguments, outputs and workspace are those of rbd_fit.
 * The errors are downdated as e_j^2 -= 2 t_j (g' x_j) - t_j^2 ||xi||_A^2 with
 * g = (I - Y Y')(A xi), formed each step, and certified as in rbd_fit.
 */
int rbd_fit_weighted(const void* X, rbd_dtype xt, int64_t m, int64_t n, int64_t ldx, const double* weights,
                     double tol, rbd_tol_mode mode, int32_t d_max, int64_t start,
                     double* Y, double* T, int64_t* pivots, double* col_err, double* err_hist,
                     int32_t* d_out, int32_t* status, int32_t* stop_reason,
                     void* workspace, size_t workspace_bytes, void* stream);

/*
 * Captured fits.  rbd_fit_graph_create records the launch sequence of one
 * rbd_fit (weights == NULL) or rbd_fit_weighted call -- all D greedy steps,
 * each kernel of a step returning at once after the device-side stop -- into
 * a HIP graph, without running it; rbd_fit_graph_launch replays it on any
 * stream.  Every pointer argument is baked into the graph: a replay fits
 * whatever X (and weights) then hold, into the same outputs and workspace,
 * which must stay allocated until rbd_fit_graph_destroy.  `stream` must not
 * be the null stream (capture needs a created stream); nothing runs on it
 * during creation.  Replays on one workspace must not overlap.  Arguments
 * and errors otherwise as for rbd_fit / rbd_fit_weighted; creation can also
 * fail with RBD_EDEVICE if capture is not possible.
 */
typedef struct rbd_fit_graph_s* rbd_fit_graph;
int rbd_fit_graph_create(const void* X, rbd_dtype xt, int64_t m, int64_t n, int64_t ldx, const double* weights,
                         double tol, rbd_tol_mode mode, int32_t d_max, int64_t start,
                         double* Y, double* T, int64_t* pivots, double* col_err, double* err_hist,
                         int32_t* d_out, int32_t* status, int32_t* stop_reason,
                         void* workspace, size_t workspace_bytes, void* stream, rbd_fit_graph* out);
int rbd_fit_graph_launch(rbd_fit_graph graph, void* stream);
int rbd_fit_graph_destroy(rbd_fit_graph graph);

/*
 * rbd_fit_spd -- Algorithm 1 with the A-norm of section 3.2 for a general
 * symmetric positive definite A, which can couple different entries of a
 * column (for instance an energy norm of a field on a grid), A given in CSR
 * form:
 *   a_indptr   m + 1 int64 row offsets into a_indices / a_values,
 *              non-decreasing (rows own consecutive ranges of entries)
 *   a_indices  a_nnz int32 column indices in [0, m)
 *   a_values   a_nnz FP64 values
 * The basis Y and T = Y'X are built exactly as by rbd_fit; every error of step
 * 2.3 (E_0, the relative tolerance, the argmax, col_err, err_hist) is
 * ||x_j - Y T(:, j)||_A = sqrt(r' A r), eq. (3).  Symmetry and definiteness
 * of A are the caller's responsibility; a column index outside [0, m), a
 * row range outside [0, a_nnz) or a decreasing a_indptr is reported through
 * *status as RBD_EMATRIX (d = 0), and no kernel reads outside the arrays.
 * The errors are downdated as for a diagonal A with g = (I - YY')(A xi)
 * (two sparse products per step).  Exact refreshes of queued columns
 * materialise their residuals in chunks of columns: every step enqueues the
 * chunks for the longest possible queue, and each chunk reads the queue's
 * length on the device (empty chunks return at once), so, as rbd_fit, the
 * call never waits for the device.  Other arguments, outputs and errors are
 * those of rbd_fit; workspace: rbd_fit_spd_workspace_size() bytes.
 */
int rbd_fit_spd_workspace_size(int64_t m, int64_t n, int32_t d_max, rbd_dtype xt, size_t* bytes);
int rbd_fit_spd(const void* X, rbd_dtype xt, int64_t m, int64_t n, int64_t ldx, const int64_t* a_indptr,
                const int32_t* a_indices, const double* a_values, int64_t a_nnz, double tol, rbd_tol_mode mode,
                int32_t d_max, int64_t start, double* Y, double* T, int64_t* pivots, double* col_err,
                double* err_hist, int32_t* d_out, int32_t* status, int32_t* stop_reason,
                void* workspace, size_t workspace_bytes, void* stream);

/*
 * rbd_project_workspace_size -- bytes of workspace rbd_project needs.
 */
int rbd_project_workspace_size(int64_t m, int32_t d, int64_t k, rbd_dtype vt, size_t* bytes);

/*
 * rbd_project -- out-of-sample compression (section 3.1, the
 * compression of out-of-sample data): v_C = Y' v for each column v of V,
 * with the A = I error of eq. (3), ||v - Y v_C||, as the error indicator.
 *
 *   Y        m x d row-major FP64 with leading dimension ldy >= d; columns are
 *            assumed orthonormal (as rbd_fit returns them).
 *   V        m x k row-major, leading dimension ldv >= k, storage type vt.
 *   Tv       d x k row-major FP64 (ld = k): the coordinates Y'V.
 *   err_v    k FP64: ||v_q - Y Tv(:, q)||, evaluated from the explicit
 *            residual (no cancellation).
 *   workspace at least rbd_project_workspace_size() bytes.
 *
 * 1 <= d <= RBD_MAX_D, m >= 1, k >= 1.  Returns RBD_OK, RBD_EINVAL,
 * RBD_EWORKSPACE or RBD_EDEVICE.
 */
int rbd_project(const double* Y, int64_t ldy, int64_t m, int32_t d,
                const void* V, rbd_dtype vt, int64_t k, int64_t ldv,
                double* Tv, double* err_v,
                void* workspace, size_t workspace_bytes, void* stream);

/*
 * Batched fits: many independent matrices of different sizes in one
 * persistent launch (Algorithm 1 applied to each, with the same readings and
 * certified errors as rbd_fit).  Limits: m_b <= 4096 rows, d_max <= 256.
 *
 * Packed layouts (all row-major, offsets in elements, assigned in batch order
 * by rbd_batch_plan): X holds X_b (m_b x n_b, ld n_b) back to back; Y holds
 * Y_b (m_b x d_max); T holds T_b (d_max x n_b); col_err holds n_b values per
 * matrix; pivots is batch x d_max; err_hist is batch x (d_max + 1); d_out and
 * status hold one int32 per matrix.  Unused basis columns / rows of T are
 * zeroed, pivots past d are -1, as for rbd_fit.
 */
typedef struct {
    int64_t x_elems, y_elems, t_elems, c_elems; /* sizes of the packed X, Y, T, col_err buffers */
    int64_t max_m, max_n;                       /* largest m_b and n_b                           */
    size_t workspace_bytes;                     /* device workspace rbd_fit_batched needs          */
} rbd_batch_sizes;

/* Workgroup shape of the persistent launch: threads per workgroup (64, 128,
 * 256, 512 or 1024; one workgroup handles one matrix at a time) and
 * workgroups per compute unit (1..16). */
typedef struct {
    int32_t threads;
    int32_t wg_per_cu;
} rbd_batch_config;

/*
 * rbd_batch_plan -- host-only.  From the sizes m[b], n[b] (host arrays of
 * `batch` entries) fills `desc` (host, batch x 8 int64: per-matrix sizes and
 * offsets) and `order` (host, batch int32: processing order, largest
 * m_b * n_b * min(d_max, m_b, n_b) first), and the buffer sizes.  The caller
 * copies desc and order to the device.  Returns RBD_OK or RBD_EINVAL.
 */
int rbd_batch_plan(const int64_t* m, const int64_t* n, int32_t batch, int32_t d_max, int64_t* desc,
                   int32_t* order, rbd_batch_sizes* sizes);

/*
 * rbd_fit_batched -- fits every matrix of the batch in one persistent launch
 * on `stream`.  desc / order: device copies of rbd_batch_plan's arrays;
 * max_m: sizes.max_m.  tol, mode, d_max as for rbd_fit (one setting for all
 * matrices).  Returns RBD_OK, RBD_EINVAL, RBD_EWORKSPACE or RBD_EDEVICE;
 * per-matrix non-finite input is reported in status[b].
 */
int rbd_fit_batched(const void* X, rbd_dtype xt, const int64_t* desc, const int32_t* order, int32_t batch,
                    double tol, rbd_tol_mode mode, int32_t d_max, rbd_batch_config cfg,
                    double* Y, double* T, int64_t* pivots, double* col_err, double* err_hist,
                    int32_t* d_out, int32_t* status, int64_t max_m,
                    void* workspace, size_t workspace_bytes, void* stream);

/*
 * rbd_batched_autotune -- empirical choice of rbd_batch_config: runs every
 * candidate (threads 128..1024 x 1, 2, 4, 8 workgroups per compute unit)
 * twice on the sub-batch order[0], order[s], order[2s], ... (s =
 * sample_stride), keeps the fastest second run, and writes it to *best (and
 * the 16 times in ms to trial_ms when not NULL, threads-major; -1 for a shape
 * that cannot be launched, e.g. for lack of LDS).  The sub-batch should give
 * every workgroup several matrices (at least about 4 x 8 x the number of
 * compute units), or the times measure single-matrix latency rather than
 * throughput.  Overwrites the sampled matrices' outputs and WAITS for the
 * stream.  Same arguments otherwise as rbd_fit_batched.
 */
int rbd_batched_autotune(const void* X, rbd_dtype xt, const int64_t* desc, const int32_t* order, int32_t batch,
                         double tol, rbd_tol_mode mode, int32_t d_max, int32_t sample_stride,
                         double* Y, double* T, int64_t* pivots, double* col_err, double* err_hist,
                         int32_t* d_out, int32_t* status, int64_t max_m,
                         void* workspace, size_t workspace_bytes, void* stream,
                         rbd_batch_config* best, double* trial_ms);

/*
 * rbd_reconstruct -- uncompress (section 3.1): Z = Y T, i.e. X(:, j) ~
 * Y T(:, j) for every column.  Y: m x d (ld ldy >= d), T: d x n (ld ldt >= n),
 * Z: m x n (ld ldz >= n), all FP64 device memory.  An FP64 GEMM on the matrix
 * cores; needs no workspace.  Returns RBD_OK, RBD_EINVAL or RBD_EDEVICE.
 */
int rbd_reconstruct(const double* Y, int64_t ldy, int64_t m, int32_t d, const double* T, int64_t ldt, int64_t n,
                    double* Z, int64_t ldz, void* stream);

/*
 * rbd_reconstruct_backward -- gradient of L = <G, Z>, Z = Y Y' X (the
 * reconstruction of X by its own fit), with respect to X, holding the pivots
 * fixed.  With A = X(:, pivots) = Y R (R = T(:, pivots), upper triangular):
 *   dX = Y (Y'G) + scatter_pivots( (Ybar + Y copyltu(-Ybar'Y)) R^{-T} ),
 *   Ybar = G T' + X (G'Y),   copyltu(M) = tril(M) + tril(M, -1)'.
 *
 *   X       m x n, ld ldx, storage xt (the matrix that was fitted)
 *   G       m x n, ld ldg, FP64 or FP32 (the cotangent of Z)
 *   Y, T    the fit's basis (m x d, ld ldy) and coefficients (d x n, ld ldt)
 *   pivots  d int64 (device), the fit's pivots (distinct, in [0, n); an entry
 *           outside [0, n) contributes nothing to dX)
 *   dX      m x n FP64 output, ld lddx (overwritten)
 *   workspace  rbd_reconstruct_backward_workspace_size() bytes, 256-aligned
 * 1 <= d <= min(m, n, RBD_MAX_D).  Returns RBD_OK, RBD_EINVAL, RBD_EWORKSPACE
 * or RBD_EDEVICE.
 */
int rbd_reconstruct_backward_workspace_size(int64_t m, int64_t n, int32_t d, size_t* bytes);
int rbd_reconstruct_backward(const void* X, rbd_dtype xt, int64_t ldx, const void* G, rbd_dtype gt, int64_t ldg,
                             const double* Y, int64_t ldy, const double* T, int64_t ldt, const int64_t* pivots,
                             int64_t m, int64_t n, int32_t d, double* dX, int64_t lddx,
                             void* workspace, size_t workspace_bytes, void* stream);

/*
 * rbd_classify -- recognition of out-of-sample data in the compressed
 * coordinates: each query v (a column of V) is compressed as c = Y'v
 * (section 3.1, compression of out-of-sample data) and matched
 * to the training sample j whose coordinates T(:, j) are nearest,
 *   j* = argmin_j sum_i (c_i - T(i, j))^2,
 * the differences squared and summed in FP64 term by term in ascending i; the
 * lowest index wins ties.  This is how section 4 uses the compressed faces for
 * recognition.
 *   Y         m x d FP64, row-major, leading dimension ldy >= d (the basis)
 *   T         d x n FP64, row-major, ldt >= n (training coordinates)
 *   labels    n int32 class labels of the training samples, or NULL (the
 *             label reported is then the index)
 *   V         m x k queries, row-major, ldv >= k, stored as vt
 *   C         out: d x k FP64 row-major (leading dimension k), C = Y'V
 *   nn_index  out: k int64 nearest training index
 *   nn_label  out: k int32 labels[nn_index]
 *   nn_dist2  out: k FP64 squared distance to it
 *   workspace rbd_classify_workspace_size() bytes (split-k partials of Y'V),
 *             256-byte aligned
 * All pointers are device memory owned by the caller; stream-ordered, no
 * allocation or synchronisation.  Returns RBD_EINVAL for bad sizes or
 * pointers (d > RBD_MAX_D, k >= 2^31, n < 1), RBD_EWORKSPACE when the
 * workspace is too small, RBD_EDEVICE on a launch failure.
 */
int rbd_classify_workspace_size(int64_t m, int32_t d, int64_t k, size_t* bytes);
int rbd_classify(const double* Y, int64_t ldy, int64_t m, int32_t d, const double* T, int64_t ldt, int64_t n,
                 const int32_t* labels, const void* V, rbd_dtype vt, int64_t k, int64_t ldv, double* C,
                 int64_t* nn_index, int32_t* nn_label, double* nn_dist2,
                 void* workspace, size_t workspace_bytes, void* stream);

/*
 * Optional phase timing for measurement tools.  Between rbd_profiler_begin and
 * rbd_profiler_end, every rbd_fit call made by the calling host thread records
 * HIP events on its stream around the launches of the phases selected by
 * `phase_mask` (bit i = phase i below) and at the end of every greedy step.
 * Events come from a pool owned by the library and reused across calls; no
 * device memory is allocated.  rbd_profiler_end waits for the last recorded
 * event, then returns, per phase, the summed kernel time in milliseconds and
 * the number of launches (arrays of length `nphase`, may be NULL), and for the
 * last recorded fit the elapsed milliseconds from its start to the end of each
 * step (`step_end_ms`, up to `nstep` entries; *nstep_out = steps recorded).
 * Recording adds a few microseconds per event to the stream.
 */
enum {
    RBD_PHASE_COLNORM = 0,   /* diag(X'X) pre-computation (section 3.3)          */
    RBD_PHASE_INIT = 1,      /* E_0, tau, first column                           */
    RBD_PHASE_CGS1 = 2,      /* the pass over Y (x_p read from X, or gathered)   */
    RBD_PHASE_CGS2 = 3,      /* nu and the break test; for A = I the correction   *
                              * rows of T, otherwise the second pass over Y and   *
                              * the A-norm terms                                  */
    RBD_PHASE_XSCAN = 4,     /* T(d, :) = xi' X: the stream over X                */
    RBD_PHASE_UPDATE = 5,    /* error downdate and argmax (eq. (3))               */
    RBD_PHASE_RESID = 6,     /* exact residual norms of queued columns            */
    RBD_PHASE_RESID_FINISH = 7,
    RBD_PHASE_EPILOGUE = 8,
    RBD_PHASE_LOOP = 9,      /* the persistent loop of a cache-resident fit: the  *
                              * whole of Algorithm 1 in one launch                */
    RBD_NUM_PHASES = 10
};
int rbd_profiler_begin(uint32_t phase_mask);
int rbd_profiler_end(double* phase_ms, int64_t* phase_launches, int32_t nphase,
                     double* step_end_ms, int64_t nstep, int64_t* nstep_out);

/*
 * rbd_read_stream -- a measurement tool: reads `bytes` of device memory at
 * `data` once with the X-scan's 16-byte loads (non-temporal when
 * `nontemporal` is nonzero, as the scan uses them for X above 512 MB) and
 * discards the values, so the time it takes gives the read bandwidth a scan of
 * that buffer can reach.  `sink` is 4 bytes of device memory that the kernel
 * may write.  `data` must be 16-byte aligned and `bytes` a multiple of 16.
 * Returns RBD_OK, RBD_EINVAL or RBD_EDEVICE.
 */
int rbd_read_stream(const void* data, size_t bytes, int nontemporal, void* sink, void* stream);

/* Human-readable text for a return or status code (static storage). */
const char* rbd_status_string(int code);

/* Library version string, e.g. "rbd-gfx950 0.1". */
const char* rbd_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RBD_H_ */
