/*
 * tprod.h - C ABI of the MI355X (gfx950) t-product library.
 *
 * Tensors are third-order real arrays X of size n1 x n2 x n3 stored
 * contiguously, element (i, j, k) at offset (i*n2 + j)*n3 + k: every tube
 * X_{ij:} is contiguous ("tube-major"). Fourier-domain data ("spectra") hold
 * the K = floor(n3/2) + 1 non-redundant frontal slices of fft(X, [], 3)
 * (slice K-1 is the Nyquist slice when n3 is even; the others are the
 * conjugates of these, so they are never stored) in planar form:
 * re[k][row][col] and im[k][row][col], each a contiguous K x rows x cols
 * array. The transform follows the MATLAB convention of Section 2.1: the
 * forward transform is unscaled, the inverse carries 1/n3.
 *
 * Ownership: the caller allocates and frees every buffer (inputs, outputs
 * and the workspace, whose size the *_workspace functions return). Unless a
 * parameter says "host", pointers are device pointers on the current HIP
 * device. The library keeps no per-call state; its only global state is a
 * per-device table of transform twiddles set up on first use, the fixed
 * scratch array of tp_tsample_noalloc, and a per-device side stream with
 * two events, created on first use, on which the block Jacobi sweeps of
 * the singular value thresholding (tp_tsvt, the ADMM calls, tp_tsvd_full,
 * t-project beyond 64 slices) run half of the Fourier slices when a launch
 * has more pair steps than the GPU has compute units and fewer than 7/8 of
 * twice that number (the steps that fit at once). That work is forked
 * from `stream` by an event and joined back to it before the call's later
 * work, so it stays ordered with `stream` (also under graph capture).
 *
 * Asynchrony: every call enqueues its work on `stream` (a hipStream_t;
 * NULL is the default stream) and returns without synchronising (the one
 * exception is the first call on a device that runs a tube transform,
 * which uploads the twiddle table synchronously; tp_trace_count also waits
 * for its recorded events). Values a
 * call writes to device memory (sample counts, ranks) are valid once the
 * stream has reached that point.
 *
 * Errors: arguments are validated on the host before anything is enqueued;
 * on failure a negative tp_status is returned, nothing is enqueued and
 * tp_last_error() describes the problem (thread-local). A failed kernel
 * launch returns TP_EHIP.
 *
 * Determinism: the same inputs, seed and precision give bitwise identical
 * outputs: no reduction uses floating-point atomics.
 */
#ifndef TPROD_H
#define TPROD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TP_OK = 0,
  TP_EINVAL = -1,      /* bad scalar argument or null pointer          */
  TP_ESHAPE = -2,      /* shapes do not match                          */
  TP_EDTYPE = -3,      /* unsupported dtype / precision combination    */
  TP_EWORKSPACE = -4,  /* workspace missing or too small               */
  TP_EHIP = -5,        /* a HIP runtime call or kernel launch failed    */
  TP_ENOCONV = -6,     /* an ADMM call with a stop tolerance reached its
                          iteration cap first (results still written)   */
  TP_EUNSUPPORTED = -7 /* size outside what the kernels implement      */
} tp_status;

typedef enum { TP_F32 = 0, TP_F64 = 1 } tp_dtype;

/* Arithmetic of the per-slice contractions.
 *  TP_PREC_F64    float64 operands and accumulation (TP_F64 storage).
 *  TP_PREC_F32    float32 operands and accumulation; products with at least
 *                 16 rows and columns and a contraction of at least 64 run
 *                 on the float32 matrix cores with complex products as
 *                 three real products (Re = P1 - P2, Im = P3 - P1 - P2 with
 *                 P1 = Ar Br, P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi)); smaller
 *                 ones as four (Re = Ar Br - Ai Bi, Im = Ar Bi + Ai Br).
 *  TP_PREC_BF16X3 float32 operands split as x = hi + lo, hi = bf16(x),
 *                 lo = bf16(x - hi) (round to nearest even), products
 *                 hi*hi + hi*lo + lo*hi on the bf16 matrix cores with
 *                 float32 accumulation. Complex products of float32
 *                 spectra (inside the decompositions) use three real
 *                 products, with Ar + Ai and Br + Bi formed and split while
 *                 staging; the t-product and rt-product, whose transforms
 *                 emit the split planes directly, use four (Re = Ar Br -
 *                 Ai Bi, Im = Ar Bi + Ai Br): the staging of those planes,
 *                 not the matrix cores, bounds that product, and three
 *                 products would need two more planes per operand.
 *  TP_PREC_BF16   single bf16 product (hi*hi only), float32 accumulation. */
typedef enum { TP_PREC_F64 = 0, TP_PREC_F32 = 1, TP_PREC_BF16X3 = 2, TP_PREC_BF16 = 3 } tp_prec;

/* A dense tube-major tensor. */
typedef struct {
  void* data;
  int32_t dtype; /* tp_dtype */
  int64_t n1, n2, n3;
} tp_tensor;

/* A half spectrum: planar re/im arrays of K x rows x cols. */
typedef struct {
  void* re;
  void* im;
  int32_t dtype; /* tp_dtype */
  int64_t K, rows, cols;
} tp_spectrum;

/* Where sampling probabilities come from (Section 3).
 *  TP_P_USER      caller-supplied non-negative weights w[n] (host or device
 *                 per the call's documentation), p_i = w_i / sum w.
 *  TP_P_UNIFORM   p_i = 1/n.
 *  TP_P_NORM2     p_j ~ ||A_{:j:}||_F^2, eq. nonoptimal_probs (lateral) or
 *                 ||A_{i::}||_F^2 (horizontal).
 *  TP_P_NORMPROD  p_j ~ ||A_{:j:}||_F ||B_{j::}||_F, eq. nearly_optimal_probs.
 *  TP_P_LEV       tubal leverage scores: lateral ||Vhat_{j::}||_F^2 from the
 *                 top-r right singular slices (eq. cur-col-prob); horizontal
 *                 ||Uhat_{i::}||_F^2 from the top-r left singular slices of C
 *                 (eq. colprob_rows_exact, read with the squared norm).
 *  TP_P_LEARNED   lateral slices only: the learned proposal of
 *                 tp_mlp_proposal (a network's estimate of the lateral
 *                 leverage scores, mixed with the uniform distribution), given
 *                 as a tp_mlp. Not in the paper; TP_P_LEV stays the
 *                 reference. */
typedef enum {
  TP_P_USER = 0, TP_P_UNIFORM = 1, TP_P_NORM2 = 2, TP_P_NORMPROD = 3, TP_P_LEV = 4, TP_P_LEARNED = 5
} tp_prob_kind;

/* The learned proposal's inputs (TP_P_LEARNED): params, the
 * tp_mlp_param_count() float32 network parameters; phi, the (n1 n3) x 16
 * float32 sketch matrix; alpha, the weight of the uniform distribution in
 * the mixture (see tp_mlp_proposal). Device pointers. */
typedef struct {
  const float* params;
  const float* phi;
  double alpha;
} tp_mlp;

/* How slices are picked.
 *  TP_S_BERNOULLI  Algorithm 2: slice i kept with probability min(1, c p_i),
 *                  scale 1/sqrt(min(1, c p_i)); ascending slice order; the
 *                  number kept is random (expected sum_i min(1, c p_i)).
 *  TP_S_IID        exactly c draws with replacement from p, scale
 *                  1/sqrt(c p_j); draw order.
 *  TP_S_UNIFORM    c distinct slices uniformly without replacement
 *                  (Corollaries cor:proj-main, cor:gnys-main), scale
 *                  sqrt(n/c); ascending order. It uses no weights, so the
 *                  decompositions accept it with TP_P_UNIFORM only.
 * Decisions are exact integer comparisons on weights quantised to
 * q_i = floor(w_i 2^(B-e)) (e the binary exponent of max w, B = 62 -
 * ceil(log2 n)) against Philox4x64-10 draws keyed by (seed, stream_id) at
 * counter (i or draw number, 0, 0, 0), word 0. */
typedef enum { TP_S_BERNOULLI = 0, TP_S_IID = 1, TP_S_UNIFORM = 2 } tp_sample_mode;

/* A device-resident pick: idx[0..*count) slice indices, scale[] their
 * rescaling factors; cap is the capacity of idx and scale. */
typedef struct {
  int32_t* idx;
  double* scale;
  int64_t cap;
  int64_t* count;
} tp_sample;

const char* tp_status_string(int status);
const char* tp_last_error(void);
/* Library version as major*10000 + minor*100 + patch. */
int tp_version(void);

/* ---------------------------------------------------------------------------
 * Fourier engine (Section 2.1 operators; the transforms of Algorithm 1).
 * ------------------------------------------------------------------------- */

/* Forward transform of every tube: Xh = first K slices of fft(X, [], 3).
 * Xh must be K x n1 x n2 with X's dtype. n3 >= 1. Tube lengths: any; even
 * lengths beyond one workgroup's LDS (float32 above 8192, float64 above
 * 4096) up to 2^19 with no prime factor above 13 (e.g. 500000) run a
 * four-step transform that uses Xh itself as its intermediate storage;
 * other lengths without a fast kernel fall back to a direct O(n3^2)
 * transform. The same holds for tp_tifft (which then uses X). */
int tp_tfft(const tp_tensor* X, tp_spectrum* Xh, void* stream);

/* Inverse transform: X = ifft of the conjugate-symmetric extension of Xh.
 * The imaginary parts of slice 0 and (n3 even) slice n3/2 are ignored, as
 * for a real signal they are zero. X is rows x cols x n3. */
int tp_tifft(const tp_spectrum* Xh, tp_tensor* X, void* stream);

/* Per-slice products of two spectra, C_k = op(A_k) op(B_k), k < K.
 * op_a / op_b: 0 = as stored, 1 = conjugate transpose. Slices 0 and (when
 * real_last != 0) K-1 are treated as real: their imaginary parts are neither
 * read nor computed, and C's are set to zero. `prec` selects the arithmetic
 * (TP_PREC_F64 needs TP_F64 spectra, the others TP_F32). */
int tp_spectrum_matmul(const tp_spectrum* A, int op_a, const tp_spectrum* B, int op_b, tp_spectrum* C,
                       int real_last, int prec, void* stream);

/* ---------------------------------------------------------------------------
 * Slice statistics (eqs. nearly_optimal_probs, nonoptimal_probs).
 * ------------------------------------------------------------------------- */

/* out[j] = ||A_{:j:}||_F^2 (mode 0, lateral, n2 values) or
 * out[i] = ||A_{i::}||_F^2 (mode 1, horizontal, n1 values), accumulated in
 * float64 in a fixed order. out is a device array of float64. */
int tp_slice_norms(const tp_tensor* A, int mode, double* out, void* ws, size_t ws_bytes, void* stream);
size_t tp_slice_norms_workspace(const tp_tensor* A, int mode);

/* ---------------------------------------------------------------------------
 * Sampling (the pick loops of Algorithms 2, 4 and 5).
 * ------------------------------------------------------------------------- */

/* Picks slices of a set of n candidates.
 *  kind TP_P_USER:     w is a device array of n float64 weights; A, B unused.
 *  kind TP_P_UNIFORM:  only n is used.
 *  kind TP_P_NORM2:    lateral slices of A (n = A->n2).
 *  kind TP_P_NORMPROD: lateral slices of A with horizontal slices of B
 *                      (n = A->n2 = B->n1).
 * c: 1 <= c <= n. out->cap must be >= c (TP_S_IID, TP_S_UNIFORM) or >= n
 * (TP_S_BERNOULLI). Weights must be finite, non-negative and not all zero;
 * for device weights this is checked on the device, and a violation yields
 * *count = -1. */
int tp_tsample(int kind, const tp_tensor* A, const tp_tensor* B, const double* w, int64_t n, int64_t c, int mode,
               uint64_t seed, uint64_t stream_id, tp_sample* out, void* ws, size_t ws_bytes, void* stream);
size_t tp_tsample_workspace(int64_t n);

/* tp_tsample without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses
 * that forbid allocation). Same arguments, checks, picks and errors as
 * tp_tsample; its scratch is a fixed 32 MiB device array inside the library
 * (tp_tsample_noalloc_max_bytes()), one per GPU, held until the process
 * ends. Sizes whose tp_tsample workspace (tp_tsample_workspace(n), plus the
 * slice-norm partials of A for TP_P_NORM2 / TP_P_NORMPROD) exceed it return
 * TP_EUNSUPPORTED. Calls on one GPU share that array: calls that overlap on
 * a GPU (other streams, unordered host threads) race; order them. The first
 * call on a device looks up the array's address there (no allocation). */
int tp_tsample_noalloc(int kind, const tp_tensor* A, const tp_tensor* B, const double* w, int64_t n, int64_t c,
                       int mode, uint64_t seed, uint64_t stream_id, tp_sample* out, void* stream);
size_t tp_tsample_noalloc_max_bytes(void);

/* ---------------------------------------------------------------------------
 * t-product (Algorithm 1) and rt-product (Algorithm 2).
 * ------------------------------------------------------------------------- */

/* C = A * B (sample == NULL), or C = (A*S*D) * (D*S^T*B) where S, D are the
 * picks in `sample` (the lateral slices idx of A and the matching
 * horizontal slices of B, each times scale; only the first *count entries
 * are used). A is n1 x n2 x n3, B is n2 x n4 x n3, C is n1 x n4 x n3, all of
 * the same dtype. prec: TP_PREC_F64 with TP_F64 data; TP_PREC_F32,
 * TP_PREC_BF16X3 or TP_PREC_BF16 with TP_F32 data. */
int tp_tprod(const tp_tensor* A, const tp_tensor* B, const tp_sample* sample, tp_tensor* C, int prec, void* ws,
             size_t ws_bytes, void* stream);
size_t tp_tprod_workspace(const tp_tensor* A, const tp_tensor* B, const tp_sample* sample, int prec);

/* ---------------------------------------------------------------------------
 * Randomized t-SVD and tubal leverage scores (Theorem "t-SVD", eq. circ1;
 * eqs. cur-col-prob and colprob_rows_exact).
 * ------------------------------------------------------------------------- */

/* Leading-r t-SVD of A by a range finder applied to every non-redundant
 * Fourier slice (Halko, Martinsson, Tropp 2011), with an
 * orthonormalisation through the float64 eigen-decomposition of the s x s
 * Gram matrix. The basis is
 *   slices == NULL: a Gaussian sketch of s = r + p columns (p rounded up so
 *                   that s is a multiple of 4 where the slices allow), then
 *                   q power iterations;
 *   slices != NULL: the picked lateral slices Chat_k = Ahat_k S D of
 *                   Definition t-CX / Algorithm 4 (s = slices->cap columns;
 *                   device picks as from tp_tsample, columns past *count are
 *                   zero), then q power iterations (q = 0: the rank-r
 *                   truncation of the t-CX projection C C^+ A). p unused.
 * Outputs (each may be NULL):
 *   S              device K x r float64 singular values of the Fourier
 *                  slices, descending;
 *   U              n1 x r x n3 (A's dtype): the first r left singular
 *                  slices;
 *   V              n2 x r x n3: the first r right singular slices;
 *   Z              A's shape: the tubal-rank-r approximation U * S * V^T
 *                  (the t-SVD theorem truncated to r);
 *   lev_lateral    device n2 float64 values ||Vhat_{j::}||_F^2 summed over
 *                  all n3 Fourier slices (the lateral leverage scores before
 *                  normalisation; they sum to r n3 when every slice has rank
 *                  >= r);
 *   lev_horizontal device n1 float64 values ||Uhat_{i::}||_F^2, likewise.
 * Directions whose eigenvalue is below 1e-6 (float32) or 1e-12 (float64)
 * of the slice's largest give zero columns. s <= 64 and r <= s; prec
 * TP_PREC_F64 (float64 data), TP_PREC_F32 or TP_PREC_BF16X3 (float32 data;
 * the small eigenproblems are float64 in every case). Gaussian sketches use
 * stream 2 of `seed`. Workspace: tp_tsvd_rand_workspace(A, r, p, slices,
 * prec) bytes. */
int tp_tsvd_rand(const tp_tensor* A, int64_t r, int64_t p, int32_t q, const tp_sample* slices, uint64_t seed,
                 int prec, double* S, tp_tensor* U, tp_tensor* V, tp_tensor* Z, double* lev_lateral,
                 double* lev_horizontal, void* ws, size_t ws_bytes, void* stream);
size_t tp_tsvd_rand_workspace(const tp_tensor* A, int64_t r, int64_t p, const tp_sample* slices, int prec);

/* ---------------------------------------------------------------------------
 * t-project and t-CX (Algorithms 3 and 4; Definition "t-CX", eq. ell2reg).
 * ------------------------------------------------------------------------- */

/* Z = C * C^+ * X (Algorithm 3): every Fourier slice of X projected onto the
 * range of the matching slice of C, as Q_k (Q_k^H Xhat_k) with Q_k an
 * orthonormal basis of the columns of Chat_k:
 *   c <= 64: CholeskyQR applied twice; a Cholesky pivot at or below 1e-7
 *            (float32) or 1e-13 (float64) of the largest drops its column,
 *            so repeated or dependent slices project onto the numerical
 *            range (float32 columns below ~3e-4 of the largest singular
 *            value of their slice are treated as dependent);
 *   c > 64:  float32 data with c <= min(n1, 4096): the left singular
 *            vectors of Chat_k from the block one-sided Jacobi on the rows of
 *            Chat_k^H (no squared condition number), keeping singular values
 *            above max(n1, c) eps_32 of the largest.
 * X n1 x n2 x n3, C n1 x c x n3, Z like X; one dtype; prec TP_PREC_F64
 * (float64) or TP_PREC_F32 / TP_PREC_BF16X3 (float32). Workspace:
 * tp_tproject_workspace(X, C, prec) bytes. */
int tp_tproject(const tp_tensor* X, const tp_tensor* C, tp_tensor* Z, int prec, void* ws, size_t ws_bytes,
                void* stream);
size_t tp_tproject_workspace(const tp_tensor* X, const tp_tensor* C, int prec);

/* t-CX (Algorithm 4) boosted by repetition: `rounds` independent draws of
 * exactly c lateral slices of A by col_kind (TP_P_USER with col_w, n2
 * device float64 weights; TP_P_UNIFORM; TP_P_NORM2; TP_P_LEV, lateral
 * leverage of the rank-r t-SVD as in tp_tcur), mode TP_S_IID or
 * TP_S_UNIFORM, round i from stream 16 i of `seed`; then Z = C * C^+ * A
 * with C the union of all picks. The projection onto the union is never
 * worse than any single round, which is how repetition boosts the success
 * probability of the relative-error bound. cols receives the picks round
 * after round (capacity >= c * rounds; *count = c * rounds, or -1 when the
 * weights are rejected, in which case Z is zero). The projection is that of
 * tp_tproject with c * rounds columns (more than 64: float32 data and
 * c * rounds <= min(n1, 4096)); r is used by TP_P_LEV only (r + 10 <= 64).
 * Workspace:
 * tp_tcx_workspace(A, c, rounds, r, col_kind, prec) bytes. */
int tp_tcx(const tp_tensor* A, int64_t c, int32_t rounds, int64_t r, int col_kind, const double* col_w, int mode,
           uint64_t seed, tp_sample* cols, tp_tensor* Z, int prec, void* ws, size_t ws_bytes, void* stream);
size_t tp_tcx_workspace(const tp_tensor* A, int64_t c, int32_t rounds, int64_t r, int col_kind, int prec);

/* ---------------------------------------------------------------------------
 * t-CUR (Definition "t-CUR", Algorithm 5).
 * ------------------------------------------------------------------------- */

/* Picks c lateral slices of A by col_kind and col_mode (TP_P_USER with
 * col_w, a device array of n2 float64 weights; TP_P_UNIFORM; TP_P_NORM2;
 * TP_P_LEV, lateral leverage of the rank-r t-SVD estimated as in
 * tp_tsvd_rand with p = 10, q = 1; TP_P_LEARNED with mlp), forms
 * Chat_k = Ahat_k S D, then picks l horizontal slices by row_kind and
 * row_mode (TP_P_USER with row_w, n1 weights; TP_P_UNIFORM; TP_P_NORM2 of A's
 * horizontal slices; TP_P_LEV, horizontal leverage of C from its top-r left
 * singular slices) and returns
 *     Z = ifft(Chat_k pinv_r(D S^T Chat_k) D S^T Ahat_k)
 * where pinv_r keeps the r leading singular values of every Fourier slice
 * of the core (and drops those <= max(l, c) eps sigma_1); the core is
 * computed in float64 by a range finder with 10 extra columns and 2 power
 * iterations. A TP_S_UNIFORM mode takes TP_P_UNIFORM only. The remark after
 * Corollary cor:gnys-main (lateral slices uniformly without replacement,
 * then horizontal leverage of those slices) is col_kind = TP_P_UNIFORM,
 * col_mode = TP_S_UNIFORM, row_kind = TP_P_LEV with row_mode TP_S_IID or
 * TP_S_BERNOULLI. Column picks use stream 0, row picks stream 1 of `seed`.
 * cols/rows receive the picks (capacity >= c and l, or n2 and n1 for
 * TP_S_BERNOULLI). core (may be NULL): the core Uhat_k = pinv_r(D S^T Chat_k)
 * of every non-redundant Fourier slice, a float64 spectrum of K x c x l
 * (n2 or n1 in place of c or l for Bernoulli picks; rows past the live pick
 * counts are zero). Z (same shape and dtype as A) may be NULL. With both
 * NULL only the picks are drawn. r <= min(c, l), r + 10 <= 64; mlp is read
 * for TP_P_LEARNED only (float32 data, n3 divisible by 4). */
int tp_tcur(const tp_tensor* A, int64_t c, int64_t l, int64_t r, int col_kind, const double* col_w, int col_mode,
            int row_kind, const double* row_w, int row_mode, const tp_mlp* mlp, uint64_t seed, tp_sample* cols,
            tp_sample* rows, tp_spectrum* core, tp_tensor* Z, int prec, void* ws, size_t ws_bytes, void* stream);
size_t tp_tcur_workspace(const tp_tensor* A, int64_t c, int64_t l, int64_t r, int col_kind, int col_mode,
                         int row_kind, int row_mode, int prec);

/* ---------------------------------------------------------------------------
 * Singular value thresholding, completion, robust PCA and CUR t-NN
 * (Algorithms 6-7; eqs. tnuc, tlow6, tlow7).
 * ------------------------------------------------------------------------- */

/* L = t-SVT(M, tau): in every Fourier slice, U max(Sigma - tau, 0) V^H, the
 * proximal map of tau times the tensor nuclear norm of eq. tnuc (both that
 * norm and the squared Frobenius norm carry 1/n3 in the Fourier domain, so
 * the slice threshold is tau itself). ranks (device, K int32 values, may be
 * NULL) receives the number of singular values above tau in each
 * non-redundant slice. The slice SVDs are computed exactly (block one-sided
 * Jacobi on the shorter side of the slices, until every row inner product
 * is below 1e-6 of the larger squared row norm, at most 30 sweeps).
 * unconverged (device, one int32, may be NULL) receives the number of
 * non-redundant slices whose sweeps reached that cap without meeting the
 * test (their L is still written, from the last rotations; 0 in normal
 * operation). float32 data, prec TP_PREC_F32. */
int tp_tsvt(const tp_tensor* M, double tau, tp_tensor* L, int32_t* ranks, int32_t* unconverged, int prec, void* ws,
            size_t ws_bytes, void* stream);
size_t tp_tsvt_workspace(const tp_tensor* M);

/* Dense leading-r t-SVD (the t-SVD theorem of Section 2.1) without the
 * range finder's 64-column limit. When the longer side of A's slices is at
 * most four times the shorter, the block one-sided Jacobi of tp_tsvt runs on
 * every Fourier slice A_k itself (on A_k^H, through the t-transpose, when
 * n1 > n2) and U_r comes from its accumulated rotations (or from the
 * orthogonalised rows divided by sigma). Longer slices use the Gram matrix
 * of the shorter side (A_k^H A_k when n1 > n2, A_k A_k^H otherwise,
 * float32): the same Jacobi diagonalises it and its r leading eigenvectors
 * give V_r (then U_r = A_k V_r Sigma_r^-1) or U_r directly. U (n1 x r x n3,
 * float32, caller-owned, overwritten) is the inverse transform: the first r
 * left singular slices of A, columns ordered by descending singular value
 * in every Fourier slice. S (device, K x r float64, K = n3/2 + 1; may be
 * NULL) receives the singular values. The Gram route squares the condition
 * number: there singular values below ~1e-3 of the largest lose accuracy in
 * float32 and those below ~3e-4 of it (the square root of float32 rounding)
 * are not resolved. A column whose singular value is exactly zero is zero.
 * unconverged (device, one int32, may be NULL) receives the number of
 * Fourier slices whose Jacobi sweeps reached their cap without converging,
 * as for tp_tsvt. A float32; 1 <= r <= min(n1, n2) <= 4096. Workspace:
 * tp_tsvd_full_workspace(A, r) bytes. */
int tp_tsvd_full(const tp_tensor* A, int64_t r, tp_tensor* U, double* S, int32_t* unconverged, void* ws,
                 size_t ws_bytes, void* stream);
size_t tp_tsvd_full_workspace(const tp_tensor* A, int64_t r);

/* Tensor completion by the ADMM of Algorithm 7 with the constraint
 * X = L + E, E zero on the observed entries (mask[i] != 0; X holds the
 * observed values, anything elsewhere). From L = E = Y = 0 and mu = mu0,
 * every iteration does
 *   L <- t-SVT(X - E - Y/mu, 1/mu); E <- P_unobserved(X - L - Y/mu);
 *   Y <- Y + mu (L + E - X);        mu <- min(rho mu, mu_max)
 * (the paper's values are rho = 1.1, mu0 = 1e-3, mu_max = 1e10), then
 * Algorithm 7's stop test when tol > 0: the loop ends after the first
 * iteration with max|L_{k+1} - L_k|, max|E_{k+1} - E_k| and
 * max|L_{k+1} + E_{k+1} - X| all <= tol (the paper uses 1e-8 in float64;
 * float32 iterates stall near 1e-7 of their scale). The three quantities
 * are formed on the device and read back after every iteration, so tol > 0
 * synchronises the stream once per iteration; reaching `iters` iterations
 * first returns TP_ENOCONV with the iterates written. tol <= 0 runs exactly
 * `iters` iterations without synchronising. L, E, Y are outputs (tube-major
 * float32, the shape of X); ranks (device, may be NULL) gets the last
 * iteration's per-slice ranks; iters_done (host, may be NULL) the number of
 * iterations run. Each iteration's slice SVDs start from the previous
 * iteration's left singular vectors. With tol <= 0 every iteration but the
 * first and the last spends at most two block Jacobi sweeps on them (the
 * rotations left undone resume in the next iteration; on the 256 x 256 x 100
 * completion workload L after 100 iterations is within 3e-4, relative, of a
 * loop whose thresholdings all converge); the last iteration converges, so L
 * is the exact t-SVT of its argument. With tol > 0 every iteration
 * converges. Workspace: tp_tcomplete_workspace(X). */
int tp_tcomplete(const tp_tensor* X, const uint8_t* mask, int32_t iters, double rho, double mu0, double mu_max,
                 double tol, tp_tensor* L, tp_tensor* E, tp_tensor* Y, int32_t* ranks, int32_t* iters_done, int prec,
                 void* ws, size_t ws_bytes, void* stream);
size_t tp_tcomplete_workspace(const tp_tensor* X);

/* Robust tensor PCA by Algorithm 7 as stated (eq. tlow7: minimise
 * ||L||_TNN + lambda ||E||_1 subject to X = L + E). From L = E = Y = 0 and
 * mu = mu0, every iteration does
 *   L <- t-SVT(X - E - Y/mu, 1/mu);
 *   E <- sign(V) max(|V| - lambda/mu, 0) with V = X - L - Y/mu;
 *   Y <- Y + mu (L + E - X);  mu <- min(rho mu, mu_max)
 * with the stop test, tol, iters_done, TP_ENOCONV and the sweep budget of
 * the intermediate iterations as for tp_tcomplete.
 * X, L, E, Y: tube-major float32 of one shape (caller-owned device buffers;
 * L, E, Y are overwritten); lambda > 0, or 0 for the default
 * 1/sqrt(max(n1, n2) n3) (the paper gives no value; this is the one of the
 * tensor robust PCA work eq. tlow7 comes from); ranks as for tp_tcomplete.
 * Workspace: tp_trpca_workspace(X) bytes. */
int tp_trpca(const tp_tensor* X, double lambda, int32_t iters, double rho, double mu0, double mu_max, double tol,
             tp_tensor* L, tp_tensor* E, tp_tensor* Y, int32_t* ranks, int32_t* iters_done, int prec, void* ws,
             size_t ws_bytes, void* stream);
size_t tp_trpca_workspace(const tp_tensor* X);

/* CUR t-NN (Algorithm 6): c lateral slices C of X picked by col_kind (as
 * for tp_tcur: TP_P_USER with col_w, TP_P_UNIFORM, TP_P_NORM2, or TP_P_LEV =
 * lateral leverage of X, eq. cur-col-prob), cleaned by the ADMM of
 * Algorithm 7 (Ct); l horizontal slices R of X picked by row_kind
 * (TP_P_LEV = horizontal leverage of Ct, eq. colprob_rows_exact; TP_P_NORM2
 * = squared norms of X's horizontal slices), cleaned likewise (Rt); then
 *     L = Ct * pinv_r(W) * Rt,   W = the picked horizontal slices of Ct,
 * with the rank-r pseudo-inverse of every Fourier slice computed as in
 * tp_tcur. The picked slices are used as they are (Algorithm 6 does not
 * rescale them); cols/rows receive the picks (their scales are written but
 * not used). mask != NULL: completion (eq. tlow6; X holds the observed
 * values, mask is tube-major uint8 of X's shape, nonzero where observed) and
 * lambda is ignored; mask == NULL: robust PCA (eq. tlow7) with weight
 * lambda > 0 (0: 1/sqrt(max(n1, n2) n3) of X), the same for C and R; both
 * ADMM runs take exactly `iters` iterations (with the sweep budget of
 * tp_tcomplete's fixed-count iterations). col_mode and row_mode are
 * TP_S_IID or TP_S_UNIFORM (exactly c and l picks; TP_S_UNIFORM with
 * TP_P_UNIFORM); 1 <= r <= min(c, l), r + 10 <= 64; float32 data, prec
 * TP_PREC_F32. L (float32, X's shape) is overwritten. Workspace:
 * tp_tcur_nn_workspace(X, c, l, r, col_kind, row_kind, mask != NULL). */
int tp_tcur_nn(const tp_tensor* X, const uint8_t* mask, double lambda, int64_t c, int64_t l, int64_t r, int col_kind,
               const double* col_w, int col_mode, int row_kind, const double* row_w, int row_mode, uint64_t seed,
               int32_t iters, double rho, double mu0, double mu_max, tp_sample* cols, tp_sample* rows, tp_tensor* L,
               int prec, void* ws, size_t ws_bytes, void* stream);
size_t tp_tcur_nn_workspace(const tp_tensor* X, int64_t c, int64_t l, int64_t r, int col_kind, int row_kind,
                            int masked);

/* ---------------------------------------------------------------------------
 * Learned lateral-leverage proposal (not in the paper; the exact scores of
 * eq. cur-col-prob stay its reference and fallback).
 * ------------------------------------------------------------------------- */

/* Launch tracing. tp_trace_enable(1) clears earlier records and starts
 * recording: each stage of a call (for the t-product "tprod.fft_a",
 * "tprod.fft_b", "tprod.gemm", "tprod.ifft", with the prefix "rtprod." when
 * picks are given) records a HIP event pair on the
 * caller's stream around its kernels. tp_trace_enable(2) does the same for
 * the per-slice product stages only (names ending in ".gemm"): each event
 * pair costs some device time, so a caller timing a whole step can keep the
 * pairs to the kernel it wants to see. tp_trace_enable(0) stops recording;
 * other values give TP_EINVAL.
 * tp_trace_count() waits for the recorded events, folds them into per-stage
 * totals and returns the number of stages; tp_trace_entry(i, ...) reports
 * stage i: its name (copied into name, name_cap bytes with the terminating
 * zero), the number of recorded calls and their summed duration in
 * milliseconds. Host-side bookkeeping only; the device work is unchanged. */
int tp_trace_enable(int on);
int tp_trace_count(void);
int tp_trace_entry(int i, char* name, size_t name_cap, int64_t* calls, double* total_ms);

/* Number of float32 parameters: W1 (17 x 128) | b1 (128) | W2 (128 x 128) |
 * b2 (128) | w3 (128) | b3 (1), with h1 = relu(x W1 + b1),
 * h2 = relu(h1 W2 + b2), o = h2 w3 + b3. */
int tp_mlp_param_count(void);

/* Per-lateral-slice features of a float32 tensor A (n3 % 4 == 0, any tube
 * length): the sketch s_j = Phi^T vec(A_{:j:}) (vec order i n3 + k; Phi a
 * caller-supplied device float32 (n1 n3) x 16 row-major matrix, e.g.
 * Gaussian / 4), whitened
 * as z_j = G^{-1/2} s_j sqrt(n2) with G = sum_j s_j s_j^T, followed by
 * log(n2 a_j / sum a), a_j = ||A_{:j:}||_F^2. feat: device n2 x 17 float32. */
int tp_mlp_features(const tp_tensor* A, const float* phi, float* feat, void* ws, size_t ws_bytes, void* stream);
size_t tp_mlp_features_workspace(const tp_tensor* A);

/* logits[r] = o for each of nrows feature rows (fp16 weights and activations
 * on the matrix cores, float32 accumulation). */
int tp_mlp_forward(const float* params, const float* feat, int64_t nrows, float* logits, void* stream);

/* One training step on ntensors tensors of nslices lateral slices each
 * (feat: (ntensors nslices) x 17 in tensor order; target: ntensors x nslices
 * nonnegative exact leverage scores, each row normalised to a distribution
 * inside the call, so any positive scale is accepted; a row summing to zero
 * is read as all-zero targets: zero loss, gradient softmax / ntensors). Loss:
 * mean over tensors of KL(target || softmax(logits of the tensor)). Writes
 * the loss (float, may be NULL) and the gradient (tp_mlp_param_count() float32 values,
 * may be NULL), then, if step >= 1, applies Adam (beta1 0.9, beta2 0.999, eps 1e-8,
 * bias correction with this step number) to params with moments m, v. */
int tp_mlp_train_step(float* params, float* m, float* v, int64_t step, double lr, const float* feat,
                      const float* target, int64_t ntensors, int64_t nslices, float* loss, float* grad, void* ws,
                      size_t ws_bytes, void* stream);
size_t tp_mlp_train_workspace(int64_t ntensors, int64_t nslices);

/* Sampling weights for the lateral slices of A from the network:
 * w = (1 - alpha) softmax(logits) + alpha / n2 (device float64, n2 values;
 * a defensive mixture: every slice keeps probability >= alpha / n2, so a
 * slice the network underrates is still reachable). One pass over A
 * (features), the forward pass and the mixture. Feed w to tp_tsample or
 * tp_tcur as TP_P_USER weights; the exact leverage kind stays the
 * reference. If any network output is not finite (diverged or corrupted
 * parameters), w is the uniform distribution 1 / n2 instead, so the picks
 * drawn from it stay valid (no host synchronisation is needed to detect
 * it; compare w with 1 / n2 to see it). */
int tp_mlp_proposal(const float* params, const tp_tensor* A, const float* phi, double alpha, double* w, void* ws,
                    size_t ws_bytes, void* stream);
size_t tp_mlp_proposal_workspace(const tp_tensor* A);

#ifdef __cplusplus
}
#endif

#endif /* TPROD_H */
