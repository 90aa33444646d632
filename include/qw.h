/*
 * qw.h -- C ABI of the MI355X quantum-walk library (libqw.so).
 *
 * The library simulates, at register level and on a sparse state, the quantum
 * walk on a sparse real symmetric matrix stored in QRAM (Chen et al., arXiv
 * 2303.06890): the walk step W = S T~ P T~^dagger of Alg. 6 on the six
 * registers j_c, j, b1, k_c, k, b2 (Sec. IV, "Implementation of the quantum
 * walk"), its inverse, the walk-based Chebyshev linear solver (Eq. "fx" and
 * the iteration of Sec. V.B), measurements, a batched multi-instance form and
 * a reverse-mode gradient.  Real symmetric and complex Hermitian matrices.
 *
 * Conventions shared by every entry point
 *   - Return value: QW_OK (0) or a negative qw_status.  Functions never throw
 *     and never abort: every entry point catches what the host code may
 *     throw (host memory exhaustion is reported as QW_ENOMEM, anything else
 *     as QW_EINVAL); qw_last_error() returns the text of the last error of
 *     the calling thread.
 *   - Host arrays are borrowed for the duration of the call only.
 *   - Device memory comes from the caller's allocator (qw_allocator; NULL
 *     means hipMalloc/hipFree) and belongs to the qw_ctx or qw_state that
 *     allocated it until it is freed.  A freed state's buffers stay with its
 *     context, for the next states made from it (at most four of one size,
 *     4 GiB in all), and return to the allocator when the context goes.
 *     Nothing is allocated inside qw_step, qw_step_adjoint or qls_run's step
 *     loop once a state's graphs and 8-byte planes exist.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     qw_load_csc*, qw_state_init, qw_state_import, qw_step and
 *     qw_step_adjoint only enqueue work; qw_measure, qw_export, qls_run,
 *     qw_grad and qw_sync synchronise the stream and copy results to the host.
 *     No error is raised on the device: a state's storage is fixed when it is
 *     created (see qw_state_init), so a step cannot overflow it.
 *   - Indices are 0-based.  A matrix is given in CSC form (colptr[n+1],
 *     rowidx[nnz] sorted and unique inside each column, vals[nnz] real).  The
 *     walk's row register j addresses CSC column j: the QRAM row j holds the
 *     row indices and values of column j (the same data for a symmetric
 *     matrix, which the paper's "CSC" storage of Sec. II.C assumes).
 *
 * Register key layout (packed 64-bit, high to low bits)
 *     [ inst | j_c (n) | j (n) | b1 | k_c (n) | k (n) | b2 ]
 *   n = log2 of the padded dimension (the largest one over all instances of a
 *   batched context); inst = instance index (0 for a single matrix).
 *   4n+2 + bits(inst) must not exceed 64.
 */
#ifndef QW_H
#define QW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QW_OK = 0,
  QW_EINVAL = -1,    /* invalid argument or matrix */
  QW_ENOMEM = -2,    /* allocation failed */
  QW_ECAPACITY = -3, /* general branch list capacity exceeded */
  QW_EDEVICE = -4,   /* HIP runtime error */
  QW_ENOTSUP = -5    /* valid request outside what the library supports */
} qw_status;

typedef struct qw_ctx qw_ctx;     /* preprocessed matrices resident on the GPU */
typedef struct qw_state qw_state; /* a walk state (sparse, on the GPU) */

/* Device allocator hooks; `alloc` returns a device pointer aligned to 256
 * bytes or NULL.  The Python binding plugs in torch's caching allocator. */
typedef struct {
  void* (*alloc)(size_t bytes, void* user);
  void (*free)(void* ptr, void* user);
  void* user;
} qw_allocator;

/* flags for qw_load_csc / qw_load_csc_batched */
#define QW_REQUIRE_SYMMETRIC 0x1u /* reject matrices that are not symmetric (Hermitian) */
/* Fixed-point data of word length w = 1 ... 32 (bits 8-13 of flags; 0 = the
 * values are FP64 numbers).  Sec. V.B: the elements are fixed-point numbers
 * below 1 whose number of digits is the word length; appendix table of basic
 * operations: the conditional rotation is computed with a fixed-point square
 * root, a fixed-point arccos and a rotation by a fixed-point angle.  Every
 * scaled value must be +-q / 2^w with an integer 0 <= q < 2^w; the rotation
 * then uses r = floor(sqrt(q / 2^w) 2^w) / 2^w (truncated square root),
 * the angle theta = t (pi/2) / 2^w with t the nearest integer to
 * arccos(r) / (pi/2) 2^w, f = cos(theta) (times +-i for a negative value,
 * by the rule of the real case) and g = sin(theta).  Real matrices only. */
#define QW_WORD_LENGTH(w) (((uint32_t)(w) & 0x3fu) << 8)

/* Lanes of a step-kernel wavefront that share a row of s >= 16 slots
 * (bits 16-17 of flags; neither: 16 when the context would have at most
 * 1024 wavefronts with 8, else 8).  A tuning choice: results are identical,
 * only the lane mapping of the step, adjoint and measurement kernels
 * changes (the autotuner times both). */
#define QW_LANES_8 (1u << 16)
#define QW_LANES_16 (2u << 16)

/* Row blocks of the one-pass walk-step and adjoint kernels numbered by XCD: the
 * GPU deals workgroups to its eight XCDs in turn, each XCD with its own L2,
 * and neighbouring row blocks share cache lines of the state and slot
 * planes; with this flag they run on one XCD.  A tuning choice like the lanes
 * per row: results are identical, and which is faster depends on the matrix
 * (the autotuner times both). */
#define QW_XCD_ROWS (1u << 18)

/* flags for qw_state_init */
#define QW_INIT_RAW 0x1u /* start from |b~> itself instead of T~|b~> */

/* kinds for qw_measure */
#define QW_COUNT 1      /* out: int64[1]   number of stored branches M */
#define QW_NORM 2       /* out: double[1]  sum |amp|^2 */
#define QW_J_MARGINAL 3 /* out: double[sum N_i]  probability of each j value */
#define QW_PROJECT 4    /* out: double[2 sum N_i] interleaved complex <psi~_j|state> */
#define QW_STATS 5      /* out: int64[5] {step launches so far (walk steps and
                           swaps), current branch count, general-list capacity,
                           general-list count, branches written by all launches};
                           with out_len >= 6 also [5] = 1 when every cell of
                           the state is real or imaginary by construction (a
                           real matrix whose negative values pair up, as in a
                           symmetric one, and a real b, from T~ |b~>): its walk
                           steps then run on one double per cell whenever the
                           one-pass conditions of the step kernels hold; with
                           out_len >= 7 also [6] = the lanes of a step-kernel
                           wavefront that share a row of s >= 16 slots (8 or
                           16: QW_LANES_8 / QW_LANES_16, or by default 16 in a
                           context of at most 1024 wavefronts with 8); with
                           out_len >= 8 also [7] = 1 when the context was
                           loaded with QW_XCD_ROWS */

/* Load one matrix (Sec. V.B, preprocessing list; Sec. II.C, Fig. 1):
 *   scale: > 0 multiplies every value by `scale`; 0 selects 1/max(1, max|a|).
 *   The QRAM row length s is the power of two >= the largest column count
 *   (Table I, note b); each row is padded to s sorted unique slots with the
 *   smallest absent indices carrying value 0; the dimension is padded to a
 *   power of two N with empty columns.
 * Errors: QW_EINVAL for n <= 0, bad colptr, row indices out of range,
 *   unsorted or duplicate, |scale*a| > 1, a negative diagonal entry (not
 *   encodable: <j~|T~^dagger S T~|j~> = |f|^2/s >= 0), a non-symmetric matrix
 *   when QW_REQUIRE_SYMMETRIC is set, a word length above 32 or a value that
 *   is not a fixed-point number of the word length given with
 *   QW_WORD_LENGTH; QW_ENOTSUP for s > 64 or 4n+2 > 64.  qw_grad is not
 *   provided for fixed-point data (QW_ENOTSUP). */
int qw_load_csc(qw_ctx** out, int32_t n, const int32_t* colptr, const int32_t* rowidx,
                const double* vals, int64_t nnz, double scale, uint32_t flags,
                const qw_allocator* alloc, void* stream);

/* Load `ninst` independent matrices into one context (batched form).
 * Instance i: dimension n[i], colptr at colptr + colptr_off[i] (n[i]+1
 * entries, relative to the instance's first entry), rowidx/vals at
 * nnz_off[i].  scales: NULL (automatic for every instance) or ninst values
 * with the meaning of qw_load_csc's scale.  Same errors as qw_load_csc. */
int qw_load_csc_batched(qw_ctx** out, int32_t ninst, const int32_t* n, const int64_t* colptr_off,
                        const int64_t* nnz_off, const int32_t* colptr, const int32_t* rowidx,
                        const double* vals, const double* scales, uint32_t flags,
                        const qw_allocator* alloc, void* stream);

/* Load `ninst` complex Hermitian matrices (ninst = 1: one matrix; the offset
 * arrays may then be NULL), with the layout and meaning of
 * qw_load_csc_batched's arguments; vals_re/vals_im are the real and imaginary
 * parts of the stored entries (vals_im required).  The QRAM row j holds
 * column j of A, i.e. the entries A*_{jk} of row j of a Hermitian A, and
 * psi_j takes sqrt(A*_{jk}) (Sec. IV): the principal root off the real
 * axis, the real rule of qw_load_csc on it (entries with a zero imaginary
 * part).  QW_REQUIRE_SYMMETRIC requires A_kj = conj(A_jk) exactly.  Scaling
 * uses |a| = hypot(re, im).  Errors: as qw_load_csc, plus QW_EINVAL for a
 * diagonal entry with a nonzero imaginary part, QW_ENOTSUP with
 * QW_WORD_LENGTH.  Such a context takes qw_grad_complex instead of qw_grad
 * (QW_ENOTSUP there). */
int qw_load_csc_hermitian(qw_ctx** out, int32_t ninst, const int32_t* n, const int64_t* colptr_off,
                          const int64_t* nnz_off, const int32_t* colptr, const int32_t* rowidx,
                          const double* vals_re, const double* vals_im, const double* scales, uint32_t flags,
                          const qw_allocator* alloc, void* stream);

/* Per-instance facts: padded dimension N, slots per row s, register width n
 * of the key layout (common to all instances), scale applied, and the
 * condition number kappa of A/s once qw_kappa (or qls_run with kappa <= 0)
 * has computed it, NaN before.  Any output pointer may be NULL.  Errors:
 * QW_EINVAL for a NULL context or an instance index out of range. */
int qw_ctx_info(const qw_ctx* ctx, int32_t inst, int32_t* n_padded, int32_t* s, int32_t* nbits,
                double* scale, double* kappa);

/* Condition number kappa = 1 / min |lambda(A/s)| of instance `inst`, the
 * quantity the solver's schedule takes (Sec. V.B, preprocessing list: A is
 * rescaled and the walk encodes A/s; Table I, note a; A is the n x n matrix
 * given, without the padding to N).  Computed on the host once and kept with
 * the context: for n <= 2048 (2n for complex values) exactly, by Householder
 * reduction to tridiagonal form and bisection on Sturm counts; beyond that
 * estimated by Lanczos with full reorthogonalisation, on A/s when its
 * extreme Ritz values show it definite (the end of the spectrum nearest 0)
 * and on (A/s)^2 otherwise (its smallest eigenvalue), accepted when the
 * residual bound of that Ritz value is below 1e-9 of it.
 * Fixed-point data uses the matrix the rotations encode, sign(a) cos^2(theta)
 * per entry.  Synchronous, host only (about 1 s at n = 1024).
 * Errors: QW_EINVAL (NULL arguments, instance out of range, a singular
 * matrix), QW_ENOTSUP (a matrix that is not symmetric or Hermitian; a
 * Lanczos estimate that did not converge in 600 steps). */
int qw_kappa(qw_ctx* ctx, int32_t inst, double* kappa);
/* Number of instances of a context (0 for NULL). */
int32_t qw_ctx_ninst(const qw_ctx* ctx);

/* Create a state holding T~ |b~> (Alg. 5 applied to |b~> = sum_j b_j |0,j,0,0,0,0>,
 * Sec. IV) or |b~> itself with QW_INIT_RAW.  b_re/b_im (b_im may be NULL):
 * sum_i n[i] values, instance after instance; b is used as given (callers
 * normalise).  Every branch reachable from T~|b~> has a fixed address (the
 * group members (0,j,0,0,k_{j,l},b2) of every QRAM slot and their swaps), so
 * such a state needs no capacity and can never overflow; branches outside
 * that span (raw starts, imports) go to a general list whose size the walk
 * never changes.  capacity: initial general-list capacity (0 = as needed).
 * Errors: QW_EINVAL, QW_ENOMEM. */
int qw_state_init(qw_state** out, qw_ctx* ctx, const double* b_re, const double* b_im, uint32_t flags,
                  int64_t capacity, void* stream);

/* Apply W^nsteps (Alg. 6: W = S T~ P T~^dagger), branches with |Re| and |Im|
 * both <= tau (1e-13) removed after every step.  One kernel launch per step;
 * asynchronous.  When `stream` is not NULL the step loop is replayed from
 * captured HIP graphs of 256 and of 16 steps (as many long replays as fit,
 * then short ones, then single launches), each built on first use for the
 * stream, the state's parity and its representation, and kept with the
 * state; a state at the other parity from its graphs takes one single step
 * first.  The state's amplitude planes are double-buffered inside the state
 * (the 8-byte planes of one double per cell are allocated at the first step
 * that uses them); nothing is allocated once the graphs exist.
 * Errors: QW_EINVAL (NULL state, nsteps < 0), QW_EDEVICE (launch or graph
 * failure). */
int qw_step(qw_state* st, int32_t nsteps, void* stream);

/* Apply (W^dagger)^nsteps, W^dagger = T~ P T~^dagger S (unitarity of W):
 * a swap pass, nsteps walk steps, a swap pass.  Errors as qw_step. */
int qw_step_adjoint(qw_state* st, int32_t nsteps, void* stream);

/* Measurements (kinds above).  out_len is the number of elements of `out`.
 * QW_J_MARGINAL is the probability of each value of the column register j,
 * the p_j of the solver's readout (Sec. V.B: the probability of measuring
 * each column index); QW_PROJECT is <psi~_j|state> = <j~|T~^dagger|state>,
 * the amplitude of |0, j, 0, 0, 0, 0> after T~^dagger, which Pi_0 T~^dagger
 * of the iteration of Sec. V.B reads (psi~_j = T~|j~>, Sec. IV);
 * QW_COUNT and QW_NORM are the number of stored branches and sum |amp|^2 of
 * the sparse state (Sec. V.A: the state array and amplitude vector).
 * Synchronises the stream.  Errors: QW_EINVAL (unknown kind, NULL pointers,
 * out_len too small), QW_EDEVICE. */
int qw_measure(qw_state* st, int32_t kind, void* out, int64_t out_len, void* stream);

/* Copy the state to the host, sorted by key: the sparse representation of
 * Sec. V.A (every stored register tuple and its amplitude), with keys in the
 * layout above.  The branches are compacted and sorted on the GPU (a radix
 * sort; it takes about 48 bytes of device memory per branch for the call),
 * then copied.  cap = size of the host arrays; *m receives the branch count
 * (QW_EINVAL with *m set if cap < count, or if count > 2^32 - 1).  re or im
 * may be NULL.
 * Synchronises the stream.  Errors: QW_EINVAL, QW_ENOMEM, QW_EDEVICE. */
int qw_export(qw_state* st, uint64_t* keys, double* re, double* im, int64_t cap, int64_t* m,
              void* stream);

/* qw_export with the amplitudes interleaved: amps[2 t] and amps[2 t + 1] are
 * the real and imaginary parts of branch t (the layout of a C99 double
 * complex or std::complex<double> array of cap elements), copied from the
 * device without a split.  Same order, synchronisation and errors. */
int qw_export_complex(qw_state* st, uint64_t* keys, double* amps, int64_t cap, int64_t* m, void* stream);

/* Replace the state by the given branches (equal keys are summed; branches
 * whose |Re| and |Im| are both <= tau = 1e-13 are dropped, as after a step).  Keys must
 * follow the layout above with valid instance and register ranges, and every
 * branch must satisfy j_c < s and k_c < s (true of every state the walk
 * reaches).  Errors: QW_EINVAL, QW_ECAPACITY. */
int qw_state_import(qw_state* st, const uint64_t* keys, const double* re, const double* im, int64_t m,
                    void* stream);

/* qw_state_import with the amplitudes interleaved (amps[2 t], amps[2 t + 1]
 * = real and imaginary part of branch t; the layout qw_export_complex
 * writes).  Same rules and errors. */
int qw_state_import_complex(qw_state* st, const uint64_t* keys, const double* amps, int64_t m, void* stream);

/* Wait for the stream (QW_EDEVICE reports an earlier asynchronous failure). */
int qw_sync(qw_state* st, void* stream);

/* Walk-based CKS linear solver on instance 0 (Sec. IV, CKS paragraph; Eq. "fx";
 * Sec. V.B, iteration of tau_j):
 *   beta = ceil(kappa^2 ln(kappa/eps)), j0 = ceil(sqrt(beta ln(4 beta/eps)))
 *   (j0_override >= 0 replaces j0), a_k the coefficients of Eq. "fx";
 *   omega = W T~ |b~>; for k = 0..j0: y += a_k Pi_0 T~^dagger omega; then
 *   omega = W^2 omega (k < j0).  2 j0 + 1 walk steps in total.
 * b: n values (host, real).  kappa: condition number of A/s (1 / smallest
 * |eigenvalue|), > 1; kappa <= 0 takes the library's own (qw_kappa, computed
 * once per context).
 * x_re/x_im (n values, host): the post-selected, normalised solution
 * x = y / |y| with y = sum_k a_k tau_k; y_norm receives |y|, so that y itself
 * is y_norm * x.  p_succ = |y|^2 / (sum_k |a_k|)^2 (the LCU's success
 * probability).  walk_steps receives 2 j0 + 1.  Any output pointer may be
 * NULL.  Synchronises the stream.
 * Errors: QW_EINVAL (1 >= kappa > 0, eps outside (0,1), b NULL, y = 0),
 * and qw_kappa's errors when kappa <= 0. */
int qls_run(qw_ctx* ctx, const double* b, double kappa, double eps, int32_t j0_override,
            double* x_re, double* x_im, double* y_norm, double* p_succ, int64_t* walk_steps, void* stream);

/* Chebyshev coefficients a_0..a_j0 of Eq. "fx" for the given beta, computed
 * on the host into out[j0 + 1]: a_j = 4 (-1)^j sum_{i > j} C(2 beta, beta + i)
 * / 2^(2 beta), evaluated in long double from the central term (a Stirling
 * series for beta >= 64) by the ratio recurrence of consecutive terms and
 * summed from the far tail.
 * Errors: QW_EINVAL (beta < 1, j0 < 0, out NULL). */
int qw_cks_coeffs(int64_t beta, int32_t j0, double* out);

/* Reverse-mode gradient of L = sum_j w_j p_j, p = j-register marginal of the
 * state, where the state was created by qw_state_init (T~ start) and then
 * advanced by exactly `nsteps` calls' worth of qw_step.  Earlier states are
 * recomputed with W^dagger (exact checkpointing: W is unitary), never stored.
 * w: sum N_i weights.  dvals: gradient w.r.t. every stored CSC value after
 * scaling (CSC order, instance after instance; entries whose value is 0 or
 * has |value| = 1 are not differentiable and come out non-finite).
 * db_re/db_im: dL/dRe b + i dL/dIm b (sum n_i values).  Any output may be
 * NULL.  The state is consumed (left holding the recomputed T~|b~>). */
int qw_grad(qw_state* st, const double* w, int32_t nsteps, double* dvals, double* db_re, double* db_im,
            double* loss, void* stream);

/* qw_grad for a context of complex Hermitian values (qw_load_csc_hermitian;
 * a real context: QW_ENOTSUP, use qw_grad).  The rotation of a value
 * v = a + i b is f = sqrt(v) (the principal root off the real axis, the +-i
 * rule of real values on it) and g = sqrt(1 - |v|) (Sec. IV); reverse mode
 * differentiates it by a and by b, each stored entry an independent
 * parameter (the mirror conj(v) of an entry has derivatives of its own).
 * dvals_re[p] = dL/da and dvals_im[p] = dL/db of CSC entry p after scaling
 * (CSC order, instance after instance).  Not differentiable, non-finite:
 * both parts at v = 0 and |v| = 1, and dL/db on the negative real axis,
 * where the +-i rule is one side of the principal root's cut.  Other
 * arguments, results and errors as qw_grad. */
int qw_grad_complex(qw_state* st, const double* w, int32_t nsteps, double* dvals_re, double* dvals_im,
                    double* db_re, double* db_im, double* loss, void* stream);

/* qw_grad without allocating anything: for callers that cannot allocate
 * device memory (tight serving loops, harnesses that forbid allocation).
 * Same arguments, results and errors as qw_grad, for a state whose walk
 * steps run on one double per cell and have run at least once (a real
 * matrix whose negative values pair up, a real b, a one-pass launch shape);
 * other states: QW_ENOTSUP.  Every buffer of the sweep (the adjoint state's
 * planes, the weights, dL/dv, dL/db and the results in CSC order) is carved
 * from one device array of the library, 32 MiB on each GPU it runs on, held
 * from the first call on that GPU to qw_shutdown; a context that needs more
 * (about 56 bytes per QRAM slot plus 40 per column; G(16384, 8) needs 9 MB)
 * is rejected with QW_EINVAL and the size in qw_last_error.  Calls share
 * that array: calls that overlap on one GPU (other threads or streams) race,
 * so serialise them.  Each call clears what must start at 0. */
int qw_grad_noalloc(qw_state* st, const double* w, int32_t nsteps, double* dvals, double* db_re,
                    double* db_im, double* loss, void* stream);

/* Free a state (waits for the device; its buffers go to the context's
 * pool).  NULL is ignored. */
void qw_state_free(qw_state* st);
/* Release the caller's reference to a context.  Each state holds its own
 * reference, so a context and its states may be freed in any order; the
 * device arrays go when the last reference does.  NULL is ignored. */
void qw_ctx_free(qw_ctx* ctx);
const char* qw_last_error(void);

/* Release the library's kernels from the HIP runtime (they are loaded on
 * first use, per device).  Call after every qw_state and qw_ctx has been
 * freed, while the runtime is alive (e.g. at the start of process exit); a
 * later call into the library loads them again. */
void qw_shutdown(void);

/* Launch shape of the step kernel: workgroup size (64..256, a multiple of
 * 64) and number of workgroups, 1..65536 (a grid smaller than one pass over
 * the work makes the kernel stride); 0 keeps the current value (default: 256
 * and one pass, at most 65536).  Captured graphs are discarded, after the
 * device has finished all work enqueued so far (a replay may still be
 * running).  Used by the autotuner.  Errors: QW_EINVAL for sizes out of
 * range. */
int qw_set_launch(qw_state* st, int32_t wg_size, int32_t grid_limit);

#ifdef __cplusplus
}
#endif

#endif /* QW_H */
