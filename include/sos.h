/*
 * sos.h -- C ABI of libsos: the loss, gradient and first-order loop of the
 * over-parameterised sum-of-squares method (Keren, Osadchy, Poranne,
 * "A practical, fast method for solving sum-of-squares problems for very
 * large polynomials"), on one AMD Instinct MI355X (gfx950).
 *
 * The problem (Section 1.1, eq. basicsos and eq. nonconvex): a polynomial p
 * of degree 2d in n variables is a sum of squares iff p = m_d^T G m_d for a
 * PSD Gram matrix G, m_d being the vector of all monomials of degree <= d.
 * Writing G = W W^T with an unconstrained N x k factor W, the method
 * minimises
 *
 *     L(W) = || coeff(m_d^T W W^T m_d) - p ||^2
 *
 * in coefficient space with Adam (Section 3), using a full-rank, over-
 * parameterised W (Section 1.3).
 *
 * Conventions used by every entry point:
 *   - Basis order: all monomials of degree <= d, higher total degree first,
 *     then lexicographically larger exponent vector first with x1 most
 *     significant (the order of the n = d = 2 example of Section 1.1).
 *     N = C(n+d, d).  Coefficient monomials (degree <= 2d) use the same
 *     order; M = C(n+2d, 2d) and p, r, c are indexed by it.
 *   - coeff(G)_beta = sum over ORDERED pairs (i, j) with alpha_i + alpha_j =
 *     beta of G_ij.  The residual is r = coeff(W W^T) - p, the loss
 *     L = ||r||^2 (not normalised, Section 3), the gradient 4 R W with
 *     R_ij = r[rank(alpha_i + alpha_j)].
 *   - W is N x k, row-major (row i = basis monomial i, column l = square l),
 *     leading dimension k.  Its element type is double for SOS_FP64 and
 *     float for every other precision (an FP32 master copy).
 *   - d_* arguments are device pointers owned by the caller; h_* are host
 *     pointers.  The library never allocates device memory: the caller
 *     provides a workspace (sos_plan_bind) and per-problem optimiser state.
 *   - `stream` is a hipStream_t passed as void* (NULL: the null stream).
 *     Device work is enqueued on it; only sos_plan_bind, sos_solve,
 *     sos_verify and sos_exponents block the host.
 *   - Return value: SOS_OK (0), a positive status, or a negative error.  On
 *     error sos_last_error() returns a message (thread-local).  Arguments
 *     are validated before anything is enqueued.  No entry point aborts the
 *     process or throws across the ABI.
 *   - A plan's workspace holds scratch of the call in flight: calls that
 *     use one plan must be ordered (one stream, or synchronised); separate
 *     plans may run concurrently.
 */
#ifndef SOS_H
#define SOS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sos_plan_s* sos_plan_t;

/* Arithmetic of the two contractions (Gram forward, R W backward).  The
 * residual r, the loss and the certificate are FP64 in every mode.        */
enum sos_precision {
  SOS_FP64 = 0,    /* W double; FP64 MFMA for both contractions            */
  SOS_FP32 = 1,    /* W float;  FP32 MFMA for both contractions            */
  SOS_BF16X3 = 2,  /* W float master; each operand split into bf16 hi + lo,
                      three bf16 MFMA products (hi*hi + hi*lo + lo*hi) with
                      FP32 accumulation                                    */
  SOS_FP16X3 = 3,  /* as SOS_BF16X3 with fp16 halves (11 significant bits
                      each against bf16's 8, at the same MFMA rate).  fp16
                      has a narrow exponent range, so the W copies are
                      scaled by 2^sW (2^sW max|W| < 2^12, set when the
                      copies are built from W and kept by the fused steps:
                      W may grow 16x before the copies overflow) and R by
                      2^sR (2^sR max|r| < 2^14, every step); the GEMM
                      epilogues divide the powers of two out exactly.
                      Halves below fp16's normal range keep an absolute
                      error of 2^-25 in scaled units.                      */
};

enum sos_status {
  SOS_OK = 0,
  SOS_NOT_CONVERGED = 1, /* sos_solve: budget spent before the target      */
  SOS_EINVAL = -1,       /* bad argument                                   */
  SOS_ERANGE = -2,       /* problem outside the supported sizes            */
  SOS_ENOMEM = -3,       /* workspace too small                            */
  SOS_EHIP = -4,         /* HIP runtime error                              */
  SOS_ENUMERIC = -5,     /* loss became NaN or Inf                         */
};

/* Flags for sos_loss_grad / sos_step. */
enum sos_flags {
  /* Forward in FP64: the FP32 master W is converted exactly to FP64 and the
   * Gram tiles use FP64 MFMA.  Used to reach residuals below the FP32 or
   * split-bf16 floor; ignored for SOS_FP64 (already exact).               */
  SOS_FLAG_EXACT_FORWARD = 1,
  /* sos_step only, a promise by the caller: W has not been modified since
   * the previous sos_step on this plan returned.  A SOS_BF16X3 step with
   * SOS_FLAG_SINGLE_BACKWARD (fast or exact forward) updates W inside the
   * backward GEMM's epilogue and writes there the operand copies the next
   * step reads; with this flag the next step on the same W pointer and
   * forward mode skips rebuilding them.  Ignored whenever the library holds
   * no such copies (other modes, another call on the plan in between).    */
  SOS_FLAG_COPIES_VALID = 2,
  /* SOS_BF16X3 and SOS_FP16X3: the backward takes one 16-bit product per
   * element pair (hi * hi) instead of three.  The gradient 4 R W then
   * carries a relative error of about 2^-8 (bf16) or 2^-11 (fp16) per term;
   * it still vanishes where R does (at an exact fit), so the fixed point is
   * unchanged.  Ignored for other modes.                                   */
  SOS_FLAG_SINGLE_BACKWARD = 4,
  /* SOS_BF16X3 and SOS_FP16X3: forward with FP32 MFMA on the FP32 master W
   * (between the split forward and the FP64 one in accuracy and cost).
   * SOS_FLAG_EXACT_FORWARD takes precedence.                              */
  SOS_FLAG_FP32_FORWARD = 8,
  /* SOS_FP32 and SOS_BF16X3 plans: an FP64-accurate forward from int8
   * MFMA (Ozaki splitting, Ozaki-Ogita-Oishi-Rump 2012).  Each row of W is
   * scaled by a power of two and cut into 6 signed 7-bit digit slices; the
   * slice products of levels s + t < 6 are summed exactly in int32, the
   * levels combined in FP64.  Per Gram entry the error is at most
   * 7.05 * 2^-42 * rank * 2^(e_i + e_j), 2^e_i being the least power of two
   * above row i's largest magnitude (plus FP64 rounding), so it reaches the
   * residuals the exact forward reaches, on matrix cores of twice the BF16
   * rate.  SOS_ERANGE when rank exceeds 87,360 (the int32 level sums would
   * overflow); SOS_EINVAL for SOS_FP64 plans.  SOS_FLAG_EXACT_FORWARD takes
   * precedence.  sos_verify keeps the FP64-MFMA forward.                  */
  SOS_FLAG_OZAKI_FORWARD = 16,
  /* SOS_FP32 and SOS_FP64 plans with N <= SOS_BATCH_MAX_N, the plan's own
   * forward only: instead of adding each Gram entry into r by FP64 atomics
   * (whose order varies from run to run), the gram stores its tiles (one
   * copy per contraction slice) and each coefficient then sums its pairs in
   * the plan's fixed pair order.  Results then depend on W and p alone:
   * repeated runs, and a run resumed from a checkpoint, follow the same
   * trajectory bit for bit.  SOS_EINVAL for other plans or with
   * SOS_FLAG_EXACT_FORWARD / SOS_FLAG_OZAKI_FORWARD on an FP32 plan.      */
  SOS_FLAG_DETERMINISTIC = 32,
  /* SOS_BF16X3 plans, fast forward, a measurement variant: the gram stores
   * its FP32 tiles (256 x 256 per upper tile, in the workspace) instead of
   * scattering them in its epilogue, and a separate kernel (timing class
   * SOS_K_SCATTER) ranks and adds them into r.  Same result as the fused
   * forward up to the order of the FP64 additions; slower.                */
  SOS_FLAG_UNFUSED_SCATTER = 64,
  /* SOS_BF16X3 and SOS_FP16X3 plans, fused fast forward, a measurement
   * variant: the gram's epilogue ranks each Gram entry and adds it into r by
   * its own FP64 atomic, as the allocation-free entry point does, instead
   * of first merging the entries of each 64 x 256 segment that share a
   * coefficient in LDS (the merge maps that sos_plan_bind builds).  Same
   * result up to the order of the FP64 additions; slower.                 */
  SOS_FLAG_UNMERGED_SCATTER = 128,
  /* With SOS_FLAG_OZAKI_FORWARD: 5 digit slices instead of 6 (levels
   * s + t < 5: 15 slice products instead of 21, about 0.7x the time).  Per
   * Gram entry the error is then at most 6.05 * 2^-35 * rank * 2^(e_i + e_j)
   * plus FP64 rounding, about 128x the six-slice figure; for Gaussian rows
   * the coefficients come out within ~3e-10 of ||coeff(W W^T)||, far below
   * residual targets such as 1e-8, so it serves as a finisher's forward
   * (sos_solve's finisher 2).  SOS_EINVAL without SOS_FLAG_OZAKI_FORWARD. */
  SOS_FLAG_OZAKI_FIVE_SLICES = 256,
  /* SOS_BF16X3 and SOS_FP16X3 plans, fast forward: the gram takes one
   * 16-bit product per element pair (hi * hi) instead of three.  Each
   * coefficient is then off by at most about 2^-7 (bf16) or 2^-10 (fp16)
   * of coeff(|W||W|^T), the gram costs about a third, and the answer is that
   * of the rounded W; for the first phase of a solve, while the residual is
   * far above that level (sos_solve's single_rel).  SOS_FLAG_EXACT_FORWARD,
   * SOS_FLAG_OZAKI_FORWARD and SOS_FLAG_FP32_FORWARD take precedence;
   * SOS_EINVAL on other plans or with SOS_FLAG_UNFUSED_SCATTER,
   * SOS_FLAG_UNMERGED_SCATTER or SOS_FLAG_DETERMINISTIC.                 */
  SOS_FLAG_SINGLE_FORWARD = 512,
  /* With SOS_FLAG_OZAKI_FORWARD: 4 digit slices (levels s + t < 4: 10
   * slice products).  Per Gram entry the error is at most
   * 5.05 * 2^-28 * rank * 2^(e_i + e_j) plus FP64 rounding, about 128x the
   * five-slice figure (~4e-8 of ||coeff(W W^T)|| for Gaussian rows); for
   * the start of a finisher (sos_solve's four_rel).  SOS_EINVAL without
   * SOS_FLAG_OZAKI_FORWARD or with SOS_FLAG_OZAKI_FIVE_SLICES.             */
  SOS_FLAG_OZAKI_FOUR_SLICES = 1024,
};

/* Adam hyper-parameters (Kingma and Ba; the paper's optimiser, Section 3). */
typedef struct {
  double lr, beta1, beta2, eps;
} sos_adam_t;

/* sos_solve options.  The loop follows the paper's first-order method
 * (Adam from the given start, success judged on the best iterate); the
 * precision ladder and the step-size guard are this library's additions,
 * needed because a residual measured with a rounded forward cannot go below
 * that forward's rounding level, and Adam with a fixed step size turns
 * unstable once the gradient is dominated by that rounding noise.        */
typedef struct {
  double tol;            /* target: FP64 ||r|| / ||p|| <= tol                */
  int64_t max_steps;     /* step budget                                     */
  int64_t check_every;   /* read the loss back every this many steps        */
  int32_t ladder;        /* 1: start with the plan's fast forward and switch
                            to SOS_FLAG_EXACT_FORWARD (see switch_rel and
                            stall_checks)                                   */
  int32_t stall_checks;  /* checks without `stall_ratio` progress count as a
                            stall, on which the ladder switches; 0: off     */
  double stall_ratio;    /* progress means rel < stall_ratio * reference    */
  double switch_rel;     /* ladder: switch once the fast forward's rel <=
                            switch_rel (0: switch on a stall only)          */
  double lr_exact;       /* Adam step size in the exact phase (0: adam->lr) */
  double rollback_ratio; /* rel > rollback_ratio * best rel: restore the best
                            W, zero the Adam moments (the bias correction
                            restarts) and halve the step size (0: off).  A
                            non-finite loss after a finite check always rolls
                            back this way; before any finite check it ends
                            the solve with SOS_ENUMERIC                     */
  int32_t single_backward; /* 1: steps use SOS_FLAG_SINGLE_BACKWARD         */
  int32_t finisher;      /* forward of the exact phase: 0 FP64 MFMA
                            (SOS_FLAG_EXACT_FORWARD), 1 six int8 slices
                            (SOS_FLAG_OZAKI_FORWARD), 2 five int8 slices
                            (with SOS_FLAG_OZAKI_FIVE_SLICES).  The result
                            is certified by the FP64-MFMA forward in every
                            case                                            */
  double mid_rel;        /* SOS_BF16X3 ladder with a middle rung: after the
                            fast phase, steps use SOS_FLAG_FP32_FORWARD until
                            rel <= mid_rel (or a stall), then the exact
                            forward (0: no middle rung)                     */
  int32_t step_flags;    /* SOS_FLAG_DETERMINISTIC or 0: added to the steps
                            of the plan's own forward                       */
  int32_t reserved;
  double single_rel;     /* SOS_BF16X3 / SOS_FP16X3 ladder: the fast phase
                            starts with SOS_FLAG_SINGLE_FORWARD and goes on
                            to the three-product forward once rel <=
                            single_rel (or on a stall); same Adam state and
                            step size (0: three products from the start)    */
  double four_rel;       /* finisher 2: the exact phase takes four int8
                            slices (SOS_FLAG_OZAKI_FOUR_SLICES) until rel <=
                            four_rel (or a stall), then five (0: five
                            throughout)                                     */
} sos_solve_opts_t;

typedef struct {
  int64_t steps;         /* steps taken                                     */
  int64_t exact_steps;   /* of which with the FP64 forward                  */
  double loss;           /* last loss (as measured at the last check)       */
  double rel;            /* FP64-verified ||r||/||p|| of the returned W     */
  double best_rel;       /* best relative residual seen at any check        */
  int32_t status;        /* SOS_OK or SOS_NOT_CONVERGED                     */
  int32_t phase;         /* forward at the end: 0 fast, 1 FP32 (middle rung),
                            2 exact                                         */
} sos_result_t;

/* Plan a problem (host only; enumerates the bases of Section 1.1, builds
 * the ranking tables and sizes the buffers).  n, d, rank >= 1.  Up to 16
 * variables the ranking uses 4-bit suffix-sum codes (2d <= 15); with more
 * variables it uses sorted variable lists (2d <= 8, n <= 255, as for the
 * paper's quartics in 100 variables).  SOS_ERANGE outside these, or when
 * M >= 2^31 or N*N >= 2^31.  The plan must be bound to a workspace before
 * any device call.                                                        */
int sos_plan(int n, int d, int rank, int precision, sos_plan_t* out);

/* Sizes: basis length N, coefficient count M, workspace bytes (one per
 * plan, see sos_plan_bind) and optimiser-state bytes (one per problem:
 * Adam moments m, v and the best W seen, each N x rank in W's type).
 * Any output pointer may be NULL.                                         */
int sos_plan_query(sos_plan_t plan, int64_t* N, int64_t* M, size_t* ws_bytes,
                   size_t* state_bytes);

/* Attach a device workspace of at least ws_bytes (256-byte aligned) and
 * upload the ranking tables into it, on `stream`.  For SOS_BF16X3 and
 * SOS_FP16X3 plans it also builds the gram epilogue's merge maps there (per
 * 64 x 256 segment of every upper Gram tile: the slot of each pair among the
 * segment's distinct coefficients, and their ranks; about 10 ms and 0.7 GB
 * at n = 12, d = 6) and keeps them only where merging saves atomics (at least
 * 1.5 pairs per coefficient of a segment on the whole).  Returns once the
 * stream has done this work.  The workspace must stay allocated while the
 * plan is used.                                                           */
int sos_plan_bind(sos_plan_t plan, void* d_ws, size_t ws_bytes, void* stream);

/* Free the host side of a plan (the workspace stays the caller's). */
void sos_plan_destroy(sos_plan_t plan);

/* Exponent vectors in the library's order: which = 0 gives the N basis
 * monomials, which = 1 the M coefficient monomials; h_out holds rows x n
 * bytes.  Host only; needs no binding.                                    */
int sos_exponents(sos_plan_t plan, int which, uint8_t* h_out);

/* Test hook: d_out[i*N + j] = rank of alpha_i + alpha_j among the
 * coefficient monomials, computed by the same in-kernel ranking the
 * forward and backward use.  d_out holds N*N int32.                       */
int sos_pair_ranks(sos_plan_t plan, int32_t* d_out, void* stream);

/* Loss and gradient at W (eq. nonconvex; gradient 4 R W).
 *   d_W:    N x rank, row-major (double for SOS_FP64, else float); read only
 *   d_p:    M doubles
 *   d_loss: 1 double, receives L = ||r||^2
 *   d_grad: N x rank in W's type, receives 4 R W; may be NULL (forward only)
 *   d_r:    M doubles, receives r = coeff(W W^T) - p; may be NULL
 *   flags:  0 (the plan's own forward) or the SOS_FLAG_* values above that
 *           select a forward (EXACT, OZAKI with FIVE_SLICES or FOUR_SLICES,
 *           FP32, SINGLE) or a variant of it (DETERMINISTIC, UNFUSED_SCATTER,
 *           UNMERGED_SCATTER), and SOS_FLAG_SINGLE_BACKWARD; each flag's
 *           comment states the plans it applies to and its SOS_EINVAL cases;
 *           any other bit is SOS_EINVAL                                    */
int sos_loss_grad(sos_plan_t plan, const void* d_W, const double* d_p, double* d_loss,
                  void* d_grad, double* d_r, int flags, void* stream);

/* Size of the library's static device workspace behind
 * sos_loss_grad_noalloc: 64 MiB per GPU, held from the library's first use
 * of a GPU until the process ends.  It covers every plan of the serving
 * sizes (n <= 8, d <= 4, rank 2N: at most 23 MiB, any precision).        */
#define SOS_NOALLOC_MAX_WS (64u << 20)

/* sos_loss_grad for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Arguments, flags and results are those of sos_loss_grad (the caller still
 * passes W, p and the outputs), but the plan must be UNBOUND: the call uses
 * the library's static workspace on the stream's GPU instead of one from
 * sos_plan_bind, uploads the plan's ranking tables into it, and leaves the
 * plan unbound again on return.  It calls no hipMalloc, hipFree or other
 * allocating routine (kernel timing from sos_timing is not recorded).
 * Every call on one GPU shares that GPU's workspace, which keeps the last
 * call's contents; the call writes every region before reading it.  Calls
 * that overlap on one GPU (other streams, other threads) race: order them.
 * Errors as sos_loss_grad, plus SOS_EINVAL for a bound plan and SOS_ERANGE
 * when the plan's ws_bytes (sos_plan_query) exceeds SOS_NOALLOC_MAX_WS.   */
int sos_loss_grad_noalloc(sos_plan_t plan, const void* d_W, const double* d_p, double* d_loss,
                          void* d_grad, double* d_r, int flags, void* stream);

/* One Adam step at iteration t (1-based): computes the loss and gradient
 * at W (written to d_loss), then updates W, m, v in place.
 *   d_state: state_bytes from sos_plan_query; zero it before t = 1.
 *   flags:   those of sos_loss_grad, and SOS_FLAG_COPIES_VALID.            */
int sos_step(sos_plan_t plan, void* d_W, void* d_state, int64_t t, const double* d_p,
             const sos_adam_t* adam, double* d_loss, int flags, void* stream);

/* The first-order loop (Section 3): Adam steps from the given W until the
 * FP64-verified relative residual ||r||/||p|| <= opts->tol or max_steps.
 * Success is judged on the best iterate (the minimum error over all
 * iterations, Section 3): on return W holds the best W found.  Returns
 * SOS_OK only if sos_verify of that W meets tol, else SOS_NOT_CONVERGED.
 * d_state is zeroed by the call.  Blocks until done.                      */
int sos_solve(sos_plan_t plan, void* d_W, void* d_state, const double* d_p,
              const sos_adam_t* adam, const sos_solve_opts_t* opts, sos_result_t* h_res,
              void* stream);

/* Certificate check (eq. basicsos): FP64 Gram of the exactly converted W,
 * r = coeff(W W^T) - p in FP64, *h_rel = ||r|| / ||p||.  d_r may be NULL.
 * Blocks until done.                                                      */
int sos_verify(sos_plan_t plan, const void* d_W, const double* d_p, double* h_rel,
               double* d_r, void* stream);

/* Largest basis size N for which a plan supports the grouped (serving)
 * calls below.                                                            */
#define SOS_BATCH_MAX_N 1024

/* Serving: one Adam step (Section 3 loop body) for `count` independent small
 * problems in one set of grouped launches.  plans[q] must be bound SOS_FP32
 * plans with N <= SOS_BATCH_MAX_N and distinct workspaces (SOS_EINVAL when
 * two entries share one); d_W[q] (N x k
 * FP32, row-major), d_state[q] (sos_plan_query's state_bytes; m and v as in
 * sos_step), t[q] (1-based Adam step count) and d_p[q] (M FP64) as in
 * sos_step.  d_losses[q] (device) receives L of problem q at the W before
 * the update.  Any count >= 0 is accepted; the library launches in groups
 * of problems of similar size (largest basis first).
 *
 * Numerics: the forward forms every Gram entry from exact FP64 products of
 * the FP32 entries, summed in FP64, then each coefficient sums its (i <= j)
 * pairs in one fixed order (eq. basicsos, no atomics); the backward 4 R W
 * is FP32; Adam is FP32.  Every problem's arithmetic is independent of the
 * others in the call, and the order of every sum is fixed, so a problem's
 * results are bitwise the same alone and in any mix.  Asynchronous on
 * `stream`.  Errors: SOS_EINVAL for NULL arrays, unbound or non-FP32 plans,
 * t < 1; SOS_ERANGE for a plan with N > SOS_BATCH_MAX_N.                  */
int sos_step_batch(const sos_plan_t* plans, void* const* d_W, void* const* d_state,
                   const int64_t* t, const double* const* d_p, const sos_adam_t* adam,
                   double* d_losses, int count, void* stream);

/* Serving certificate: the grouped forward of sos_step_batch alone.
 * d_losses[q] = ||coeff(W_q W_q^T) - p_q||^2 in FP64 (exact FP64 products of
 * the FP32 entries, fixed summation order), so sqrt(d_losses[q]) / ||p_q||
 * is the FP64-verified relative residual of W_q.  Same plan requirements
 * and errors as sos_step_batch; asynchronous on `stream`.               */
int sos_loss_batch(const sos_plan_t* plans, const void* const* d_W, const double* const* d_p,
                   double* d_losses, int count, void* stream);

/* ---------------------------------------------------------------------
 * Two-layer network (Section 2, eq. NN): a quartic form in n variables as
 * ||B Z A x||^2 with A (m x n), B (k x n m) and the augmentation
 * Z(x) A x = (x_1 A x, .., x_n A x); output l is the quadratic form
 * f_l = sum_{a,c} P[l,a,c] x_a x_c, P[l,a,c] = sum_b B[l, a m + b] A[b, c].
 * Forms of degree 4 in n variables are the polynomials of degree <= 4 in
 * x_1 .. x_{n-1} (x_n = 1), so these calls take a bound plan (n - 1, 2) of
 * rank k: p is indexed like that plan's
 * coefficients, and the network's factor W = net(A, B) (N x k, the
 * coefficients of each f_l over the plan's basis, in the plan's W type)
 * goes through the plan's loss, gradient and certificate.  With an
 * SOS_FP64 plan W is formed in FP64 from exact products of the FP32
 * weights; with FP32 and split plans W is rounded to FP32 after the map,
 * which puts a floor of about 3e-8 under the reachable relative residual.
 * The weights are stored transposed, row-major FP32: d_At = A^T (n x m),
 * d_Bt = B^T (n m x k).  d_state is caller memory of sos_net_query's size
 * (Adam moments of both, W, scratch); its first call uploads small index
 * maps into it.  Errors: SOS_EINVAL for a plan that is not (n - 1, 2),
 * n < 2, m < 1; SOS_ERANGE when n^2 k or n m k reaches 2^31.              */
int sos_net_query(sos_plan_t plan, int n, int m, size_t* state_bytes);

/* d_W (N x k, the plan's W type) = net(At, Bt).  Asynchronous.          */
int sos_net_weights(sos_plan_t plan, int n, int m, const float* d_At, const float* d_Bt, void* d_W,
                    void* d_state, void* stream);

/* L of W = net(At, Bt) (d_loss, device) and its gradient with respect to
 * the weights: d_dBt (n m x k) and, unless d_dAt is NULL, d_dAt (n x m),
 * FP32, by the chain rule through dL/dW = 4 R W (flags as for
 * sos_loss_grad).  Asynchronous on stream.                                */
int sos_net_grad(sos_plan_t plan, int n, int m, const float* d_At, const float* d_Bt, void* d_state,
                 const double* d_p, double* d_loss, float* d_dAt, float* d_dBt, int flags, void* stream);

/* One Adam step on the weights at iteration t (1-based): W = net(At, Bt),
 * the plan's loss and dL/dW (flags: SOS_FLAG_EXACT_FORWARD,
 * SOS_FLAG_SINGLE_BACKWARD as in sos_loss_grad), the chain rule to dL/dAt
 * and dL/dBt (FP32 GEMMs), then Adam on Bt, and on At when train_first is
 * nonzero (train_first = 0 keeps the first layer fixed, e.g. A = I).
 * d_loss (device) receives L at the weights before the update.            */
int sos_net_step(sos_plan_t plan, int n, int m, float* d_At, float* d_Bt, void* d_state, int64_t t,
                 const double* d_p, const sos_adam_t* adam, double* d_loss, int flags, int train_first,
                 void* stream);

/* Adam on the weights from their current values until the FP64-verified
 * relative residual of W = net(At, Bt) is <= opts->tol or opts->max_steps
 * (uses tol, max_steps, check_every, ladder, switch_rel, lr_exact,
 * rollback_ratio and single_backward of opts: the fast forward until
 * rel <= switch_rel, then the exact forward with step size lr_exact).  As in
 * sos_solve, success is judged on the best weights seen at a check, which
 * are returned in d_At, d_Bt; a check whose rel exceeds rollback_ratio times
 * the best (or is not finite, after a finite one) restores the best weights,
 * zeroes the Adam moments and halves the step size (0: off).  The Adam
 * moments are zeroed first; d_state holds two extra copies of the weights
 * for the rollback.  h_res as for sos_solve (steps, exact_steps, the
 * verified rel of the returned weights).  Blocks until done.               */
int sos_net_solve(sos_plan_t plan, int n, int m, float* d_At, float* d_Bt, void* d_state, const double* d_p,
                  const sos_adam_t* adam, const sos_solve_opts_t* opts, int train_first, sos_result_t* h_res,
                  void* stream);

/* Kernel classes reported by sos_timing_read. */
enum sos_kernel_class {
  SOS_K_PREP = 0,    /* operand copies / bf16 split of W                  */
  SOS_K_INIT = 1,    /* r <- -p                                           */
  SOS_K_GRAM = 2,    /* gram-scatter forward                              */
  SOS_K_LOSS = 3,    /* sum of squares                                    */
  SOS_K_GATHER = 4,  /* R from r                                          */
  SOS_K_RW = 5,      /* R W backward                                      */
  SOS_K_ADAM = 6,    /* Adam update                                       */
  SOS_K_SCATTER = 7, /* scatter of stored Gram tiles (SOS_FLAG_UNFUSED_SCATTER) */
  SOS_K_COUNT = 8
};

/* Per-kernel timing with HIP events around this plan's launches (tracing
 * aid; adds one event pair per launch).  enable = 1 clears the totals and
 * starts recording, enable = 0 stops.                                     */
int sos_timing(sos_plan_t plan, int enable);

/* Wait for the recorded events and return, per kernel class, the summed
 * milliseconds (h_ms[SOS_K_COUNT]) and launch counts (h_calls[SOS_K_COUNT],
 * may be NULL).  Clears the totals.                                       */
int sos_timing_read(sos_plan_t plan, double* h_ms, int64_t* h_calls);

/* Message for the last error on this thread ("" if none). */
const char* sos_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SOS_H */
