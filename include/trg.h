/*
 * trg.h -- C ABI of the MI355X (gfx950) implementation of the coarse-graining
 * step of ATRG and triad-ATRG for the d-dimensional Ising model.
 *
 * Method: Y. Sugimoto and S. Sasaki, "Triad representation for the
 * anisotropic tensor renormalization group in four dimensions",
 * arXiv:2507.21909.  Section, equation and appendix labels below are the
 * paper's.
 *
 * Conventions shared by every entry point
 *   - All calls return TRG_OK (0) or a negative TRG_E_* code; they never
 *     abort or throw across the ABI.  trg_strerror() names a code,
 *     trg_last_error() gives the message of the last failure on a state.
 *   - A state owns every device buffer it uses; no pointer into device
 *     memory escapes.  Host pointers passed in are only read (or written,
 *     for outputs) during the call.
 *   - Work is enqueued on the state's HIP stream (opt.stream, or the null
 *     stream when NULL).  A step reads the convergence flags of its
 *     eigensolvers and SVDs and its numerical status back on the host, so it
 *     returns with the stream synchronised; log_z_per_site and the
 *     export/inspection calls synchronise it too.  The asynchronous form of
 *     a step is a captured one (trg_graph_launch).  The caller keeps a stream
 *     it passed alive until trg_destroy.
 *   - A step that fails leaves the state as it was before the step (tensors,
 *     step count and log-norm accumulator), so log_z_per_site still gives
 *     the value before the failed step.  If even that cannot be restored
 *     (HIP error) the state asks for a new tensor_init (TRG_E_STATE).
 *   - Device: opt.device selects the GPU; the library makes it current for
 *     the duration of each call.
 */
#ifndef TRG_H
#define TRG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------ */
#define TRG_OK           0
#define TRG_E_INVALID   -1   /* NULL pointer, D < 1, beta < 0, axis out of range, triad with dim != 4, ... */
#define TRG_E_STATE     -2   /* step or query before tensor_init                                      */
#define TRG_E_NOMEM     -3   /* device allocation failed or exceeds opt.workspace_cap                 */
#define TRG_E_NUMERICAL -4   /* NaN/Inf, non-positive norm, Jacobi not converged in max_sweeps       */
#define TRG_E_HIP       -5   /* HIP runtime error (message kept in trg_last_error)                    */
#define TRG_E_UNSUPPORTED -6 /* a shape outside the kernels' documented limits                       */
#define TRG_E_MULTIPLET -7   /* a truncation cut falls inside a multiplet of more than 32 values      */

/* ---- options ---------------------------------------------------------- */
#define TRG_MODEL_ISING 0

#define TRG_FP64   0   /* every contraction in FP64 (MFMA f64)                                     */
#define TRG_FP32   1   /* coarse-graining contractions (makeMG/makeMH) in FP32 MFMA; rest FP64     */
#define TRG_BF16X3 2   /* coarse-graining contractions as split BF16 MFMA, 3 products, FP32 acc.   */
#define TRG_BF16X6 3   /* same with the 6 split products i + j <= 2 (about FP32 accuracy)          */

#define TRG_TAN_BETA 1   /* carry d/dbeta of the site tensor (needs beta > 0)                     */
#define TRG_TAN_H    2   /* carry d/dh of the site tensor                                          */

#define TRG_SVD_SKETCH 0  /* bond swap by the randomized SVD of App. A (power_iters passes)         */
#define TRG_SVD_EXACT  1  /* bond swap by the exact SVD of the QR-reduced core of App. A            */

typedef struct trg_options {
    int dim;            /* lattice dimension: 4 (the GPU path implements d = 4 only)               */
    int r;              /* overspanning parameter r of Sec. II A (triad bond R = min(r D, d1 d2))   */
    int sketch_mult;    /* sketch width m = sketch_mult * D (App. A footnote: eta D)                */
    int power_iters;    /* extra power passes of the randomized SVD (App. A loop count q = this+1) */
    uint64_t seed;      /* Philox4x32-10 key of the Gaussian sketch                                */
    uint32_t instance;  /* Philox counter word 2 (distinguishes independent solves)                */
    int precision;      /* TRG_FP64 / TRG_FP32 / TRG_BF16X3 / TRG_BF16X6                           */
    int bond_svd;       /* TRG_SVD_SKETCH / TRG_SVD_EXACT                                          */
    int max_sweeps;     /* Jacobi sweep limit (0: default 300)                                      */
    size_t workspace_cap; /* bytes of device workspace the state may hold (0: unlimited)           */
    void *stream;       /* hipStream_t to enqueue on, or NULL for the null stream                  */
    int device;         /* HIP device ordinal                                                      */
    double tau_deg;     /* multiplet tolerance of every truncation and canonical basis, relative
                           to the largest value (0: default 1e-9); see kept-count rule           */
    int tangents;       /* impurity tangents carried by triad_atrg_step (Sec. III D):
                           TRG_TAN_BETA | TRG_TAN_H (0: none); see impurity_derivatives     */
    int r_bond;         /* bond-swap overspanning of ILO triad-ATRG (Sec. II C, App. A): the bond
                           swap keeps r_bond * D values, which the next step's alpha and beta
                           carry; 1 is the plain bond swap.  Needs sketch_mult >= r_bond (the
                           paper oversamples with sketch_mult = r_bond + 1), r_bond * D <= 256
                           and sketch_mult * D <= 512 (tensor_init: TRG_E_UNSUPPORTED)          */
} trg_options;

/* Fills *opt with the defaults: dim 4, r 7, sketch_mult 2, power_iters 1,
 * seed 0, instance 0, FP64, sketch, max_sweeps 300, no cap, NULL stream,
 * device 0, tau_deg 1e-9, no tangents, r_bond 1. */
void trg_default_options(trg_options *opt);

typedef struct trg_state trg_state;

/* Creates a state (no tensors yet).  *out is NULL on failure. */
int trg_create(const trg_options *opt, trg_state **out);

/* Frees the state and its device memory.  NULL is accepted (no-op). */
int trg_destroy(trg_state *s);

/*
 * tensor_init -- Ising initial tensor in CP form (Sec. III):
 *   T[i_1..i_d; j_1..j_d] = sum_a exp(h s_a) prod_mu W[a,i_mu] W[a,j_mu],
 *   W = [[sqrt cosh beta, sqrt sinh beta], [sqrt cosh beta, -sqrt sinh beta]],
 * kept as the pair (Phi, Psi) with T = sum_g Phi[.., g] Psi[.., g].
 * model must be TRG_MODEL_ISING, beta >= 0, D >= 2 (bond dimension cap).
 * Resets the step count and the log-norm accumulator; may be called again.
 */
int tensor_init(trg_state *s, int model, double beta, double h, int D);

/*
 * atrg_step -- one ATRG coarse-graining step along `axis` (0..dim-1):
 * exact re-split of T (Fig. 5f), bond swap (eq. of the bond swap, App. A),
 * squeezers from the canonical Gamma^ATRG and makeG / makeH (Sec. II A).
 * Halves the lattice along `axis`.  Returns with the stream synchronised
 * (it reads its status back); trg_graph_launch replays a captured step
 * asynchronously.
 */
int atrg_step(trg_state *s, int axis);

/*
 * triad_atrg_step -- one triad-ATRG step along `axis` (dim must be 4):
 * re-split, bond swap, triad isometries from the truncated HOSVD of
 * Gamma^ATRG (eq. HOSVD), triad tensors E..L, squeezers from Gamma^Triad
 * with the Gram matrices O and P (Sec. II D), makeMG / makeMH (Sec. II B).
 * Synchronises as atrg_step does.
 */
int triad_atrg_step(trg_state *s, int axis);

/*
 * log_z_per_site -- log Z / V of the torus the state represents (extent
 * 2^(steps along mu) on axis mu): sum_k 2^-k log c_k + 2^-n log tTr T^(n)
 * (eq. Z), with c_k the norm removed at the k-th re-split.  Synchronises;
 * writes one double to *out (host).  TRG_E_NUMERICAL if the trace <= 0.
 */
int log_z_per_site(trg_state *s, double *out);

/*
 * gu_wen_x -- the dimensionless ratio X = (Tr A)^2 / Tr(A A) of Sec. III D,
 * A[k, l] = sum of the current coarse tensor T over every forward/backward
 * leg pair traced except those along `axis` (k forward, l backward; the
 * paper keeps the fourth leg open: axis = 3).  X counts the ground-state
 * degeneracy: 2 in the ordered phase (h = 0), 1 in the disordered phase, so
 * its jump over a beta scan locates T_c.  Computed on the device (one
 * contraction over D^(d-1) chi entries, fixed-order sums); synchronises and
 * writes one double to *out (host).  TRG_E_INVALID for a bad axis,
 * TRG_E_STATE before tensor_init, TRG_E_NUMERICAL if Tr(A A) <= 0.
 */
int gu_wen_x(trg_state *s, int axis, double *out);

/*
 * impurity_derivatives -- d(log Z/V)/d(beta) and d(log Z/V)/dh of the torus the
 * state represents, by the impurity-tensor method (Sec. III D): the derivative
 * of the site tensor, summed over the sites, is carried through every step:
 * the re-split and bond-swap tangents taken in the tangent space of the
 * rank-chi matrices, the triad isometries' kept subspaces moved with their
 * Grams (first-order invariant-subspace perturbation; kept / discarded pairs
 * whose eigenvalues differ by at most 1e-12 of the largest are treated as
 * degenerate and not rotated), the squeezers and norms held; then
 * d(log Z/V) = 2^-n Tr dT^(n) / Tr T^(n).  Exact where
 * nothing is truncated; otherwise it differs from the derivative of the
 * truncated flow by what the held squeezers and the bond swap's tangent-space
 * form leave out (about 4e-4 relative at D = 8 near T_c).  The internal
 * energy per site is u = -(*dbeta) and the magnetisation m = *dh.
 * The state must be created with opt.tangents; each output pointer (host,
 * may be NULL) receives its derivative, or NaN if that tangent is not
 * carried.  Synchronises.  TRG_E_STATE without tangents or before
 * tensor_init, TRG_E_NUMERICAL if the trace is not positive.
 */
int impurity_derivatives(trg_state *s, double *dbeta, double *dh);

/*
 * trg_release_workspace -- frees the state's step workspace (the device
 * arena that a step's temporaries live in; the next step allocates it
 * again).  The state tensors stay.  Synchronises the state's stream first.
 */
int trg_release_workspace(trg_state *s);

/*
 * Captured steps (HIP graphs) -- the RG loop without host round trips.
 *
 * trg_graph_capture records one step of `method` (TRG_METHOD_ATRG or
 * TRG_METHOD_TRIAD) along `axis` into a HIP graph, at the state's current
 * shapes, without running it; *out receives the graph.  The state must have
 * run at least one eager step of the same method at these shapes since its
 * last tensor_init: that step sized the workspace (nothing may be allocated
 * while recording) and logged how many sweeps each Jacobi solve needed.
 * Otherwise TRG_E_STATE, and the state is unchanged.  The recorded step
 * reads nothing back: the panel Jacobi solves run at most twice the most
 * sweeps logged for them plus 8, stopping early on device flags, and
 * numerical failures set the state's device status flag.  Neither an
 * n > 1024 squeezer Gram nor the eigensolver fallback can be recorded
 * (TRG_E_UNSUPPORTED).
 *
 * trg_graph_launch enqueues the recorded step on the state's stream; the
 * state then holds the next step's tensors, step count, spectra and
 * log-norm, bit for bit those of the eager step (same kernels in the same
 * order).  check = 0: returns without waiting; a failure inside the step
 * (including a Jacobi solve that needs more sweeps than recorded) is
 * reported by the next call that reads the status (log_z_per_site) as
 * TRG_E_NUMERICAL or TRG_E_MULTIPLET, with no rollback.  check != 0: waits
 * for the step and reads its status; on a failure the state goes back to
 * where the step started (the recorded step keeps a copy of it) and the
 * error is returned, as for an eager step, so the caller can take that step
 * eagerly (which logs the sweeps it needed) and record again.  TRG_E_STATE
 * if the state's shapes differ from those at capture, or if tensor_init or
 * trg_release_workspace ran on the state since the capture.  Recording
 * allocates that copy once per state (twice the state tensors, tangents
 * included).
 *
 * trg_graph_destroy frees a graph (NULL: no-op); destroy graphs before their
 * state.  One graph per (method, axis) covers a steady RG loop: the shapes
 * stop changing once the bond dimension reaches its cap.
 */
#define TRG_METHOD_ATRG  0
#define TRG_METHOD_TRIAD 1
typedef struct trg_graph trg_graph;
int trg_graph_capture(trg_state *s, int method, int axis, trg_graph **out);
int trg_graph_launch(trg_graph *g, int check);
int trg_graph_destroy(trg_graph *g);

/* ---- many instances ------------------------------------------------------ */

typedef struct trg_batch trg_batch;

/*
 * trg_batch_create -- n independent triad-ATRG solves of the 4D Ising model
 * (betas[i], hs[i], Ds[i]), each with the options *opt except that instance
 * i draws its sketches with Philox counter word opt->instance + i and runs on
 * a stream the batch creates (opt->stream must be NULL).  Arrays are host
 * memory, read during the call.  On error nothing is left allocated.
 */
int trg_batch_create(int n, const double *betas, const double *hs, const int *Ds,
                     const trg_options *opt, trg_batch **out);

/*
 * trg_batch_run -- nsteps triad-ATRG steps on every instance, along
 * axes[0..nsteps) (NULL: 0, 1, 2, 3, 0, ...).  Host workers (up to 8) run
 * instances concurrently on their own streams; each instance gives the same
 * bits as a lone solver with the same options.  An instance's step workspace
 * is released when its steps are done, so the device holds at most one
 * workspace per worker besides the instances' state tensors.  Returns after all steps are
 * issued and their host read-backs done; the first error code of any
 * instance is returned (trg_batch_last_error names the instance).
 */
int trg_batch_run(trg_batch *b, int nsteps, const int *axes);

/*
 * trg_batch_run_graphs -- trg_batch_run with the steady part of each flow
 * replayed from HIP graphs: an instance steps eagerly until a step leaves
 * its shapes unchanged, then records one step per axis (trg_graph_capture)
 * and replays them for its remaining steps, checked (one status read per
 * step instead of one per Jacobi sweep).  A replay that fails is rolled
 * back and taken eagerly, and the steps are recorded again; the graphs are
 * destroyed when the instance is done.  Same bits as trg_batch_run.
 */
int trg_batch_run_graphs(trg_batch *b, int nsteps, const int *axes);

/* log Z / V of every instance into out_n[0..n) (host).  Synchronises. */
int trg_batch_log_z(trg_batch *b, double *out_n);

int trg_batch_size(const trg_batch *b);
const char *trg_batch_last_error(const trg_batch *b);

/* Frees every instance and stream; NULL is a no-op. */
int trg_batch_destroy(trg_batch *b);

/* ---- device-memory building blocks ------------------------------------- */

/*
 * trg_qr -- thin QR factorisation A = Q R of a tall matrix in device memory,
 * the factorisation of the re-split (Fig. 5f: QR of Phi and of Psi) and of
 * the randomized SVD's sketches (App. A, the QR steps after eq. bond1 and
 * eq. bond2), by the library's tall-skinny Householder QR.
 *   A  device pointer, m x n row-major (read only), 1 <= n <= 64, m >= n;
 *   Q  device pointer, m x n row-major (written), orthonormal columns;
 *   R  device pointer, n x n row-major (written), upper triangular with a
 *      non-negative diagonal.
 * All three live on the calling thread's current HIP device and must not
 * overlap.  stream: hipStream_t to enqueue on (NULL: the null stream).  The
 * call allocates its scratch (about 3 m n doubles) with hipMalloc, runs,
 * synchronises the stream and frees it.  TRG_E_INVALID for NULL pointers or
 * bad sizes, TRG_E_NOMEM if the scratch cannot be allocated, TRG_E_HIP for a
 * runtime error; trg_last_error(NULL) gives the message.
 */
int trg_qr(const double *A, int64_t m, int n, double *Q, double *R, void *stream);

/*
 * trg_qr_noalloc -- trg_qr for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, kernels and results as trg_qr, bit for bit,
 * but the call allocates nothing: its scratch is a fixed 64 MiB device array
 * inside the library (one per GPU, held until the process ends), and it does
 * not synchronise: the QR is enqueued on `stream` and the call returns.
 *   Limit: the QR's scratch (about 3 m n doubles: 256-row blocks of every
 *   TSQR level plus two Q-rebuild buffers) must fit 8 Mi doubles; every
 *   m * n <= 2097152 does (e.g. m <= 35584 at n = 64).  Larger sizes return
 *   TRG_E_UNSUPPORTED before anything is enqueued; use trg_qr for them.
 * Every call on one GPU shares that GPU's scratch: calls that overlap on one
 * device (two streams, or two host threads) race and give wrong results;
 * serialise them on one stream.  The scratch keeps the last call's contents,
 * which no call reads.  TRG_E_INVALID for NULL pointers or bad sizes,
 * TRG_E_HIP for a runtime error; trg_last_error(NULL) gives the message.
 */
int trg_qr_noalloc(const double *A, int64_t m, int n, double *Q, double *R, void *stream);

/* ---- inspection (tests and benchmarks) --------------------------------- */

/* Names accepted by trg_export (host copy of a device tensor). */
#define TRG_T_PHI    0   /* Phi  [dims..., chi], natural axis order, FP64 */
#define TRG_T_PSI    1   /* Psi  [dims..., chi]                           */
#define TRG_T_SIGMA  2   /* bond-swap singular values of the last step    */
#define TRG_T_RESPLIT 3  /* re-split singular values / c_k of the last step */

/* Shape of the current state: dims[0..dim-1] leg dims, *chi the bond. */
int trg_shape(trg_state *s, int *dims, int *chi, int *steps);

/* Copies tensor `which` to host_dst (bytes must equal its size in bytes). */
int trg_export(trg_state *s, int which, void *host_dst, size_t bytes);

/* Byte size of tensor `which` (0 if not available). */
size_t trg_export_size(trg_state *s, int which);

/*
 * Per-kernel timing of the last step: the library records HIP events
 * around the coarse-graining GEMMs (makeMG / makeMH) when enabled.
 * trg_set_timing(s, 1) enables; trg_kernel_time returns the summed
 * milliseconds and the algorithmic flop count of those GEMMs since the
 * last reset, and resets them.
 */
int trg_set_timing(trg_state *s, int enable);
int trg_kernel_time(trg_state *s, double *ms, double *flops, int *launches);

const char *trg_strerror(int code);
const char *trg_last_error(trg_state *s);

/* ---- kernel self-tests (host buffers in and out; tests only) ------------
 * Each copies its host inputs to the device, runs one kernel of the path,
 * and copies the result back.  Row-major storage throughout. */

/* C[b] = A[b] op B[b] in FP64 MFMA: A (M x K, or K x M if ta), B (K x N, or
 * N x K if tb), C (M x N), batch b with strides M*K, K*N, M*N.  precision
 * selects FP64 / FP32 / BF16X3 / BF16X6 arithmetic. */
int trg_selftest_gemm(int precision, int ta, int tb, int M, int N, int K, int batch,
                      const double *A, const double *B, double *C);

/* Thin QR of A (m x n, m >= n; n <= 512) by the Householder TSQR (n > 64:
 * blocked over 64-column panels): Q (m x n), R (n x n) with diag(R) >= 0. */
int trg_selftest_tsqr(int m, int n, const double *A, double *Q, double *R);

/* dst = src with its axes permuted, as the contractions reshape tensor legs
 * between GEMMs: src has nd <= 8 axes of sizes dims[0..nd) (row-major), dst
 * axis i is src axis perm[i] (row-major, the same number of elements).
 * TRG_E_INVALID if perm is not a permutation of 0..nd-1 or a size is < 1. */
int trg_selftest_permute(int nd, const int *dims, const int *perm, const double *src, double *dst);

/* One-sided Jacobi SVD of A (m x n, m >= n): U (m x n), s (n) descending,
 * V (n x n).  Returns the number of sweeps in *sweeps. */
int trg_selftest_svd(int m, int n, const double *A, double *U, double *s, double *V, int *sweeps);

/* Two-sided block Jacobi eigen-decomposition of `count` symmetric n x n
 * matrices K (batch stride n*n; symmetrised on load): lam (count x n)
 * descending, V (count x n x n) with eigenvector j in column j.  Returns the
 * number of sweeps in *sweeps. */
int trg_selftest_eigh(int count, int n, const double *K, double *lam, double *V, int *sweeps);

/* Diagonally pivoted Cholesky factor of `count` symmetric positive
 * semi-definite n x n matrices K (n <= 1024, batch stride n*n): X (count x n
 * x n) with K = X X^T, X = P L (P a row permutation, L lower triangular).  A
 * matrix's factorisation stops at its first pivot at or below tol times its
 * first (largest) pivot, 0 <= tol < 1, and the columns of X from there on are
 * zero; rank (count ints) receives the columns formed.  TRG_E_NUMERICAL for a
 * pivot that is not finite, or, with tol = 0, not positive. */
int trg_selftest_pchol(int count, int n, const double *K, double tol, double *X, int *rank);

/* Eigen-decomposition of `count` symmetric positive semi-definite n x n Grams
 * K (n <= 1024) as the triad isometries take it: one-sided Jacobi SVD of the
 * pivoted Cholesky factor X (K = X X^T), eigenvectors the left singular
 * vectors, eigenvalues the squared singular values.  lam, V and *sweeps as
 * for trg_selftest_eigh. */
int trg_selftest_gram_eig(int count, int n, const double *K, double *lam, double *V, int *sweeps);

/* Gaussian sketch entries Omega[beta, j1, j2, j3, m] (layout as named) drawn
 * exactly as the bond swap of step `step` draws them. */
int trg_selftest_sketch(uint64_t seed, int step, uint32_t instance, int chi,
                        int j1, int j2, int j3, int m, double *out);

#ifdef __cplusplus
}
#endif
#endif /* TRG_H */
