// Shared declarations of the gfx950 kernels and the host engine.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <stdexcept>
#include <array>
#include <functional>
#include <string>
#include <vector>

namespace trg {

// Error raised inside the library; converted to a TRG_E_* code at the ABI.
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define TRG_HIP_CHECK(expr)                                                              \
    do {                                                                                 \
        hipError_t _e = (expr);                                                          \
        if (_e != hipSuccess) {                                                          \
            (void)hipGetLastError();                                                     \
            throw ::trg::Error(-5, std::string(#expr) + ": " + hipGetErrorString(_e));   \
        }                                                                                \
    } while (0)

#define TRG_REQUIRE(cond, code, msg)                                                     \
    do {                                                                                 \
        if (!(cond)) throw ::trg::Error((code), (msg));                                   \
    } while (0)

enum Prec { P_FP64 = 0, P_FP32 = 1, P_BF16X3 = 2, P_BF16X6 = 3 };

// ---- GEMM: C[b] = alpha * sum_k A[b](r,k) B[b](k,n) + beta * C[b] -----------------
// Element (r, k) of A[b] is at A + b*sAb + r*sAr + k*sAk (likewise B, C).
// With inner > 1 the batch is two-level: z = outer * inner + i, outer < batch,
// and operand offsets add i * sAi (sBi, sCi) to outer * sAb (sBb, sCb) (split K).
struct GemmArgs {
    int M, N, K, batch;
    const double *A; long sAr, sAk, sAb;
    const double *B; long sBk, sBn, sBb;
    double *C; long sCr, sCn, sCb;
    double alpha, beta;
    int inner; long sAi, sBi, sCi;
    // optional two-level C index: with cR2 > 0 row r lands at
    // (r / cR2) * sCr + (r % cR2) * sCr2 (likewise columns with cN2, sCn2),
    // which writes C directly in a layout that interleaves the row and column
    // legs; 0 keeps r * sCr (c * sCn)
    int cR2, cN2; long sCr2, sCn2;
    // tile rows per L2 group of the tile walk (0: the default, 8); any value
    // gives the same bits (it only reorders which workgroup takes which tile)
    int gm;
};
// Tile-walk autotuning (gemm.hip).  The first eager launch of a large shape
// with beta = 0 (a rerun writes the same C) runs once per candidate group size
// {4, 8, 16}, timed with events on its stream, and the fastest is kept for the
// key (kernel variant and shape); later launches, launches being recorded into
// a graph and small shapes take the cached or default value.  The group size
// only reorders tiles over workgroups, so every choice gives the same bits.
// TRG_AUTOTUNE=0 switches tuning off, TRG_GEMM_GM=g forces g.
int tuned_gm(const std::array<long, 8> &key, hipStream_t st, bool eligible, const std::function<void(int)> &launch);
// ev0 / ev1 (optional): events stamped at the kernel's start and end
void gemm(const GemmArgs &g, Prec prec, hipStream_t st, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
void gemm_f64(const GemmArgs &g, hipStream_t st, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// mode 1: FP32, 2: BF16 split, 3 products; 3: BF16 split, 6 products
void gemm_mixed(const GemmArgs &g, int mode, hipStream_t st, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// ---- element-wise / layout kernels (kernels.hip) -----------------------------------
// dst = src with axes permuted: dst dims = src dims[perm[i]].
void permute(const double *src, double *dst, const std::vector<int> &dims,
             const std::vector<int> &perm, hipStream_t st);
// t[..., i_axis, ...] *= v[i_axis]^power (power 1 or 2 or -0.5) ; in place.
void scale_axis(double *t, const std::vector<int> &dims, int axis, const double *v,
                int mode, hipStream_t st);
void fill(double *p, size_t n, double v, hipStream_t st);
// C[r * sCr + c * sCn] = sum over s of w[s][r][c] (w: nslices x M x N), fixed order
void sum_slices(const double *w, int nslices, long M, long N, double *C, long sCr, long sCn, hipStream_t st);
void copy(double *dst, const double *src, size_t n, hipStream_t st);

// ---- small device helpers (kernels.hip) ---------------------------------------------
// kept count of a descending vector (rule shared with every truncation)
void kept_count(const double *vals, int n, int cap, double eps_rel, double tau_deg,
                int *kept_dev, hipStream_t st);
// zero columns j >= *kept of a row-major (rows x cols) matrix; also vals[j] if given
void zero_tail_cols(double *a, long rows, int cols, long ld, const int *kept_dev,
                    hipStream_t st);
// sign convention: sg[j] = sign(sum_i w(i) Q[i,j]); row multi-index decoded from
// `dims` (row-major over the GPU layout), each leg contributing idx * pw[leg].
// ws: weight_ws_doubles(rows, cols, 1) doubles of scratch.
void sign_vector(const double *q, long rows, int cols, long ld, const std::vector<int> &dims,
                 const std::vector<double> &pw, double *sg, double *ws, hipStream_t st);
// scratch for the weight sums of `cols` columns of `rows` rows with L weights
size_t weight_ws_doubles(long rows, int cols, int L);
// largest multiplet the canonical basis forms (a cut inside a larger one sets status 2)
constexpr int CANON_L = 32;
// Canonical basis within multiplets: rot (cols x cols, block diagonal) such that
// q rot has, in every group of the first *k_dev values closer than tau * vals[0],
// the columns Q_m Q_z with Q_z the Q factor of Q_m^T W (fixed weights w_l of the
// row multi-index).  z_work holds weight_ws_doubles(rows, cols, CANON_L) doubles;
// status gets 2 if a group is larger than 16.
void canonical_rotation(const double *q, long rows, int cols, long ld, const std::vector<int> &dims,
                        const std::vector<double> &pw, const double *vals, const int *k_dev, double tau,
                        double *z_work, double *rot, int *status, hipStream_t st);
// a[:, j] *= sg[j]
void scale_cols(double *a, long rows, int cols, long ld, const double *sg, hipStream_t st);

// step_dev (optional): the step index is read there, on the device, instead of `step`
void philox_sketch(double *out, uint64_t seed, int step, uint32_t instance,
                   const std::vector<int> &jdims, int chi, int m, int layout_jbm,
                   hipStream_t st, const int *step_dev = nullptr);

// ---- split-BF16 planes (gemm_bf16.hip) --------------------------------------------
// An FP64 operand split into three BF16 planes x = x0 + x1 + x2, laid out
// [plane][batch][row][Kp] (K contiguous, Kp a multiple of 32, zero padded).
struct PlaneGemm {
    const void *A, *B;          // planes of A (rows = M) and of B (rows = N)
    long sAp, sAb, sBp, sBb;    // plane and batch strides (elements)
    int M, N, Kp, batch;
    int kslice, inner;          // K split in `inner` z-slices of kslice (multiples of 32)
    double *C;
    long sCr, sCn, sCb, sCi;    // C[batch][slice] strides, as GemmArgs
    int cR2, cN2;
    long sCr2, sCn2;
    double alpha, beta;
    int gm;   // tile rows per L2 group (0: 8); bit-neutral, as GemmArgs::gm
};
size_t bf16_planes_elems(long rows, long Kp, int batch);
// src[b][r][k] at src + b sB + r sR + k sK (rows x K, batch entries) -> planes in dst
void split_bf16x3(const double *src, long sR, long sK, long sB, int rows, int K, int batch, int Kp, void *dst,
                  hipStream_t st);
// C = alpha sum_{i+j<=2} A_i B_j^T (+ beta C), FP32 MFMA accumulators flushed to FP64 per K tile
void gemm_planes(const PlaneGemm &g, hipStream_t st, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// ---- factorizations -----------------------------------------------------------------
// Thin QR of a (m x n, row-major, ld = n), n <= 64: q (m x n), r (n x n), diag r >= 0.
// ws must hold tsqr_ws_doubles(m, n) doubles.
size_t tsqr_ws_doubles(long m, int n);
void tsqr(const double *a, long m, int n, double *q, double *r, double *ws, hipStream_t st);

// One-sided Jacobi SVD of `count` matrices.  Each matrix is given column-major
// (ut: n columns of m entries, column j at ut + j*m); on return the columns hold
// U S (unsorted) and vt holds V column-major (n columns of n).  Returns sweeps.
struct JacobiBatch {
    int count, m, n;
    double *ut;   // count * n * m
    double *vt;   // count * n * n
    long strideU, strideV;
};
// Device-driven convergence (graph capture): the solver enqueues `sweeps`
// sweeps and reads nothing back; once a sweep makes no rotation the remaining
// launches return at once.  Rotations still made in the last sweep set
// *status = code, non-finite pairs *status = code + 2.
struct DevLoop {
    int sweeps;
    int *status;
    int code;
};
// work: count * (n + 1) doubles (per-matrix scale, then column norms); flags_dev:
// 2 * count + 1 ints.  With dl the return value is -1 (sweeps not known on the host).
int jacobi_svd(const JacobiBatch &jb, int max_sweeps, int *flags_dev, double *work, hipStream_t st,
               const DevLoop *dl = nullptr);
// true when jacobi_svd solves the batch in a single launch (its sweeps loop on
// the device; no sweep cap is needed when it is recorded)
bool jacobi_one_launch(const JacobiBatch &jb);
// After jacobi_svd: s (count x n) descending singular values, U columns normalized
// and sorted into u_sorted (row-major m x n, may be null), V sorted into v_sorted
// (row-major n x n).
// Symmetric eigen-decomposition (two-sided block Jacobi) of `count` n x n
// matrices K (row-major, symmetrised on load): lam (count x n) descending,
// vec (count x n x n) row-major with eigenvector j in column j.  ws / iws:
// device scratch of eigh_ws_doubles / eigh_iws_ints entries.  Returns sweeps.
size_t eigh_ws_doubles(int count, int n);
size_t eigh_iws_ints(int count, int n);
int eigh_sym(const double *K, int count, int n, double *lam, double *vec, double *ws, int *iws, int max_sweeps,
             hipStream_t st);
// Batched Cholesky K = L L^T in place (lower, upper zeroed) of `count` n x n
// matrices; ws: chol_ws_doubles entries; status_dev: count ints.  Returns
// false (after synchronising) if any pivot was not positive and finite.
size_t chol_ws_doubles(int count, int n);
bool cholesky_batched(double *K, int count, int n, double *ws, int *status_dev, hipStream_t st);
// Pivoted variant: K (count x n x n, n <= 1024) is overwritten; X (count x n x n)
// receives X = P L with K = X X^T.  iws: pchol_iws_ints ints, 8-byte aligned.
// tol = 0: false if a pivot was not positive and finite (X then undefined).
// tol > 0: a matrix's factorisation stops at the first pivot at or below tol
// times its first pivot and the remaining columns of X are zero; false only for
// a non-finite pivot.  rank (host, count ints, optional): columns formed.
// dstatus (device int, optional): nothing is read back; a failed pivot sets
// *dstatus = 4 and the call returns true.
size_t pchol_iws_ints(int count, int n);
bool pivoted_cholesky_batched(double *K, int count, int n, double *X, int *iws, hipStream_t st, double tol = 0.0,
                              int *rank = nullptr, int *dstatus = nullptr);
void jacobi_finish(const JacobiBatch &jb, double *s, double *u_sorted, double *v_sorted,
                   double *work, hipStream_t st);

inline unsigned cdiv(size_t a, size_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace trg
