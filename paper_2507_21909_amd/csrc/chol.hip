// Batched Cholesky factorisation K = L L^T of symmetric positive definite
// matrices, for the square roots of the squeezer environment Grams (Sec. II A):
// R = L^T satisfies R^T R = K, and any two square roots of K differ by an
// orthogonal factor on the left, which cancels in the squeezer pair
// E = R_b^T V S^-1/2, F = R_f^T U S^-1/2 (U S V^T the SVD of R_f R_b^T).
//
// Right-looking, blocks of 64: the diagonal block is factorised in LDS by one
// workgroup per matrix (which also inverts it), the panel below is multiplied
// by that inverse (GEMM), and the trailing matrix takes the rank-64 update
// (GEMM, alpha = -1, beta = 1).  The pivoted variant (diagonal pivoting, as
// LAPACK's dpstrf) factors 24-column panels in one 1024-thread workgroup per
// matrix, each row in one thread's registers, and gives K = X X^T with
// X = P L, whose columns are graded like the eigen-decomposition's
// W Lambda^{1/2}.  A pivot that is not positive and finite marks
// the matrix in status[] (the caller then takes the eigen-decomposition route),
// unless a relative tolerance is given: then the factorisation of a matrix stops
// at the first pivot at or below tol times its first (largest) one, and the
// columns from there on are zero.  The Schur complement left out is positive
// semi-definite with every diagonal entry at or below that pivot, so for a
// tolerance at the rounding level of K the truncated X X^T is K to that level.
#include <algorithm>
#include <cmath>
#include <cstdint>

#include "common.h"

namespace trg {

namespace {
constexpr int CB = 64;       // block edge
constexpr int CT = 256;      // threads per workgroup
constexpr int CLD = CB + 1;  // LDS row stride

// Factor K[j0:j0+nb, j0:j0+nb] of matrix blockIdx.x in place (lower triangle,
// upper set to zero); winv <- (L_jj^-1)^T (nb x nb, row-major, stride CB).
__global__ __launch_bounds__(CT) void chol_diag_kernel(double *K, int n, int j0, int nb, double *winv,
                                                      int *status) {
    __shared__ double a[CB * CLD];
    __shared__ double x[CB * CLD];
    const int mat = blockIdx.x, t = threadIdx.x;
    double *Km = K + (size_t)mat * n * n;
    for (int e = t; e < nb * nb; e += CT) {
        const int i = e / nb, j = e % nb;
        a[i * CLD + j] = Km[(size_t)(j0 + i) * n + j0 + j];
    }
    __syncthreads();
    for (int k = 0; k < nb; ++k) {
        if (t == 0) {
            double d = a[k * CLD + k];
            if (!(d > 0.0) || !isfinite(d)) {
                status[mat] = 1;
                d = 1.0;
            }
            a[k * CLD + k] = sqrt(d);
        }
        __syncthreads();
        const double dk = a[k * CLD + k];
        for (int i = k + 1 + t; i < nb; i += CT) a[i * CLD + k] /= dk;
        __syncthreads();
        const int m = nb - k - 1;
        for (int e = t; e < m * m; e += CT) {
            const int i = k + 1 + e / m, j = k + 1 + e % m;
            if (j <= i) a[i * CLD + j] -= a[i * CLD + k] * a[j * CLD + k];
        }
        __syncthreads();
    }
    // X = L^-1 by forward substitution, one column per thread
    if (t < nb) {
        const int c = t;
        for (int i = 0; i < nb; ++i) {
            double s = i == c ? 1.0 : 0.0;
            for (int k = c; k < i; ++k) s -= a[i * CLD + k] * x[k * CLD + c];
            x[i * CLD + c] = i < c ? 0.0 : s / a[i * CLD + i];
        }
    }
    __syncthreads();
    for (int e = t; e < nb * nb; e += CT) {
        const int i = e / nb, j = e % nb;
        Km[(size_t)(j0 + i) * n + j0 + j] = j <= i ? a[i * CLD + j] : 0.0;
        winv[(size_t)mat * CB * CB + i * CB + j] = x[j * CLD + i];   // (L^-1)^T
    }
}

// Pivoted Cholesky without row or column exchanges: X = P L is formed in the
// original row order.  S (overwritten) holds the Schur complement
// K - X[:, :j0] X[:, :j0]^T in original indices, brought up to date after each
// panel of PCW columns by one GEMM over the whole matrix.  Thread i keeps row i
// of the panel's columns in registers.  Column j takes the unchosen index p with
// the largest remaining diagonal d_p (ties: lowest index), reads row p of S
// (contiguous), and sets x_i = (S[p, i] - sum over the panel's earlier columns
// k of X[i, k] X[p, k]) / sqrt(d_p), with x_p = sqrt(d_p) and x = 0 at indices
// chosen before; then d_i -= x_i^2.
constexpr int PCW = 24;     // panel width (the row, 2 * PCW registers, fits 1024 threads)
constexpr int PCT = 1024;   // threads: one per row (n <= 1024)

// rk[mat]: columns formed (n unless the factorisation stopped); dtop[mat]: the
// first pivot; perm[mat][j]: the index chosen for column j.
__global__ __launch_bounds__(PCT) void pchol_panel_kernel(double *S, int n, int j0, int nb, int *perm,
                                                         int *status, int *rk, double *dtop, double tol,
                                                         double *X) {
    __shared__ unsigned char chosen[PCT];
    __shared__ double pv[PCT / 64];
    __shared__ int pi[PCT / 64];
    __shared__ double rowp[PCW];
    const int mat = blockIdx.x, i = threadIdx.x, lane = i & 63, w = i >> 6;
    if (rk[mat] < n || status[mat]) return;   // stopped in an earlier panel (uniform)
    const double *Sm = S + (size_t)mat * n * n;
    double *Xm = X + (size_t)mat * n * n;
    int *pm = perm + (size_t)mat * n;
    chosen[i] = 0;
    __syncthreads();
    for (int k = i; k < j0; k += PCT) chosen[pm[k]] = 1;
    __syncthreads();
    bool mine = i >= n || chosen[i];   // row i already has its pivot (or is padding)
    double dd = mine ? 0.0 : Sm[(size_t)i * n + i];
    double d0 = j0 > 0 ? dtop[mat] : 0.0;
    double xr[PCW];
#pragma unroll
    for (int k = 0; k < PCW; ++k) xr[k] = 0.0;
    // xr[k] = 0 for the panel's columns not formed yet, so every step runs the
    // full-width dot product and all register indices are compile-time constants
    for (int jj = 0; jj < nb; ++jj) {
        // argmax over the unchosen rows; NaN never wins
        double bv = (mine || !(dd == dd)) ? -INFINITY : dd;
        int bi = mine ? PCT : i;
        for (int o = 32; o > 0; o >>= 1) {
            const double ov = __shfl_xor(bv, o, 64);
            const int oi = __shfl_xor(bi, o, 64);
            if (ov > bv || (ov == bv && oi < bi)) {
                bv = ov;
                bi = oi;
            }
        }
        if (lane == 0) {
            pv[w] = bv;
            pi[w] = bi;
        }
        __syncthreads();
        double v = pv[0];
        int p = pi[0];
        for (int x = 1; x < PCT / 64; ++x) {
            const double ov = pv[x];
            const int oi = pi[x];
            if (ov > v || (ov == v && oi < p)) {
                v = ov;
                p = oi;
            }
        }
        if (j0 + jj == 0) d0 = v;
        // every thread reaches the same verdict from the same LDS values
        int stop = 0;
        if (!isfinite(v) || p >= n)
            stop = 1;
        else if (tol > 0.0 ? v <= tol * d0 : !(v > 0.0))
            stop = tol > 0.0 ? 2 : 1;
        if (stop) {
            if (i == 0) {
                if (stop == 1) status[mat] = 1;   // the caller falls back
                else rk[mat] = j0 + jj;           // rank j0 + jj: columns from here on stay zero
            }
            break;
        }
        if (i == p) {
#pragma unroll
            for (int k = 0; k < PCW; ++k) rowp[k] = xr[k];
        }
        if (i == 0) pm[j0 + jj] = p;
        __syncthreads();
        if (i < n) {
            const double ljj = sqrt(v);
            double a = Sm[(size_t)p * n + i];
#pragma unroll
            for (int k = 0; k < PCW; ++k) a -= xr[k] * rowp[k];
            const double x = i == p ? ljj : (mine ? 0.0 : a / ljj);
#pragma unroll
            for (int k = 0; k < PCW; ++k) xr[k] = k == jj ? x : xr[k];
            if (i == p) mine = true;
            if (!mine) dd -= x * x;
        }
    }
    if (j0 == 0 && i == 0) dtop[mat] = d0;
    if (i < n) {
#pragma unroll
        for (int k = 0; k < PCW; ++k)
            if (k < nb) Xm[(size_t)i * n + j0 + k] = xr[k];
    }
}

__global__ void perm_init_kernel(int *perm, int *rk, int *status, int n, int count) {
    const long tot = (long)count * n;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
        perm[e] = (int)(e % n);
        if (e < count) {
            rk[e] = n;
            status[e] = 0;
        }
    }
}

// zero above the diagonal and, with rk, the columns past each matrix's rank
__global__ void zero_upper_kernel(double *K, int n, int count, const int *rk) {
    const long tot = (long)count * n * n;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
        const long mat = e / ((long)n * n), rem = e % ((long)n * n);
        const int i = (int)(rem / n), j = (int)(rem % n);
        if (j > i || (rk && j >= rk[mat])) K[e] = 0.0;
    }
}

// device-side verdict of the pivoted factorisation: a non-finite pivot in any
// matrix sets *dstatus = 4
__global__ void pchol_check_kernel(const int *status, int count, int *dstatus) {
    if (threadIdx.x) return;
    for (int i = 0; i < count; ++i)
        if (status[i]) *dstatus = 4;
}
}  // namespace

size_t chol_ws_doubles(int count, int n) { return (size_t)count * (CB * CB + (size_t)n * CB) + 64; }

// ints: dtop (count doubles), status (count), rk (count), perm (count * n)
size_t pchol_iws_ints(int count, int n) { return (size_t)count * (n + 4) + 16; }

bool pivoted_cholesky_batched(double *K, int count, int n, double *X, int *iws, hipStream_t st, double tol,
                              int *rank, int *dstatus) {
    TRG_REQUIRE(!(dstatus && rank), -1, "pivoted Cholesky: no host rank with a device status");
    if (count == 0 || n == 0) return true;
    TRG_REQUIRE(n <= 1024, -6, "pivoted Cholesky: n > 1024");
    TRG_REQUIRE(tol >= 0.0 && tol < 1.0, -1, "pivoted Cholesky: tolerance outside [0, 1)");
    TRG_REQUIRE(reinterpret_cast<uintptr_t>(iws) % alignof(double) == 0, -1, "pivoted Cholesky: iws not 8-aligned");
    double *dtop = reinterpret_cast<double *>(iws);
    int *status = iws + 2 * count, *rk = status + count, *perm = rk + count;
    const unsigned gb = (unsigned)std::min<size_t>(((size_t)count * n + 255) / 256, 65536);
    hipLaunchKernelGGL(perm_init_kernel, dim3(gb), dim3(256), 0, st, perm, rk, status, n, count);
    fill(X, (size_t)count * n * n, 0.0, st);
    for (int j0 = 0; j0 < n; j0 += PCW) {
        const int nb = std::min(PCW, n - j0);
        hipLaunchKernelGGL(pchol_panel_kernel, dim3(count), dim3(PCT), 0, st, K, n, j0, nb, perm, status, rk, dtop,
                           tol, X);
        TRG_HIP_CHECK(hipGetLastError());
        if (j0 + nb == n) break;
        // Schur complement: K -= X[:, j0:j0+nb] X[:, j0:j0+nb]^T
        GemmArgs h{};
        h.M = n; h.N = n; h.K = nb; h.batch = count;
        h.A = X + j0; h.sAr = n; h.sAk = 1; h.sAb = (long)n * n;
        h.B = X + j0; h.sBk = 1; h.sBn = n; h.sBb = (long)n * n;
        h.C = K; h.sCr = n; h.sCn = 1; h.sCb = (long)n * n;
        h.alpha = -1.0; h.beta = 1.0;
        gemm(h, P_FP64, st);
    }
    if (dstatus) {
        hipLaunchKernelGGL(pchol_check_kernel, dim3(1), dim3(64), 0, st, status, count, dstatus);
        TRG_HIP_CHECK(hipGetLastError());
        return true;
    }
    std::vector<int> fl(2 * count);   // status, then rk
    TRG_HIP_CHECK(hipMemcpyAsync(fl.data(), status, sizeof(int) * 2 * count, hipMemcpyDeviceToHost, st));
    TRG_HIP_CHECK(hipStreamSynchronize(st));
    if (rank) std::copy(fl.begin() + count, fl.end(), rank);
    for (int i = 0; i < count; ++i)
        if (fl[i]) return false;
    return true;
}

bool cholesky_batched(double *K, int count, int n, double *ws, int *status_dev, hipStream_t st) {
    if (count == 0 || n == 0) return true;
    TRG_HIP_CHECK(hipMemsetAsync(status_dev, 0, sizeof(int) * count, st));
    double *winv = ws, *tmp = ws + (size_t)count * CB * CB;
    for (int j0 = 0; j0 < n; j0 += CB) {
        const int nb = std::min(CB, n - j0), rows = n - j0 - nb;
        hipLaunchKernelGGL(chol_diag_kernel, dim3(count), dim3(CT), 0, st, K, n, j0, nb, winv, status_dev);
        TRG_HIP_CHECK(hipGetLastError());
        if (rows == 0) break;
        // panel: L[j0+nb:, j0:j0+nb] = K[j0+nb:, j0:j0+nb] L_jj^-T
        GemmArgs g{};
        g.M = rows; g.N = nb; g.K = nb; g.batch = count;
        g.A = K + (size_t)(j0 + nb) * n + j0; g.sAr = n; g.sAk = 1; g.sAb = (long)n * n;
        g.B = winv; g.sBk = CB; g.sBn = 1; g.sBb = (long)CB * CB;
        g.C = tmp; g.sCr = nb; g.sCn = 1; g.sCb = (long)rows * nb;
        g.alpha = 1.0; g.beta = 0.0;
        gemm(g, P_FP64, st);
        for (int m = 0; m < count; ++m)
            TRG_HIP_CHECK(hipMemcpy2DAsync(K + (size_t)m * n * n + (size_t)(j0 + nb) * n + j0, sizeof(double) * n,
                                           tmp + (size_t)m * rows * nb, sizeof(double) * nb, sizeof(double) * nb,
                                           rows, hipMemcpyDeviceToDevice, st));
        // trailing update: K[j0+nb:, j0+nb:] -= L_panel L_panel^T
        GemmArgs h{};
        h.M = rows; h.N = rows; h.K = nb; h.batch = count;
        h.A = K + (size_t)(j0 + nb) * n + j0; h.sAr = n; h.sAk = 1; h.sAb = (long)n * n;
        h.B = K + (size_t)(j0 + nb) * n + j0; h.sBk = 1; h.sBn = n; h.sBb = (long)n * n;
        h.C = K + (size_t)(j0 + nb) * n + j0 + nb; h.sCr = n; h.sCn = 1; h.sCb = (long)n * n;
        h.alpha = -1.0; h.beta = 1.0;
        gemm(h, P_FP64, st);
    }
    hipLaunchKernelGGL(zero_upper_kernel, dim3(std::min<size_t>(((size_t)count * n * n + 255) / 256, 65536)),
                       dim3(256), 0, st, K, n, count, nullptr);
    TRG_HIP_CHECK(hipGetLastError());
    std::vector<int> fl(count);
    TRG_HIP_CHECK(hipMemcpyAsync(fl.data(), status_dev, sizeof(int) * count, hipMemcpyDeviceToHost, st));
    TRG_HIP_CHECK(hipStreamSynchronize(st));
    for (int f : fl)
        if (f) return false;
    return true;
}

}  // namespace trg
