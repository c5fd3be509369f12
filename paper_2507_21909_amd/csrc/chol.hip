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
// LAPACK's dpstrf) factors each 64-column panel in one workgroup per matrix
// and gives K = X X^T with X = P L, whose columns are graded like the
// eigen-decomposition's W Lambda^{1/2}.  A pivot that is not positive and finite marks
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

// Pivoted panel: columns j0 .. j0 + nb - 1 of matrix blockIdx.x with diagonal
// (symmetric) pivoting.  Before step j the trailing matrix A[j:, j:] holds K
// minus the updates of all earlier panels (not yet those of this panel's
// columns, which are applied to column j and to the diagonal as they are
// needed).  Step j picks the largest remaining diagonal, swaps rows and
// columns j and p of the whole matrix (and perm), and forms column j of L.
// rk[mat]: columns formed (n unless the factorisation stopped); dtop[mat]: the first pivot.
__global__ __launch_bounds__(CT) void pchol_panel_kernel(double *K, int n, int j0, int nb, int *perm,
                                                        int *status, int *rk, double *dtop, double tol) {
    __shared__ double dd[1024];
    __shared__ double rowj[CB];
    __shared__ double rv[CT / 64];
    __shared__ int ri[CT / 64];
    __shared__ int piv;
    __shared__ double dpiv;
    __shared__ double d0;
    __shared__ int stop;
    const int mat = blockIdx.x, t = threadIdx.x, lane = t & 63, w = t >> 6;
    if (rk[mat] < n || status[mat]) return;   // stopped in an earlier panel
    double *A = K + (size_t)mat * n * n;
    int *pm = perm + (size_t)mat * n;
    if (t == 0) d0 = j0 > 0 ? dtop[mat] : 0.0;
    // diagonal of the trailing matrix, corrected for nothing yet in this panel
    for (int i = j0 + t; i < n; i += CT) dd[i] = A[(size_t)i * n + i];
    __syncthreads();
    for (int j = j0; j < j0 + nb; ++j) {
        // argmax of dd[j:] (ties: lowest index)
        double bv = -1.0;
        int bi = j;
        for (int i = j + t; i < n; i += CT)
            if (dd[i] > bv) { bv = dd[i]; bi = i; }
        for (int o = 32; o > 0; o >>= 1) {
            const double ov = __shfl_xor(bv, o, 64);
            const int oi = __shfl_xor(bi, o, 64);
            if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
        }
        if (lane == 0) { rv[w] = bv; ri[w] = bi; }
        __syncthreads();
        if (t == 0) {
            double v = rv[0];
            int id = ri[0];
            for (int x = 1; x < CT / 64; ++x)
                if (rv[x] > v || (rv[x] == v && ri[x] < id)) { v = rv[x]; id = ri[x]; }
            piv = id;
            dpiv = v;
            if (j == 0) {
                d0 = v;
                dtop[mat] = v;
            }
            int st = 0;
            if (!isfinite(v))
                st = 1;
            else if (tol > 0.0 ? v <= tol * d0 : !(v > 0.0))
                st = tol > 0.0 ? 2 : 1;
            if (st == 1) status[mat] = 1;   // the caller falls back
            if (st == 2) rk[mat] = j;       // rank j: columns j.. stay zero
            stop = st;
        }
        __syncthreads();
        if (stop) return;   // uniform
        const int p = piv;
        if (p != j) {
            for (int c = t; c < n; c += CT) {
                const double x = A[(size_t)j * n + c];
                A[(size_t)j * n + c] = A[(size_t)p * n + c];
                A[(size_t)p * n + c] = x;
            }
            __syncthreads();
            for (int r = t; r < n; r += CT) {
                const double x = A[(size_t)r * n + j];
                A[(size_t)r * n + j] = A[(size_t)r * n + p];
                A[(size_t)r * n + p] = x;
            }
            if (t == 0) {
                const double x = dd[j];
                dd[j] = dd[p];
                dd[p] = x;
                const int y = pm[j];
                pm[j] = pm[p];
                pm[p] = y;
            }
            __syncthreads();
        }
        // row j of this panel's earlier columns
        if (t < j - j0) rowj[t] = A[(size_t)j * n + j0 + t];
        __syncthreads();
        const double ljj = sqrt(dd[j]);
        if (t == 0) A[(size_t)j * n + j] = ljj;
        for (int i = j + 1 + t; i < n; i += CT) {
            double a = A[(size_t)i * n + j];
            const double *li = A + (size_t)i * n + j0;
            for (int k = 0; k < j - j0; ++k) a -= li[k] * rowj[k];
            a /= ljj;
            A[(size_t)i * n + j] = a;
            dd[i] -= a * a;
        }
        __syncthreads();
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

// X[perm[i], :] = L[i, :] (K = X X^T with X = P L)
__global__ void unpermute_rows_kernel(const double *L, const int *perm, int n, int count, double *X) {
    const long tot = (long)count * n * n;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
        const long mat = e / ((long)n * n), rem = e % ((long)n * n);
        const int i = (int)(rem / n), c = (int)(rem % n);
        X[mat * n * n + (long)perm[mat * n + i] * n + c] = L[e];
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
}  // namespace

size_t chol_ws_doubles(int count, int n) { return (size_t)count * (CB * CB + (size_t)n * CB) + 64; }

// ints: dtop (count doubles), status (count), rk (count), perm (count * n)
size_t pchol_iws_ints(int count, int n) { return (size_t)count * (n + 4) + 16; }

bool pivoted_cholesky_batched(double *K, int count, int n, double *X, int *iws, hipStream_t st, double tol,
                              int *rank) {
    if (count == 0 || n == 0) return true;
    TRG_REQUIRE(n <= 1024, -6, "pivoted Cholesky: n > 1024");
    TRG_REQUIRE(tol >= 0.0 && tol < 1.0, -1, "pivoted Cholesky: tolerance outside [0, 1)");
    TRG_REQUIRE(reinterpret_cast<uintptr_t>(iws) % alignof(double) == 0, -1, "pivoted Cholesky: iws not 8-aligned");
    double *dtop = reinterpret_cast<double *>(iws);
    int *status = iws + 2 * count, *rk = status + count, *perm = rk + count;
    const unsigned gb = (unsigned)std::min<size_t>(((size_t)count * n * n + 255) / 256, 65536);
    hipLaunchKernelGGL(perm_init_kernel, dim3(gb), dim3(256), 0, st, perm, rk, status, n, count);
    for (int j0 = 0; j0 < n; j0 += CB) {
        const int nb = std::min(CB, n - j0), rows = n - j0 - nb;
        hipLaunchKernelGGL(pchol_panel_kernel, dim3(count), dim3(CT), 0, st, K, n, j0, nb, perm, status, rk, dtop,
                           tol);
        TRG_HIP_CHECK(hipGetLastError());
        if (rows == 0) break;
        GemmArgs h{};
        h.M = rows; h.N = rows; h.K = nb; h.batch = count;
        h.A = K + (size_t)(j0 + nb) * n + j0; h.sAr = n; h.sAk = 1; h.sAb = (long)n * n;
        h.B = K + (size_t)(j0 + nb) * n + j0; h.sBk = 1; h.sBn = n; h.sBb = (long)n * n;
        h.C = K + (size_t)(j0 + nb) * n + j0 + nb; h.sCr = n; h.sCn = 1; h.sCb = (long)n * n;
        h.alpha = -1.0; h.beta = 1.0;
        gemm(h, P_FP64, st);
    }
    hipLaunchKernelGGL(zero_upper_kernel, dim3(gb), dim3(256), 0, st, K, n, count, rk);
    hipLaunchKernelGGL(unpermute_rows_kernel, dim3(gb), dim3(256), 0, st, K, perm, n, count, X);
    TRG_HIP_CHECK(hipGetLastError());
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
