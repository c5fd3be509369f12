// Tall-skinny Householder QR (TSQR) for the QR factorizations of the RG step:
// the re-split QR(Phi), QR(Psi) (Fig. 5f), the QR of the bond-swap sketches
// (App. A, eq. bond1 / bond2) and, in exact mode, the QR of B and C (App. A).
//
// Level l splits its rows into blocks of BR rows; one workgroup loads a block
// into LDS, factors it with Householder reflections (LAPACK dlarfg / dlarf
// order) and writes the n x n R factor and the explicit BR x n thin Q (dorg2r,
// formed in place).  The stacked R factors are the next level's input; the
// last level (one block) fixes diag(R) >= 0.  Q is then rebuilt top-down:
// Q_l[block b] = Q_l,b * Q_{l+1}[b*n:(b+1)*n, :], a batched GEMM per level.
#include <cmath>

#include "common.h"

namespace trg {

namespace {
constexpr int NT = 256;

// LDS per workgroup available to one kernel (queried once; 64 KiB if unknown)
size_t lds_limit() {
    static size_t lim = 0;
    if (!lim) {
        int dev = 0, v = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0) {
            (void)hipGetLastError();
            v = 65536;
        }
        lim = (size_t)v;
    }
    return lim;
}

inline size_t lds_bytes(int br, int n) { return ((size_t)br * n + 64 + 8 + 256) * sizeof(double) + 64 * sizeof(double); }

// rows per block: the largest of 1024, 512, 256, 128, 64 (and >= n) whose tile fits in LDS
inline int block_rows(int n) {
    for (int br : {1024, 512, 256, 128, 64})
        if (br >= n && lds_bytes(br, n) <= lds_limit() && (size_t)br * n <= 16384) return br;
    return 64;
}

__device__ double block_sum(double v, double *red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) red[w] = v;
    __syncthreads();
    double s = red[0] + red[1] + red[2] + red[3];
    return s;
}

// a: rows x n row-major (this level's input); block b covers rows [b*BR, b*BR+BR)
__global__ __launch_bounds__(NT) void qr_block_kernel(const double *a, long rows, int n, int BR,
                                                      double *rout,   // (nb*n) x n stacked R
                                                      double *qout,   // nb x BR x n thin Q
                                                      int final_level) {
    extern __shared__ double lds[];
    double *A = lds;                    // BR x n
    double *tau = lds + (long)BR * n;   // n
    double *red = tau + 64;             // 8
    double *wv = red + 8;               // 4 x 64 partial dots
    const int b = blockIdx.x;
    const long r0 = (long)b * BR;
    const int t = threadIdx.x;
    for (int i = t; i < BR * n; i += NT) {
        long r = r0 + i / n;
        A[i] = r < rows ? a[r * n + (i % n)] : 0.0;
    }
    __syncthreads();
    const int cc = t & 63, part = t >> 6;   // column / row-quarter for the dot products
    for (int j = 0; j < n; ++j) {
        // norm of A[j+1:, j]
        double s = 0.0;
        for (int i = j + 1 + t; i < BR; i += NT) s += A[i * n + j] * A[i * n + j];
        double xnorm2 = block_sum(s, red);
        double alpha = A[j * n + j];
        double tj = 0.0, beta = alpha, scal = 0.0;
        if (xnorm2 > 0.0) {
            double nrm = sqrt(alpha * alpha + xnorm2);
            beta = alpha >= 0.0 ? -nrm : nrm;
            tj = (beta - alpha) / beta;
            scal = 1.0 / (alpha - beta);
        }
        __syncthreads();
        if (tj != 0.0)
            for (int i = j + 1 + t; i < BR; i += NT) A[i * n + j] *= scal;
        if (t == 0) { tau[j] = tj; A[j * n + j] = beta; }
        __syncthreads();
        if (tj == 0.0) continue;
        // w_c = v^T A[j:, c], v = [1; A[j+1:, j]]
        const int nc = n - j - 1;
        if (cc < nc) {
            const int c = j + 1 + cc;
            double acc = 0.0;
            for (int i = j + part; i < BR; i += 4) {
                double vi = (i == j) ? 1.0 : A[i * n + j];
                acc += vi * A[i * n + c];
            }
            wv[part * 64 + cc] = acc;
        }
        __syncthreads();
        for (int idx = t; idx < (BR - j) * nc; idx += NT) {
            int i = j + idx / nc, c = j + 1 + idx % nc;
            double vi = (i == j) ? 1.0 : A[i * n + j];
            double w = wv[c - j - 1] + wv[64 + c - j - 1] + wv[128 + c - j - 1] + wv[192 + c - j - 1];
            A[i * n + c] -= tj * vi * w;
        }
        __syncthreads();
    }
    // R (upper triangle), with the sign of the final level
    __shared__ double dsg[64];
    if (t < n) dsg[t] = (final_level && A[t * n + t] < 0.0) ? -1.0 : 1.0;
    __syncthreads();
    for (int i = t; i < n * n; i += NT) {
        int r = i / n, c = i % n;
        rout[((long)b * n + r) * n + c] = c >= r ? dsg[r] * A[r * n + c] : 0.0;
    }
    __syncthreads();
    // explicit thin Q in place (dorg2r)
    for (int j = n - 1; j >= 0; --j) {
        const double tj = tau[j];
        const int nc = n - j - 1;
        if (nc > 0) {
            if (t == 0) A[j * n + j] = 1.0;
            __syncthreads();
            if (cc < nc && tj != 0.0) {
                const int c = j + 1 + cc;
                double acc = 0.0;
                for (int i = j + part; i < BR; i += 4) acc += A[i * n + j] * A[i * n + c];
                wv[part * 64 + cc] = acc;
            }
            __syncthreads();
            if (tj != 0.0)
                for (int idx = t; idx < (BR - j) * nc; idx += NT) {
                    int i = j + idx / nc, c = j + 1 + idx % nc;
                    double w = wv[c - j - 1] + wv[64 + c - j - 1] + wv[128 + c - j - 1] + wv[192 + c - j - 1];
                    A[i * n + c] -= tj * A[i * n + j] * w;
                }
            __syncthreads();
        }
        for (int i = j + 1 + t; i < BR; i += NT) A[i * n + j] *= -tj;
        if (t == 0) A[j * n + j] = 1.0 - tj;
        for (int i = t; i < j; i += NT) A[i * n + j] = 0.0;
        __syncthreads();
    }
    double *q = qout + (long)b * BR * n;
    for (int i = t; i < BR * n; i += NT) q[i] = A[i] * dsg[i % n];
}

struct Level {
    long rows;
    int nb;
    double *in;   // rows x n
    double *q;    // nb x BR x n
};
}  // namespace

size_t tsqr_ws_doubles(long m, int n) {
    const int BR = block_rows(n);
    size_t tot = 0;
    long rows = m;
    while (true) {
        long nb = (rows + BR - 1) / BR;
        tot += (size_t)nb * BR * n;           // q of this level
        tot += (size_t)nb * n * n;            // stacked R (next level input / final R)
        if (nb == 1) break;
        rows = nb * n;
    }
    long nb0 = (m + BR - 1) / BR;
    tot += 2 * (size_t)nb0 * BR * n;          // ping-pong for the rebuilt Q
    return tot + 64;
}

void tsqr(const double *a, long m, int n, double *q, double *r, double *ws, hipStream_t st) {
    TRG_REQUIRE(n >= 1 && n <= 64, -6, "tsqr: n must be in [1, 64]");
    TRG_REQUIRE(m >= n, -6, "tsqr: needs m >= n");
    const int BR = block_rows(n);
    const size_t lds = ((size_t)BR * n + 64 + 8 + 256) * sizeof(double);
    TRG_REQUIRE(lds_bytes(BR, n) <= lds_limit(), -6, "tsqr: LDS tile does not fit");
    static size_t attr_set = 0;
    if (lds > 65536 && lds > attr_set) {
        if (hipFuncSetAttribute(reinterpret_cast<const void *>(qr_block_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
            (void)hipGetLastError();
        attr_set = lds;
    }
    std::vector<Level> lv;
    double *p = ws;
    const double *in = a;
    long rows = m;
    while (true) {
        Level L;
        L.rows = rows;
        L.nb = (int)((rows + BR - 1) / BR);
        L.in = const_cast<double *>(in);
        L.q = p;
        p += (size_t)L.nb * BR * n;
        double *rs = p;
        p += (size_t)L.nb * n * n;
        bool fin = L.nb == 1;
        hipLaunchKernelGGL(qr_block_kernel, dim3(L.nb), dim3(NT), lds, st, in, rows, n, BR, rs, L.q, fin ? 1 : 0);
        TRG_HIP_CHECK(hipGetLastError());
        lv.push_back(L);
        if (fin) {
            copy(r, rs, (size_t)n * n, st);
            break;
        }
        in = rs;
        rows = (long)L.nb * n;
    }
    // rebuild Q top-down
    long nb0 = lv[0].nb;
    double *bufA = p, *bufB = p + (size_t)nb0 * BR * n;
    const double *upper = lv.back().q;   // rows_L x n (padded to BR)
    for (int l = (int)lv.size() - 2; l >= 0; --l) {
        double *dst = (l % 2 == 0) ? bufA : bufB;
        GemmArgs g{};
        g.M = BR; g.N = n; g.K = n; g.batch = lv[l].nb;
        g.A = lv[l].q; g.sAr = n; g.sAk = 1; g.sAb = (long)BR * n;
        g.B = upper; g.sBk = n; g.sBn = 1; g.sBb = (long)n * n;
        g.C = dst; g.sCr = n; g.sCn = 1; g.sCb = (long)BR * n;
        g.alpha = 1.0; g.beta = 0.0;
        gemm(g, P_FP64, st);
        upper = dst;
    }
    copy(q, upper, (size_t)m * n, st);
}

}  // namespace trg
