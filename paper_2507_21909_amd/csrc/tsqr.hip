// Tall-skinny Householder QR (TSQR) for the QR factorizations of the RG step:
// the re-split QR(Phi), QR(Psi) (Fig. 5f), the QR of the bond-swap sketches
// (App. A, eq. bond1 / bond2) and, in exact mode, the QR of B and C (App. A).
//
// Level l splits its rows into blocks of 256 rows; one workgroup factors a
// block with Householder reflections (LAPACK dlarfg / dlarf order), one row of
// the block per thread held in registers, and writes the n x n R factor and
// the explicit 256 x n thin Q (dorg2r order).  The reflectors wait in the
// block's own rows of the Q output (each thread reads back only its row), so
// the kernel needs no large LDS buffer and, at up to 256 registers per lane,
// two blocks share a CU and hide each other's reduction latency.  The stacked R factors are the
// next level's input; the last level (one block) fixes diag(R) >= 0.  Q is
// then rebuilt top-down: Q_l[block b] = Q_l,b * Q_{l+1}[b*n:(b+1)*n, :], a
// batched GEMM per level.
#include <cmath>

#include <cstdio>
#include <cstdlib>

#include "common.h"

namespace trg {

namespace {
constexpr int NT = 256;

// Block factorisation: one row of the 256-row block per thread (NC >= n
// columns in registers), Householder column by column with the dot products of
// the reflector with every column (v^T A) reduced at once: a reduce-scatter
// butterfly across the wavefront, then the 4 wavefronts in LDS.
constexpr int RB = 256;   // rows per block

// reduce-scatter halving steps: CNT live values in v[0..CNT); the partner
// (lane ^ off) keeps the other half; all indices compile-time.  The first step
// (off 32) is wg_sum's own, so v holds NC / 2 values
template <int NC, int CNT>
__device__ inline void halve_rest(double (&v)[NC / 2], int lane, int &idx) {
    if constexpr (CNT > 1) {
        constexpr int half = CNT / 2, off = 32 * CNT / NC;
        const bool hi = lane & off;
#pragma unroll
        for (int i = 0; i < half; ++i) {
            const double send = hi ? v[i] : v[half + i], keep = hi ? v[half + i] : v[i];
            v[i] = keep + __shfl_xor(send, off, 64);
        }
        idx += hi ? half : 0;
        halve_rest<NC, half>(v, lane, idx);
    }
}

// sum over the workgroup of s * x[0..NC) (per thread); result in out[0..NC)
// (LDS).  The first halving step reads s * x directly, so the products never
// take NC registers of their own.
template <int NC>
__device__ inline void wg_sum(const double (&x)[NC], double s, double (*red)[NC], double *out) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    constexpr int H = NC / 2;
    const bool hi = lane & 32;
    double v[H];
#pragma unroll
    for (int i = 0; i < H; ++i) {
        const double send = s * (hi ? x[i] : x[H + i]), keep = s * (hi ? x[H + i] : x[i]);
        v[i] = keep + __shfl_xor(send, 32, 64);
    }
    int idx = hi ? H : 0;
    halve_rest<NC, H>(v, lane, idx);
    // v[0] holds value idx summed over the lanes that differ in the top bits;
    // finish over the low 64 / NC lanes
#pragma unroll
    for (int off = (64 / NC) / 2; off > 0; off >>= 1) v[0] += __shfl_xor(v[0], off, 64);
    if ((lane & (64 / NC - 1)) == 0) red[w][idx] = v[0];
    __syncthreads();
    if ((int)threadIdx.x < NC) out[threadIdx.x] = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] +
                                                 red[3][threadIdx.x];
    __syncthreads();
}

template <int NC>
__global__ __launch_bounds__(NT, 2) void qr_block_reg_kernel(const double *a_in, long rows, int n, double *rout,
                                                             double *qout, int final_level) {
    __shared__ double red[4][NC];
    __shared__ double wsum[NC], taus[NC], dsg[NC];
    __shared__ double ab[2];
    const int t = threadIdx.x, b = blockIdx.x;
    const long row = (long)b * RB + t;
    double a[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) a[c] = (row < rows && c < n) ? a_in[row * n + c] : 0.0;
    for (int j = 0; j < n; ++j) {
        double x = 0.0;
#pragma unroll
        for (int c = 0; c < NC; ++c) x = c == j ? a[c] : x;
        // xnorm2 = sum_{i > j} x_i^2, alpha = x_j
        {
            double p2[2] = {t > j ? x * x : 0.0, t == j ? x : 0.0};
            const int lane = t & 63, w = t >> 6;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                p2[0] += __shfl_xor(p2[0], off, 64);
                p2[1] += __shfl_xor(p2[1], off, 64);
            }
            if (lane == 0) {
                red[w][0] = p2[0];
                red[w][1] = p2[1];
            }
            __syncthreads();
            if (t < 2) ab[t] = red[0][t] + red[1][t] + red[2][t] + red[3][t];
            __syncthreads();
        }
        const double xnorm2 = ab[0], alpha = ab[1];
        double tau = 0.0, beta = alpha, scal = 0.0;
        if (xnorm2 > 0.0) {
            const double nrm = sqrt(alpha * alpha + xnorm2);
            beta = alpha >= 0.0 ? -nrm : nrm;
            tau = (beta - alpha) / beta;
            scal = 1.0 / (alpha - beta);
        }
        if (t == 0) taus[j] = tau;
        double vt = 0.0;
        if (t == j) vt = 1.0;
        else if (t > j) vt = tau != 0.0 ? x * scal : x;
        const double newx = t == j ? beta : (t > j ? vt : x);
#pragma unroll
        for (int c = 0; c < NC; ++c) a[c] = c == j ? newx : a[c];
        if (tau == 0.0) continue;   // uniform
        wg_sum<NC>(a, vt, red, wsum);
        const double tv = tau * vt;
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (c > j) a[c] -= tv * wsum[c];
    }
    // R rows (thread t < n owns row t) with the final level's sign
    if (t < n) {
        double d = 0.0;
#pragma unroll
        for (int c = 0; c < NC; ++c) d = c == t ? a[c] : d;
        dsg[t] = (final_level && d < 0.0) ? -1.0 : 1.0;
    }
    // reflectors (row t of V, below the diagonal) into this thread's own row of
    // the Q output, read back by the same thread below
    double *qo = qout + (long)b * RB * n;
#pragma unroll
    for (int c = 0; c < NC; ++c)
        if (c < n) qo[(long)t * n + c] = a[c];
    __syncthreads();
    if (t < n) {
        const double sg = dsg[t];
#pragma unroll
        for (int c = 0; c < NC; ++c)
            if (c < n) rout[((long)b * n + t) * n + c] = c >= t ? sg * a[c] : 0.0;
    }
    // explicit thin Q (dorg2r): Q = H_0 ... H_{n-1} [I; 0], row t in registers
    double q[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) q[c] = (t == c && c < n) ? 1.0 : 0.0;
    // v of the next column is fetched one step ahead (barriers wait on LDS only,
    // so the load overlaps the current step's reductions)
    double vnext = t > n - 1 ? qo[(long)t * n + n - 1] : 0.0;
    for (int j = n - 1; j >= 0; --j) {
        const double vcur = vnext;
        if (j > 0) vnext = t > j - 1 ? qo[(long)t * n + j - 1] : 0.0;
        const double tau = taus[j];
        if (tau == 0.0) continue;   // uniform
        const double vt = t == j ? 1.0 : (t > j ? vcur : 0.0);
        wg_sum<NC>(q, vt, red, wsum);
        const double tv = tau * vt;
#pragma unroll
        for (int c = 0; c < NC; ++c) q[c] -= tv * wsum[c];
    }
#pragma unroll
    for (int c = 0; c < NC; ++c)
        if (c < n) qo[(long)t * n + c] = q[c] * dsg[c];
}

struct Level {
    long rows;
    int nb;
    double *in;   // rows x n
    double *q;    // nb x BR x n
};
}  // namespace

size_t tsqr_ws_doubles(long m, int n) {
    const int BR = RB;
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

namespace {
template <int NC>
void launch_block_reg(int nb, const double *in, long rows, int n, double *rs, double *q, bool fin, hipStream_t st) {
    hipLaunchKernelGGL(qr_block_reg_kernel<NC>, dim3(nb), dim3(NT), 0, st, in, rows, n, rs, q, fin ? 1 : 0);
}
}  // namespace

void tsqr(const double *a, long m, int n, double *q, double *r, double *ws, hipStream_t st) {
    TRG_REQUIRE(n >= 1 && n <= 64, -6, "tsqr: n must be in [1, 64]");
    TRG_REQUIRE(m >= n, -6, "tsqr: needs m >= n");
    static const bool trace = [] {
        const char *e = getenv("TRG_SHAPE_TRACE");
        return e && *e && *e != '0';
    }();
    if (trace) fprintf(stderr, "[tsqr] m %ld n %d\n", m, n);
    const int BR = RB;
    Level lv[64];   // rows shrink by 4x or more per level: far fewer levels than this
    int nlv = 0;
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
        if (n <= 16) launch_block_reg<16>(L.nb, in, rows, n, rs, L.q, fin, st);
        else if (n <= 32) launch_block_reg<32>(L.nb, in, rows, n, rs, L.q, fin, st);
        else launch_block_reg<64>(L.nb, in, rows, n, rs, L.q, fin, st);
        TRG_HIP_CHECK(hipGetLastError());
        TRG_REQUIRE(nlv < 64, -6, "tsqr: too many levels");
        lv[nlv++] = L;
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
    const double *upper = lv[nlv - 1].q;   // rows_L x n (padded to BR)
    for (int l = nlv - 2; l >= 0; --l) {
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
