// Tall-skinny Householder QR (TSQR) for the QR factorizations of the RG step:
// the re-split QR(Phi), QR(Psi) (Fig. 5f), the QR of the bond-swap sketches
// (App. A, eq. bond1 / bond2) and, in exact mode, the QR of B and C (App. A).
//
// Level l splits its rows into blocks of 256 rows; one workgroup factors a
// block with Householder reflections (LAPACK dlarfg / dlarf order) and writes
// the n x n R factor and the explicit 256 x n thin Q (dorg2r order).  The
// stacked R factors are the next level's input; the last level (one block)
// fixes diag(R) >= 0.  Q is then rebuilt top-down: Q_l[block b] = Q_l,b *
// Q_{l+1}[b*n:(b+1)*n, :], a batched GEMM per level.
#include <cmath>

#include <cstdio>
#include <cstdlib>
#include <type_traits>

#include "common.h"

namespace trg {

namespace {
constexpr int RB = 256;   // rows per block

// Block factorisation with the block's columns spread over the workgroup: a
// group of TPC = NTH / NC adjacent lanes owns column c, lane q of the group
// holding rows TPC i + q (i < RPT = 256 / TPC) in registers, so every dot
// product of a column with the reflector is RPT products summed pairwise in a
// lane and a log2(TPC)-step butterfly inside the group (the depth of a tree
// over the block's 256 rows).  Step j: the lanes of
// column j form the reflector (norm by the same butterfly) and write it, zero
// above row j, to LDS; after one barrier every column right of j reads it
// there and updates itself, and the workgroup copies it, one row a thread,
// to the block's Q output.  Runs of SK registers whose rows all lie above j
// are skipped (a workgroup-uniform test).  The reflector buffer alternates
// between two slots, so a step needs no second barrier.  Q = H_0 ... H_{n-1}
// [I; 0] is then built the same way, column c of Q in the registers of column
// c's lanes.  1024 threads keep the per-step chain at 16 rows a lane.
// Row tests are written as TPC i against a per-lane offset (j - q, n - q, ...)
// so that no per-register row index is held in registers.
constexpr int NTH = 1024;

// pairwise (tree) sum of f(L) .. f(L + N - 1), N a power of two, with every
// index a compile-time constant so that f can pick registers.  The left half
// is finished before the right half's loads start (an empty asm with a memory
// clobber), which keeps the register count of a sequential sum
template <int L, int N, class F>
__device__ __forceinline__ double tree_sum(const F &f) {
    if constexpr (N == 1) {
        return f(std::integral_constant<int, L>{});
    } else {
        double lo = tree_sum<L, N / 2>(f);
        asm volatile("" : "+v"(lo) : : "memory");
        return lo + tree_sum<L + N / 2, N / 2>(f);
    }
}

template <int NC>
__global__ __launch_bounds__(NTH, 8) void qr_block_kernel(const double *a_in, long rows, int n, double *rout,
                                                       double *qout, int final_level) {
    constexpr int TPC = NTH / NC, RPT = RB / TPC;
    constexpr int SK = RPT >= 16 ? 4 : RPT;
    static_assert(TPC <= 64 && RPT >= 1 && RPT % SK == 0, "column groups must fit a wavefront");
    __shared__ double vb[2][RB];
    __shared__ double taus[NC], betas[NC], dsg[NC], tb[2];
    const int t = threadIdx.x, b = blockIdx.x;
    const int c = t / TPC, q = t % TPC;
    const long row0 = (long)b * RB;
    double *qo = qout + (long)b * RB * n;
    const int lim = (int)(rows - row0 < RB ? rows - row0 : RB) - q;   // rows TPC i + q < rows: TPC i < lim
    double a[RPT];
    {
        const double *src = a_in + (row0 + q) * n + c;
#pragma unroll
        for (int i = 0; i < RPT; ++i) a[i] = (TPC * i < lim && c < n) ? src[(long)TPC * i * n] : 0.0;
    }
    for (int j = 0; j < n; ++j) {
        const int p = j & 1;
        if (c == j) {
            // row TPC i + q is below j when TPC i > jq.  j is laundered so that
            // the compiler does not rewrite it as c and hoist every row test of
            // the loop out of it
            int jj = j;
            asm volatile("" : "+v"(jj));
            const int jq = jj - q;
            // xnorm2 = sum_{r > j} x_r^2, alpha = x_j (dlarfg); x (rows >= j)
            // to the reflector slot
            double al = 0.0;
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                al = TPC * i == jq ? a[i] : al;
                vb[p][TPC * i + q] = TPC * i >= jq ? a[i] : 0.0;
            }
            double s2 = tree_sum<0, RPT>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                return TPC * i > jq ? a[i] * a[i] : 0.0;
            });
#pragma unroll
            for (int off = 1; off < TPC; off <<= 1) {
                s2 += __shfl_xor(s2, off, 64);
                al += __shfl_xor(al, off, 64);
            }
            double tau = 0.0, beta = al, scal = 0.0;
            if (s2 > 0.0) {
                const double nrm = sqrt(al * al + s2);
                beta = al >= 0.0 ? -nrm : nrm;
                tau = (beta - al) / beta;
                scal = 1.0 / (al - beta);
            }
            const double sc = tau != 0.0 ? scal : 1.0;
            // v = (0 above j, 1 at j, x scal below); the column's own
            // registers keep x (R above j)
#pragma unroll
            for (int i = 0; i < RPT; ++i) vb[p][TPC * i + q] *= sc;
            if (q == (j % TPC)) vb[p][j] = 1.0;
            if (q == 0) {
                taus[j] = tau;
                betas[j] = beta;
                tb[p] = tau;
            }
        }
        __syncthreads();
        if (t < RB) qo[(long)j * RB + t] = vb[p][t];   // the reflector, column-major in the block's Q output
        const double tau = tb[p];
        if (c > j && c < n && tau != 0.0) {
            // pairwise over the lane's rows (runs of SK above row j skipped)
            double d = tree_sum<0, RPT / SK>([&](auto kc) {
                constexpr int i0 = decltype(kc)::value * SK;
                if (TPC * (i0 + SK) - 1 < j) return 0.0;
                return tree_sum<i0, SK>([&](auto ic) {
                    constexpr int i = decltype(ic)::value;
                    return vb[p][TPC * i + q] * a[i];
                });
            });
#pragma unroll
            for (int off = 1; off < TPC; off <<= 1) d += __shfl_xor(d, off, 64);
            const double k = tau * d;
            asm volatile("" ::: "memory");   // read the reflector again: 64 registers keep two blocks on a CU
#pragma unroll
            for (int i0 = 0; i0 < RPT; i0 += SK)
                if (TPC * (i0 + SK) - 1 >= j) {
#pragma unroll
                    for (int i = i0; i < i0 + SK; ++i) a[i] -= k * vb[p][TPC * i + q];
                }
        }
    }
    // diagonal signs (the final level makes diag(R) >= 0)
    if (t < n) dsg[t] = (final_level && betas[t] < 0.0) ? -1.0 : 1.0;
    __syncthreads();
    const int cq = c - q;
    if (c < n) {
        const int nq = n - q;
        double *dst = rout + ((long)b * n + q) * n + c;
#pragma unroll
        for (int i = 0; i < RPT; ++i)
            if (TPC * i < nq)
                dst[(long)TPC * i * n] = TPC * i < cq ? dsg[TPC * i + q] * a[i]
                                                      : (TPC * i == cq ? dsg[c] * betas[c] : 0.0);
    }
    // explicit thin Q (dorg2r): the reflector of step j is staged in LDS (row t
    // by thread t < 256, fetched one step ahead)
    double qv[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) qv[i] = TPC * i == cq ? 1.0 : 0.0;
    double vnext = t < RB ? qo[(long)(n - 1) * RB + t] : 0.0;
    for (int j = n - 1; j >= 0; --j) {
        const int p = j & 1;
        if (t < RB) {
            vb[p][t] = vnext;
            if (j > 0) vnext = qo[(long)(j - 1) * RB + t];
        }
        __syncthreads();
        const double tau = taus[j];
        // columns left of j are e_c, untouched by H_j (zero in rows >= j)
        if (c >= j && c < n && tau != 0.0) {
            // pairwise over the lane's rows (runs of SK above row j skipped)
            double d = tree_sum<0, RPT / SK>([&](auto kc) {
                constexpr int i0 = decltype(kc)::value * SK;
                if (TPC * (i0 + SK) - 1 < j) return 0.0;
                return tree_sum<i0, SK>([&](auto ic) {
                    constexpr int i = decltype(ic)::value;
                    return vb[p][TPC * i + q] * qv[i];
                });
            });
#pragma unroll
            for (int off = 1; off < TPC; off <<= 1) d += __shfl_xor(d, off, 64);
            const double k = tau * d;
            asm volatile("" ::: "memory");
#pragma unroll
            for (int i0 = 0; i0 < RPT; i0 += SK)
                if (TPC * (i0 + SK) - 1 >= j) {
#pragma unroll
                    for (int i = i0; i < i0 + SK; ++i) qv[i] -= k * vb[p][TPC * i + q];
                }
        }
    }
    __syncthreads();   // every reflector has been read from qo
    if (c < n) {
        const double sg = dsg[c];
        double *dst = qo + (long)q * n + c;
#pragma unroll
        for (int i = 0; i < RPT; ++i) dst[(long)TPC * i * n] = qv[i] * sg;
    }
}

struct Level {
    long rows;
    int nb;
    double *in;   // rows x n
    double *q;    // nb x BR x n
};
}  // namespace

size_t tsqr_ws_narrow(long m, int n) {
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
void launch_block(int nb, const double *in, long rows, int n, double *rs, double *q, bool fin, hipStream_t st) {
    hipLaunchKernelGGL(qr_block_kernel<NC>, dim3(nb), dim3(NTH), 0, st, in, rows, n, rs, q, fin ? 1 : 0);
}
}  // namespace

void tsqr_narrow(const double *a, long m, int n, double *q, double *r, double *ws, hipStream_t st) {
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
        if (n <= 16) launch_block<16>(L.nb, in, rows, n, rs, L.q, fin, st);
        else if (n <= 32) launch_block<32>(L.nb, in, rows, n, rs, L.q, fin, st);
        else launch_block<64>(L.nb, in, rows, n, rs, L.q, fin, st);
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
    // rebuild Q top-down; the first level's product goes straight into q (its
    // blocks that lie inside q in one batch, a last block that runs past row
    // m on its own)
    long nb0 = lv[0].nb;
    double *bufA = p, *bufB = p + (size_t)nb0 * BR * n;
    const double *upper = lv[nlv - 1].q;   // rows_L x n (padded to BR)
    for (int l = nlv - 2; l >= 0; --l) {
        double *dst = l == 0 ? q : ((l % 2 == 0) ? bufA : bufB);
        GemmArgs g{};
        g.M = BR; g.N = n; g.K = n; g.batch = lv[l].nb;
        g.A = lv[l].q; g.sAr = n; g.sAk = 1; g.sAb = (long)BR * n;
        g.B = upper; g.sBk = n; g.sBn = 1; g.sBb = (long)n * n;
        g.C = dst; g.sCr = n; g.sCn = 1; g.sCb = (long)BR * n;
        g.alpha = 1.0; g.beta = 0.0;
        if (l > 0) {
            gemm(g, P_FP64, st);
        } else {
            const long full = m / BR;
            const int rem = (int)(m - full * BR);
            if (full > 0) {
                g.batch = (int)full;
                gemm(g, P_FP64, st);
            }
            if (rem > 0) {
                GemmArgs h = g;
                h.M = rem; h.batch = 1;
                h.A = lv[0].q + full * BR * n;
                h.B = upper + full * n * n;
                h.C = q + full * BR * n;
                gemm(h, P_FP64, st);
            }
        }
        upper = dst;
    }
    if (nlv == 1) copy(q, upper, (size_t)m * n, st);
}


// ---------------------------------------------------------------------------
// Wide thin QR (64 < n <= 512): blocked Householder QR whose 64-column panels
// are factored by the TSQR above.  TSQR returns an explicit Q_p; the
// Householder form of the same panel, H = I - Y T Y^T with H[:, :b] = Q_p S
// (S = diag(+-1)), follows from an LU factorisation without pivoting of
// [I; 0] - Q_p S = Y (T Y_1^T), the signs chosen column by column so every
// pivot is 1 + |.| >= 1 (Householder reconstruction; Ballard et al.,
// "Reconstructing Householder vectors from tall-skinny QR", 2014).  The block
// reflector updates the trailing columns with GEMMs, and Q = H_1 .. H_k [I; 0]
// is accumulated the same way.  Unlike Gram-Schmidt on panels this stays
// orthogonal for rank-deficient input (zero-padded bond columns).
namespace {
constexpr int WB = 64;   // panel width

__global__ void copy2d_kernel(double *dst, long ldd, const double *src, long lds, long rows, int cols) {
    const long tot = rows * cols;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < tot; i += (long)gridDim.x * blockDim.x) {
        const long r = i / cols;
        const int c = (int)(i - r * cols);
        dst[r * ldd + c] = src[r * lds + c];
    }
}

// q (rows x n, ld n) = [I_n; 0]
__global__ void eye_rect_kernel(double *q, long rows, int n) {
    const long tot = rows * n;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < tot; i += (long)gridDim.x * blockDim.x) {
        const long r = i / n;
        q[i] = (r == i - r * n) ? 1.0 : 0.0;
    }
}

// Householder reconstruction of one panel from the top b x b block of its
// TSQR factor (qtop, row-major, ld b), b <= 64.  Writes s (b signs), the unit
// lower L into ytop (b x b, ld b: the first b rows of Y), V = -S U^-1 and
// T = U L^-T (both b x b), with [I; 0] - Q_p S = Y U.  One workgroup.
__global__ __launch_bounds__(256) void hh_reconstruct_kernel(const double *qtop, int b, double *svec,
                                                            double *ytop, double *vmat, double *tmat) {
    __shared__ double Z[WB][WB + 1];
    __shared__ double U[WB][WB + 1];
    __shared__ double X[WB][WB + 1];
    __shared__ double sg[WB];
    const int t = threadIdx.x;
    for (int e = t; e < b * b; e += blockDim.x) Z[e / b][e % b] = qtop[e];
    __syncthreads();
    for (int k = 0; k < b; ++k) {
        const double z = Z[k][k];
        const double sk = z >= 0.0 ? -1.0 : 1.0;
        const double piv = 1.0 + fabs(z);
        __syncthreads();
        if (t == 0) {
            sg[k] = sk;
            U[k][k] = piv;
        }
        // multipliers l_ik = -s_k Z_ik / piv, kept in Z's strict lower part
        for (int i = k + 1 + t; i < b; i += blockDim.x) Z[i][k] = -sk * Z[i][k] / piv;
        __syncthreads();
        const int w = b - k - 1;
        for (int e = t; e < w * w; e += blockDim.x) {
            const int i = k + 1 + e / w, j = k + 1 + e % w;
            Z[i][j] -= Z[i][k] * Z[k][j];
        }
        __syncthreads();
    }
    // U (upper): U_kj = -s_j Z_kj for j > k; L (unit lower) to ytop
    for (int e = t; e < b * b; e += blockDim.x) {
        const int i = e / b, j = e % b;
        if (j > i) U[i][j] = -sg[j] * Z[i][j];
        else if (j < i) U[i][j] = 0.0;
        ytop[e] = j < i ? Z[i][j] : (j == i ? 1.0 : 0.0);
    }
    __syncthreads();
    // X = U^-1, column j by thread j (back substitution)
    if (t < b) {
        const int j = t;
        for (int i = b - 1; i >= 0; --i) {
            double acc = i == j ? 1.0 : 0.0;
            for (int l = i + 1; l <= j; ++l) acc -= U[i][l] * X[l][j];
            X[i][j] = i <= j ? acc / U[i][i] : 0.0;
        }
    }
    __syncthreads();
    for (int e = t; e < b * b; e += blockDim.x) {
        const int i = e / b, j = e % b;
        vmat[e] = -sg[i] * X[i][j];
    }
    __syncthreads();
    // X = L^-1 (unit lower), column j by thread j (forward substitution)
    if (t < b) {
        const int j = t;
        for (int i = 0; i < b; ++i) {
            double acc = i == j ? 1.0 : 0.0;
            for (int l = j; l < i; ++l) acc -= Z[i][l] * X[l][j];
            X[i][j] = i >= j ? acc : 0.0;
        }
    }
    __syncthreads();
    // T = U L^-T: T_ij = sum_l U_il (L^-1)_jl, l in [i, j]
    for (int e = t; e < b * b; e += blockDim.x) {
        const int i = e / b, j = e % b;
        double acc = 0.0;
        for (int l = i; l <= j; ++l) acc += U[i][l] * X[j][l];
        tmat[e] = j >= i ? acc : 0.0;
    }
    if (t < b) svec[t] = sg[t];
}

// R block (b x b at r, ld ldr) = S Rp
__global__ void scale_rows_kernel(double *r, long ldr, const double *rp, int b, const double *svec) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < b * b; e += gridDim.x * blockDim.x) {
        const int i = e / b, j = e % b;
        r[(long)i * ldr + j] = svec[i] * rp[e];
    }
}

// d_i = sign of R_ii (+1 for 0); rows of R and columns of Q scaled by d
__global__ void diag_sign_kernel(const double *r, int n, double *d) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        d[i] = r[(long)i * n + i] < 0.0 ? -1.0 : 1.0;
}
__global__ void row_scale_kernel(double *r, int n, const double *d) {
    const long tot = (long)n * n;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x)
        r[e] *= d[e / n];
}

inline unsigned g256(long n) { return (unsigned)std::max(1L, std::min((n + 255) / 256, 65536L)); }

void copy2d(double *dst, long ldd, const double *src, long lds, long rows, int cols, hipStream_t st) {
    if (rows <= 0 || cols <= 0) return;
    hipLaunchKernelGGL(copy2d_kernel, dim3(g256(rows * cols)), dim3(256), 0, st, dst, ldd, src, lds, rows, cols);
    TRG_HIP_CHECK(hipGetLastError());
}

// slices of the split-K product W = Y^T E (b x nc) over K = rows
int wide_splits(long rows) {
    int s = 1;
    while (s < 256 && rows / (2 * s) >= 1024) s *= 2;
    return s;
}

// W (b x nc, dense) = Y^T E with Y (rows x b, ld b) and E (rows x nc, ld lde):
// K split into equal slices (+ a remainder) summed in a fixed order
void gemm_yt_e(const double *y, int b, const double *e, long lde, long rows, int nc, double *w, double *slices,
               hipStream_t st) {
    const int sp = wide_splits(rows);
    const long kc = rows / sp, rem = rows - kc * sp;
    GemmArgs g{};
    g.M = b; g.N = nc; g.K = (int)kc; g.batch = 1;
    g.A = y; g.sAr = 1; g.sAk = b;
    g.B = e; g.sBk = lde; g.sBn = 1;
    g.C = slices; g.sCr = nc; g.sCn = 1; g.sCb = (long)(sp + 1) * b * nc;
    g.alpha = 1.0; g.beta = 0.0;
    g.inner = sp; g.sAi = kc * b; g.sBi = kc * lde; g.sCi = (long)b * nc;
    gemm(g, P_FP64, st);
    int ns = sp;
    if (rem > 0) {
        GemmArgs h = g;
        h.K = (int)rem; h.inner = 1; h.sAi = h.sBi = h.sCi = 0;
        h.A = y + kc * sp * b;
        h.B = e + kc * sp * lde;
        h.C = slices + (long)sp * b * nc;
        gemm(h, P_FP64, st);
        ns = sp + 1;
    }
    sum_slices(slices, ns, b, nc, w, nc, 1, st);
}

long wide_rows_total(long m, int n) {
    long tot = 0;
    for (int c0 = 0; c0 < n; c0 += WB) tot += m - c0;
    return tot;
}
}  // namespace

size_t tsqr_ws_doubles(long m, int n) {
    if (n <= 64) return tsqr_ws_narrow(m, n);
    const int np = (n + WB - 1) / WB;
    size_t tot = 0;
    tot += (size_t)m * n;                       // working copy of A
    tot += 2 * (size_t)m * WB;                  // panel and its TSQR Q
    tot += tsqr_ws_narrow(m, WB);               // panel TSQR scratch
    tot += (size_t)wide_rows_total(m, n) * WB;  // Y of every panel
    tot += (size_t)np * WB * WB;                // T of every panel
    tot += 3 * (size_t)WB * WB + 2 * WB;        // Rp, V, s, d
    tot += (size_t)(256 + 1) * WB * n + (size_t)WB * n * 2;   // split-K slices, W, W2
    return tot + 64;
}

void tsqr(const double *a, long m, int n, double *q, double *r, double *ws, hipStream_t st) {
    if (n <= 64) {
        tsqr_narrow(a, m, n, q, r, ws, st);
        return;
    }
    TRG_REQUIRE(n <= 512, -6, "tsqr: n must be <= 512");
    TRG_REQUIRE(m >= n, -6, "tsqr: needs m >= n");
    const int np = (n + WB - 1) / WB;
    double *p = ws;
    double *aw = p; p += (size_t)m * n;
    double *pan = p; p += (size_t)m * WB;
    double *qp = p; p += (size_t)m * WB;
    double *pws = p; p += tsqr_ws_narrow(m, WB);
    double *yall = p; p += (size_t)wide_rows_total(m, n) * WB;
    double *tall = p; p += (size_t)np * WB * WB;
    double *rp = p; p += WB * WB;
    double *vm = p; p += WB * WB;
    double *sv = p; p += WB;
    double *dv = p; p += WB > n ? WB : n;
    double *w1 = p; p += (size_t)WB * n;
    double *w2 = p; p += (size_t)WB * n;
    double *slices = p;
    copy(aw, a, (size_t)m * n, st);
    fill(r, (size_t)n * n, 0.0, st);
    std::vector<double *> ys(np);
    long yoff = 0;
    for (int j = 0; j < np; ++j) {
        const int c0 = j * WB, b = std::min(WB, n - c0);
        const long rows = m - c0;
        const int n2 = n - c0 - b;
        double *y = yall + yoff;
        ys[j] = y;
        yoff += rows * WB;
        double *tj = tall + (size_t)j * WB * WB;
        copy2d(pan, b, aw + (long)c0 * n + c0, n, rows, b, st);
        tsqr_narrow(pan, rows, b, qp, rp, pws, st);
        hipLaunchKernelGGL(hh_reconstruct_kernel, dim3(1), dim3(256), 0, st, qp, b, sv, y, vm, tj);
        TRG_HIP_CHECK(hipGetLastError());
        hipLaunchKernelGGL(scale_rows_kernel, dim3(g256((long)b * b)), dim3(256), 0, st, r + (long)c0 * n + c0, (long)n,
                           rp, b, sv);
        TRG_HIP_CHECK(hipGetLastError());
        if (rows > b) {   // Y_bot = Q_p[b:, :] V
            GemmArgs g{};
            g.M = (int)(rows - b); g.N = b; g.K = b; g.batch = 1;
            g.A = qp + (long)b * b; g.sAr = b; g.sAk = 1;
            g.B = vm; g.sBk = b; g.sBn = 1;
            g.C = y + (long)b * b; g.sCr = b; g.sCn = 1;
            g.alpha = 1.0; g.beta = 0.0;
            gemm(g, P_FP64, st);
        }
        if (n2 > 0) {
            double *a2 = aw + (long)c0 * n + c0 + b;   // rows x n2, ld n
            gemm_yt_e(y, b, a2, n, rows, n2, w1, slices, st);
            GemmArgs g{};
            g.M = b; g.N = n2; g.K = b; g.batch = 1;    // W2 = T^T W
            g.A = tj; g.sAr = 1; g.sAk = b;
            g.B = w1; g.sBk = n2; g.sBn = 1;
            g.C = w2; g.sCr = n2; g.sCn = 1;
            g.alpha = 1.0; g.beta = 0.0;
            gemm(g, P_FP64, st);
            GemmArgs h{};                               // A2 -= Y W2
            h.M = (int)rows; h.N = n2; h.K = b; h.batch = 1;
            h.A = y; h.sAr = b; h.sAk = 1;
            h.B = w2; h.sBk = n2; h.sBn = 1;
            h.C = a2; h.sCr = n; h.sCn = 1;
            h.alpha = -1.0; h.beta = 1.0;
            gemm(h, P_FP64, st);
            copy2d(r + (long)c0 * n + c0 + b, n, a2, n, b, n2, st);
        }
    }
    // Q = H_0 H_1 .. H_{np-1} [I; 0], applied last panel first; columns left
    // of a panel are still zero in its rows when it is applied
    hipLaunchKernelGGL(eye_rect_kernel, dim3(g256((long)m * n)), dim3(256), 0, st, q, m, n);
    TRG_HIP_CHECK(hipGetLastError());
    for (int j = np - 1; j >= 0; --j) {
        const int c0 = j * WB, b = std::min(WB, n - c0);
        const long rows = m - c0;
        const int nc = n - c0;
        double *e = q + (long)c0 * n + c0;   // rows x nc, ld n
        const double *y = ys[j], *tj = tall + (size_t)j * WB * WB;
        gemm_yt_e(y, b, e, n, rows, nc, w1, slices, st);
        GemmArgs g{};
        g.M = b; g.N = nc; g.K = b; g.batch = 1;        // W2 = T W
        g.A = tj; g.sAr = b; g.sAk = 1;
        g.B = w1; g.sBk = nc; g.sBn = 1;
        g.C = w2; g.sCr = nc; g.sCn = 1;
        g.alpha = 1.0; g.beta = 0.0;
        gemm(g, P_FP64, st);
        GemmArgs h{};                                   // E -= Y W2
        h.M = (int)rows; h.N = nc; h.K = b; h.batch = 1;
        h.A = y; h.sAr = b; h.sAk = 1;
        h.B = w2; h.sBk = nc; h.sBn = 1;
        h.C = e; h.sCr = n; h.sCn = 1;
        h.alpha = -1.0; h.beta = 1.0;
        gemm(h, P_FP64, st);
    }
    // diag(R) >= 0
    hipLaunchKernelGGL(diag_sign_kernel, dim3(1), dim3(256), 0, st, r, n, dv);
    hipLaunchKernelGGL(row_scale_kernel, dim3(g256((long)n * n)), dim3(256), 0, st, r, n, dv);
    TRG_HIP_CHECK(hipGetLastError());
    scale_cols(q, m, n, n, dv, st);
}

}  // namespace trg
