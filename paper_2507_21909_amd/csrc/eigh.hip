// Symmetric eigen-decomposition by two-sided block Jacobi, for the Gram
// matrices of the RG step: the triad HOSVD Grams (eq. HOSVD) and the
// environment Grams whose square roots build the squeezers (Sec. II A).
//
// The matrix (scaled to unit max entry, padded to a multiple of 64) is cut
// into blocks of 32 indices.  A sweep runs the circle-method tournament over
// the blocks; in each round the blocks are paired, and for every pair (I, J):
//   solve: the 64 x 64 sub-matrix A[IJ, IJ] is diagonalised in LDS by cyclic
//          scalar Jacobi (parallel rounds of 32 disjoint rotations) until no
//          pair exceeds the threshold, accumulating its rotation Q_IJ;
//   apply: every 64 x 64 tile A[P, R] <- Q_P^T A[P, R] Q_R (tiles P < R, the
//          mirror written as the transpose, so A stays exactly symmetric;
//          diagonal tiles take the solved sub-matrix) and V[:, P] <- V[:, P] Q_P.
// A sweep in which no sub-problem rotates ends the iteration; the diagonal of A
// holds the eigenvalues, the columns of V the eigenvectors.  The rotation
// threshold is relative, |a_pq| > n eps sqrt(|a_pp a_qq|), as in cyclic
// two-sided Jacobi, so small eigenvalues of a graded matrix are resolved too.
//
// Every pair of indices meets in some sub-problem once per sweep, so the
// convergence test covers all off-diagonal entries.  FP64 throughout; the
// tile products run on the FP64 vector units (CDNA4 issues FP64 FMA at the
// same rate as FP64 MFMA) with 4 x 4 register blocking from LDS.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <mutex>

#include "common.h"

namespace trg {

namespace {
constexpr int EB = 32;          // indices per block
constexpr int ET = 2 * EB;      // sub-problem / tile edge
constexpr int LDT = ET + 1;     // LDS row stride (odd: conflict-free column reads)
constexpr int NT = 256;
constexpr size_t TILE_LDS = 2 * (size_t)ET * LDT * sizeof(double);

__device__ inline int player(int mm, int i, int r) { return i == 0 ? 0 : 1 + ((i - 1 + r) % (mm - 1)); }

struct PairMap {
    int I, J;
};
__device__ inline PairMap pair_blocks(int nb, int k, int r) { return {player(nb, k, r), player(nb, nb - 1 - k, r)}; }
// global index of local index l (0..63) of a block pair
__device__ inline int gidx(PairMap pm, int l) { return l < EB ? pm.I * EB + l : pm.J * EB + (l - EB); }

// per-matrix max |K| (one workgroup per matrix)
__global__ __launch_bounds__(NT) void eh_scale_kernel(const double *K, int n, double *scale) {
    const int mat = blockIdx.x;
    const double *k = K + (size_t)mat * n * n;
    double mx = 0.0;
    for (long i = threadIdx.x; i < (long)n * n; i += NT) mx = fmax(mx, fabs(k[i]));
    __shared__ double red[NT];
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) scale[mat] = red[0] > 0.0 ? red[0] : 1.0;
}

// A = sym(K) / scale padded with zeros to N x N; V = identity
__global__ void eh_init_kernel(const double *K, int n, int N, int count, const double *scale, double *A, double *V) {
    const long tot = (long)count * N * N;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
        const int mat = (int)(e / ((long)N * N));
        const long rem = e - (long)mat * N * N;
        const int i = (int)(rem / N), j = (int)(rem % N);
        double a = 0.0;
        if (i < n && j < n) {
            const double *k = K + (size_t)mat * n * n;
            a = 0.5 * (k[(long)i * n + j] + k[(long)j * n + i]) / scale[mat];
        }
        A[e] = a;
        V[e] = i == j ? 1.0 : 0.0;
    }
}

// Diagonalise the sub-matrix of block pair blockIdx.x of round r (matrix blockIdx.y).
__global__ __launch_bounds__(NT) void eh_solve_kernel(const double *A, int N, int nb, int r, double tol,
                                                      int max_inner, double *Qbuf, double *Sbuf, int *flags,
                                                      int *qflag) {
    extern __shared__ double sh[];
    double *S = sh;               // ET x LDT
    double *Q = sh + ET * LDT;    // ET x LDT
    __shared__ double cc[EB], ss[EB], tt[EB];
    __shared__ int pp[EB], qq[EB];
    __shared__ int any_round, any_sweep, total;
    const int k = blockIdx.x, mat = blockIdx.y, t = threadIdx.x;
    const int npair = nb / 2;
    const PairMap pm = pair_blocks(nb, k, r);
    const double *Am = A + (size_t)mat * N * N;
    for (int e = t; e < ET * ET; e += NT) {
        const int i = e / ET, j = e % ET;
        S[i * LDT + j] = Am[(size_t)gidx(pm, i) * N + gidx(pm, j)];
        Q[i * LDT + j] = i == j ? 1.0 : 0.0;
    }
    if (t == 0) total = 0;
    __syncthreads();
    for (int sw = 0; sw < max_inner; ++sw) {
        if (t == 0) any_sweep = 0;
        for (int rr = 0; rr < ET - 1; ++rr) {
            if (t < EB) {
                const int a = player(ET, t, rr), b = player(ET, ET - 1 - t, rr);
                const int p = a < b ? a : b, q = a < b ? b : a;
                const double app = S[p * LDT + p], aqq = S[q * LDT + q], apq = S[p * LDT + q];
                double c = 1.0, s = 0.0, tn = 0.0;
                const bool rot = fabs(apq) > 1e-300 && fabs(apq) > tol * sqrt(fabs(app)) * sqrt(fabs(aqq));
                if (rot) {
                    const double zeta = (aqq - app) / (2.0 * apq);
                    tn = zeta == 0.0 ? 1.0 : copysign(1.0, zeta) / (fabs(zeta) + hypot(zeta, 1.0));
                    c = 1.0 / sqrt(1.0 + tn * tn);
                    s = c * tn;
                }
                pp[t] = p;
                qq[t] = q;
                cc[t] = c;
                ss[t] = s;
                tt[t] = tn;
                const unsigned long long bal = __ballot(rot);
                if (t == 0) {
                    any_round = bal != 0ull;
                    if (bal) {
                        any_sweep = 1;
                        total += __popcll(bal);
                    }
                }
            }
            __syncthreads();
            if (any_round) {
                // S <- J^T S J on 2 x 2 blocks (u <= v); the mirror block is the transpose.
                // Thread t always takes column pair v = t % 32 with row pairs u = t / 32 + 8 i,
                // and in the Q update pair t % 32 on rows t / 32 + 8 i.  All LDS reads of a
                // phase are issued before its writes, so their latencies overlap.
                const int vv = t % EB;
                const int pv = pp[vv], qv = qq[vv];
                const double cv = cc[vv], sv = ss[vv];
                double m00[4], m01[4], m10[4], m11[4];
                int pu[4], qu[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int u = t / EB + 8 * i;
                    pu[i] = pp[u];
                    qu[i] = qq[u];
                    if (u <= vv) {
                        m00[i] = S[pu[i] * LDT + pv];
                        m01[i] = S[pu[i] * LDT + qv];
                        m10[i] = S[qu[i] * LDT + pv];
                        m11[i] = S[qu[i] * LDT + qv];
                    }
                }
                double qx[8], qy[8];
                const bool qrot = cv != 1.0 || sv != 0.0;
                if (qrot) {
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        const int i = t / EB + 8 * k;
                        qx[k] = Q[i * LDT + pv];
                        qy[k] = Q[i * LDT + qv];
                    }
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int u = t / EB + 8 * i;
                    if (u > vv) continue;
                    double n00, n01, n10, n11;
                    if (u == vv) {
                        const double app = m00[i], aqq = m11[i], apq = m01[i];
                        const double tn = tt[u];
                        if (tn != 0.0) {
                            n00 = app - tn * apq;
                            n11 = aqq + tn * apq;
                            n01 = n10 = 0.0;
                        } else {
                            n00 = app;
                            n11 = aqq;
                            n01 = n10 = apq;
                        }
                        S[pu[i] * LDT + pu[i]] = n00;
                        S[qu[i] * LDT + qu[i]] = n11;
                        S[pu[i] * LDT + qu[i]] = n01;
                        S[qu[i] * LDT + pu[i]] = n10;
                        continue;
                    }
                    const double cu = cc[u], su = ss[u];
                    // columns (pv, qv) by J_v
                    const double r00 = cv * m00[i] - sv * m01[i], r01 = sv * m00[i] + cv * m01[i];
                    const double r10 = cv * m10[i] - sv * m11[i], r11 = sv * m10[i] + cv * m11[i];
                    // rows (pu, qu) by J_u^T
                    n00 = cu * r00 - su * r10;
                    n10 = su * r00 + cu * r10;
                    n01 = cu * r01 - su * r11;
                    n11 = su * r01 + cu * r11;
                    S[pu[i] * LDT + pv] = n00;
                    S[pu[i] * LDT + qv] = n01;
                    S[qu[i] * LDT + pv] = n10;
                    S[qu[i] * LDT + qv] = n11;
                    S[pv * LDT + pu[i]] = n00;
                    S[qv * LDT + pu[i]] = n01;
                    S[pv * LDT + qu[i]] = n10;
                    S[qv * LDT + qu[i]] = n11;
                }
                // Q <- Q J (columns p, q of every row)
                if (qrot) {
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        const int i = t / EB + 8 * k;
                        Q[i * LDT + pv] = cv * qx[k] - sv * qy[k];
                        Q[i * LDT + qv] = sv * qx[k] + cv * qy[k];
                    }
                }
            }
            __syncthreads();
        }
        const int more = any_sweep;
        __syncthreads();
        if (!more) break;
    }
    // unit columns: the rotations are orthogonal, their rounded product drifts in norm
    {
        const int w = t >> 6, lane = t & 63;
        for (int j = w; j < ET; j += NT / 64) {
            const double x = Q[lane * LDT + j];
            double ss2 = x * x;
            for (int o = 32; o > 0; o >>= 1) ss2 += __shfl_xor(ss2, o, 64);
            Q[lane * LDT + j] = x / sqrt(ss2);
        }
    }
    __syncthreads();
    const size_t off = ((size_t)mat * npair + k) * ET * ET;
    for (int e = t; e < ET * ET; e += NT) {
        const int i = e / ET, j = e % ET;
        Qbuf[off + e] = Q[i * LDT + j];
        Sbuf[off + e] = S[i * LDT + j];
    }
    if (t == 0) {
        qflag[mat * npair + k] = total > 0;
        if (total > 0) atomicAdd(&flags[mat], total);
    }
}

// acc (4 x 4 per thread: rows ti + 16a, cols tj + 16b) = op(X) * Y over 64 terms
// op(X) = X (xt = false) or X^T (xt = true)
__device__ inline void tile_mm(const double *X, const double *Y, bool xt, double acc[4][4]) {
    const int ti = threadIdx.x >> 4, tj = threadIdx.x & 15;
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
    for (int kk = 0; kk < ET; ++kk) {
        double xa[4], yb[4];
        for (int a = 0; a < 4; ++a) xa[a] = xt ? X[kk * LDT + ti + 16 * a] : X[(ti + 16 * a) * LDT + kk];
        for (int b = 0; b < 4; ++b) yb[b] = Y[kk * LDT + tj + 16 * b];
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) acc[a][b] = fma(xa[a], yb[b], acc[a][b]);
    }
}

__device__ inline void tile_store(double *X, const double acc[4][4]) {
    const int ti = threadIdx.x >> 4, tj = threadIdx.x & 15;
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) X[(ti + 16 * a) * LDT + tj + 16 * b] = acc[a][b];
}

// Apply the rotations of round r: tiles [0, nA) of A (P <= R), then V tiles.
__global__ __launch_bounds__(NT) void eh_apply_kernel(double *A, double *V, int N, int nb, int r,
                                                      const double *Qbuf, const double *Sbuf, const int *qflag) {
    extern __shared__ double sh[];
    double *X = sh, *Y = sh + ET * LDT;
    const int mat = blockIdx.y, npair = nb / 2, t = threadIdx.x;
    const int nA = npair * (npair + 1) / 2;
    const int tile = blockIdx.x;
    double *Am = A + (size_t)mat * N * N, *Vm = V + (size_t)mat * N * N;
    const double *Qm = Qbuf + (size_t)mat * npair * ET * ET;
    const int *qf = qflag + mat * npair;
    double acc[4][4];
    if (tile < nA) {
        int P = 0, rem = tile;
        while (rem >= npair - P) {
            rem -= npair - P;
            ++P;
        }
        const int R = P + rem;
        const PairMap mp = pair_blocks(nb, P, r), mr = pair_blocks(nb, R, r);
        if (P == R) {
            if (!qf[P]) return;
            const double *Sm = Sbuf + ((size_t)mat * npair + P) * ET * ET;
            for (int e = t; e < ET * ET; e += NT) {
                const int i = e / ET, j = e % ET;
                Am[(size_t)gidx(mp, i) * N + gidx(mp, j)] = Sm[e];
            }
            return;
        }
        if (!qf[P] && !qf[R]) return;
        for (int e = t; e < ET * ET; e += NT) {
            const int i = e / ET, j = e % ET;
            X[i * LDT + j] = Am[(size_t)gidx(mp, i) * N + gidx(mr, j)];
            Y[i * LDT + j] = Qm[(size_t)R * ET * ET + e];
        }
        __syncthreads();
        tile_mm(X, Y, false, acc);           // T = A_PR Q_R
        __syncthreads();
        tile_store(Y, acc);                  // Y <- T
        for (int e = t; e < ET * ET; e += NT) X[(e / ET) * LDT + e % ET] = Qm[(size_t)P * ET * ET + e];
        __syncthreads();
        tile_mm(X, Y, true, acc);            // Z = Q_P^T T
        __syncthreads();
        tile_store(X, acc);
        __syncthreads();
        for (int e = t; e < ET * ET; e += NT) {
            const int i = e / ET, j = e % ET;
            Am[(size_t)gidx(mp, i) * N + gidx(mr, j)] = X[i * LDT + j];
        }
        for (int e = t; e < ET * ET; e += NT) {
            const int j = e / ET, i = e % ET;
            Am[(size_t)gidx(mr, j) * N + gidx(mp, i)] = X[i * LDT + j];
        }
        return;
    }
    const int vt = tile - nA;
    const int P = vt % npair, c = vt / npair;
    if (!qf[P]) return;
    const PairMap mp = pair_blocks(nb, P, r);
    for (int e = t; e < ET * ET; e += NT) {
        const int i = e / ET, j = e % ET;
        X[i * LDT + j] = Vm[(size_t)(c * ET + i) * N + gidx(mp, j)];
        Y[i * LDT + j] = Qm[(size_t)P * ET * ET + e];
    }
    __syncthreads();
    tile_mm(X, Y, false, acc);
    __syncthreads();
    tile_store(X, acc);
    __syncthreads();
    for (int e = t; e < ET * ET; e += NT) {
        const int i = e / ET, j = e % ET;
        Vm[(size_t)(c * ET + i) * N + gidx(mp, j)] = X[i * LDT + j];
    }
}

// eigenvalue j -> rank in descending order (ties by index); gather values and vectors
__global__ __launch_bounds__(NT) void eh_sort_kernel(const double *A, const double *V, int n, int N,
                                                     const double *scale, double *lam, double *vec) {
    const int j = blockIdx.x, mat = blockIdx.y;
    const double *Am = A + (size_t)mat * N * N;
    const double lj = Am[(size_t)j * N + j];
    __shared__ int rank_sh;
    if (threadIdx.x == 0) rank_sh = 0;
    __syncthreads();
    int cnt = 0;
    for (int k = threadIdx.x; k < n; k += NT) {
        const double lk = Am[(size_t)k * N + k];
        cnt += (lk > lj || (lk == lj && k < j)) ? 1 : 0;
    }
    atomicAdd(&rank_sh, cnt);
    __syncthreads();
    const int rk = rank_sh;
    if (threadIdx.x == 0) lam[(size_t)mat * n + rk] = lj * scale[mat];
    const double *Vm = V + (size_t)mat * N * N;
    // unit eigenvector (removes the norm drift of the accumulated rotations)
    __shared__ double red[NT / 64];
    double s2 = 0.0;
    for (int i = threadIdx.x; i < n; i += NT) {
        const double x = Vm[(size_t)i * N + j];
        s2 += x * x;
    }
    for (int o = 32; o > 0; o >>= 1) s2 += __shfl_xor(s2, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s2;
    __syncthreads();
    const double inv = 1.0 / sqrt(red[0] + red[1] + red[2] + red[3]);
    double *vo = vec + (size_t)mat * n * n;
    for (int i = threadIdx.x; i < n; i += NT) vo[(size_t)i * n + rk] = Vm[(size_t)i * N + j] * inv;
}

bool eh_trace() {
    static const bool on = [] {
        const char *e = getenv("TRG_JACOBI_TRACE");
        return e && *e && *e != '0';
    }();
    return on;
}

inline int padded(int n) { return ((n + ET - 1) / ET) * ET; }

inline unsigned g_blocks(size_t n) { return (unsigned)std::max<size_t>(1, std::min<size_t>((n + 255) / 256, 65536)); }

void set_lds_attr(const void *fn) {
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)TILE_LDS) != hipSuccess)
        (void)hipGetLastError();
}
}  // namespace

size_t eigh_ws_doubles(int count, int n) {
    const size_t N = padded(n), npair = N / ET;
    return (size_t)count * (2 * N * N + 2 * npair * ET * ET + 1) + 64;
}

size_t eigh_iws_ints(int count, int n) { return (size_t)count * (1 + padded(n) / ET) + 16; }

int eigh_sym(const double *K, int count, int n, double *lam, double *vec, double *ws, int *iws, int max_sweeps,
             hipStream_t st) {
    if (count == 0 || n == 0) return 0;
    TRG_REQUIRE(n > 0 && count > 0, -1, "eigh: bad sizes");
    static std::once_flag attr;
    std::call_once(attr, [] {
        set_lds_attr(reinterpret_cast<const void *>(eh_solve_kernel));
        set_lds_attr(reinterpret_cast<const void *>(eh_apply_kernel));
    });
    const int N = padded(n), nb = N / EB, npair = nb / 2;
    double *A = ws, *V = A + (size_t)count * N * N;
    double *Qb = V + (size_t)count * N * N, *Sb = Qb + (size_t)count * npair * ET * ET;
    double *scale = Sb + (size_t)count * npair * ET * ET;
    int *flags = iws, *qflag = iws + count;
    const double tol = (double)n * 2.220446049250313e-16;
    // one inner sweep per sub-problem: the outer sweeps converge about as fast
    // as with fully solved sub-problems, at a third of the inner work
    const int max_inner = 1;
    hipLaunchKernelGGL(eh_scale_kernel, dim3(count), dim3(NT), 0, st, K, n, scale);
    hipLaunchKernelGGL(eh_init_kernel, dim3(g_blocks((size_t)count * N * N)), dim3(256), 0, st, K, n, N, count,
                       scale, A, V);
    TRG_HIP_CHECK(hipGetLastError());
    const int ntiles = npair * (npair + 1) / 2 + (N / ET) * npair;
    std::vector<int> fl(count);
    int sweep = 0;
    for (;; ++sweep) {
        TRG_REQUIRE(sweep < max_sweeps, -4, "symmetric Jacobi eigensolver did not converge");
        TRG_HIP_CHECK(hipMemsetAsync(flags, 0, sizeof(int) * count, st));
        for (int r = 0; r < nb - 1; ++r) {
            hipLaunchKernelGGL(eh_solve_kernel, dim3(npair, count), dim3(NT), TILE_LDS, st, A, N, nb, r, tol,
                               max_inner, Qb, Sb, flags, qflag);
            hipLaunchKernelGGL(eh_apply_kernel, dim3(ntiles, count), dim3(NT), TILE_LDS, st, A, V, N, nb, r, Qb,
                               Sb, qflag);
        }
        TRG_HIP_CHECK(hipGetLastError());
        TRG_HIP_CHECK(hipMemcpyAsync(fl.data(), flags, sizeof(int) * count, hipMemcpyDeviceToHost, st));
        TRG_HIP_CHECK(hipStreamSynchronize(st));
        long tot = 0;
        for (int f : fl) tot += f;
        if (eh_trace()) fprintf(stderr, "[eigh] count %d n %d sweep %d rotations %ld\n", count, n, sweep, tot);
        if (tot == 0) break;
    }
    hipLaunchKernelGGL(eh_sort_kernel, dim3(n, count), dim3(NT), 0, st, A, V, n, N, scale, lam, vec);
    TRG_HIP_CHECK(hipGetLastError());
    return sweep;
}

}  // namespace trg
