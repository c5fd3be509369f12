// One-sided (Hestenes) Jacobi SVD for the truncated SVDs and eigen-
// decompositions of the RG step: the re-split SVD (Fig. 5f), the SVD of the
// projected bond-swap matrix (App. A), the exact bond-swap SVD, the triad
// HOSVD Grams (eq. HOSVD) and the squeezer square roots and SVDs (Sec. II A).
// For a symmetric positive semi-definite Gram K, K V = U S gives its
// eigenvectors V and eigenvalues S.
//
// Matrices are held column by column (column j contiguous, m entries).  A
// round of the circle-method tournament rotates n/2 disjoint column pairs; one
// wavefront owns one pair: three dot products over the m rows (wave
// reductions), the rotation of Rutishauser's formulas, and the update of the
// two columns of U and of V.  Large n: one launch per round, all matrices of a
// batch together.  Small n: one workgroup per matrix loops over every round
// and sweep in a single launch.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "common.h"

namespace trg {

namespace {
constexpr int NT = 256;

__device__ inline int player_at(int mm, int i, int r) { return i == 0 ? 0 : 1 + ((i - 1 + r) % (mm - 1)); }

__device__ inline double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Rotation (c, s) that makes two columns with x.x = al, y.y = be, x.y = ga
// orthogonal: t = tan(theta) the root of t^2 + 2 zeta t - 1 = 0 of smaller
// magnitude, zeta = (be - al) / (2 ga), c = 1 / sqrt(1 + t^2), s = c t.
// false (c = 1, s = 0) when the pair is orthogonal to tol already or a column
// is (numerically) zero.
__device__ inline bool jacobi_rotation(double al, double be, double ga, double tol, double &c, double &s) {
    c = 1.0;
    s = 0.0;
    if (al < 1e-280 || be < 1e-280 || fabs(ga) <= tol * sqrt(al) * sqrt(be)) return false;
    const double zeta = (be - al) / (2.0 * ga);
    const double az = fabs(zeta);
    // sqrt(1 + zeta^2); past 1e150 the 1 is far below zeta's last bit
    const double h = az < 1e150 ? sqrt(fma(az, az, 1.0)) : az;
    const double t = (zeta < 0.0 ? -1.0 : 1.0) / (az + h);
    c = 1.0 / sqrt(fma(t, t, 1.0));
    s = c * t;
    return true;
}

// v from the lane that DPP control CTRL selects (all lanes active)
template <int CTRL>
__device__ inline double dpp_d(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// lane l's value of v, as a wave-uniform value
__device__ inline double read_lane(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// rotate pair k of round r of matrix (u, v); returns 1 if rotated, 2 if the
// pair's dot products are not finite (the pair is then left alone), else 0
__device__ int rotate_pair(double *u, double *v, int m, int n, int mm, int r, int k, double tol) {
    const int lane = threadIdx.x & 63;
    int a = player_at(mm, k, r), b = player_at(mm, mm - 1 - k, r);
    if (a >= n || b >= n) return 0;
    int p = a < b ? a : b, q = a < b ? b : a;
    double *up = u + (long)p * m, *uq = u + (long)q * m;
    double al = 0.0, be = 0.0, ga = 0.0;
    for (int i = lane; i < m; i += 64) {
        double x = up[i], y = uq[i];
        al += x * x;
        be += y * y;
        ga += x * y;
    }
    al = wave_sum(al);
    be = wave_sum(be);
    ga = wave_sum(ga);
    if (!isfinite(al + be + ga)) return 2;
    double c, s;
    if (!jacobi_rotation(al, be, ga, tol, c, s)) return 0;
    for (int i = lane; i < m; i += 64) {
        double x = up[i], y = uq[i];
        up[i] = c * x - s * y;
        uq[i] = s * x + c * y;
    }
    if (v) {
        double *vp = v + (long)p * n, *vq = v + (long)q * n;
        for (int i = lane; i < n; i += 64) {
            double x = vp[i], y = vq[i];
            vp[i] = c * x - s * y;
            vq[i] = s * x + c * y;
        }
    }
    return 1;
}

// flags[mat]: rotations of this sweep; flags[count + mat]: non-finite pairs seen
__global__ __launch_bounds__(NT) void round_kernel(JacobiBatch jb, int r, double tol, int *flags) {
    if (flags[2 * jb.count]) return;   // solve already converged (device-driven sweeps)
    const int mat = blockIdx.y;
    const int k = blockIdx.x * (NT / 64) + (threadIdx.x >> 6);
    const int mm = jb.n + (jb.n & 1);
    if (k >= mm / 2) return;
    double *u = jb.ut + (long)mat * jb.strideU;
    double *v = jb.vt ? jb.vt + (long)mat * jb.strideV : nullptr;
    const int rc = rotate_pair(u, v, jb.m, jb.n, mm, r, k, tol);
    if ((threadIdx.x & 63) == 0) {
        if (rc == 1) atomicAdd(&flags[mat], 1);
        if (rc == 2) flags[jb.count + mat] = 1;
    }
}

// One workgroup per matrix loops over every round and sweep.  All column
// pairs of a round are rotated at once: pair k takes a group of tp lanes (a
// power of two, np tp <= NT, inside one wavefront), each lane summing every
// tp-th row, the group reducing its three dot products by an xor butterfly
// (fixed order, so the bits do not depend on the schedule) and rotating its
// rows of U and V; one barrier per round.
__global__ __launch_bounds__(NT) void full_kernel(JacobiBatch jb, int max_sweeps, double tol, int *flags) {
    const int mat = blockIdx.x;
    double *u = jb.ut + (long)mat * jb.strideU;
    double *v = jb.vt ? jb.vt + (long)mat * jb.strideV : nullptr;
    const int n = jb.n, m = jb.m, mm = n + (n & 1), np = mm / 2;
    int tp = 64;
    while (tp > 1 && np * tp > NT) tp >>= 1;
    const int k = threadIdx.x / tp, l = threadIdx.x % tp;
    __shared__ int rot, bad;
    if (threadIdx.x == 0) bad = 0;
    int sweep = 0;
    for (; sweep < max_sweeps; ++sweep) {
        if (threadIdx.x == 0) rot = 0;
        __syncthreads();
        for (int r = 0; r < mm - 1; ++r) {
            const int a = k < np ? player_at(mm, k, r) : n, b = k < np ? player_at(mm, mm - 1 - k, r) : n;
            if (a < n && b < n) {   // uniform within the lane group
                const int p = a < b ? a : b, q = a < b ? b : a;
                double *up = u + (long)p * m, *uq = u + (long)q * m;
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int i = l; i < m; i += tp) {
                    const double x = up[i], y = uq[i];
                    al += x * x;
                    be += y * y;
                    ga += x * y;
                }
                for (int off = tp / 2; off > 0; off >>= 1) {
                    al += __shfl_xor(al, off, 64);
                    be += __shfl_xor(be, off, 64);
                    ga += __shfl_xor(ga, off, 64);
                }
                if (!isfinite(al + be + ga)) {
                    if (l == 0) bad = 1;
                } else {
                    double c, s;
                    if (jacobi_rotation(al, be, ga, tol, c, s)) {
                        for (int i = l; i < m; i += tp) {
                            const double x = up[i], y = uq[i];
                            up[i] = c * x - s * y;
                            uq[i] = s * x + c * y;
                        }
                        if (v) {
                            double *vp = v + (long)p * n, *vq = v + (long)q * n;
                            for (int i = l; i < n; i += tp) {
                                const double x = vp[i], y = vq[i];
                                vp[i] = c * x - s * y;
                                vq[i] = s * x + c * y;
                            }
                        }
                        if (l == 0) atomicAdd(&rot, 1);
                    }
                }
            }
            __syncthreads();
        }
        if (rot == 0) break;
        __syncthreads();
    }
    // flags[mat]: sweeps used (-1 - rotations of the last sweep if not converged)
    if (threadIdx.x == 0) {
        flags[mat] = sweep < max_sweeps ? sweep : -1 - rot;
        flags[jb.count + mat] = bad;
    }
}

// ---- panel variant (n > 96, m <= 1024) ------------------------------------
// The columns are cut into blocks of 8; a round of the circle-method tournament
// over the blocks pairs them, and one workgroup takes the 16-column panel of a
// block pair with its m rows held in registers (row t + 256 j of every panel
// column in thread t).  Inside the panel, cyclic one-sided Jacobi runs up to
// max_inner sweeps of 15 parallel rounds of 8 disjoint column pairs, the
// round-robin played on slots: slots k and 15 - k meet, then the columns in
// slots 1..15 move one slot on (register moves), so every register index is a
// compile-time constant and 15 rounds bring each column back to its slot.
// Only a sweep's first launch plays all 15 rounds, which covers the pairs
// inside every block (each block sits in exactly one panel per launch); the
// later launches play just the 8 rounds of pairs between the two blocks, so
// a sweep visits each column pair once in about n sequential rounds.
// The dot products are per-thread partial sums reduced across the wavefront by
// a reduce-scatter butterfly and across the 4 wavefronts in LDS; every
// wavefront then computes the round's rotations itself (jacobi_rotation, as in
// rotate_pair), so a round needs one barrier.  The panel's rotations are
// accumulated in a 16 x 16 matrix and applied to the 16 columns of V at the
// end.  HBM sees each panel once per tournament round instead of once per pair
// round, and a sweep needs nb - 1 launches instead of n - 1.
constexpr int PW = 16;
constexpr int PANEL_INNER = 1;   // inner sweeps per panel and tournament round

template <int ROWS>
__device__ inline void shift_slots(double (&u)[PW][ROWS], double (&vrow)[PW]) {
#pragma unroll
    for (int j = 0; j < ROWS; ++j) {
        const double tmp = u[PW - 1][j];
#pragma unroll
        for (int c = PW - 1; c > 1; --c) u[c][j] = u[c - 1][j];
        u[1][j] = tmp;
    }
    const double tmp = vrow[PW - 1];
#pragma unroll
    for (int c = PW - 1; c > 1; --c) vrow[c] = vrow[c - 1];
    vrow[1] = tmp;
}

// cross rounds: the columns in slots 8..15 move one slot on, cyclically
template <int ROWS>
__device__ inline void shift_cross(double (&u)[PW][ROWS], double (&vrow)[PW]) {
#pragma unroll
    for (int j = 0; j < ROWS; ++j) {
        const double tmp = u[PW - 1][j];
#pragma unroll
        for (int c = PW - 1; c > PW / 2; --c) u[c][j] = u[c - 1][j];
        u[PW / 2][j] = tmp;
    }
    const double tmp = vrow[PW - 1];
#pragma unroll
    for (int c = PW - 1; c > PW / 2; --c) vrow[c] = vrow[c - 1];
    vrow[PW / 2] = tmp;
}

// cross != 0: only the 64 pairs between the two blocks, in 8 rounds (slot k
// meets slot 15 - k while the second block's columns cycle through slots
// 8..15); the pairs inside each block are left to the full rounds of the
// sweep's first launch.
// WV: V is accumulated (without it the 16 x 16 panel rotation is dead code)
template <int ROWS, bool WV>
__global__ __launch_bounds__(NT) void panel_kernel(JacobiBatch jb, int nb, int r, double tol, int max_inner,
                                                   int cross, int *flags) {
    if (flags[2 * jb.count]) return;   // solve already converged (device-driven sweeps)
    const int k = blockIdx.x, mat = blockIdx.y, t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int I = player_at(nb, k, r), J = player_at(nb, nb - 1 - k, r);
    double *U = jb.ut + (long)mat * jb.strideU;
    double *V = jb.vt ? jb.vt + (long)mat * jb.strideV : nullptr;
    const int m = jb.m, n = jb.n;
    __shared__ double red[2][NT / 64][24];   // by round parity: one barrier per round
    __shared__ double vpan[PW][PW + 1];
    __shared__ int sweep_rot, total_rot, nonfinite;

    double u[PW][ROWS];
#pragma unroll
    for (int c = 0; c < PW; ++c) {
        const int g = c < 8 ? I * 8 + c : J * 8 + (c - 8);
#pragma unroll
        for (int j = 0; j < ROWS; ++j) {
            const int row = t + NT * j;
            // nontemporal: a panel is read and written once per launch and the
            // next launch takes it on another XCD, so it gains nothing in L2
            u[c][j] = (g < n && row < m) ? __builtin_nontemporal_load(&U[(long)g * m + row]) : 0.0;
        }
    }
    double vrow[PW];
#pragma unroll
    for (int c = 0; c < PW; ++c) vrow[c] = c == t ? 1.0 : 0.0;
    if (t == 0) {
        sweep_rot = 0;
        total_rot = 0;
        nonfinite = 0;
    }
    __syncthreads();
    const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8;
    const int slot = (b5 ? 12 : 0) + (b4 ? 6 : 0) + (b3 ? 3 : 0);
    const int nrounds = cross ? PW / 2 : PW - 1;
    int buf = 0;
    for (int sw = 0; sw < max_inner; ++sw) {
        for (int rr = 0; rr < nrounds; ++rr) {
            double v[24];
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) {
                double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
                for (int j = 0; j < ROWS; ++j) {
                    al += u[kk][j] * u[kk][j];
                    be += u[PW - 1 - kk][j] * u[PW - 1 - kk][j];
                    ga += u[kk][j] * u[PW - 1 - kk][j];
                }
                v[3 * kk] = al;
                v[3 * kk + 1] = be;
                v[3 * kk + 2] = ga;
            }
            // reduce-scatter: after the xor-32/16/8 steps a lane holds 3 of the 24
            // sums (slots `slot` .. slot + 2) over 8 lanes; xor 4/2/1 completes them
            double w12[12], w6[6], w3[3];
#pragma unroll
            for (int i = 0; i < 12; ++i) {
                const double send = b5 ? v[i] : v[12 + i], keep = b5 ? v[12 + i] : v[i];
                w12[i] = keep + __shfl_xor(send, 32, 64);
            }
#pragma unroll
            for (int i = 0; i < 6; ++i) {
                const double send = b4 ? w12[i] : w12[6 + i], keep = b4 ? w12[6 + i] : w12[i];
                w6[i] = keep + __shfl_xor(send, 16, 64);
            }
            // inside 16-lane rows the partners come from DPP: row_mirror pairs
            // lane l with l ^ 15 (opposite bit 3), then half-mirror (l ^ 7) and
            // the quad permutations l ^ 2, l ^ 1 finish the sums over 8 lanes
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const double send = b3 ? w6[i] : w6[3 + i], keep = b3 ? w6[3 + i] : w6[i];
                w3[i] = keep + dpp_d<0x140>(send);
            }
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                w3[i] += dpp_d<0x141>(w3[i]);
                w3[i] += dpp_d<0x4E>(w3[i]);
                w3[i] += dpp_d<0xB1>(w3[i]);
            }
            if ((lane & 7) == 0) {
                red[buf][w][slot] = w3[0];
                red[buf][w][slot + 1] = w3[1];
                red[buf][w][slot + 2] = w3[2];
            }
            __syncthreads();
            // every wavefront computes the 8 rotations (lane kk: pair kk) from the
            // same sums in the same order, so all rows see identical (c, s); the
            // parity buffer keeps the next round's writes off this round's sums
            double cl = 1.0, sl = 0.0;
            if (lane < 8) {
                double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
                for (int x = 0; x < NT / 64; ++x) {
                    al += red[buf][x][3 * lane];
                    be += red[buf][x][3 * lane + 1];
                    ga += red[buf][x][3 * lane + 2];
                }
                if (!isfinite(al + be + ga)) {
                    if (w == 0) nonfinite = 1;
                } else if (jacobi_rotation(al, be, ga, tol, cl, sl)) {
                    if (w == 0) atomicAdd(&sweep_rot, 1);
                }
            }
            buf ^= 1;
#pragma unroll
            for (int kk = 0; kk < 8; ++kk) {
                const double c = read_lane(cl, kk), s = read_lane(sl, kk);
#pragma unroll
                for (int j = 0; j < ROWS; ++j) {
                    const double x = u[kk][j], y = u[PW - 1 - kk][j];
                    u[kk][j] = c * x - s * y;
                    u[PW - 1 - kk][j] = s * x + c * y;
                }
                const double x = vrow[kk], y = vrow[PW - 1 - kk];
                vrow[kk] = c * x - s * y;
                vrow[PW - 1 - kk] = s * x + c * y;
            }
            if (cross)
                shift_cross<ROWS>(u, vrow);
            else
                shift_slots<ROWS>(u, vrow);
        }
        __syncthreads();   // the last round's counts
        const int more = sweep_rot;
        __syncthreads();
        if (t == 0) {
            total_rot += more;
            sweep_rot = 0;
        }
        if (!more) break;
    }
    __syncthreads();
    const int total = total_rot;
    if (t == 0) {
        if (total > 0) atomicAdd(&flags[mat], total);
        if (nonfinite) flags[jb.count + mat] = 1;
    }
    if (total == 0) return;
#pragma unroll
    for (int c = 0; c < PW; ++c) {
        const int g = c < 8 ? I * 8 + c : J * 8 + (c - 8);
#pragma unroll
        for (int j = 0; j < ROWS; ++j) {
            const int row = t + NT * j;
            if (g < n && row < m) {
                __builtin_nontemporal_store(u[c][j], &U[(long)g * m + row]);
            }
        }
    }
    if constexpr (!WV) return;
    if (t < PW) {
#pragma unroll
        for (int c = 0; c < PW; ++c) vpan[t][c] = vrow[c];
    }
    __syncthreads();
    // V[:, panel] <- V[:, panel] * (panel rotation); thread t holds rows t + 256 j
    // (n <= m, so ROWS covers them); each thread reads its rows before writing them
    double vv[PW][ROWS];
#pragma unroll
    for (int c = 0; c < PW; ++c) {
        const int g = c < 8 ? I * 8 + c : J * 8 + (c - 8);
#pragma unroll
        for (int j = 0; j < ROWS; ++j) {
            const int row = t + NT * j;
            vv[c][j] = (g < n && row < n) ? V[(long)g * n + row] : 0.0;
        }
    }
#pragma unroll
    for (int c2 = 0; c2 < PW; ++c2) {
        const int g = c2 < 8 ? I * 8 + c2 : J * 8 + (c2 - 8);
        double acc[ROWS];
#pragma unroll
        for (int j = 0; j < ROWS; ++j) acc[j] = 0.0;
#pragma unroll
        for (int c = 0; c < PW; ++c) {
            const double wv = vpan[c][c2];
#pragma unroll
            for (int j = 0; j < ROWS; ++j) acc[j] = fma(vv[c][j], wv, acc[j]);
        }
#pragma unroll
        for (int j = 0; j < ROWS; ++j) {
            const int row = t + NT * j;
            if (g < n && row < n) V[(long)g * n + row] = acc[j];
        }
    }
}

__global__ void init_v_kernel(JacobiBatch jb) {
    long tot = (long)jb.count * jb.n * jb.n;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < tot; i += (long)gridDim.x * blockDim.x) {
        long mat = i / ((long)jb.n * jb.n), rem = i - mat * jb.n * jb.n;
        int col = (int)(rem / jb.n), row = (int)(rem % jb.n);
        jb.vt[mat * jb.strideV + (long)col * jb.n + row] = row == col ? 1.0 : 0.0;
    }
}

// per-matrix max |u| -> scale[mat]; u /= scale.  Three passes so that the
// whole GPU takes part (a batch holds only a few matrices): partial maxima of
// P slices per matrix, their maximum, then the division (max is exact in any
// order, so the result does not depend on P).
__global__ void absmax_partial_kernel(JacobiBatch jb, int P, double *part) {
    const int mat = blockIdx.y, b = blockIdx.x;
    const double *u = jb.ut + (long)mat * jb.strideU;
    const long tot = (long)jb.m * jb.n;
    double mx = 0.0;
    for (long i = (long)b * NT + threadIdx.x; i < tot; i += (long)P * NT) mx = fmax(mx, fabs(u[i]));
    __shared__ double red[NT];
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(long)mat * P + b] = red[0];
}

__global__ void absmax_final_kernel(const double *part, int P, double *scale) {
    const int mat = blockIdx.x;
    if (threadIdx.x) return;
    double mx = 0.0;
    for (int b = 0; b < P; ++b) mx = fmax(mx, part[(long)mat * P + b]);
    scale[mat] = mx > 0.0 ? mx : 1.0;
}

__global__ void divide_kernel(JacobiBatch jb, const double *scale) {
    const long per = (long)jb.m * jb.n, tot = per * jb.count;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
        const long mat = e / per;
        jb.ut[mat * jb.strideU + (e - mat * per)] /= scale[mat];
    }
}

// norms of the columns (one wave per column)
__global__ void norms_kernel(JacobiBatch jb, const double *scale, double *nrm) {
    const int mat = blockIdx.y;
    const int j = blockIdx.x * (NT / 64) + (threadIdx.x >> 6);
    if (j >= jb.n) return;
    const double *u = jb.ut + (long)mat * jb.strideU + (long)j * jb.m;
    double s = 0.0;
    for (int i = threadIdx.x & 63; i < jb.m; i += 64) s += u[i] * u[i];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) nrm[(long)mat * jb.n + j] = sqrt(s);
}

// rank of every column in descending norm order (ties by index), then gather
__global__ void sort_gather_kernel(JacobiBatch jb, const double *scale, const double *nrm, double *s,
                                   double *us, double *vs) {
    const int mat = blockIdx.y;
    const int j = blockIdx.x;
    const double *nm = nrm + (long)mat * jb.n;
    const double sj = nm[j];
    __shared__ int rank_sh;
    if (threadIdx.x == 0) rank_sh = 0;
    __syncthreads();
    int cnt = 0;
    for (int k = threadIdx.x; k < jb.n; k += blockDim.x) {
        double sk = nm[k];
        cnt += (sk > sj || (sk == sj && k < j)) ? 1 : 0;
    }
    atomicAdd(&rank_sh, cnt);
    __syncthreads();
    const int rk = rank_sh;
    if (threadIdx.x == 0) s[(long)mat * jb.n + rk] = sj * scale[mat];
    const double *u = jb.ut + (long)mat * jb.strideU + (long)j * jb.m;
    double inv = sj > 0.0 ? 1.0 / sj : 0.0;
    if (us) {
        double *uo = us + (long)mat * jb.m * jb.n;
        for (int i = threadIdx.x; i < jb.m; i += blockDim.x) uo[(long)i * jb.n + rk] = u[i] * inv;
    }
    if (vs && jb.vt) {
        const double *v = jb.vt + (long)mat * jb.strideV + (long)j * jb.n;
        double *vo = vs + (long)mat * jb.n * jb.n;
        for (int i = threadIdx.x; i < jb.n; i += blockDim.x) vo[(long)i * jb.n + rk] = v[i];
    }
}

// flags layout: [0, count) rotations of the sweep, [count, 2 count) non-finite
// pairs seen, [2 count] done (no launch of the solve does anything once set)
__global__ void flags_init_kernel(int *flags, int count) {
    for (int i = threadIdx.x; i <= 2 * count; i += blockDim.x) flags[i] = 0;
}

__global__ void sweep_begin_kernel(int *flags, int count) {
    if (flags[2 * count]) return;
    for (int i = threadIdx.x; i < 2 * count; i += blockDim.x) flags[i] = 0;
}

// end of a device-driven sweep: the solve is done once no matrix rotated;
// rotations left after the last allowed sweep set *status = code, a
// non-finite pair *status = code + 2
__global__ void sweep_end_kernel(int *flags, int count, int last, int *status, int code) {
    if (threadIdx.x || flags[2 * count]) return;
    int any = 0, bad = 0;
    for (int i = 0; i < count; ++i) {
        any |= flags[i] != 0;
        bad |= flags[count + i] != 0;
    }
    if (bad) *status = code + 2;
    else if (any && last) *status = code;
    if (bad || !any || last) flags[2 * count] = 1;
}

// the one-launch solver's verdict, device side: flags[i] < 0 is no convergence
__global__ void full_check_kernel(const int *flags, int count, int *status, int code) {
    if (threadIdx.x) return;
    for (int i = 0; i < count; ++i) {
        if (flags[count + i] != 0) *status = code + 2;
        else if (flags[i] < 0) *status = code;
    }
}
}  // namespace

namespace {
// sweep statistics of every call, printed when TRG_JACOBI_TRACE is set
bool trace_on() {
    static const bool on = [] {
        const char *e = getenv("TRG_JACOBI_TRACE");
        return e && *e && *e != '0';
    }();
    return on;
}

[[noreturn]] void not_converged(const JacobiBatch &jb, const std::vector<int> &fl, bool full_path) {
    char msg[256];
    int stuck = 0, nonfinite = 0, worst_rot = 0;
    for (int i = 0; i < jb.count; ++i) {
        nonfinite += fl[jb.count + i] != 0;
        int rot = full_path ? (fl[i] < 0 ? -1 - fl[i] : 0) : fl[i];
        stuck += rot > 0;
        worst_rot = std::max(worst_rot, rot);
    }
    snprintf(msg, sizeof msg,
             "Jacobi SVD did not converge: %d of %d matrices (m %d, n %d) still rotating, up to %d "
             "rotations in the last sweep; %d with non-finite entries",
             stuck, jb.count, jb.m, jb.n, worst_rot, nonfinite);
    throw Error(-4, msg);
}
}  // namespace

bool jacobi_one_launch(const JacobiBatch &jb) { return jb.n <= 96; }

// flags_dev: 2 * count + 1 ints of device scratch
int jacobi_svd(const JacobiBatch &jb, int max_sweeps, int *flags_dev, double *work, hipStream_t st,
               const DevLoop *dl) {
    if (jb.count == 0 || jb.n == 0) return 0;
    const double tol = sqrt((double)jb.m) * 2.220446049250313e-16;
    {   // the column-norm area of work (count * n doubles) holds the partial maxima
        const int P = std::min(jb.n, 64);
        hipLaunchKernelGGL(absmax_partial_kernel, dim3(P, jb.count), dim3(NT), 0, st, jb, P, work + jb.count);
        hipLaunchKernelGGL(absmax_final_kernel, dim3(jb.count), dim3(64), 0, st, work + jb.count, P, work);
        const size_t tot = (size_t)jb.count * jb.m * jb.n;
        hipLaunchKernelGGL(divide_kernel, dim3((unsigned)std::min<size_t>(cdiv(tot, 256), 65536)), dim3(256), 0, st,
                           jb, work);
    }
    if (jb.vt)
        hipLaunchKernelGGL(init_v_kernel, dim3(cdiv((size_t)jb.count * jb.n * jb.n, 256)), dim3(256), 0, st, jb);
    TRG_HIP_CHECK(hipGetLastError());
    const int mm = jb.n + (jb.n & 1);
    std::vector<int> fl(2 * jb.count);
    if (jacobi_one_launch(jb)) {
        hipLaunchKernelGGL(full_kernel, dim3(jb.count), dim3(NT), 0, st, jb, max_sweeps, tol, flags_dev);
        TRG_HIP_CHECK(hipGetLastError());
        if (dl) {
            hipLaunchKernelGGL(full_check_kernel, dim3(1), dim3(64), 0, st, flags_dev, jb.count, dl->status, dl->code);
            TRG_HIP_CHECK(hipGetLastError());
            return -1;
        }
        TRG_HIP_CHECK(hipMemcpyAsync(fl.data(), flags_dev, sizeof(int) * 2 * jb.count, hipMemcpyDeviceToHost, st));
        TRG_HIP_CHECK(hipStreamSynchronize(st));
        int worst = 0;
        bool bad = false;
        for (int i = 0; i < jb.count; ++i) {
            bad |= fl[i] < 0 || fl[jb.count + i] != 0;
            worst = std::max(worst, fl[i]);
        }
        if (trace_on()) fprintf(stderr, "[jacobi] count %d m %d n %d sweeps %d (one launch)\n", jb.count, jb.m, jb.n, worst);
        if (bad) not_converged(jb, fl, true);
        return worst;
    }
    const bool panel = jb.m <= 4 * NT;
    const int nbk = ((jb.n + PW - 1) / PW) * PW / 8;   // blocks of 8 columns (even)
    hipLaunchKernelGGL(flags_init_kernel, dim3(1), dim3(256), 0, st, flags_dev, jb.count);
    const int nsweeps = dl ? std::min(dl->sweeps, max_sweeps) : max_sweeps;
    for (int sweep = 0; sweep < nsweeps; ++sweep) {
        hipLaunchKernelGGL(sweep_begin_kernel, dim3(1), dim3(256), 0, st, flags_dev, jb.count);
        if (panel) {
            dim3 grid(nbk / 2, jb.count);
            // the first launch of a sweep also takes the pairs inside every block
            const bool wv = jb.vt != nullptr;
            auto kern = jb.m <= NT       ? (wv ? panel_kernel<1, true> : panel_kernel<1, false>)
                        : jb.m <= 2 * NT ? (wv ? panel_kernel<2, true> : panel_kernel<2, false>)
                                         : (wv ? panel_kernel<4, true> : panel_kernel<4, false>);
            for (int r = 0; r < nbk - 1; ++r) {
                const int cross = r > 0;
                hipLaunchKernelGGL(kern, grid, dim3(NT), 0, st, jb, nbk, r, tol, PANEL_INNER, cross, flags_dev);
            }
        } else {
            dim3 grid(cdiv(mm / 2, NT / 64), jb.count);
            for (int r = 0; r < mm - 1; ++r)
                hipLaunchKernelGGL(round_kernel, grid, dim3(NT), 0, st, jb, r, tol, flags_dev);
        }
        TRG_HIP_CHECK(hipGetLastError());
        if (dl) {
            hipLaunchKernelGGL(sweep_end_kernel, dim3(1), dim3(64), 0, st, flags_dev, jb.count,
                               sweep + 1 == nsweeps ? 1 : 0, dl->status, dl->code);
            TRG_HIP_CHECK(hipGetLastError());
            continue;
        }
        TRG_HIP_CHECK(hipMemcpyAsync(fl.data(), flags_dev, sizeof(int) * 2 * jb.count, hipMemcpyDeviceToHost, st));
        TRG_HIP_CHECK(hipStreamSynchronize(st));
        bool any = false, bad = false;
        long tot = 0;
        for (int i = 0; i < jb.count; ++i) {
            any |= fl[i] != 0;
            bad |= fl[jb.count + i] != 0;
            tot += fl[i];
        }
        if (trace_on()) fprintf(stderr, "[jacobi] count %d m %d n %d sweep %d rotations %ld\n", jb.count, jb.m, jb.n, sweep, tot);
        if (bad) not_converged(jb, fl, false);
        if (!any) return sweep;
        if (sweep + 1 == max_sweeps) not_converged(jb, fl, false);
    }
    if (dl) return -1;
    throw Error(-4, "Jacobi SVD did not converge");
}

void jacobi_finish(const JacobiBatch &jb, double *s, double *u_sorted, double *v_sorted, double *work,
                   hipStream_t st) {
    // work: count (scale) + count*n (norms)
    double *scale = work, *nrm = work + jb.count;
    hipLaunchKernelGGL(norms_kernel, dim3(cdiv(jb.n, NT / 64), jb.count), dim3(NT), 0, st, jb, scale, nrm);
    hipLaunchKernelGGL(sort_gather_kernel, dim3(jb.n, jb.count), dim3(NT), 0, st, jb, scale, nrm, s, u_sorted,
                       v_sorted);
    TRG_HIP_CHECK(hipGetLastError());
}

}  // namespace trg
