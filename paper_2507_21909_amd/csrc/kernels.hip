// Layout, element-wise and bookkeeping kernels of the RG step.
#include <cmath>

#include <cstdio>
#include <cstdlib>

#include "common.h"

namespace trg {

namespace {
constexpr int MAXD = 8;
struct PermArgs {
    int nd;
    long dd[MAXD];   // dst dims
    long ss[MAXD];   // src stride of the axis that becomes dst axis i
    long total;
};

__global__ void permute_kernel(const double *__restrict__ src, double *__restrict__ dst, PermArgs a) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < a.total; i += (long)gridDim.x * blockDim.x) {
        long rem = i, off = 0;
        for (int d = a.nd - 1; d >= 0; --d) {
            long q = rem / a.dd[d];
            off += (rem - q * a.dd[d]) * a.ss[d];
            rem = q;
        }
        dst[i] = src[off];
    }
}

// General permutation whose destination's last axis is not the source's unit
// stride axis: 32 x 32 tiles over dst axis ka (source stride 1) and dst axis
// nd - 1, staged through LDS so that reads run along the source's unit stride
// and writes along the destination's; block id = (batch, tile_b, tile_a) with
// the batch over the other destination axes.  dst strides are row-major.
__global__ __launch_bounds__(256) void permute_tiled_kernel(const double *__restrict__ src, double *__restrict__ dst,
                                                            PermArgs a, int ka, long nta, long ntb) {
    __shared__ double tile[32][33];
    const int L = a.nd - 1, tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    long bid = blockIdx.x;
    const long ta = bid % nta;
    bid /= nta;
    const long tb = bid % ntb;
    long batch = bid / ntb;
    // destination strides (row-major) and the batch's base offsets
    long ostr[MAXD];
    ostr[L] = 1;
    for (int d = L - 1; d >= 0; --d) ostr[d] = ostr[d + 1] * a.dd[d + 1];
    long in_base = 0, out_base = 0;
    for (int d = L - 1; d >= 0; --d) {
        if (d == ka) continue;
        const long q = batch / a.dd[d];
        const long idx = batch - q * a.dd[d];
        in_base += idx * a.ss[d];
        out_base += idx * ostr[d];
        batch = q;
    }
    const long a0 = ta * 32, b0 = tb * 32, na = a.dd[ka], nb = a.dd[L];
    // read: x along ka (source stride 1), y along the destination's last axis
    for (int y = ty; y < 32; y += 8) {
        const long ai = a0 + tx, bi = b0 + y;
        if (ai < na && bi < nb) tile[y][tx] = src[in_base + ai + bi * a.ss[L]];
    }
    __syncthreads();
    // write: x along the destination's last axis (stride 1), y along ka
    for (int y = ty; y < 32; y += 8) {
        const long ai = a0 + y, bi = b0 + tx;
        if (ai < na && bi < nb) dst[out_base + ai * ostr[ka] + bi] = tile[tx][y];
    }
}

// tiled 2-D transpose for the common case "swap two contiguous groups":
// dst[b][c][r] = src[b][r][c]
__global__ void transpose_kernel(const double *__restrict__ src, double *__restrict__ dst, long R, long Cc) {
    __shared__ double tile[32][33];
    long b = blockIdx.z;
    long r0 = blockIdx.y * 32L, c0 = blockIdx.x * 32L;
    const double *s = src + b * R * Cc;
    double *d = dst + b * R * Cc;
    int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    for (int k = ty; k < 32; k += 8) {
        long r = r0 + k, c = c0 + tx;
        tile[k][tx] = (r < R && c < Cc) ? s[r * Cc + c] : 0.0;
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        long c = c0 + k, r = r0 + tx;
        if (r < R && c < Cc) d[c * R + r] = tile[tx][k];
    }
}

__global__ void scale_axis_kernel(double *t, long total, long inner, long dim, const double *v, int mode) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
        long ax = (i / inner) % dim;
        double x = v[ax];
        double f = mode == 1 ? x : mode == 2 ? x * x : (x > 0.0 ? 1.0 / sqrt(x) : 0.0);
        t[i] *= f;
    }
}

__global__ void fill_kernel(double *p, long n, double v) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void copy_kernel(double *d, const double *s, long n) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) d[i] = s[i];
}

__global__ void kept_kernel(const double *v, int n, int cap, double eps, double tau, int *out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int k = 0;
    double top = n > 0 ? v[0] : 0.0;
    if (n > 0 && top > 0.0) {
        int nz = 0;
        for (int i = 0; i < n; ++i) nz += v[i] > eps * top ? 1 : 0;
        k = cap < nz ? cap : nz;
        if (k < nz)
            while (k > 0 && (v[k - 1] - v[k]) <= tau * top) --k;
    }
    *out = k;
}

__global__ void zero_tail_kernel(double *a, long rows, int cols, long ld, const int *kept) {
    int k = *kept;
    long n = rows * (long)cols;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        long r = i / cols;
        int c = (int)(i - r * cols);
        if (c >= k) a[r * ld + c] = 0.0;
    }
}

struct SignArgs {
    int nd;
    long dd[MAXD];
    double pw[MAXD];
};

__global__ void scale_cols_kernel(double *a, long rows, int cols, long ld, const double *sg) {
    long n = rows * (long)cols;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        long r = i / cols;
        int c = (int)(i - r * cols);
        a[r * ld + c] *= sg[c];
    }
}

// Philox4x32-10 (Salmon et al., SC'11)
__device__ inline void philox(uint32_t c[4], uint32_t k0, uint32_t k1) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = (uint64_t)M0 * c[0], p1 = (uint64_t)M1 * c[2];
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    }
}

struct SketchArgs {
    uint32_t k0, k1, instance, step;
    const int *stepp;   // step index read on the device (replayed graphs), else step
    int j1, j2, j3, chi, m, layout_jbm;
    long total;
};

// Omega entry for multi-index (beta, j1, j2, j3, m): standard normal from the
// first two Philox words (Box-Muller, cosine branch).
__global__ void sketch_kernel(double *out, SketchArgs a) {
    const uint32_t step = a.stepp ? (uint32_t)*a.stepp : a.step;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < a.total; i += (long)gridDim.x * blockDim.x) {
        long rem = i;
        int mm = (int)(rem % a.m); rem /= a.m;
        int b, x1, x2, x3;
        if (a.layout_jbm) {   // [j1, j2, j3, beta, m]
            b = (int)(rem % a.chi); rem /= a.chi;
            x3 = (int)(rem % a.j3); rem /= a.j3;
            x2 = (int)(rem % a.j2); rem /= a.j2;
            x1 = (int)rem;
        } else {              // [beta, j1, j2, j3, m]
            x3 = (int)(rem % a.j3); rem /= a.j3;
            x2 = (int)(rem % a.j2); rem /= a.j2;
            x1 = (int)(rem % a.j1); rem /= a.j1;
            b = (int)rem;
        }
        uint32_t c[4] = {(uint32_t)x1 | ((uint32_t)x2 << 8) | ((uint32_t)x3 << 16) | ((uint32_t)b << 24),
                         (uint32_t)mm | ((step & 0xFFFFu) << 16), a.instance, 0x4F4D4547u};
        philox(c, a.k0, a.k1);
        double u1 = ((double)c[0] + 0.5) * 0x1p-32;
        double u2 = ((double)c[1] + 0.5) * 0x1p-32;
        out[i] = sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
    }
}

// Z[j][l] = sum_i Q[i, j] w_l(i), w_l(i) = 0.5 + frac(g (1 + code(i)) + l (sqrt 2 - 1)),
// l < L <= LM (1 for the sign vectors, CANON_L for the canonical bases), with
// code(i) = sum_d idx_d(i) pw_d over the row multi-index.
// First pass: workgroup (x, y) takes 64 columns and the y-th chunk of rpb rows;
// each wavefront reads whole 64-column row segments (coalesced), every 4th row
// of the chunk, and the 4 wavefronts' sums are added in a fixed order into
// part[(y * cols + j) * L + l].  Second pass: Z = the chunk partials added in
// chunk order (and, with sg, the sign of Z[j][0]).  Both orders are fixed, so
// the sums are the same bits on every run.
template <int LM>
__global__ __launch_bounds__(256) void weights_partial_kernel(const double *q, long rows, int cols, long ld,
                                                              SignArgs a, int L, long rpb, double *part) {
    const double golden = 0.6180339887498949, c2 = 0.41421356237309515;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + lane;
    const long r0 = (long)blockIdx.y * rpb, r1 = r0 + rpb < rows ? r0 + rpb : rows;
    double acc[LM];
#pragma unroll
    for (int l = 0; l < LM; ++l) acc[l] = 0.0;
    for (long r = r0 + w; r < r1; r += 4) {
        long rem = r;
        double code = 0.0;
        for (int d = a.nd - 1; d >= 0; --d) {
            long qd = rem / a.dd[d];
            code += (double)(rem - qd * a.dd[d]) * a.pw[d];
            rem = qd;
        }
        const double x = golden * (1.0 + code);
        const double v = j < cols ? q[r * ld + j] : 0.0;
#pragma unroll
        for (int l = 0; l < LM; ++l)
            if (l < L) {
                const double y = x + l * c2;
                acc[l] += (0.5 + (y - floor(y))) * v;
            }
    }
    __shared__ double red[4][64][LM + 1];
#pragma unroll
    for (int l = 0; l < LM; ++l)
        if (l < L) red[w][lane][l] = acc[l];
    __syncthreads();
    if (w == 0 && j < cols)
        for (int l = 0; l < L; ++l)
            part[((long)blockIdx.y * cols + j) * L + l] =
                ((red[0][lane][l] + red[1][lane][l]) + red[2][lane][l]) + red[3][lane][l];
}

__global__ void weights_final_kernel(const double *part, int nchunk, int cols, int L, double *z, double *sg) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;   // j * L + l
    if (i >= cols * L) return;
    double acc = 0.0;
    for (int b = 0; b < nchunk; ++b) acc += part[(long)b * cols * L + i];
    z[i] = acc;
    if (sg) sg[i] = acc < 0.0 ? -1.0 : 1.0;   // L == 1
}

// Block-diagonal canonical rotation (n x n): identity, except on each multiplet
// [a, a+d) of the first k values (neighbours within tau * v[0]) where it is the
// Q factor (positive diagonal R) of Z_m[r][c] = z[(a+r)*L + c], c < d.
__global__ void canon_rot_kernel(const double *v, int n, const int *kdev, double tau, const double *z, int L,
                                 double *rot, int *status) {
    if (threadIdx.x || blockIdx.x) return;
    int k = *kdev;
    for (long i = 0; i < (long)n * n; ++i) rot[i] = (i / n == i % n) ? 1.0 : 0.0;
    if (k <= 0) return;
    int a = 0;
    for (int i = 1; i <= k; ++i) {
        if (i < k && (v[i - 1] - v[i]) <= tau * v[0]) continue;
        int d = i - a;
        if (d > L) {
            *status = 2;
        } else {
            double qm[CANON_L][CANON_L];
            for (int c = 0; c < d; ++c) {
                double col[CANON_L];
                for (int r = 0; r < d; ++r) col[r] = z[(long)(a + r) * L + c];
                for (int pass = 0; pass < 2; ++pass)
                    for (int p = 0; p < c; ++p) {
                        double dot = 0.0;
                        for (int r = 0; r < d; ++r) dot += qm[r][p] * col[r];
                        for (int r = 0; r < d; ++r) col[r] -= dot * qm[r][p];
                    }
                double nrm = 0.0;
                for (int r = 0; r < d; ++r) nrm += col[r] * col[r];
                nrm = sqrt(nrm);
                for (int r = 0; r < d; ++r) qm[r][c] = nrm > 0.0 ? col[r] / nrm : (r == c ? 1.0 : 0.0);
            }
            for (int r = 0; r < d; ++r)
                for (int c = 0; c < d; ++c) rot[(long)(a + r) * n + (a + c)] = qm[r][c];
        }
        a = i;
    }
}

inline unsigned grid_for(long n) { return (unsigned)std::min<long>((n + 255) / 256, 65536L); }
}  // namespace

void permute(const double *src, double *dst, const std::vector<int> &dims, const std::vector<int> &perm,
             hipStream_t st) {
    int nd = (int)dims.size();
    TRG_REQUIRE(nd <= MAXD && (int)perm.size() == nd, -1, "permute: bad rank");
    long total = 1;
    for (int d : dims) total *= d;
    if (total == 0) return;
    // drop trivial permutations
    bool ident = true;
    for (int i = 0; i < nd; ++i) ident &= perm[i] == i;
    if (ident) {
        if (src != dst) copy(dst, src, (size_t)total, st);
        return;
    }
    std::vector<long> sstr(nd);
    long s = 1;
    for (int d = nd - 1; d >= 0; --d) { sstr[d] = s; s *= dims[d]; }
    // fast path: dst = [P, C, R] from src = [P, R, C] (two contiguous groups swapped)
    for (int split_a = 0; split_a < nd; ++split_a) {
        // prefix [0, split_a) fixed
        bool pre = true;
        for (int i = 0; i < split_a; ++i) pre &= perm[i] == i;
        if (!pre) break;
        for (int split_b = split_a + 1; split_b < nd; ++split_b) {
            // src groups: R = [split_a, split_b), C = [split_b, nd); dst = prefix, C, R
            bool ok = true;
            int p = split_a;
            for (int i = split_b; i < nd; ++i) ok &= perm[p++] == i;
            for (int i = split_a; i < split_b; ++i) ok &= perm[p++] == i;
            if (!ok) continue;
            long P = 1, R = 1, Cc = 1;
            for (int i = 0; i < split_a; ++i) P *= dims[i];
            for (int i = split_a; i < split_b; ++i) R *= dims[i];
            for (int i = split_b; i < nd; ++i) Cc *= dims[i];
            if (P <= 65535) {
                dim3 grid(cdiv(Cc, 32), cdiv(R, 32), (unsigned)P);
                if (grid.y <= 65535) {
                    hipLaunchKernelGGL(transpose_kernel, grid, dim3(256), 0, st, src, dst, R, Cc);
                    TRG_HIP_CHECK(hipGetLastError());
                    return;
                }
            }
        }
    }
    static const bool trace = [] {
        const char *e = getenv("TRG_SHAPE_TRACE");
        return e && *e && *e != '0';
    }();
    if (trace) {
        fprintf(stderr, "[permute] total %ld dims", total);
        for (int i = 0; i < nd; ++i) fprintf(stderr, " %d", dims[i]);
        fprintf(stderr, " perm");
        for (int i = 0; i < nd; ++i) fprintf(stderr, " %d", perm[i]);
        fprintf(stderr, "\n");
    }
    PermArgs a{};
    a.nd = nd;
    a.total = total;
    for (int i = 0; i < nd; ++i) { a.dd[i] = dims[perm[i]]; a.ss[i] = sstr[perm[i]]; }
    // the source's unit-stride axis lands at dst axis ka; tile it against the
    // dst's last axis when both are long enough to fill 32-wide rows
    int ka = -1;
    for (int i = 0; i < nd; ++i)
        if (a.ss[i] == 1) ka = i;
    if (ka >= 0 && ka != nd - 1 && a.dd[ka] >= 16 && a.dd[nd - 1] >= 16) {
        const long nta = (a.dd[ka] + 31) / 32, ntb = (a.dd[nd - 1] + 31) / 32;
        const long nbatch = total / (a.dd[ka] * a.dd[nd - 1]);
        const long blocks = nta * ntb * nbatch;
        if (blocks <= 2147483647L) {
            hipLaunchKernelGGL(permute_tiled_kernel, dim3((unsigned)blocks), dim3(256), 0, st, src, dst, a, ka, nta,
                               ntb);
            TRG_HIP_CHECK(hipGetLastError());
            return;
        }
    }
    hipLaunchKernelGGL(permute_kernel, dim3(grid_for(total)), dim3(256), 0, st, src, dst, a);
    TRG_HIP_CHECK(hipGetLastError());
}

void scale_axis(double *t, const std::vector<int> &dims, int axis, const double *v, int mode, hipStream_t st) {
    long total = 1, inner = 1;
    for (size_t d = 0; d < dims.size(); ++d) {
        total *= dims[d];
        if ((int)d > axis) inner *= dims[d];
    }
    if (total == 0) return;
    hipLaunchKernelGGL(scale_axis_kernel, dim3(grid_for(total)), dim3(256), 0, st, t, total, inner,
                       (long)dims[axis], v, mode);
    TRG_HIP_CHECK(hipGetLastError());
}

namespace {
__global__ void sum_slices_kernel(const double *w, int nslices, long M, long N, double *C, long sCr, long sCn) {
    const long tot = M * N;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int s = 0; s < nslices; ++s) acc += w[(long)s * tot + e];
        C[(e / N) * sCr + (e % N) * sCn] = acc;
    }
}
}  // namespace

void sum_slices(const double *w, int nslices, long M, long N, double *C, long sCr, long sCn, hipStream_t st) {
    if (M * N == 0) return;
    hipLaunchKernelGGL(sum_slices_kernel, dim3(grid_for(M * N)), dim3(256), 0, st, w, nslices, M, N, C, sCr, sCn);
    TRG_HIP_CHECK(hipGetLastError());
}

void fill(double *p, size_t n, double v, hipStream_t st) {
    if (!n) return;
    hipLaunchKernelGGL(fill_kernel, dim3(grid_for((long)n)), dim3(256), 0, st, p, (long)n, v);
    TRG_HIP_CHECK(hipGetLastError());
}

void copy(double *dst, const double *src, size_t n, hipStream_t st) {
    if (!n) return;
    hipLaunchKernelGGL(copy_kernel, dim3(grid_for((long)n)), dim3(256), 0, st, dst, src, (long)n);
    TRG_HIP_CHECK(hipGetLastError());
}

void kept_count(const double *vals, int n, int cap, double eps_rel, double tau_deg, int *kept_dev, hipStream_t st) {
    hipLaunchKernelGGL(kept_kernel, dim3(1), dim3(64), 0, st, vals, n, cap, eps_rel, tau_deg, kept_dev);
    TRG_HIP_CHECK(hipGetLastError());
}

void zero_tail_cols(double *a, long rows, int cols, long ld, const int *kept_dev, hipStream_t st) {
    long n = rows * cols;
    if (!n) return;
    hipLaunchKernelGGL(zero_tail_kernel, dim3(grid_for(n)), dim3(256), 0, st, a, rows, cols, ld, kept_dev);
    TRG_HIP_CHECK(hipGetLastError());
}

namespace {
// rows per chunk of the weight sums: at most 512 chunks, at least 256 rows each
long weight_rpb(long rows) {
    long r = (rows + 511) / 512;
    r = (r + 3) / 4 * 4;
    return r < 256 ? 256 : r;
}

}  // namespace

size_t weight_ws_doubles(long rows, int cols, int L) {
    const long rpb = weight_rpb(rows), nchunk = (rows + rpb - 1) / rpb;
    return (size_t)(nchunk + 1) * cols * L + 16;
}

namespace {
// Z (cols x L) into z, the chunk partials in ws (weight_ws_doubles)
void weight_sums(const double *q, long rows, int cols, long ld, const SignArgs &a, int L, double *ws, double *z,
                 double *sg, hipStream_t st) {
    const long rpb = weight_rpb(rows);
    const int nchunk = (int)((rows + rpb - 1) / rpb);
    TRG_REQUIRE(L == 1 || L == CANON_L, -1, "weight sums: L must be 1 or CANON_L");
    dim3 grid((cols + 63) / 64, nchunk);
    if (L == 1) hipLaunchKernelGGL(weights_partial_kernel<1>, grid, dim3(256), 0, st, q, rows, cols, ld, a, L, rpb, ws);
    else hipLaunchKernelGGL(weights_partial_kernel<CANON_L>, grid, dim3(256), 0, st, q, rows, cols, ld, a, L, rpb, ws);
    hipLaunchKernelGGL(weights_final_kernel, dim3((cols * L + 255) / 256), dim3(256), 0, st, ws, nchunk, cols, L,
                       z, sg);
    TRG_HIP_CHECK(hipGetLastError());
}
}  // namespace

void sign_vector(const double *q, long rows, int cols, long ld, const std::vector<int> &dims,
                 const std::vector<double> &pw, double *sg, double *ws, hipStream_t st) {
    SignArgs a{};
    a.nd = (int)dims.size();
    TRG_REQUIRE(a.nd <= MAXD && pw.size() == dims.size(), -1, "sign_vector: bad dims");
    long prod = 1;
    for (int i = 0; i < a.nd; ++i) { a.dd[i] = dims[i]; a.pw[i] = pw[i]; prod *= dims[i]; }
    TRG_REQUIRE(prod == rows, -1, "sign_vector: dims do not match rows");
    if (cols == 0) return;
    const long rpb = weight_rpb(rows), nchunk = (rows + rpb - 1) / rpb;
    weight_sums(q, rows, cols, ld, a, 1, ws, ws + nchunk * cols, sg, st);
}

void scale_cols(double *a, long rows, int cols, long ld, const double *sg, hipStream_t st) {
    long n = rows * cols;
    if (!n) return;
    hipLaunchKernelGGL(scale_cols_kernel, dim3(grid_for(n)), dim3(256), 0, st, a, rows, cols, ld, sg);
    TRG_HIP_CHECK(hipGetLastError());
}

void philox_sketch(double *out, uint64_t seed, int step, uint32_t instance, const std::vector<int> &jdims,
                   int chi, int m, int layout_jbm, hipStream_t st, const int *step_dev) {
    SketchArgs a{};
    a.stepp = step_dev;
    a.k0 = (uint32_t)(seed & 0xFFFFFFFFu);
    a.k1 = (uint32_t)(seed >> 32);
    a.instance = instance;
    a.step = (uint32_t)step;
    a.j1 = jdims.size() > 0 ? jdims[0] : 1;
    a.j2 = jdims.size() > 1 ? jdims[1] : 1;
    a.j3 = jdims.size() > 2 ? jdims[2] : 1;
    TRG_REQUIRE(a.j1 <= 256 && a.j2 <= 256 && a.j3 <= 256 && chi <= 256 && m <= 65536 && step <= 0xFFFF, -6,
                "sketch: leg dims must be < 256 and m < 65536");
    a.chi = chi;
    a.m = m;
    a.layout_jbm = layout_jbm;
    a.total = (long)a.j1 * a.j2 * a.j3 * chi * m;
    if (!a.total) return;
    hipLaunchKernelGGL(sketch_kernel, dim3(grid_for(a.total)), dim3(256), 0, st, out, a);
    TRG_HIP_CHECK(hipGetLastError());
}

}  // namespace trg

namespace trg {
void canonical_rotation(const double *q, long rows, int cols, long ld, const std::vector<int> &dims,
                        const std::vector<double> &pw, const double *vals, const int *k_dev, double tau,
                        double *z_work, double *rot, int *status, hipStream_t st) {
    SignArgs a{};
    a.nd = (int)dims.size();
    TRG_REQUIRE(a.nd <= MAXD && pw.size() == dims.size(), -1, "canonical_rotation: bad dims");
    long prod = 1;
    for (int i = 0; i < a.nd; ++i) { a.dd[i] = dims[i]; a.pw[i] = pw[i]; prod *= dims[i]; }
    TRG_REQUIRE(prod == rows, -1, "canonical_rotation: dims do not match rows");
    if (cols == 0) return;
    const int L = CANON_L;
    double *z = z_work, *part = z_work + (size_t)cols * L;
    weight_sums(q, rows, cols, ld, a, L, part, z, nullptr, st);
    hipLaunchKernelGGL(canon_rot_kernel, dim3(1), dim3(64), 0, st, vals, cols, k_dev, tau, z, L, rot, status);
    TRG_HIP_CHECK(hipGetLastError());
}
}  // namespace trg
