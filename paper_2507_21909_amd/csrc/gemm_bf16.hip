// Split-BF16 contractions over pre-split operand planes on the gfx950 matrix
// cores, for the coarse-graining GEMMs of makeMG / makeMH (Sec. II B) in mixed
// precision.
//
// Each FP64 operand is split once into three BF16 planes, x = x0 + x1 + x2,
// with the residuals formed exactly in FP64, and laid out K-contiguous
// ([plane][batch][row][Kp], Kp a multiple of 32, zero padded), so the GEMM
// reads 16-byte chunks that are already MFMA operands.  The product sums the
// six plane products x_i y_j with i + j <= 2 (about FP32 accuracy) on
// v_mfma_f32_32x32x16_bf16.  FP32 accumulators are added into FP64 registers
// after every K tile of 32, so FP32 rounding stays within partial sums of 32
// terms per product however long the contraction.
//
// Tiling: a 512-thread workgroup owns a 128 x 128 tile of C; its eight
// wavefronts (4 x 2) own 32 x 64 strips (one row block and two column blocks
// of 32 x 32).  K tiles of the three planes of both operands (48 KB each) are
// double-buffered in LDS, one barrier per tile, the tile after next
// prefetched into registers meanwhile.
// Workgroups are mapped to tiles XCD by XCD, in groups of 8 tile rows, so a
// group's A panels and the current B panel stay in one XCD's L2.
#include <hip/hip_ext.h>

#include "common.h"

namespace trg {
namespace {
typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int PT = 128;        // tile edge (rows and columns of C)
constexpr int PK = 32;         // K tile
constexpr int PNT = 512;       // threads per workgroup
constexpr int PPAD = 8;        // LDS row padding (bf16 elements; rows stay 16-byte aligned)
constexpr int PGM = 8;         // tile rows per L2 group

// x = a + b + c in BF16 with the residuals taken exactly in FP64 (a subtraction
// of two numbers within a factor 2 of each other is exact)
__device__ inline void split3(double x, __bf16 &a, __bf16 &b, __bf16 &c) {
    a = (__bf16)(float)x;
    double r = x - (double)(float)a;
    b = (__bf16)(float)r;
    r -= (double)(float)b;
    c = (__bf16)(float)r;
}

// planes[p][bt][r][k] = part p of src[bt][r][k] (zero for k >= K), Kp columns.
// 64 x 64 tiles through LDS: the source is read along whichever of its two
// axes is contiguous (rows_fast: sR == 1), the planes are written along k.
__global__ __launch_bounds__(256) void split3_kernel(const double *src, long sR, long sK, long sB, int rows, int K,
                                                     int Kp, long plane, __bf16 *dst, int rows_fast) {
    __shared__ double t[64][65];
    const int bt = blockIdx.z, r0 = blockIdx.y * 64, k0 = blockIdx.x * 64;
    const double *s = src + (long)bt * sB;
    for (int e = threadIdx.x; e < 4096; e += 256) {
        const int i = rows_fast ? (e & 63) : (e >> 6), j = rows_fast ? (e >> 6) : (e & 63);
        const int r = r0 + i, k = k0 + j;
        t[i][j] = (r < rows && k < K) ? s[(long)r * sR + (long)k * sK] : 0.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 4096; e += 256) {
        const int i = e >> 6, j = e & 63;
        const int r = r0 + i, k = k0 + j;
        if (r < rows && k < Kp) {
            __bf16 a, b, c;
            split3(t[i][j], a, b, c);
            const long o = ((long)bt * rows + r) * Kp + k;
            dst[o] = a;
            dst[o + plane] = b;
            dst[o + 2 * plane] = c;
        }
    }
}

__device__ inline void pdivmod(int x, int d, int &q, int &r) {
    if ((d & (d - 1)) == 0) {
        const int sh = __ffs(d) - 1;
        q = x >> sh;
        r = x & (d - 1);
    } else {
        q = x / d;
        r = x - q * d;
    }
}

__device__ inline long pc_off(const PlaneGemm &g, int r, int c) {
    long ro = (long)r * g.sCr, co = (long)c * g.sCn;
    if (g.cR2 > 0) {
        int q, m;
        pdivmod(r, g.cR2, q, m);
        ro = (long)q * g.sCr + (long)m * g.sCr2;
    }
    if (g.cN2 > 0) {
        int q, m;
        pdivmod(c, g.cN2, q, m);
        co = (long)q * g.sCn + (long)m * g.sCn2;
    }
    return ro + co;
}

__device__ inline void ptile_of(int &mt, int &nt, int gm) {
    const int G = gm > 0 ? gm : PGM;
    const int nx = gridDim.x, ny = gridDim.y, T = nx * ny;
    const int h = blockIdx.y * nx + blockIdx.x;
    const int L = (T % 8 == 0) ? (h % 8) * (T / 8) + h / 8 : h;
    const int in_group = G * nx, first = (L / in_group) * G;
    const int gs = min(ny - first, G);
    mt = first + (L % in_group) % gs;
    nt = (L % in_group) / gs;
}

// TAG only names the instance (1: the timed coarse-graining launches)
template <int TAG>
__global__ __launch_bounds__(PNT) void gemm_planes_kernel(PlaneGemm g) {
    const int bz = blockIdx.z, bo = bz / g.inner, bi = bz - (bz / g.inner) * g.inner;
    const __bf16 *A = static_cast<const __bf16 *>(g.A) + (long)bo * g.sAb;
    const __bf16 *B = static_cast<const __bf16 *>(g.B) + (long)bo * g.sBb;
    double *C = g.C + (long)bo * g.sCb + (long)bi * g.sCi;
    const int kbeg = bi * g.kslice, kend = min(g.Kp, kbeg + g.kslice);
    int mt, nt;
    ptile_of(mt, nt, g.gm);
    const int m0 = mt * PT, n0 = nt * PT;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wr = w >> 1, wc = w & 1;

    // two K tiles of both operands' planes (double-buffered, 120 KB)
    __shared__ __bf16 As[2][3][PT][PK + PPAD];
    __shared__ __bf16 Bs[2][3][PT][PK + PPAD];

    // loader: thread t moves the 16-byte chunk (row t / 4, k chunk t % 4) of each plane
    const int lr = t >> 2, lk = (t & 3) * 8;
    const bool a_in = m0 + lr < g.M, b_in = n0 + lr < g.N;
    const __bf16 *ga = A + (long)(m0 + lr) * g.Kp + lk;
    const __bf16 *gb = B + (long)(n0 + lr) * g.Kp + lk;
    uint4 ra[3], rb[3];
    auto load = [&](int k0) {
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            ra[p] = a_in ? *reinterpret_cast<const uint4 *>(ga + p * g.sAp + k0) : make_uint4(0, 0, 0, 0);
            rb[p] = b_in ? *reinterpret_cast<const uint4 *>(gb + p * g.sBp + k0) : make_uint4(0, 0, 0, 0);
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            *reinterpret_cast<uint4 *>(&As[buf][p][lr][lk]) = ra[p];
            *reinterpret_cast<uint4 *>(&Bs[buf][p][lr][lk]) = rb[p];
        }
    };

    f16v acc[2];
    double dacc[2][16];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            acc[j][e] = 0.0f;
            dacc[j][e] = 0.0;
        }
    }
    const int arow = wr * 32 + (lane & 31), kl = (lane >> 5) * 8;
    const int bcol = wc * 64 + (lane & 31);

    // tile i is multiplied from buffer i % 2 while tile i + 1 goes from the
    // registers into the other buffer and tile i + 2 is fetched: one barrier a tile
    if (kbeg < kend) {
        load(kbeg);
        store(0);
        if (kbeg + PK < kend) load(kbeg + PK);
    }
    __syncthreads();
    int buf = 0;
    for (int k0 = kbeg; k0 < kend; k0 += PK) {
        // raised priority while this wave's MFMAs issue; the other waves' LDS
        // traffic fills in around them
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int ks = 0; ks < PK; ks += 16) {
            bf8 a[3], b[2][3];
#pragma unroll
            for (int p = 0; p < 3; ++p) {
                a[p] = *reinterpret_cast<const bf8 *>(&As[buf][p][arow][ks + kl]);
                b[0][p] = *reinterpret_cast<const bf8 *>(&Bs[buf][p][bcol][ks + kl]);
                b[1][p] = *reinterpret_cast<const bf8 *>(&Bs[buf][p][bcol + 32][ks + kl]);
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                // small products first
                acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[2], b[j][0], acc[j], 0, 0, 0);
                acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], b[j][2], acc[j], 0, 0, 0);
                acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[1], b[j][1], acc[j], 0, 0, 0);
                acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[1], b[j][0], acc[j], 0, 0, 0);
                acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], b[j][1], acc[j], 0, 0, 0);
                acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], b[j][0], acc[j], 0, 0, 0);
            }
        }
        __builtin_amdgcn_s_setprio(0);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                dacc[j][e] += (double)acc[j][e];
                acc[j][e] = 0.0f;
            }
        }
        if (k0 + PK < kend) {
            store(buf ^ 1);
            if (k0 + 2 * PK < kend) load(k0 + 2 * PK);
        }
        __syncthreads();
        buf ^= 1;
    }
    // 32 x 32 block output: element e of lane l is row 8 (e / 4) + 4 (l / 32) + e % 4, column l % 32
#pragma unroll
    for (int j = 0; j < 2; ++j) {
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int r = m0 + wr * 32 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
            const int c = n0 + wc * 64 + j * 32 + (lane & 31);
            if (r < g.M && c < g.N) {
                double *p = C + pc_off(g, r, c);
                double v = g.alpha * dacc[j][e];
                if (g.beta != 0.0) v += g.beta * *p;
                *p = v;
            }
        }
    }
}
}  // namespace

size_t bf16_planes_elems(long rows, long Kp, int batch) { return 3 * (size_t)batch * rows * Kp; }

void split_bf16x3(const double *src, long sR, long sK, long sB, int rows, int K, int batch, int Kp, void *dst,
                  hipStream_t st) {
    TRG_REQUIRE(Kp % PK == 0 && Kp >= K && batch <= 65535, -6, "split_bf16x3: bad padding or batch");
    if (rows <= 0 || Kp <= 0 || batch <= 0) return;
    const long plane = (long)batch * rows * Kp;
    dim3 grid(cdiv(Kp, 64), cdiv(rows, 64), batch);
    hipLaunchKernelGGL(split3_kernel, grid, dim3(256), 0, st, src, sR, sK, sB, rows, K, Kp, plane,
                       static_cast<__bf16 *>(dst), sR == 1 && sK != 1 ? 1 : 0);
    TRG_HIP_CHECK(hipGetLastError());
}

void gemm_planes(const PlaneGemm &g, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
    if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return;
    TRG_REQUIRE(g.Kp % PK == 0 && g.kslice % PK == 0 && g.kslice > 0 && g.inner >= 1 &&
                    (long)g.inner * g.kslice >= g.Kp && (long)g.batch * g.inner <= 65535,
                -6, "gemm_planes: bad K slicing");
    dim3 grid(cdiv(g.N, PT), cdiv(g.M, PT), g.batch * g.inner);
    PlaneGemm h = g;
    if (h.gm == 0) {
        const double fl = 6.0 * 2.0 * h.M * (double)h.N * (double)h.Kp * h.batch;
        const std::array<long, 8> key{10, h.M, h.N, (long)h.Kp, h.batch, h.inner, h.kslice, h.cR2 > 0 || h.cN2 > 0};
        h.gm = tuned_gm(key, st, h.beta == 0.0 && fl >= 2e10, [&](int gm) {
            PlaneGemm x = h;
            x.gm = gm;
            hipLaunchKernelGGL(gemm_planes_kernel<0>, grid, dim3(PNT), 0, st, x);
        });
    }
    if (ev0) hipExtLaunchKernelGGL(gemm_planes_kernel<1>, grid, dim3(PNT), 0, st, ev0, ev1, 0, h);
    else hipLaunchKernelGGL(gemm_planes_kernel<0>, grid, dim3(PNT), 0, st, h);
    TRG_HIP_CHECK(hipGetLastError());
}

}  // namespace trg
