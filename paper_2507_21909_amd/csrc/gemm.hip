// Batched GEMM over arbitrarily strided operands on the gfx950 matrix cores.
//
// Every contraction of the RG step (Sec. II A-B) is evaluated as a GEMM over
// reshaped tensor legs; the strides let one kernel read operands in the
// layout the previous step left them in (row- or column-major, batched).
//
// FP64 path: v_mfma_f64_16x16x4_f64.  A 256-thread workgroup owns a 64x64
// tile of C; its four wavefronts own 32x32 quadrants (2x2 MFMA tiles).  K is
// staged through LDS in slabs of 16, K-major, and the next slab is fetched
// into registers while the current one is multiplied.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>

#include <hip/hip_ext.h>

#include "common.h"

#ifndef VEC_KB
#define VEC_KB 32
#endif

namespace trg {

typedef double d4 __attribute__((ext_vector_type(4)));

namespace {
constexpr int BM = 64, BN = 64, BK = 16, NT = 256, LP = 4;  // LP: LDS row padding

// operand pointers of batch entry blockIdx.z (two-level when g.inner > 1)
__device__ inline void batch_ptrs(const GemmArgs &g, const double *&A, const double *&B, double *&C) {
    const int bz = blockIdx.z;
    const int bo = g.inner > 1 ? bz / g.inner : bz, bi = g.inner > 1 ? bz % g.inner : 0;
    A = g.A + (long)bo * g.sAb + (long)bi * g.sAi;
    B = g.B + (long)bo * g.sBb + (long)bi * g.sBi;
    C = g.C + (long)bo * g.sCb + (long)bi * g.sCi;
}


// TAG only names the instance: 1 for the timed coarse-graining contractions
// (makeMG / makeMH), so a kernel trace separates them from the other GEMMs.
// KB: K slab staged per barrier pair (32 measured slower than 16 on the
// coarse-graining shapes: occupancy falls from 4 to 3 wavefronts per SIMD).
// TM: tile edge (64 or 128); each wavefront owns a (TM/2)^2 quadrant of
// (TM/32)^2 MFMA tiles.  128 doubles the flops per byte staged (16 flop/B).
// Tile order: workgroups go to the 8 XCDs round-robin by linear id, so the id
// is first remapped to give each XCD a contiguous eighth of the tiles, which
// it then walks in groups of GM tile rows (column by column inside a group):
// the group's A panels and the current B panel stay in that XCD's L2.
constexpr int GM = 8;

// x / d and x % d, by shift and mask when d is a power of two (d > 0)
__device__ inline void divmod(int x, int d, int &q, int &r) {
    if ((d & (d - 1)) == 0) {
        const int sh = __ffs(d) - 1;
        q = x >> sh;
        r = x & (d - 1);
    } else {
        q = x / d;
        r = x - q * d;
    }
}

// element (r, c) of C relative to the batch entry's base
__device__ inline long c_off(const GemmArgs &g, int r, int c) {
    long ro = (long)r * g.sCr, co = (long)c * g.sCn;
    if (g.cR2 > 0) {
        int q, m;
        divmod(r, g.cR2, q, m);
        ro = (long)q * g.sCr + (long)m * g.sCr2;
    }
    if (g.cN2 > 0) {
        int q, m;
        divmod(c, g.cN2, q, m);
        co = (long)q * g.sCn + (long)m * g.sCn2;
    }
    return ro + co;
}

__device__ inline void tile_of(int &mt, int &nt, int gm) {
    const int G = gm > 0 ? gm : GM;
    const int nx = gridDim.x, ny = gridDim.y, T = nx * ny;
    const int h = blockIdx.y * nx + blockIdx.x;
    const int L = (T % 8 == 0) ? (h % 8) * (T / 8) + h / 8 : h;
    const int in_group = G * nx, first = (L / in_group) * G;
    const int gs = min(ny - first, G);
    mt = first + (L % in_group) % gs;
    nt = (L % in_group) / gs;
}

template <int TAG, int TM, int KB = 16>
__global__ __launch_bounds__(NT) void gemm_f64_kernel(GemmArgs g) {
    constexpr int NI = TM / 32;            // MFMA tiles per wave and dimension
    constexpr int EPT = TM * KB / NT;      // elements per thread per operand and K tile
    constexpr int TPR = KB / EPT;          // threads per row (k-fast loads)
    const double *A, *B;
    double *C;
    batch_ptrs(g, A, B, C);
    int mt, nt;
    tile_of(mt, nt, g.gm);
    const int m0 = mt * TM, n0 = nt * TM;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wr = w >> 1, wc = w & 1;

    __shared__ double As[KB][TM + LP];
    __shared__ double Bs[KB][TM + LP];

    // loader mapping (EPT elements per thread per operand)
    const bool a_kfast = (g.sAk == 1) || (g.sAr != 1);
    const bool b_nfast = (g.sBn == 1) || (g.sBk != 1);
    int ar, ak, br, bk;  // base row/k of this thread's A elements, k/col of B
    if (a_kfast) { ar = t / TPR; ak = (t % TPR) * EPT; } else { ak = t / (TM / EPT); ar = (t % (TM / EPT)) * EPT; }
    if (b_nfast) { bk = t / (TM / EPT); br = (t % (TM / EPT)) * EPT; } else { br = t / TPR; bk = (t % TPR) * EPT; }

    double ra[EPT], rb[EPT];
    auto load = [&](int k0) {
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            int r = m0 + (a_kfast ? ar : ar + i), k = k0 + (a_kfast ? ak + i : ak);
            ra[i] = (r < g.M && k < g.K) ? A[(long)r * g.sAr + (long)k * g.sAk] : 0.0;
            int c = n0 + (b_nfast ? br + i : br), kb = k0 + (b_nfast ? bk : bk + i);
            rb[i] = (c < g.N && kb < g.K) ? B[(long)kb * g.sBk + (long)c * g.sBn] : 0.0;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
            if (a_kfast) As[ak + i][ar] = ra[i]; else As[ak][ar + i] = ra[i];
            if (b_nfast) Bs[bk][br + i] = rb[i]; else Bs[bk + i][br] = rb[i];
        }
    };

    d4 acc[NI][NI];
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int j = 0; j < NI; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

    const int nk = (g.K + KB - 1) / KB;
    load(0);
    store();
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        if (kt + 1 < nk) load((kt + 1) * KB);
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int kk = 0; kk < KB; kk += 4) {
            const int kr = kk + (lane >> 4);
            double af[NI], bf[NI];
#pragma unroll
            for (int i = 0; i < NI; ++i) af[i] = As[kr][wr * (TM / 2) + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < NI; ++j) bf[j] = Bs[kr][wc * (TM / 2) + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < NI; ++i)
#pragma unroll
                for (int j = 0; j < NI; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
        }
        __builtin_amdgcn_s_setprio(0);
        __syncthreads();
        if (kt + 1 < nk) {
            store();
            __syncthreads();
        }
    }
    // epilogue: item e of lane l holds D[l/16 + 4e][l%16] of each 16x16 tile
    // (the f64 16x16x4 output layout, checked against a host GEMM)
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int j = 0; j < NI; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                int r = m0 + wr * (TM / 2) + i * 16 + (lane >> 4) + 4 * e;
                int c = n0 + wc * (TM / 2) + j * 16 + (lane & 15);
                if (r < g.M && c < g.N) {
                    double *p = C + c_off(g, r, c);
                    double v = g.alpha * acc[i][j][e];
                    if (g.beta != 0.0) v += g.beta * *p;
                    *p = v;
                }
            }
}

// The same 64 x 64 tile as gemm_f64_kernel with a K slab of KB (32 measured
// 1.6 % faster than 16 on the makeMG/makeMH shapes), for launches whose tiles
// all lie inside C (M, N multiples of 64, K of KB) and whose operands have a
// unit stride along one index with 16-byte aligned rows: each thread fetches
// its KB / 4 elements per operand and slab as 16-byte loads from a pointer
// that advances by one slab, with no per-element index arithmetic or bounds
// checks.  AK1: A is k-contiguous (sAk = 1), else m-contiguous (sAr = 1);
// BN1: B is n-contiguous (sBn = 1), else k-contiguous (sBk = 1).
template <int TAG, bool AK1, bool BN1, int KB = 16>
__global__ __launch_bounds__(NT) void gemm_f64_vec_kernel(GemmArgs g) {
    constexpr int TM = 64;
    constexpr int KQ = KB / 16;   // k rows per thread along a 64-contiguous operand
    constexpr int KV = KB / 8;    // 16-byte loads per thread along a k-contiguous operand
    const double *A, *B;
    double *C;
    batch_ptrs(g, A, B, C);
    int mt, nt;
    tile_of(mt, nt, g.gm);
    const int m0 = mt * TM, n0 = nt * TM;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wr = w >> 1, wc = w & 1;
    __shared__ double As[KB][TM + LP];
    __shared__ double Bs[KB][TM + LP];
    // A: AK1 -> row t/4, k (t%4)*(KB/4) .. +KB/4-1; else k t/16 + 16q, rows (t%16)*4 .. +3
    const int ar = AK1 ? t / 4 : (t % 16) * 4, ak = AK1 ? (t % 4) * (KB / 4) : t / 16;
    // B: BN1 -> k t/16 + 16q, cols (t%16)*4 .. +3; else col t/4, k (t%4)*(KB/4) .. +KB/4-1
    const int bc = BN1 ? (t % 16) * 4 : t / 4, bk = BN1 ? t / 16 : (t % 4) * (KB / 4);
    const double *pa = A + (long)(m0 + ar) * g.sAr + (long)ak * g.sAk;
    const double *pb = B + (long)bk * g.sBk + (long)(n0 + bc) * g.sBn;
    const long da = (long)KB * g.sAk, db = (long)KB * g.sBk;   // one slab on
    const long qa = 16 * g.sAk, qb = 16 * g.sBk;               // 16 k rows on
    typedef double d2 __attribute__((ext_vector_type(2)));
    d2 ra[KB / 8], rb[KB / 8];
    auto load = [&]() {
        if (AK1) {
#pragma unroll
            for (int v = 0; v < KV; ++v) ra[v] = *reinterpret_cast<const d2 *>(pa + 2 * v);
        } else {
#pragma unroll
            for (int q = 0; q < KQ; ++q) {
                ra[2 * q] = *reinterpret_cast<const d2 *>(pa + q * qa);
                ra[2 * q + 1] = *reinterpret_cast<const d2 *>(pa + q * qa + 2);
            }
        }
        if (BN1) {
#pragma unroll
            for (int q = 0; q < KQ; ++q) {
                rb[2 * q] = *reinterpret_cast<const d2 *>(pb + q * qb);
                rb[2 * q + 1] = *reinterpret_cast<const d2 *>(pb + q * qb + 2);
            }
        } else {
#pragma unroll
            for (int v = 0; v < KV; ++v) rb[v] = *reinterpret_cast<const d2 *>(pb + 2 * v);
        }
        pa += da;
        pb += db;
    };
    auto store = [&]() {
#pragma unroll
        for (int i = 0; i < KB / 4; ++i) {
            const double x = ra[i / 2][i % 2], y = rb[i / 2][i % 2];
            if (AK1) As[ak + i][ar] = x;
            else As[ak + 16 * (i / 4)][ar + i % 4] = x;
            if (BN1) Bs[bk + 16 * (i / 4)][bc + i % 4] = y;
            else Bs[bk + i][bc] = y;
        }
    };
    d4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    const int nk = g.K / KB;
    load();
    store();
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        if (kt + 1 < nk) load();
        // raised wave priority while issuing the slab's MFMAs (measured +5 %
        // on the makeMG/makeMH shapes): the other waves' loads and LDS stores
        // fill in around them
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int kk = 0; kk < KB; kk += 4) {
            const int kr = kk + (lane >> 4);
            double af[2], bf[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) af[i] = As[kr][wr * 32 + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 2; ++j) bf[j] = Bs[kr][wc * 32 + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
        }
        __builtin_amdgcn_s_setprio(0);
        __syncthreads();
        if (kt + 1 < nk) {
            store();
            __syncthreads();
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int r = m0 + wr * 32 + i * 16 + (lane >> 4) + 4 * e;
                const int c = n0 + wc * 32 + j * 16 + (lane & 15);
                double *p = C + c_off(g, r, c);
                double v = g.alpha * acc[i][j][e];
                if (g.beta != 0.0) v += g.beta * *p;
                *p = v;
            }
}

// the vector kernel's preconditions; *ak1, *bn1 name its layout variant
constexpr int VKB = VEC_KB;   // K slab of the vector kernel

bool vec_ok(const GemmArgs &g, bool *ak1, bool *bn1) {
    if (g.M % 64 || g.N % 64 || g.K % VKB || g.K == 0) return false;
    auto even = [](long x) { return (x & 1) == 0; };
    auto al16 = [](const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
    if (!al16(g.A) || !al16(g.B)) return false;
    if (!even(g.sAb) || !even(g.sBb) || (g.inner > 1 && (!even(g.sAi) || !even(g.sBi)))) return false;
    if (g.sAk == 1 && even(g.sAr)) *ak1 = true;
    else if (g.sAr == 1 && even(g.sAk)) *ak1 = false;
    else return false;
    if (g.sBn == 1 && even(g.sBk)) *bn1 = true;
    else if (g.sBk == 1 && even(g.sBn)) *bn1 = false;
    else return false;
    return true;
}

template <int TAG>
void launch_vec(bool ak1, bool bn1, dim3 grid, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1, const GemmArgs &h) {
    auto kern = ak1 ? (bn1 ? gemm_f64_vec_kernel<TAG, true, true, VKB> : gemm_f64_vec_kernel<TAG, true, false, VKB>)
                    : (bn1 ? gemm_f64_vec_kernel<TAG, false, true, VKB> : gemm_f64_vec_kernel<TAG, false, false, VKB>);
    if (ev0) hipExtLaunchKernelGGL(kern, grid, dim3(NT), 0, st, ev0, ev1, 0, h);
    else hipLaunchKernelGGL(kern, grid, dim3(NT), 0, st, h);
}
std::mutex tune_mu;
std::map<std::array<long, 8>, int> tune_cache;

int env_int(const char *name, int dflt) {
    const char *e = getenv(name);
    return e && *e ? atoi(e) : dflt;
}
}  // namespace

int tuned_gm(const std::array<long, 8> &key, hipStream_t st, bool eligible, const std::function<void(int)> &launch) {
    static const int forced = env_int("TRG_GEMM_GM", 0);
    static const bool on = env_int("TRG_AUTOTUNE", 1) != 0;
    static const bool trace = env_int("TRG_GEMM_TRACE", 0) != 0;
    if (forced > 0) return forced;
    {
        std::lock_guard<std::mutex> lk(tune_mu);
        auto it = tune_cache.find(key);
        if (it != tune_cache.end()) return it->second;
    }
    if (!on || !eligible) return 0;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    TRG_HIP_CHECK(hipStreamIsCapturing(st, &cs));
    if (cs != hipStreamCaptureStatusNone) return 0;
    const int cand[3] = {4, 8, 16};
    hipEvent_t ev[4];
    for (auto &e : ev) TRG_HIP_CHECK(hipEventCreate(&e));
    TRG_HIP_CHECK(hipEventRecord(ev[0], st));
    for (int i = 0; i < 3; ++i) {
        launch(cand[i]);
        TRG_HIP_CHECK(hipEventRecord(ev[i + 1], st));
    }
    TRG_HIP_CHECK(hipEventSynchronize(ev[3]));
    int best = 0;
    float best_ms = 0.0f;
    for (int i = 0; i < 3; ++i) {
        float ms = 0.0f;
        TRG_HIP_CHECK(hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
        if (i == 0 || ms < best_ms) {
            best_ms = ms;
            best = cand[i];
        }
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    if (trace)
        fprintf(stderr, "[tune] kind %ld M %ld N %ld K %ld batch %ld inner %ld: group %d (%.3f ms)\n", key[0], key[1],
                key[2], key[3], key[4], key[5], best, best_ms);
    std::lock_guard<std::mutex> lk(tune_mu);
    tune_cache[key] = best;
    return best;
}

void gemm_f64(const GemmArgs &g, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
    if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return;
    // a ragged last column tile keeps the whole launch off the vector kernel:
    // the 64-aligned columns go to it and the rest to the general kernel (each
    // element of C sums its K terms in the same MFMA order in both, so the
    // split changes no bits)
    if (!ev0 && g.N > 64 && g.N % 64 != 0 && g.cN2 == 0) {
        GemmArgs h = g;
        h.N = g.N - g.N % 64;
        bool ak1 = false, bn1 = false;
        if (vec_ok(h, &ak1, &bn1)) {
            gemm_f64(h, st, nullptr, nullptr);
            GemmArgs r = g;
            r.N = g.N % 64;
            r.B = g.B + (long)h.N * g.sBn;
            r.C = g.C + (long)h.N * g.sCn;
            gemm_f64(r, st, nullptr, nullptr);
            return;
        }
    }
    const int inner = std::max(1, g.inner);
    // shapes of every launch on stderr when TRG_GEMM_TRACE is set
    static const bool trace = [] {
        const char *e = getenv("TRG_GEMM_TRACE");
        return e && *e && *e != '0';
    }();
    if (trace)
        fprintf(stderr, "[gemm] M %d N %d K %ld batch %d inner %d sA %ld,%ld sB %ld,%ld sC %ld,%ld beta %g\n", g.M,
                g.N, (long)g.K, g.batch, inner, g.sAr, g.sAk, g.sBk, g.sBn, g.sCr, g.sCn, g.beta);
    TRG_REQUIRE(inner == 1 || (long)g.batch * inner <= 65535, -6, "gemm: two-level batch too large");
    for (int b0 = 0; b0 < g.batch; b0 += 65535 / inner) {
        GemmArgs h = g;
        h.batch = std::min(65535 / inner, g.batch - b0);
        h.A += (long)b0 * g.sAb;
        h.B += (long)b0 * g.sBb;
        h.C += (long)b0 * g.sCb;
        // 128-edge tiles measured slower than 64 on the coarse-graining shapes
        // (one wavefront per SIMD at 218 VGPRs); kept selectable for tuning
        constexpr bool kBigTiles = false;
        const bool big = kBigTiles && h.M >= 256 && h.N >= 256 &&
                         (long)cdiv(h.N, 128) * cdiv(h.M, 128) * h.batch >= 256;
        const int tm = big ? 128 : 64;
        dim3 grid(cdiv(h.N, tm), cdiv(h.M, tm), h.batch * inner);
        bool ak1 = false, bn1 = false;
        if (!big && vec_ok(h, &ak1, &bn1)) {
            if (h.gm == 0) {
                const double fl = 2.0 * h.M * (double)h.N * (double)h.K * h.batch;
                const std::array<long, 8> key{(long)(ak1 ? 2 : 0) + (bn1 ? 1 : 0), h.M, h.N, (long)h.K, h.batch, inner,
                                              h.cR2 > 0 || h.cN2 > 0, 0};
                h.gm = tuned_gm(key, st, h.beta == 0.0 && fl >= 2e10, [&](int gm) {
                    GemmArgs x = h;
                    x.gm = gm;
                    launch_vec<0>(ak1, bn1, grid, st, nullptr, nullptr, x);
                });
            }
            if (ev0 && (long)g.batch * inner <= 65535) launch_vec<1>(ak1, bn1, grid, st, ev0, ev1, h);
            else launch_vec<0>(ak1, bn1, grid, st, nullptr, nullptr, h);
            continue;
        }
        if (ev0 && (long)g.batch * inner <= 65535) {   // kernel start / end timestamps
            if (big) hipExtLaunchKernelGGL(gemm_f64_kernel<1, 128>, grid, dim3(NT), 0, st, ev0, ev1, 0, h);
            else hipExtLaunchKernelGGL(gemm_f64_kernel<1, 64>, grid, dim3(NT), 0, st, ev0, ev1, 0, h);
        } else {
            auto kern = big ? gemm_f64_kernel<0, 128> : gemm_f64_kernel<0, 64>;
            hipLaunchKernelGGL(kern, grid, dim3(NT), 0, st, h);
        }
    }
    TRG_HIP_CHECK(hipGetLastError());
}

}  // namespace trg

// ---------------------------------------------------------------------------
// Mixed-precision paths for the coarse-graining contractions.
//
// FP32: operands rounded to FP32, v_mfma_f32_16x16x4_f32.
// BF16xN: each operand x (rounded to FP32) is split by round-to-nearest into
// x = x0 + x1 + x2 with x0 = bf16(x), x1 = bf16(x - x0), x2 = bf16(x - x0 - x1);
// the product sums the split products x_i y_j with i + j <= 1 (N = 3 products)
// or i + j <= 2 (N = 6), each on v_mfma_f32_16x16x32_bf16.
// In both paths the FP32 MFMA accumulators are added into FP64 registers after
// every K tile, so FP32 rounding stays within partial sums of 16 (FP32) or 32
// (BF16) terms however long the contraction.
namespace trg {
namespace {
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int FLUSH_K = 16;   // FP32 partial sums span one K tile at most

// FP32 path: same tiling as the FP64 kernel (BK 16), LDS in FP32
__global__ __launch_bounds__(NT) void gemm_f32_kernel(GemmArgs g) {
    const double *A, *B;
    double *C;
    batch_ptrs(g, A, B, C);
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wr = w >> 1, wc = w & 1;
    __shared__ float As[BK][BM + LP];
    __shared__ float Bs[BK][BN + LP];
    const bool a_kfast = (g.sAk == 1) || (g.sAr != 1);
    const bool b_nfast = (g.sBn == 1) || (g.sBk != 1);
    int ar, ak, br, bk;
    if (a_kfast) { ar = t >> 2; ak = (t & 3) * 4; } else { ak = t >> 4; ar = (t & 15) * 4; }
    if (b_nfast) { bk = t >> 4; br = (t & 15) * 4; } else { br = t >> 2; bk = (t & 3) * 4; }
    float ra[4], rb[4];
    auto load = [&](int k0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            int r = m0 + (a_kfast ? ar : ar + i), k = k0 + (a_kfast ? ak + i : ak);
            ra[i] = (r < g.M && k < g.K) ? (float)A[(long)r * g.sAr + (long)k * g.sAk] : 0.0f;
            int c = n0 + (b_nfast ? br + i : br), kb = k0 + (b_nfast ? bk : bk + i);
            rb[i] = (c < g.N && kb < g.K) ? (float)B[(long)kb * g.sBk + (long)c * g.sBn] : 0.0f;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (a_kfast) As[ak + i][ar] = ra[i]; else As[ak][ar + i] = ra[i];
            if (b_nfast) Bs[bk][br + i] = rb[i]; else Bs[bk + i][br] = rb[i];
        }
    };
    f4 acc[2][2];
    d4 dacc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) { acc[i][j] = f4{0, 0, 0, 0}; dacc[i][j] = d4{0, 0, 0, 0}; }
    const int nk = (g.K + BK - 1) / BK;
    load(0);
    store();
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        if (kt + 1 < nk) load((kt + 1) * BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            const int kr = kk + (lane >> 4);
            float af[2], bf[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) af[i] = As[kr][wr * 32 + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 2; ++j) bf[j] = Bs[kr][wc * 32 + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bf[j], acc[i][j], 0, 0, 0);
        }
        if (((kt + 1) * BK) % FLUSH_K == 0 || kt + 1 == nk) {
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
#pragma unroll
                    for (int e = 0; e < 4; ++e) { dacc[i][j][e] += (double)acc[i][j][e]; acc[i][j][e] = 0.0f; }
        }
        __syncthreads();
        if (kt + 1 < nk) {
            store();
            __syncthreads();
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                int r = m0 + wr * 32 + i * 16 + 4 * (lane >> 4) + e;
                int c = n0 + wc * 32 + j * 16 + (lane & 15);
                if (r < g.M && c < g.N) {
                    double *p = C + c_off(g, r, c);
                    double v = g.alpha * dacc[i][j][e];
                    if (g.beta != 0.0) v += g.beta * *p;
                    *p = v;
                }
            }
}

// BF16 split path: BK 32; LDS tiles row-major with k contiguous (8 bf16 per lane per MFMA)
constexpr int BKB = 32, KP = 8;   // KP: padding in bf16 elements

template <int NSPLIT, int NPROD>
__global__ __launch_bounds__(NT) void gemm_bf16_kernel(GemmArgs g) {
    const double *A, *B;
    double *C;
    batch_ptrs(g, A, B, C);
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int wr = w >> 1, wc = w & 1;
    __shared__ __bf16 As[NSPLIT][BM][BKB + KP];
    __shared__ __bf16 Bs[NSPLIT][BN][BKB + KP];
    // 64 x 32 tile = 2048 elements: 8 per thread
    const bool a_kfast = (g.sAk == 1) || (g.sAr != 1);
    const bool b_kfast = (g.sBk == 1) || (g.sBn != 1);
    int ar, ak, br, bk;
    if (a_kfast) { ar = t >> 2; ak = (t & 3) * 8; } else { ak = t >> 3; ar = (t & 7) * 8; }
    if (b_kfast) { br = t >> 2; bk = (t & 3) * 8; } else { bk = t >> 3; br = (t & 7) * 8; }
    float ra[8], rb[8];
    auto load = [&](int k0) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            int r = m0 + (a_kfast ? ar : ar + i), k = k0 + (a_kfast ? ak + i : ak);
            ra[i] = (r < g.M && k < g.K) ? (float)A[(long)r * g.sAr + (long)k * g.sAk] : 0.0f;
            int c = n0 + (b_kfast ? br : br + i), kb = k0 + (b_kfast ? bk + i : bk);
            rb[i] = (c < g.N && kb < g.K) ? (float)B[(long)kb * g.sBk + (long)c * g.sBn] : 0.0f;
        }
    };
    auto split_store = [&](float x, __bf16 *dst0, long plane) {
        __bf16 x0 = (__bf16)x;
        float r1 = x - (float)x0;
        __bf16 x1 = (__bf16)r1;
        dst0[0] = x0;
        dst0[plane] = x1;
        if (NSPLIT > 2) {
            float r2 = r1 - (float)x1;
            dst0[2 * plane] = (__bf16)r2;
        }
    };
    auto store = [&]() {
        const long pa = (long)BM * (BKB + KP), pb = (long)BN * (BKB + KP);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            if (a_kfast) split_store(ra[i], &As[0][ar][ak + i], pa);
            else split_store(ra[i], &As[0][ar + i][ak], pa);
            if (b_kfast) split_store(rb[i], &Bs[0][br][bk + i], pb);
            else split_store(rb[i], &Bs[0][br + i][bk], pb);
        }
    };
    f4 acc[2][2];
    d4 dacc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) { acc[i][j] = f4{0, 0, 0, 0}; dacc[i][j] = d4{0, 0, 0, 0}; }
    const int nk = (g.K + BKB - 1) / BKB;
    load(0);
    store();
    __syncthreads();
    const int kq = (lane >> 4) * 8;
    for (int kt = 0; kt < nk; ++kt) {
        if (kt + 1 < nk) load((kt + 1) * BKB);
        bf8 af[NSPLIT][2], bfr[NSPLIT][2];
#pragma unroll
        for (int s = 0; s < NSPLIT; ++s)
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                af[s][i] = *reinterpret_cast<const bf8 *>(&As[s][wr * 32 + i * 16 + (lane & 15)][kq]);
                bfr[s][i] = *reinterpret_cast<const bf8 *>(&Bs[s][wc * 32 + i * 16 + (lane & 15)][kq]);
            }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                // smallest products first
                if (NPROD == 6) {
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[2 % NSPLIT][i], bfr[0][j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][i], bfr[2 % NSPLIT][j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[1][i], bfr[1][j], acc[i][j], 0, 0, 0);
                }
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[1][i], bfr[0][j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][i], bfr[1][j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0][i], bfr[0][j], acc[i][j], 0, 0, 0);
            }
        if (((kt + 1) * BKB) % FLUSH_K == 0 || kt + 1 == nk) {
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
#pragma unroll
                    for (int e = 0; e < 4; ++e) { dacc[i][j][e] += (double)acc[i][j][e]; acc[i][j][e] = 0.0f; }
        }
        __syncthreads();
        if (kt + 1 < nk) {
            store();
            __syncthreads();
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                int r = m0 + wr * 32 + i * 16 + 4 * (lane >> 4) + e;
                int c = n0 + wc * 32 + j * 16 + (lane & 15);
                if (r < g.M && c < g.N) {
                    double *p = C + c_off(g, r, c);
                    double v = g.alpha * dacc[i][j][e];
                    if (g.beta != 0.0) v += g.beta * *p;
                    *p = v;
                }
            }
}

template <typename K>
void launch_batched(K kern, const GemmArgs &g, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
    if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return;
    const int inner = std::max(1, g.inner);
    TRG_REQUIRE(inner == 1 || (long)g.batch * inner <= 65535, -6, "gemm: two-level batch too large");
    for (int b0 = 0; b0 < g.batch; b0 += 65535 / inner) {
        GemmArgs h = g;
        h.batch = std::min(65535 / inner, g.batch - b0);
        h.A += (long)b0 * g.sAb;
        h.B += (long)b0 * g.sBb;
        h.C += (long)b0 * g.sCb;
        dim3 grid(cdiv(h.N, BN), cdiv(h.M, BM), h.batch * inner);
        if (ev0 && (long)g.batch * inner <= 65535)
            hipExtLaunchKernelGGL(kern, grid, dim3(NT), 0, st, ev0, ev1, 0, h);
        else
            hipLaunchKernelGGL(kern, grid, dim3(NT), 0, st, h);
    }
    TRG_HIP_CHECK(hipGetLastError());
}
}  // namespace

void gemm_mixed(const GemmArgs &g, int mode, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
    switch (mode) {
        case 1: launch_batched(gemm_f32_kernel, g, st, ev0, ev1); break;
        case 2: launch_batched(gemm_bf16_kernel<2, 3>, g, st, ev0, ev1); break;
        case 3: launch_batched(gemm_bf16_kernel<3, 6>, g, st, ev0, ev1); break;
        default: gemm_f64(g, st, ev0, ev1);
    }
}

}  // namespace trg
