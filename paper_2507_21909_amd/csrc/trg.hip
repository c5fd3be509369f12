// The RG step of ATRG and triad-ATRG on one GPU, behind the C ABI of trg.h.
//
// Step along axis a, transverse axes (t1, t2, t3) = (a+1, a+2, a+3) mod 4:
//  1. re-split T = Phi Psi^T exactly (Fig. 5f): TSQR of Phi and Psi, Jacobi SVD
//     of R_Phi R_Psi^T, norm c_k into the log-norm accumulator;
//  2. bond swap (App. A): randomized SVD applying M = sum_x B C directly to the
//     sketch (no QR of B and C), or the exact SVD of the QR-reduced core;
//  3a. ATRG (Sec. II A): squeezers from canonical Gamma^ATRG, makeG / makeH;
//  3b. triad-ATRG (Sec. II B): triad isometries (eq. HOSVD), E..L, Gram
//     matrices O and P (Sec. II D), squeezers from Gamma^Triad, makeMG / makeMH.
// Every truncation keeps at most its cap, drops values at or below the
// relative threshold and never cuts a multiplet (kept_count); kept vectors
// get the sign convention of the weight w(multi-index).
#include <array>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "engine.h"

struct trg_state {
    trg_options opt;
    hipStream_t st = nullptr;
    trg::Arena ar;
    bool init = false;
    int D = 0, k = 0, chi = 0;
    double beta = 0.0, h = 0.0;
    std::vector<int> dims;
    double *phi = nullptr, *psi = nullptr;   // persistent state
    // impurity tangents (dPhi, dPsi) of d/dbeta and d/dh, when opt.tangents asks for them
    int ntan = 0, tan_kind[2] = {0, 0};
    double *dphi[2] = {nullptr, nullptr}, *dpsi[2] = {nullptr, nullptr};
    size_t cap_tan = 0;
    size_t cap_state = 0;
    double *dscal = nullptr;   // [0] logacc, [1] trace, [3] logacc before the step, [4..6) Gu-Wen traces,
                               // [6] norm c_k of the last re-split, [8..11) impurity traces,
                               // [1024..2048) trace partials
    int *dint = nullptr;       // [0] numerical status, [1] status before the step, [2] step index k,
                               // [8..] kept counts
    std::vector<double> sigma_last;    // bond-swap singular values of the last step
    std::vector<double> resplit_last;  // re-split singular values / c_k of the last step
    // the same two spectra on the device ([0, 1024) sigma, [1024, 2048) re-split,
    // [2048, 4096) their values before the step); after a graph launch the host
    // copies are refreshed from here on demand
    double *dspec = nullptr;
    // a recorded step's copy of the state it starts from (phi, psi, then the
    // tangents' pairs; cap_state each), for the rollback of a checked replay
    double *bak = nullptr;
    size_t bak_cap = 0;
    bool spec_stale = false;
    size_t nsig = 0, nrsv = 0;
    // graph capture: most sweeps an eager step's iterative solve took, keyed by
    // (call order in the step, batch count, m, n); capture_on while a step is recorded
    std::map<std::array<int, 4>, int> sweep_log;
    bool capture_on = false;
    unsigned long gen = 0;   // bumped when device buffers a graph may hold are replaced
    std::string err;
    bool timing = false;
    double t_ms = 0.0, t_flops = 0.0;
    int t_launch = 0;
};

namespace trg {
namespace {

constexpr double EPS_S = 1e-14, EPS_LAM = 1e-14, EPS_SQ = 1e-14, TAU_DEG_DEFAULT = 1e-9;
// pivoted Cholesky of a Gram stops at pivots at the rounding level of its largest
// entry (the Gram itself is only known to about that)
constexpr double PCHOL_TOL = 2.220446049250313e-16;

// ---------------------------------------------------------------- small kernels
// kp: the step index k (device)
__global__ void resplit_norm_kernel(double *s, int n, const int *kp, double *logacc, double eps, int *status,
                                    double *cout) {
    if (threadIdx.x || blockIdx.x) return;
    const int k = *kp;
    double c = s[0];
    if (!(c > 0.0) || !isfinite(c)) {
        *status = 1;
        c = 1.0;
    }
    *cout = c;
    *logacc += ldexp(log(c), -k);
    for (int i = 0; i < n; ++i) {
        double v = s[i] / c;
        s[i] = v > eps ? v : 0.0;
    }
}

// S' = R^T diag(s) R (n x n)
__global__ void sprime_kernel(const double *rot, const double *s, int n, double *sp) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * n) return;
    int r = i / n, c = i % n;
    double acc = 0.0;
    for (int k = 0; k < n; ++k) acc += rot[(long)k * n + r] * s[k] * rot[(long)k * n + c];
    sp[i] = acc;
}

// S'^+ = R^T diag(s^+) R with s^+ = 1/s on the kept values, 0 elsewhere
__global__ void sprime_inv_kernel(const double *rot, const double *s, int n, double *sp) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * n) return;
    int r = i / n, c = i % n;
    double acc = 0.0;
    for (int k = 0; k < n; ++k) {
        const double si = s[k] > 0.0 ? 1.0 / s[k] : 0.0;
        acc += rot[(long)k * n + r] * si * rot[(long)k * n + c];
    }
    sp[i] = acc;
}

// y = (y + a x) * scale, scale = 1 / *cinv_of when cinv_of is given
__global__ void axpy_scale_kernel(double *y, const double *x, long n, double a, const double *cinv_of) {
    const double sc = cinv_of ? 1.0 / *cinv_of : 1.0;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        y[i] = (y[i] + (x ? a * x[i] : 0.0)) * sc;
}

// out[j] = 1 / v[j] for v[j] > 0, else 0
__global__ void inv_pos_kernel(const double *v, double *out, int n) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) out[j] = v[j] > 0.0 ? 1.0 / v[j] : 0.0;
}

// out[j] = sqrt(lam[j]) if lam[j] > eps * lam[0] else 0
__global__ void sqrt_clamp_kernel(const double *lam, double *out, int n, double eps) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double top = lam[0] > 0.0 ? lam[0] : 0.0;
    double v = lam[j];
    out[j] = v > eps * top ? sqrt(v) : 0.0;
}

// out[j] = j < kept ? S[j]^-1/2 : 0
__global__ void isqrt_kept_kernel(const double *s, double *out, int n, const int *kept) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    out[j] = j < *kept ? 1.0 / sqrt(s[j]) : 0.0;
}

__global__ void zero_tail_vec_kernel(double *v, int n, const int *kept) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n && j >= *kept) v[j] = 0.0;
}

__global__ void square_kernel(const double *v, double *o, int n) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) o[j] = v[j] * v[j];
}

__global__ void eye_kernel(double *a, int n) {
    long tot = (long)n * n;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < tot; i += (long)gridDim.x * blockDim.x)
        a[i] = (i / n == i % n) ? 1.0 : 0.0;
}

// partial dot products of two vectors, then a final single-block sum
__global__ void dot_partial_kernel(const double *a, const double *b, long n, double *part) {
    double acc = 0.0;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        acc += a[i] * b[i];
    __shared__ double red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void sum_kernel(const double *part, int n, double *out) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) acc += part[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// Gu-Wen traces of A (n x n, row-major): out[0] = Tr A, out[1] = Tr(A A) =
// sum_{k,l} A[k,l] A[l,k]; one workgroup, fixed summation order
__global__ void gu_wen_kernel(const double *a, int n, double *out) {
    __shared__ double r1[256], r2[256];
    double t1 = 0.0, t2 = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) t1 += a[(long)i * n + i];
    for (long e = threadIdx.x; e < (long)n * n; e += 256) {
        const long k = e / n, l = e % n;
        t2 += a[e] * a[l * n + k];
    }
    r1[threadIdx.x] = t1;
    r2[threadIdx.x] = t2;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            r1[threadIdx.x] += r1[threadIdx.x + s];
            r2[threadIdx.x] += r2[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = r1[0];
        out[1] = r2[0];
    }
}

inline unsigned g1(long n) { return (unsigned)std::max(1L, std::min((n + 255) / 256, 65536L)); }

// ---------------------------------------------------------------- helpers
struct Step {
    trg_state *S;
    Ctx c;
    int *kept;   // next free device int for a kept count
    double *scr; // device scalar scratch
    Step(trg_state *s) : S(s) {
        c.st = s->st;
        c.ar = &s->ar;
        c.prec = (Prec)s->opt.precision;
        c.timing = s->timing && !s->capture_on;
        c.capture = s->capture_on;
        c.dstatus = s->dint;
        c.sweep_log = &s->sweep_log;
        kept = s->dint + 8;
    }
    int *new_kept() { return kept++; }
};

std::vector<double> pow131(int nd) {
    std::vector<double> p(nd);
    double m = 1.0;
    for (int i = 0; i < nd; ++i) { p[i] = m; m *= 131.0; }
    return p;
}

// dst (rows x k) = first k columns of src (rows x cols), both row-major
void col_slice(Ctx &c, const double *src, long rows, long cols, int k, double *dst) {
    TRG_HIP_CHECK(hipMemcpy2DAsync(dst, sizeof(double) * k, src, sizeof(double) * cols, sizeof(double) * k, rows,
                                   hipMemcpyDeviceToDevice, c.st));
}

// One-sided Jacobi under the step's convergence policy.  Eager: the host reads
// every sweep's rotation count and the sweeps used are logged for the solve
// (its call order in the step and its shape).  Captured: nothing is read back;
// the panel solver (more than 96 columns) runs
// device-driven up to twice the most sweeps logged for the same solve, plus 8
// (status 3 if that is not enough: a squeezer solve can take 10 sweeps in one
// step and 40 a few steps later), the one-launch solver up to max_sweeps as
// eagerly.
int run_jacobi(Ctx &c, const JacobiBatch &jb, int ms, int *flags, double *work) {
    const std::array<int, 4> key{c.solve_idx++, jb.count, jb.m, jb.n};
    if (!c.capture) {
        const int sw = jacobi_svd(jb, ms, flags, work, c.st);
        if (c.sweep_log) {
            int &v = (*c.sweep_log)[key];
            v = std::max(v, sw + 1);
        }
        return sw;
    }
    int cap = ms;
    if (!jacobi_one_launch(jb)) {
        auto it = c.sweep_log ? c.sweep_log->find(key) : std::map<std::array<int, 4>, int>::iterator();
        TRG_REQUIRE(c.sweep_log && it != c.sweep_log->end(), TRG_E_STATE,
                    "graph capture: no eager step of this method at these shapes has run on the state");
        cap = std::min(ms, 2 * it->second + 8);
    }
    const char *env = getenv("TRG_GRAPH_SWEEP_CAP");   // test hook: a smaller cap for recorded solves
    const int forced = env && *env ? atoi(env) : 0;
    if (forced > 0 && !jacobi_one_launch(jb)) cap = std::min(cap, forced);
    DevLoop dl{cap, c.dstatus, 3};
    return jacobi_svd(jb, ms, flags, work, c.st, &dl);
}

// SVD of `count` matrices given column-major (a + i*m*n holds n columns of m):
// s (count x n) descending, u (count x m x n) and v (count x n x n) row-major, sorted.
void svd_colmajor(Step &T, const double *a, int count, int m, int n, double *s, double *u, double *v) {
    Ctx &c = T.c;
    double *ut = c.ar->dalloc((size_t)count * m * n);
    copy(ut, a, (size_t)count * m * n, c.st);
    double *vt = v ? c.ar->dalloc((size_t)count * n * n) : nullptr;   // no V wanted: not accumulated
    double *work = c.ar->dalloc((size_t)count * (n + 1));
    int *flags = reinterpret_cast<int *>(c.ar->dalloc((size_t)count + 1));   // 2 * count + 1 ints
    JacobiBatch jb{count, m, n, ut, vt, (long)m * n, (long)n * n};
    int ms = T.S->opt.max_sweeps > 0 ? T.S->opt.max_sweeps : 300;
    run_jacobi(c, jb, ms, flags, work);
    jacobi_finish(jb, s, u, v, work, c.st);
}

// SVD of a row-major matrix a (m x n, m >= n)
void svd_rowmajor(Step &T, const DT &a, double *s, double *u, double *v) {
    int m = a.d[0], n = a.d[1];
    DT at = permuted(T.c, a, "ij", "ji");   // column-major copy
    svd_colmajor(T, at.p, 1, m, n, s, u, v);
}

// eigen-decomposition of symmetric PSD matrices (count x n x n): lam desc, vecs row-major
void eig_psd(Step &T, const double *k, int count, int n, double *lam, double *vec) {
    Ctx &c = T.c;
    double *ws = c.ar->dalloc(eigh_ws_doubles(count, n));
    int *iws = reinterpret_cast<int *>(c.ar->dalloc((eigh_iws_ints(count, n) + 1) / 2));
    int ms = T.S->opt.max_sweeps > 0 ? T.S->opt.max_sweeps : 300;
    eigh_sym(k, count, n, lam, vec, ws, iws, ms, c.st);
}

// Eigen-decomposition of symmetric PSD Grams K = X X^T (count x n x n, n <= 1024)
// through the pivoted Cholesky factor X = P L: K's eigenvectors are X's left
// singular vectors and its eigenvalues X's squared singular values.  X's
// columns come graded (pivot order), and the one-sided solver on them needs
// about half the sweeps of the two-sided solver on K.  Pivots at or below
// PCHOL_TOL of the first end the factor (the rest of the spectrum is then
// zero).  lam desc, vec row-major (columns), as eig_psd.  false (lam, vec
// untouched) if n > 1024 or a pivot is not finite.
bool gram_eig_pchol(Ctx &c, const double *k, int count, int n, int max_sweeps, double *lam, double *vec,
                    int *sweeps) {
    if (n > 1024) return false;
    const size_t nn = (size_t)n * n;
    Arena::Mark mk = c.ar->mark();
    double *kw = c.ar->dalloc(count * nn), *xs = c.ar->dalloc(count * nn);
    copy(kw, k, count * nn, c.st);
    int *piws = reinterpret_cast<int *>(c.ar->dalloc((pchol_iws_ints(count, n) + 1) / 2));
    if (!pivoted_cholesky_batched(kw, count, n, xs, piws, c.st, PCHOL_TOL, nullptr,
                                  c.capture ? c.dstatus : nullptr)) {
        c.ar->release(mk);
        return false;
    }
    // the one-sided solver takes column-major matrices: X^T row-major
    permute(xs, kw, {count, n, n}, {0, 2, 1}, c.st);
    double *work = c.ar->dalloc((size_t)count * (n + 1)), *s = c.ar->dalloc((size_t)count * n);
    int *flags = reinterpret_cast<int *>(c.ar->dalloc((size_t)count + 1));   // 2 * count + 1 ints
    JacobiBatch jb{count, n, n, kw, nullptr, (long)nn, (long)nn};
    const int sw = run_jacobi(c, jb, max_sweeps, flags, work);
    jacobi_finish(jb, s, vec, nullptr, work, c.st);
    hipLaunchKernelGGL(square_kernel, dim3(g1(count * n)), dim3(256), 0, c.st, s, lam, count * n);
    TRG_HIP_CHECK(hipGetLastError());
    if (sweeps) *sweeps = sw;
    c.ar->release(mk);
    return true;
}

// ---------------------------------------------------------------- re-split
struct Split {
    DT A, B, C, Dm;   // step order [a, t1, t2, t3, chi]
    DT s;             // chi
    DT a_nat, dm_nat, rot;   // natural order A, D as F x chi matrices; canonical rotation
};

Split resplit(Step &T, const std::vector<int> &order) {
    trg_state *S = T.S;
    Ctx &c = T.c;
    const int d = (int)S->dims.size();
    long F = 1;
    for (int v : S->dims) F *= v;
    const int chi = S->chi;
    TRG_REQUIRE(chi <= 512, -6, "bond dimension above 512 not supported by the QR");
    TRG_REQUIRE(F >= chi, -6, "re-split: fewer rows than columns");
    DT q1 = talloc(c, {(int)F, chi}), r1 = talloc(c, {chi, chi});
    DT q2 = talloc(c, {(int)F, chi}), r2 = talloc(c, {chi, chi});
    double *ws = c.ar->dalloc(tsqr_ws_doubles(F, chi));
    tsqr(S->phi, F, chi, q1.p, r1.p, ws, c.st);
    tsqr(S->psi, F, chi, q2.p, r2.p, ws, c.st);
    DT w = contract(c, r1, "ia", r2, "ja", "ij");
    DT s = talloc(c, {chi}), u = talloc(c, {chi, chi}), v = talloc(c, {chi, chi});
    svd_rowmajor(T, w, s.p, u.p, v.p);
    hipLaunchKernelGGL(resplit_norm_kernel, dim3(1), dim3(1), 0, c.st, s.p, chi, S->dint + 2, S->dscal, EPS_S,
                       S->dint, S->dscal + 6);
    DT A = contract(c, q1, "Fa", u, "ab", "Fb");
    DT Dm = contract(c, q2, "Fa", v, "ab", "Fb");
    // canonical bond basis: rotation within multiplets of s, B = Dm S', C = A S'
    int *kpos = T.new_kept();
    kept_count(s.p, chi, chi, 0.0, -1.0, kpos, c.st);           // number of s > 0
    std::vector<int> nd(S->dims.begin(), S->dims.end());
    DT rot = talloc(c, {chi, chi});
    double *zw = c.ar->dalloc(weight_ws_doubles(F, chi, CANON_L));
    canonical_rotation(A.p, F, chi, chi, nd, pow131(d), s.p, kpos, T.S->opt.tau_deg, zw, rot.p, S->dint, c.st);
    DT A2 = contract(c, A, "Fa", rot, "ab", "Fb");
    DT D2 = contract(c, Dm, "Fa", rot, "ab", "Fb");
    zero_tail_cols(A2.p, F, chi, chi, kpos, c.st);
    zero_tail_cols(D2.p, F, chi, chi, kpos, c.st);
    DT sp = talloc(c, {chi, chi});
    hipLaunchKernelGGL(sprime_kernel, dim3(g1((long)chi * chi)), dim3(256), 0, c.st, rot.p, s.p, chi, sp.p);
    DT B2 = contract(c, D2, "Fa", sp, "ab", "Fb");
    DT C2 = contract(c, A2, "Fa", sp, "ab", "Fb");
    Split o;
    o.a_nat = A2;
    o.dm_nat = D2;
    o.rot = rot;
    // tensors in step order
    std::string nat, stp;
    for (int i = 0; i < d; ++i) nat += (char)('a' + i);
    for (int i = 0; i < d; ++i) stp += (char)('a' + order[i]);
    nat += 'z';
    stp += 'z';
    std::vector<int> fd = nd;
    fd.push_back(chi);
    A2.d = fd;
    D2.d = fd;
    B2.d = fd;
    C2.d = fd;
    o.A = permuted(c, A2, nat, stp);
    o.Dm = permuted(c, D2, nat, stp);
    o.B = permuted(c, B2, nat, stp);
    o.C = permuted(c, C2, nat, stp);
    o.s = s;
    return o;
}

// ---------------------------------------------------------------- bond swap
struct Swap {
    DT X, Y, sig;   // X [alpha, t1.., g], Y [beta, t1.., g], sig [g]
};

Swap bond_swap(Step &T, const Split &sp) {
    trg_state *S = T.S;
    Ctx &c = T.c;
    const DT &Bt = sp.B, &Ct = sp.C;
    const int nd = (int)Bt.d.size();   // 1 + (d-1) + 1
    const int x = Bt.d[0], chi = Bt.d[nd - 1];
    std::vector<int> td(Bt.d.begin() + 1, Bt.d.end() - 1);
    long J = 1;
    for (int v : td) J *= v;
    const long I = J;
    const long p = std::min(J, (long)x * chi), q = std::min(I, (long)x * chi);
    const long rowsN = chi * q, colsN = chi * p;
    const int gcap = (int)std::min<long>((long)S->opt.r_bond * S->D, std::min(rowsN, colsN));
    const int m = S->opt.sketch_mult * S->D;
    const bool exact = S->opt.bond_svd == TRG_SVD_EXACT || m >= std::min(rowsN, colsN);
    // label strings: x, t legs (i j k / u v w), chi
    const std::string tl = std::string("ijk").substr(0, td.size());
    const std::string tu = std::string("uvw").substr(0, td.size());
    Swap o;
    o.sig = talloc(c, {gcap});
    int *kept = T.new_kept();
    std::vector<int> sdims;   // sign multi-index dims in GPU row order, with their weights
    if (exact) {
        const int nb = x * chi;
        TRG_REQUIRE(nb <= 512 && J >= nb, -6, "exact bond swap: x*chi must be <= 512 and <= prod(transverse)");
        DT Bp = permuted(c, Bt, "x" + tl + "a", tl + "xa");
        DT Cp = permuted(c, Ct, "x" + tl + "b", tl + "xb");
        DT qb = talloc(c, {(int)J, nb}), rb = talloc(c, {nb, nb});
        DT qc = talloc(c, {(int)I, nb}), rc = talloc(c, {nb, nb});
        double *ws = c.ar->dalloc(tsqr_ws_doubles(J, nb));
        tsqr(Bp.p, J, nb, qb.p, rb.p, ws, c.st);
        tsqr(Cp.p, I, nb, qc.p, rc.p, ws, c.st);
        rb.d = {nb, x, chi};
        rc.d = {nb, x, chi};
        DT N = contract(c, rb, "pxa", rc, "qxb", "aqbp");
        N.d = {(int)rowsN, (int)colsN};
        DT s = talloc(c, {(int)colsN}), u = talloc(c, {(int)rowsN, (int)colsN}), v = talloc(c, {(int)colsN, (int)colsN});
        svd_rowmajor(T, N, s.p, u.p, v.p);
        kept_count(s.p, (int)colsN, gcap, EPS_S, T.S->opt.tau_deg, kept, c.st);
        copy(o.sig.p, s.p, gcap, c.st);
        hipLaunchKernelGGL(zero_tail_vec_kernel, dim3(1), dim3(256), 0, c.st, o.sig.p, gcap, kept);
        // U_bond[(alpha, q), g], V_bond[(beta, p), g]: first gcap columns, zero beyond kept
        DT ub = talloc(c, {chi, (int)q, gcap}), vb = talloc(c, {chi, (int)p, gcap});
        col_slice(c, u.p, rowsN, colsN, gcap, ub.p);
        col_slice(c, v.p, colsN, colsN, gcap, vb.p);
        zero_tail_cols(ub.p, rowsN, gcap, gcap, kept, c.st);
        zero_tail_cols(vb.p, colsN, gcap, gcap, kept, c.st);
        DT X = contract(c, ub, "aqg", qc, "iq", "aig");
        DT Y = contract(c, vb, "bpg", qb, "jp", "bjg");
        std::vector<int> sd{chi};
        sd.insert(sd.end(), td.begin(), td.end());
        double *sg = c.ar->dalloc(gcap);
        sign_vector(X.p, chi * I, gcap, gcap, sd, pow131((int)sd.size()), sg,
                    c.ar->dalloc(weight_ws_doubles((long)chi * I, gcap, 1)), c.st);
        scale_cols(X.p, chi * I, gcap, gcap, sg, c.st);
        scale_cols(Y.p, chi * J, gcap, gcap, sg, c.st);
        o.X = X;
        o.X.d = sd;
        o.X.d.push_back(gcap);
        o.Y = Y;
        o.Y.d = o.X.d;
        return o;
    }
    // ---- randomized SVD of M applied directly (App. A, eq. bond1 / bond2)
    DT Bp = permuted(c, Bt, "x" + tl + "a", tl + "xa");   // [j, x, alpha]
    DT Cp = permuted(c, Ct, "x" + tl + "b", tl + "xb");   // [i, x, beta]
    Bp.d = {(int)J, x, chi};
    Cp.d = {(int)I, x, chi};
    DT om = talloc(c, {(int)J, chi, m});
    philox_sketch(om.p, S->opt.seed, S->k, S->opt.instance, td, chi, m, 1, c.st, S->dint + 2);
    DT Q = talloc(c, {(int)(I * chi), m}), Qp = talloc(c, {(int)(J * chi), m}), Rp = talloc(c, {m, m}), Rq = talloc(c, {m, m});
    double *ws = c.ar->dalloc(std::max(tsqr_ws_doubles(I * chi, m), tsqr_ws_doubles(J * chi, m)));
    DT cur = om;
    for (int it = 0; it <= S->opt.power_iters; ++it) {
        // Y[i, alpha, m] = sum_{x, beta} C[x, i, beta] sum_j B[x, j, alpha] Omega[j, beta, m]
        // t1[(x, alpha), (beta, m)] = sum_j Bp[j, (x, alpha)] Omega[j, (beta, m)]: one GEMM
        // with rows (x, alpha) contiguous in Bp
        DT t1;
        {
            t1 = talloc(c, {x, chi, chi, m});
            GemmArgs g{};
            g.M = x * chi; g.N = chi * m; g.K = (int)J; g.batch = 1;
            g.A = Bp.p; g.sAr = 1; g.sAk = (long)x * chi;
            g.B = cur.p; g.sBk = (long)chi * m; g.sBn = 1;
            g.C = t1.p; g.sCr = (long)chi * m; g.sCn = 1;
            g.alpha = 1.0; g.beta = 0.0;
            gemm(g, P_FP64, c.st);
        }
        DT t1p = permuted(c, t1, "xabm", "xbam");
        DT y = contract(c, Cp, "ixb", t1p, "xbam", "iam");
        y.d = {(int)(I * chi), m};
        tsqr(y.p, I * chi, m, Q.p, Rq.p, ws, c.st);
        // Yt[j, beta, m] = sum_{x, alpha} B[x, j, alpha] sum_i C[x, i, beta] Q[i, alpha, m]
        DT t2;
        {
            t2 = talloc(c, {x, chi, chi, m});
            GemmArgs g{};
            g.M = x * chi; g.N = chi * m; g.K = (int)I; g.batch = 1;
            g.A = Cp.p; g.sAr = 1; g.sAk = (long)x * chi;
            g.B = Q.p; g.sBk = (long)chi * m; g.sBn = 1;
            g.C = t2.p; g.sCr = (long)chi * m; g.sCn = 1;
            g.alpha = 1.0; g.beta = 0.0;
            gemm(g, P_FP64, c.st);
        }
        DT t2p = permuted(c, t2, "xbam", "xabm");
        DT yt = contract(c, Bp, "jxa", t2p, "xabm", "jbm");
        yt.d = {(int)(J * chi), m};
        tsqr(yt.p, J * chi, m, Qp.p, Rp.p, ws, c.st);
        cur = Qp;
        cur.d = {(int)J, chi, m};
    }
    // SVD of Q^T M = Rp^T Qp^T: Jacobi on Rp^T, whose columns are the rows of Rp
    DT s = talloc(c, {m}), ut = talloc(c, {m, m}), w = talloc(c, {m, m});
    svd_colmajor(T, Rp.p, 1, m, m, s.p, ut.p, w.p);
    kept_count(s.p, m, gcap, EPS_S, T.S->opt.tau_deg, kept, c.st);
    copy(o.sig.p, s.p, gcap, c.st);
    hipLaunchKernelGGL(zero_tail_vec_kernel, dim3(1), dim3(256), 0, c.st, o.sig.p, gcap, kept);
    // U_bond = Q Ut[:, :gcap] rows (i, alpha); V_bond = Qp W[:, :gcap] rows (j, beta)
    DT ub = talloc(c, {(int)(I * chi), gcap}), vb = talloc(c, {(int)(J * chi), gcap});
    {
        GemmArgs g{};
        g.M = (int)(I * chi); g.N = gcap; g.K = m; g.batch = 1;
        g.A = Q.p; g.sAr = m; g.sAk = 1; g.sAb = 0;
        g.B = ut.p; g.sBk = m; g.sBn = 1; g.sBb = 0;
        g.C = ub.p; g.sCr = gcap; g.sCn = 1; g.sCb = 0;
        g.alpha = 1.0; g.beta = 0.0;
        gemm(g, P_FP64, c.st);
        g.M = (int)(J * chi); g.A = Qp.p; g.B = w.p; g.C = vb.p;
        gemm(g, P_FP64, c.st);
    }
    zero_tail_cols(ub.p, I * chi, gcap, gcap, kept, c.st);
    zero_tail_cols(vb.p, J * chi, gcap, gcap, kept, c.st);
    // sign convention over the multi-index (alpha, i_t1, i_t2, i_t3)
    std::vector<int> sd(td.begin(), td.end());
    sd.push_back(chi);
    std::vector<double> pw;
    double mlt = 131.0;
    for (size_t i = 0; i < td.size(); ++i) { pw.push_back(mlt); mlt *= 131.0; }
    pw.push_back(1.0);
    double *sg = c.ar->dalloc(gcap);
    sign_vector(ub.p, I * chi, gcap, gcap, sd, pw, sg, c.ar->dalloc(weight_ws_doubles((long)I * chi, gcap, 1)), c.st);
    scale_cols(ub.p, I * chi, gcap, gcap, sg, c.st);
    scale_cols(vb.p, J * chi, gcap, gcap, sg, c.st);
    ub.d = td;
    ub.d.push_back(chi);
    ub.d.push_back(gcap);
    vb.d = ub.d;
    o.X = permuted(c, ub, tl + "ag", "a" + tl + "g");
    o.Y = permuted(c, vb, tl + "bg", "b" + tl + "g");
    return o;
}

// ---------------------------------------------------------------- squeezers
// K_f, K_b of transverse position pos; tf: top of the upper half [x, t.., alpha],
// bf: bottom of the upper half [alpha, b.., g] closed through penv on g;
// tb: top of the lower half [beta, t.., g] closed through oenv; bb: [x, b.., beta].
void env_grams(Step &T, const DT &tf, const DT &bf, const DT &penv, const DT &tb, const DT &bb, const DT &oenv,
               int pos, DT &kf, DT &kb) {
    Ctx &c = T.c;
    const int nt = (int)tf.d.size() - 2;   // number of transverse legs
    std::string L = std::string("ijk").substr(0, nt);
    auto open = [&](char ch) {
        std::string s = L;
        s[pos] = ch;
        return s;
    };
    // zt[a, t, A, T] = sum tf[x, .., t, .., a] tf[x, .., T, .., A]
    DT zt = contract(c, tf, "x" + L + "a", tf, "x" + open('T') + "A", std::string("a") + L[pos] + "AT");
    DT bp = contract(c, bf, "a" + L + "g", penv, "gh", "a" + L + "h");
    DT zb = contract(c, bp, "a" + L + "h", bf, "A" + open('B') + "h", std::string("a") + L[pos] + "AB");
    zt.d = {zt.d[0], zt.d[1], zt.d[2], zt.d[3]};
    DT k1 = contract(c, zt, "atAT", zb, "abAB", "tbTB");
    int dt = k1.d[0], db = k1.d[1];
    kf = k1;
    kf.d = {dt * db, dt * db};
    DT yo = contract(c, tb, "b" + L + "g", oenv, "gh", "b" + L + "h");
    DT zy = contract(c, yo, "b" + L + "h", tb, "B" + open('T') + "h", std::string("b") + L[pos] + "BT");
    DT zd = contract(c, bb, "x" + L + "b", bb, "x" + open('X') + "B", std::string("b") + L[pos] + "BX");
    DT k2 = contract(c, zy, "btBT", zd, "bxBX", "txTX");
    kb = k2;
    kb.d = {dt * db, dt * db};
}

// Projector pairs for `cnt` squeezers with the same pair dims (dt, db):
// kf, kb hold cnt matrices each (n x n, n = dt*db); E[i], F[i] are [dt, db, D].
void squeezers(Step &T, const double *kf, const double *kb, int cnt, int dt, int db, DT *E, DT *F) {
    trg_state *S = T.S;
    Ctx &c = T.c;
    const int n = dt * db, D = S->D;
    const size_t nn = (size_t)n * n;
    // square-root factors X (K = X X^T) of all K_f, K_b in one batch, [f0, b0, f1, b1, ...]:
    // R = X^T.  Pivoted Cholesky (stopped at rounding-level pivots) for n <= 1024,
    // plain Cholesky above when every Gram is positive definite; otherwise
    // X = W Lambda^{1/2} from the eigen-decomposition with eigenvalues at or
    // below EPS_LAM of the largest set to zero.  Any two square roots of K
    // differ by an orthogonal factor, which cancels in E and F below.
    double *kk = c.ar->dalloc(2 * cnt * nn);
    for (int i = 0; i < cnt; ++i) {
        copy(kk + (2 * i) * nn, kf + i * nn, nn, c.st);
        copy(kk + (2 * i + 1) * nn, kb + i * nn, nn, c.st);
    }
    // pivoted Cholesky (X = P L, columns graded like W Lambda^{1/2}) keeps the
    // one-sided Jacobi of X_f^T X_b at about half the sweeps of plain Cholesky
    double *xs = c.ar->dalloc(2 * cnt * nn);
    bool chol_ok;
    if (n <= 1024) {
        double *kw = c.ar->dalloc(2 * cnt * nn);
        copy(kw, kk, 2 * cnt * nn, c.st);
        int *piws = reinterpret_cast<int *>(c.ar->dalloc((pchol_iws_ints(2 * cnt, n) + 1) / 2));
        chol_ok = pivoted_cholesky_batched(kw, 2 * cnt, n, xs, piws, c.st, PCHOL_TOL, nullptr,
                                           c.capture ? c.dstatus : nullptr);
    } else {
        TRG_REQUIRE(!c.capture, TRG_E_UNSUPPORTED, "graph capture: squeezer Grams above 1024 are not supported");
        copy(xs, kk, 2 * cnt * nn, c.st);
        int *cst = reinterpret_cast<int *>(c.ar->dalloc(cnt + 1));
        double *cws = c.ar->dalloc(chol_ws_doubles(2 * cnt, n));
        chol_ok = cholesky_batched(xs, 2 * cnt, n, cws, cst, c.st);
    }
    if (!chol_ok) {
        DT lam = talloc(c, {2 * cnt, n}), sq = talloc(c, {2 * cnt, n});
        eig_psd(T, kk, 2 * cnt, n, lam.p, xs);
        for (int i = 0; i < 2 * cnt; ++i) {
            hipLaunchKernelGGL(sqrt_clamp_kernel, dim3(g1(n)), dim3(256), 0, c.st, lam.p + (size_t)i * n,
                               sq.p + (size_t)i * n, n, EPS_LAM);
            DT xi{xs + i * nn, {n, n}};
            scale_axis(xi.p, xi.d, 1, sq.p + (size_t)i * n, 1, c.st);
        }
    }
    // R_f R_b^T = X_f^T X_b, all cnt in one batch
    DT gm = talloc(c, {cnt, n, n});
    for (int i = 0; i < cnt; ++i) {
        GemmArgs ga{};
        ga.M = n; ga.N = n; ga.K = n; ga.batch = 1;
        ga.A = xs + (2 * i) * nn; ga.sAr = 1; ga.sAk = n;           // X_f^T
        ga.B = xs + (2 * i + 1) * nn; ga.sBk = n; ga.sBn = 1;       // X_b
        ga.C = gm.p + i * nn; ga.sCr = n; ga.sCn = 1;
        ga.alpha = 1.0;
        gemm(ga, P_FP64, c.st);
    }
    // SVDs (Jacobi wants column-major: transpose each)
    DT gt = talloc(c, {cnt, n, n});
    permute(gm.p, gt.p, {cnt, n, n}, {0, 2, 1}, c.st);
    // only U is accumulated: the kept right vectors follow as V_D = M^T U_D S^-1
    DT s = talloc(c, {cnt, n}), u = talloc(c, {cnt, n, n});
    svd_colmajor(T, gt.p, cnt, n, n, s.p, u.p, nullptr);
    for (int i = 0; i < cnt; ++i) {
        int *kept = T.new_kept();
        const double *si = s.p + (size_t)i * n;
        kept_count(si, n, D, EPS_SQ, T.S->opt.tau_deg, kept, c.st);
        DT is = talloc(c, {n});
        hipLaunchKernelGGL(isqrt_kept_kernel, dim3(g1(n)), dim3(256), 0, c.st, si, is.p, n, kept);
        DT v0 = talloc(c, {n, D});
        GemmArgs gv{};
        gv.M = n; gv.N = D; gv.K = n; gv.batch = 1;
        gv.A = gm.p + i * nn; gv.sAr = 1; gv.sAk = n;                  // M^T
        gv.B = u.p + i * nn; gv.sBk = n; gv.sBn = 1;                   // U[:, :D]
        gv.C = v0.p; gv.sCr = D; gv.sCn = 1;
        gv.alpha = 1.0;
        gemm(gv, P_FP64, c.st);
        scale_axis(v0.p, v0.d, 1, is.p, 1, c.st);
        scale_axis(v0.p, v0.d, 1, is.p, 1, c.st);                      // * S^-1 (0 past the kept ones)
        // E = X_b V[:, :D] S^-1/2 ; F = X_f U[:, :D] S^-1/2
        DT vd = talloc(c, {n, D}), ud = talloc(c, {n, D});
        GemmArgs ga{};
        ga.M = n; ga.N = D; ga.K = n; ga.batch = 1;
        ga.A = xs + (2 * i + 1) * nn; ga.sAr = n; ga.sAk = 1;
        ga.B = v0.p; ga.sBk = D; ga.sBn = 1;
        ga.C = vd.p; ga.sCr = D; ga.sCn = 1;
        ga.alpha = 1.0;
        gemm(ga, P_FP64, c.st);
        ga.A = xs + (2 * i) * nn; ga.B = u.p + i * nn; ga.sBk = n; ga.C = ud.p;
        gemm(ga, P_FP64, c.st);
        scale_axis(vd.p, vd.d, 1, is.p, 1, c.st);
        scale_axis(ud.p, ud.d, 1, is.p, 1, c.st);
        // canonical basis of the new leg within multiplets of S
        DT rot = talloc(c, {D, D});
        double *zw = c.ar->dalloc(weight_ws_doubles(n, D, CANON_L));
        canonical_rotation(vd.p, n, D, D, {dt, db}, {1.0, 131.0}, si, kept, T.S->opt.tau_deg, zw, rot.p, S->dint, c.st);
        E[i] = contract(c, vd, "pk", rot, "kl", "pl");
        E[i].d = {dt, db, D};
        F[i] = contract(c, ud, "pk", rot, "kl", "pl");
        F[i].d = {dt, db, D};
    }
}

// squeezers of the transverse positions `pos` (all non-identity), batched by pair dims
void squeezer_set(Step &T, const std::vector<int> &pos, const std::vector<int> &pd, const DT *kf, const DT *kb,
                  DT *E, DT *F) {
    Ctx &c = T.c;
    std::vector<bool> done(pos.size(), false);
    for (size_t i = 0; i < pos.size(); ++i) {
        if (done[i]) continue;
        std::vector<size_t> grp;
        for (size_t j = i; j < pos.size(); ++j)
            if (!done[j] && pd[j] == pd[i]) grp.push_back(j);
        const int n = pd[i] * pd[i];
        const size_t nn = (size_t)n * n;
        double *f = c.ar->dalloc(grp.size() * nn), *b = c.ar->dalloc(grp.size() * nn);
        for (size_t g = 0; g < grp.size(); ++g) {
            copy(f + g * nn, kf[grp[g]].p, nn, c.st);
            copy(b + g * nn, kb[grp[g]].p, nn, c.st);
        }
        std::vector<DT> e(grp.size()), ff(grp.size());
        squeezers(T, f, b, (int)grp.size(), pd[i], pd[i], e.data(), ff.data());
        for (size_t g = 0; g < grp.size(); ++g) {
            E[pos[grp[g]]] = e[g];
            F[pos[grp[g]]] = ff[g];
            done[grp[g]] = true;
        }
    }
}

void identity_squeezer(Step &T, int dt, int db, DT &E, DT &F) {
    int n = dt * db;
    E = talloc(T.c, {dt, db, n});
    hipLaunchKernelGGL(eye_kernel, dim3(g1((long)n * n)), dim3(256), 0, T.c.st, E.p, n);
    F = E;
}

// ---------------------------------------------------------------- ATRG (d = 4)
void atrg_coarse(Step &T, const Split &sp, const Swap &sw, DT &phi, DT &psi) {
    Ctx &c = T.c;
    const int D = T.S->D;
    const DT &A = sp.A, &Dm = sp.Dm;
    DT Xs = talloc(c, sw.X.d);
    copy(Xs.p, sw.X.p, Xs.n(), c.st);
    scale_axis(Xs.p, Xs.d, 4, sw.sig.p, 1, c.st);
    const int ng = sw.sig.d[0];
    DT pe = talloc(c, {ng, ng});
    hipLaunchKernelGGL(eye_kernel, dim3(g1((long)ng * ng)), dim3(256), 0, c.st, pe.p, ng);
    DT s2 = talloc(c, {ng});
    hipLaunchKernelGGL(square_kernel, dim3(g1(ng)), dim3(256), 0, c.st, sw.sig.p, s2.p, ng);
    DT oe = talloc(c, {ng, ng});
    copy(oe.p, pe.p, (size_t)ng * ng, c.st);
    scale_axis(oe.p, oe.d, 0, s2.p, 1, c.st);
    DT E[3], F[3], KF[3], KB[3];
    std::vector<int> pos_sq, pd_sq;
    for (int pos = 0; pos < 3; ++pos) {
        int dd = A.d[pos + 1];
        if (dd * dd <= D) {
            identity_squeezer(T, dd, dd, E[pos], F[pos]);
        } else {
            env_grams(T, A, Xs, pe, sw.Y, Dm, oe, pos, KF[pos_sq.size()], KB[pos_sq.size()]);
            pos_sq.push_back(pos);
            pd_sq.push_back(dd);
        }
    }
    squeezer_set(T, pos_sq, pd_sq, KF, KB, E, F);
    // makeG: G[x, k1, k2, k3, g] = A X sigma E1 E2 E3 (pairwise, as in the oracle)
    DT t = contract(c, A, "xijka", E[0], "iIp", "xjkaIp");
    t = contract(c, t, "xjkaIp", Xs, "aIJKg", "xjkpJKg");
    t = contract(c, t, "xjkpJKg", E[1], "jJq", "xkpKgq");
    phi = contract(c, t, "xkpKgq", E[2], "kKr", "xpqrg");
    DT u = contract(c, Dm, "xIJKb", F[0], "iIp", "xJKbip");
    u = contract(c, u, "xJKbip", sw.Y, "bijkg", "xJKpjkg");
    u = contract(c, u, "xJKpjkg", F[1], "jJq", "xKpkgq");
    psi = contract(c, u, "xKpkgq", F[2], "kKr", "xpqrg");
}

// ---------------------------------------------------------------- triad-ATRG
// triad isometries U[(t1, t2), k] of the four pair Grams (eq. HOSVD), one batch
// what the impurity tangents need of the triad isometries: the Grams' full
// eigenbases, the kept counts and the sign vectors of the kept columns
struct IsoKeep {
    bool truncated = false;
    int n = 0, cap = 0, d1 = 0, d2 = 0;
    DT lam, vec;          // [4, n] descending, [4, n, n] eigenvector j in column j
    int *kept[4] = {nullptr, nullptr, nullptr, nullptr};
    double *sg[4] = {nullptr, nullptr, nullptr, nullptr};
};

void triad_isos(Step &T, const DT *grams, int d1, int d2, int rcap, DT *U, IsoKeep *ik = nullptr) {
    Ctx &c = T.c;
    const int n = d1 * d2;
    const size_t nn = (size_t)n * n;
    if (ik) {
        ik->truncated = n > rcap;
        ik->n = n;
        ik->cap = rcap;
        ik->d1 = d1;
        ik->d2 = d2;
    }
    if (n <= rcap) {
        for (int i = 0; i < 4; ++i) {
            U[i] = talloc(c, {d1, d2, n});
            hipLaunchKernelGGL(eye_kernel, dim3(g1((long)nn)), dim3(256), 0, c.st, U[i].p, n);
        }
        return;
    }
    double *kk = c.ar->dalloc(4 * nn);
    for (int i = 0; i < 4; ++i) copy(kk + i * nn, grams[i].p, nn, c.st);
    DT lam = talloc(c, {4, n}), vec = talloc(c, {4, n, n});
    const int ms = T.S->opt.max_sweeps > 0 ? T.S->opt.max_sweeps : 300;
    if (!gram_eig_pchol(c, kk, 4, n, ms, lam.p, vec.p, nullptr)) eig_psd(T, kk, 4, n, lam.p, vec.p);
    for (int i = 0; i < 4; ++i) {
        int *kept = T.new_kept();
        kept_count(lam.p + (size_t)i * n, n, rcap, EPS_LAM, T.S->opt.tau_deg, kept, c.st);
        U[i] = talloc(c, {n, rcap});
        col_slice(c, vec.p + i * nn, n, n, rcap, U[i].p);
        zero_tail_cols(U[i].p, n, rcap, rcap, kept, c.st);
        double *sg = c.ar->dalloc(rcap);
        sign_vector(U[i].p, n, rcap, rcap, {d1, d2}, {1.0, 131.0}, sg, c.ar->dalloc(weight_ws_doubles(n, rcap, 1)),
                    c.st);
        scale_cols(U[i].p, n, rcap, rcap, sg, c.st);
        U[i].d = {d1, d2, rcap};
        if (ik) {
            ik->kept[i] = kept;
            ik->sg[i] = sg;
        }
    }
    if (ik) {
        ik->lam = lam;
        ik->vec = vec;
    }
}

// The two big contractions of makeMG (and, with G, H, N, of makeMH), slab by
// slab over the first leg x of E (of H), as in the paper's GPU split of
// Table I but within one device:
//   K1: Z[x, u, v, c, g] = sum_{a, s} EM[x, u, c, a, s] F[a, s, v, g]
//       (rows (u, c) and columns (v, g) of the GEMM written interleaved)
//   K2: out[x, k, l, c, g] = sum_{u, v} T23[u, v, k, l] Z[x, u, v, c, g]
// u, v are the triad bonds (kA, kX), c the squeezed t3 bond, g the bond-swap bond.
// round up to a multiple of 32 (the split planes' K padding)
inline int pad32(long k) { return (int)((k + 31) / 32 * 32); }

// planes for n elements of BF16 from the arena
void *plane_alloc(Ctx &c, size_t n) { return c.ar->alloc(n * 2); }

// makeMG / makeMH with split-BF16 contractions (BF16X6): EM, F and T23 are
// split into BF16 planes once, Z once per slab group; K1 and K2 as gemm_planes
DT coarse_half_planes(Step &T, const DT &em, const DT &fp, const DT &t23) {
    Ctx &c = T.c;
    const int X = em.d[0], U = em.d[1], C = em.d[2], Aa = em.d[3], Ss = em.d[4];
    const int V = fp.d[2], G = fp.d[3];
    const int Kk = t23.d[2], Ll = t23.d[3];
    TRG_REQUIRE(fp.d[0] == Aa && fp.d[1] == Ss && t23.d[0] == U && t23.d[1] == V, -1, "coarse_half: shapes");
    DT out = talloc(c, {X, Kk, Ll, C, G});
    const long M1 = (long)U * C, N1 = (long)V * G, K1 = (long)Aa * Ss;
    const long M2 = (long)Kk * Ll, N2 = (long)C * G, K2 = (long)U * V;
    const int K1p = pad32(K1), K2p = pad32(K2);
    Arena::Mark mk = c.ar->mark();
    void *emp = plane_alloc(c, bf16_planes_elems(M1, K1p, X));
    void *fpp = plane_alloc(c, bf16_planes_elems(N1, K1p, 1));
    void *tpp = plane_alloc(c, bf16_planes_elems(M2, K2p, 1));
    split_bf16x3(em.p, K1, 1, M1 * K1, (int)M1, (int)K1, X, K1p, emp, c.st);   // EM: rows (kA, k3), k (alpha, s)
    split_bf16x3(fp.p, 1, N1, 0, (int)N1, (int)K1, 1, K1p, fpp, c.st);       // F: rows (kX, g), k (alpha, s)
    split_bf16x3(t23.p, 1, M2, 0, (int)M2, (int)K2, 1, K2p, tpp, c.st);      // T23: rows (k1, k2), k (kA, kX)
    const long zslab = (long)U * C * V * G;
    int xs = (int)std::max(1L, std::min<long>(X, (long)(134217728L / std::max(1L, zslab))));
    DT z = talloc(c, {xs, U, V, C, G});
    void *zp = plane_alloc(c, bf16_planes_elems(N2, K2p, xs));
    // K2 has few output tiles: split K so the launch fills the CUs
    const long tiles2 = ((M2 + 127) / 128) * ((N2 + 127) / 128) * xs;
    int inner = 1;
    while (inner < 16 && tiles2 * inner < 1024 && K2p / (2 * inner) >= 2048) inner *= 2;
    const int kslice = pad32((K2p + inner - 1) / inner);
    inner = (K2p + kslice - 1) / kslice;
    const long mn = M2 * N2;
    double *kws = inner > 1 ? c.ar->dalloc((size_t)xs * inner * mn) : nullptr;
    for (int x0 = 0; x0 < X; x0 += xs) {
        const int nx = std::min(xs, X - x0);
        PlaneGemm g{};
        g.A = static_cast<const char *>(emp) + 2 * (size_t)x0 * M1 * K1p;
        g.sAp = (long)X * M1 * K1p; g.sAb = M1 * K1p;
        g.B = fpp; g.sBp = N1 * K1p; g.sBb = 0;
        g.M = (int)M1; g.N = (int)N1; g.Kp = K1p; g.batch = nx;
        g.kslice = K1p; g.inner = 1;
        // rows (kA, k3) and columns (kX, g) land in Z's [x, kA, kX, k3, g] layout
        g.C = z.p; g.sCb = zslab;
        g.cR2 = C; g.sCr = (long)V * C * G; g.sCr2 = G;
        g.cN2 = G; g.sCn = (long)C * G; g.sCn2 = 1;
        g.alpha = 1.0; g.beta = 0.0;
        timed_planes(c, g, 2.0 * M1 * N1 * K1 * nx);
        // Z as K2's B operand: rows (k3, g), k (kA, kX)
        split_bf16x3(z.p, 1, N2, zslab, (int)N2, (int)K2, nx, K2p, zp, c.st);
        PlaneGemm h{};
        h.A = tpp; h.sAp = M2 * K2p; h.sAb = 0;
        h.B = zp; h.sBp = (long)nx * N2 * K2p; h.sBb = N2 * K2p;
        h.M = (int)M2; h.N = (int)N2; h.Kp = K2p; h.batch = nx;
        h.kslice = kslice; h.inner = inner;
        h.alpha = 1.0; h.beta = 0.0;
        if (inner > 1) {
            h.C = kws; h.sCr = N2; h.sCn = 1; h.sCb = (long)inner * mn; h.sCi = mn;
            timed_planes(c, h, 2.0 * M2 * N2 * K2 * nx);
            for (int x = 0; x < nx; ++x)
                sum_slices(kws + (long)x * inner * mn, inner, M2, N2, out.p + (long)(x0 + x) * mn, N2, 1, c.st);
        } else {
            h.C = out.p + (long)x0 * mn; h.sCr = N2; h.sCn = 1; h.sCb = mn;
            timed_planes(c, h, 2.0 * M2 * N2 * K2 * nx);
        }
    }
    c.ar->release(mk);
    return out;
}

// em2 / fp2 (optional, same shapes): out = (EM F + EM2 F2) T23, the second K1
// added into the same Z before K2 (one K2 for both products)
DT coarse_half(Step &T, const DT &em, const DT &fp, const DT &t23, const DT *em2 = nullptr, const DT *fp2 = nullptr) {
    Ctx &c = T.c;
    if (c.prec == P_BF16X6) {
        DT out = coarse_half_planes(T, em, fp, t23);
        if (em2) {
            DT o2 = coarse_half_planes(T, *em2, *fp2, t23);
            hipLaunchKernelGGL(axpy_scale_kernel, dim3(g1(out.n())), dim3(256), 0, c.st, out.p, o2.p, out.n(), 1.0,
                               nullptr);
            TRG_HIP_CHECK(hipGetLastError());
        }
        return out;
    }
    const int X = em.d[0], U = em.d[1], C = em.d[2], Aa = em.d[3], Ss = em.d[4];
    const int V = fp.d[2], G = fp.d[3];
    const int Kk = t23.d[2], Ll = t23.d[3];
    TRG_REQUIRE(fp.d[0] == Aa && fp.d[1] == Ss && t23.d[0] == U && t23.d[1] == V, -1, "coarse_half: shapes");
    DT out = talloc(c, {X, Kk, Ll, C, G});
    const long zslab = (long)U * C * V * G;
    // slab group: keep one group's Z near 1 GiB
    int xs = (int)std::max(1L, std::min<long>(X, (long)(134217728L / std::max(1L, zslab))));
    Arena::Mark mk = c.ar->mark();
    DT z = talloc(c, {xs, U, V, C, G});
    const long tiles2 = (long)((Kk * Ll + 63) / 64) * ((C * G + 63) / 64) * xs;
    int ks = 1;
    while (ks < 8 && tiles2 * ks < 1024 && (U * V) % (2 * ks) == 0 && (U * V) / (2 * ks) >= 2048) ks *= 2;
    double *kws = ks > 1 ? c.ar->dalloc((size_t)xs * ks * Kk * Ll * C * G) : nullptr;
    for (int x0 = 0; x0 < X; x0 += xs) {
        const int nx = std::min(xs, X - x0);
        GemmArgs g{};
        g.M = U * C; g.N = V * G; g.K = Aa * Ss; g.batch = nx;
        g.A = em.p + (long)x0 * U * C * Aa * Ss; g.sAr = (long)Aa * Ss; g.sAk = 1; g.sAb = (long)U * C * Aa * Ss;
        g.B = fp.p; g.sBk = (long)V * G; g.sBn = 1; g.sBb = 0;
        // rows (u, c) and columns (v, g) land in Z's [x, u, v, c, g] layout, K2's operand
        g.C = z.p; g.sCb = zslab;
        g.cR2 = C; g.sCr = (long)V * C * G; g.sCr2 = G;
        g.cN2 = G; g.sCn = (long)C * G; g.sCn2 = 1;
        g.alpha = 1.0; g.beta = 0.0;
        timed_gemm(c, g, c.prec);
        if (em2) {
            TRG_REQUIRE(em2->d == em.d && fp2->d == fp.d, -1, "coarse_half: second product's shapes");
            GemmArgs g2 = g;
            g2.A = em2->p + (long)x0 * U * C * Aa * Ss;
            g2.B = fp2->p;
            g2.beta = 1.0;
            timed_gemm(c, g2, c.prec);
        }
        // K2 has few output tiles (D^2 x D^2 per slab) over a long K = R^2: split K
        // so the launch fills the CUs, then add the slices in a fixed order
        const long mn = (long)Kk * Ll * C * G;
        GemmArgs h{};
        h.M = Kk * Ll; h.N = C * G; h.K = U * V; h.batch = nx;
        h.A = t23.p; h.sAr = 1; h.sAk = (long)Kk * Ll; h.sAb = 0;
        h.B = z.p; h.sBk = (long)C * G; h.sBn = 1; h.sBb = zslab;
        h.alpha = 1.0; h.beta = 0.0;
        if (ks > 1) {
            h.K = U * V / ks;
            h.inner = ks; h.sAi = (long)h.K * h.sAk; h.sBi = (long)h.K * h.sBk;
            h.C = kws; h.sCr = (long)C * G; h.sCn = 1; h.sCb = ks * mn; h.sCi = mn;
            timed_gemm(c, h, c.prec);
            for (int x = 0; x < nx; ++x)
                sum_slices(kws + (long)x * ks * mn, ks, (long)Kk * Ll, (long)C * G, out.p + (long)(x0 + x) * mn,
                           (long)C * G, 1, c.st);
        } else {
            h.C = out.p + (long)x0 * mn; h.sCr = (long)C * G; h.sCn = 1; h.sCb = mn;
            timed_gemm(c, h, c.prec);
        }
    }
    c.ar->release(mk);
    return out;
}

// pieces of a triad step that the impurity tangents reuse (squeezers held;
// the isometries' eigenbases for their tangents)
struct TriadKeep {
    DT UA, UX, UY, UD, M2, N2, f, hh, em, fp, ijmm, hn, gp, klnn;
    DT M0, M1, N0, N1, xsx, ysy;
    IsoKeep iso;
};

void triad_coarse(Step &T, const Split &sp, const Swap &sw, DT &phi, DT &psi, TriadKeep *keep = nullptr) {
    trg_state *S = T.S;
    Ctx &c = T.c;
    const int D = S->D;
    const DT &A = sp.A, &Dm = sp.Dm, &X = sw.X, &Y = sw.Y;
    const int d1 = A.d[1], d2 = A.d[2], d3 = A.d[3];
    const int rcap = std::min(S->opt.r * D, d1 * d2);
    const int ng = sw.sig.d[0];
    DT s2 = talloc(c, {ng});
    hipLaunchKernelGGL(square_kernel, dim3(g1(ng)), dim3(256), 0, c.st, sw.sig.p, s2.p, ng);
    DT Xs2 = talloc(c, X.d), Ys2 = talloc(c, Y.d);
    copy(Xs2.p, X.p, X.n(), c.st);
    scale_axis(Xs2.p, Xs2.d, 4, s2.p, 1, c.st);
    copy(Ys2.p, Y.p, Y.n(), c.st);
    scale_axis(Ys2.p, Ys2.d, 4, s2.p, 1, c.st);
    // triad Grams (eq. HOSVD)
    DT xsx = contract(c, Xs2, "aijtg", X, "bijtg", "ab");
    DT ysy = contract(c, Ys2, "aijtg", Y, "bijtg", "ab");
    DT ax = contract(c, A, "xijta", xsx, "ab", "xijtb");
    DT ga = contract(c, ax, "xijtb", A, "xkltb", "ijkl");
    DT gx = contract(c, Xs2, "aijtg", X, "akltg", "ijkl");
    DT gy = contract(c, Ys2, "aijtg", Y, "akltg", "ijkl");
    DT dy = contract(c, Dm, "xijta", ysy, "ab", "xijtb");
    DT gd = contract(c, dy, "xijtb", Dm, "xkltb", "ijkl");
    DT grams[4] = {ga, gx, gy, gd}, Us[4];
    for (auto &gg : grams) gg.d = {d1 * d2, d1 * d2};
    IsoKeep ik;
    triad_isos(T, grams, d1, d2, rcap, Us, keep ? &ik : nullptr);
    DT &UA = Us[0], &UX = Us[1], &UY = Us[2], &UD = Us[3];
    // triad tensors
    DT e = contract(c, A, "xijta", UA, "ijk", "xkta");
    DT f = contract(c, X, "aijtg", UX, "ijk", "aktg");
    scale_axis(f.p, f.d, 3, sw.sig.p, 1, c.st);
    DT g = contract(c, Y, "bijtg", UY, "ijk", "bktg");
    DT hh = contract(c, Dm, "xijtb", UD, "ijk", "xktb");
    // O and P (Gram matrices of the upper and lower blocks)
    DT ee = contract(c, e, "xkta", e, "xktb", "ab");
    DT ef = contract(c, ee, "ab", f, "bktg", "aktg");
    DT o = contract(c, ef, "aktg", f, "akth", "gh");
    DT h2 = contract(c, hh, "xktb", hh, "xktc", "bc");
    DT hg = contract(c, h2, "bc", g, "cktg", "bktg");
    DT p = contract(c, hg, "bktg", g, "bkth", "gh");
    // projected A, X sigma, Y, D
    DT at = contract(c, e, "xkta", UA, "ijk", "xijta");
    DT xt = contract(c, f, "aktg", UX, "ijk", "aijtg");
    DT yt = contract(c, g, "bktg", UY, "ijk", "bijtg");
    DT dt = contract(c, hh, "xktb", UD, "ijk", "xijtb");
    DT M[3], N[3], KF[3], KB[3];
    const int dd[3] = {d1, d2, d3};
    std::vector<int> pos_sq, pd_sq;
    for (int pos = 0; pos < 3; ++pos) {
        if (dd[pos] * dd[pos] <= D) {
            identity_squeezer(T, dd[pos], dd[pos], M[pos], N[pos]);
        } else {
            env_grams(T, at, xt, p, yt, dt, o, pos, KF[pos_sq.size()], KB[pos_sq.size()]);
            pos_sq.push_back(pos);
            pd_sq.push_back(dd[pos]);
        }
    }
    squeezer_set(T, pos_sq, pd_sq, KF, KB, M, N);
    // makeMG: Phi = (E F M3)(I J M1 M2)
    DT im = contract(c, UA, "ijA", M[0], "ipk", "jApk");
    DT imm = contract(c, im, "jApk", M[1], "jql", "Apkql");
    DT ijmm = contract(c, imm, "Apkql", UX, "pqX", "AXkl");            // T23 [kA, kX, k1, k2]
    DT em = contract(c, e, "xAta", M[2], "tsc", "xAcas");               // [x, kA, k3, alpha, s]
    DT fp = permuted(c, f, "aXsg", "asXg");                             // [alpha, s, kX, g]
    phi = coarse_half(T, em, fp, ijmm);
    // makeMH: Psi = (G H N3)(K L N1 N2)
    DT kn = contract(c, UY, "ijY", N[0], "ipk", "jYpk");
    DT knn = contract(c, kn, "jYpk", N[1], "jql", "Ypkql");
    DT klnn = contract(c, knn, "Ypkql", UD, "pqD", "DYkl");            // [kD, kY, k1, k2]
    DT hn = contract(c, hh, "xDsb", N[2], "tsc", "xDcbt");              // [x, kD, k3, beta, t]
    DT gp = permuted(c, g, "bYtg", "btYg");                             // [beta, t, kY, g]
    psi = coarse_half(T, hn, gp, klnn);
    if (keep) *keep = TriadKeep{UA, UX, UY, UD, M[2], N[2], f, hh, em, fp, ijmm, hn, gp, klnn,
                                M[0], M[1], N[0], N[1], xsx, ysy, ik};
}

// ---------------------------------------------------------------- impurity tangents
// y += a x, then y /= *cdev when cdev is given (all on the stream)
void axpy_scale(Ctx &c, DT &y, const DT *x, double a, const double *cdev) {
    hipLaunchKernelGGL(axpy_scale_kernel, dim3(g1(y.n())), dim3(256), 0, c.st, y.p, x ? x->p : nullptr, y.n(), a, cdev);
    TRG_HIP_CHECK(hipGetLastError());
}

// Eigenvalue gap, relative to the largest, at or below which a kept /
// discarded pair gets no derivative: eigen-directions that close are not
// determined by the Gram (the cut can fall between eigenvalues a few rounding
// errors of the largest apart), so the pair is treated as degenerate
constexpr double ISO_GAP = 1e-12;

// C[j, i] (n x cap) = P[j, i] / (lam_i - lam_j) for a kept i < *kept and a
// discarded j >= *kept whose gap exceeds ISO_GAP lam_0, else 0
__global__ void iso_coef_kernel(const double *P, const double *lam, const int *kept, int n, int cap, double *C) {
    const long tot = (long)n * cap;
    const int k = *kept;
    const double cut = ISO_GAP * lam[0];
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
        const int j = (int)(e / cap), i = (int)(e - (long)j * cap);
        double v = 0.0;
        if (i < k && j >= k) {
            const double den = lam[i] - lam[j];
            v = den > cut ? P[(long)j * n + i] / den : 0.0;
        }
        C[e] = v;
    }
}

// out[p, i] = vec[p, i] / lam[i] for the kept i < *kept whose eigenvalue
// exceeds ISO_GAP lam_0 (its gap to the null space), else 0 (n x cap)
__global__ void kept_over_lam_kernel(const double *vec, const double *lam, const int *kept, int n, int cap,
                                     double *out) {
    const long tot = (long)n * cap;
    const int k = *kept;
    const double cut = ISO_GAP * lam[0];
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
        const int p = (int)(e / cap), i = (int)(e - (long)p * cap);
        out[e] = (i < k && lam[i] > cut) ? vec[(long)p * n + i] / lam[i] : 0.0;
    }
}

// g += g^T over the two halves of its labels ("ab" or "ijkl")
void sym_add(Ctx &c, DT &g, const std::string &lab, const std::string &swp) {
    DT t = permuted(c, g, lab, swp);
    axpy_scale(c, g, &t, 1.0, nullptr);
}

// Tangents dU of the four triad isometries (eq. HOSVD) along the step's
// tangents dA, d(X sigma), dY, dD (step order).  The coarse tensor depends on
// an isometry only through its projector U U^T, so only the motion of the kept
// subspace counts: dU = W C with W the discarded eigenvectors of the Gram and
// C[j, i] = w_j^T dG u_i / (lam_i - lam_j) (first-order perturbation of an
// invariant subspace), in the kept columns' sign convention.  The pivoted-
// Cholesky eigensolver returns zero columns for a rank-deficient Gram's null
// space, so that part of W enters as (1 - V V^T) dG u_i / lam_i (its
// eigenvalues are 0).  The Gram tangents follow from M_k = X sigma Y^T: X sigma^2 X^T = M_k M_k^T moves by
// d(X sigma)(X sigma)^T + transpose, Y sigma^2 Y^T = M_k^T M_k by
// Y Wg Y^T + dY sigma^2 Y^T + transpose, Wg = (X sigma)^T d(X sigma) + transpose.
void iso_tangents(Step &T, const TriadKeep &K, const DT &A, const Swap &sw, const DT &Dm, const DT &dA,
                  const DT &dxs, const DT &dY, const DT &dDm, DT *dU) {
    Ctx &c = T.c;
    const DT &X = sw.X, &Y = sw.Y;
    const int ng = sw.sig.d[0];
    DT s2 = talloc(c, {ng});
    hipLaunchKernelGGL(square_kernel, dim3(g1(ng)), dim3(256), 0, c.st, sw.sig.p, s2.p, ng);
    DT xs = talloc(c, X.d);
    copy(xs.p, X.p, X.n(), c.st);
    scale_axis(xs.p, xs.d, 4, sw.sig.p, 1, c.st);
    DT dys2 = talloc(c, dY.d);
    copy(dys2.p, dY.p, dY.n(), c.st);
    scale_axis(dys2.p, dys2.d, 4, s2.p, 1, c.st);
    DT dxsx = contract(c, dxs, "aijtg", xs, "bijtg", "ab");
    sym_add(c, dxsx, "ab", "ba");
    DT wg = contract(c, xs, "aijtg", dxs, "aijth", "gh");
    sym_add(c, wg, "gh", "hg");
    DT yw = contract(c, Y, "aijtg", wg, "gh", "aijth");
    DT dysy = contract(c, dys2, "aijtg", Y, "bijtg", "ab");
    sym_add(c, dysy, "ab", "ba");
    DT ywy = contract(c, yw, "aijth", Y, "bijth", "ab");
    axpy_scale(c, dysy, &ywy, 1.0, nullptr);
    DT dg[4];
    {   // A: sym(dA xsx A) + A dxsx A
        DT t = contract(c, dA, "xijta", K.xsx, "ab", "xijtb");
        dg[0] = contract(c, t, "xijtb", A, "xkltb", "ijkl");
        sym_add(c, dg[0], "ijkl", "klij");
        DT t2 = contract(c, A, "xijta", dxsx, "ab", "xijtb");
        DT g2 = contract(c, t2, "xijtb", A, "xkltb", "ijkl");
        axpy_scale(c, dg[0], &g2, 1.0, nullptr);
    }
    dg[1] = contract(c, dxs, "aijtg", xs, "akltg", "ijkl");             // X: sym(d(X sigma) (X sigma))
    sym_add(c, dg[1], "ijkl", "klij");
    {   // Y: sym(dY s2 Y) + Y wg Y
        dg[2] = contract(c, dys2, "aijtg", Y, "akltg", "ijkl");
        sym_add(c, dg[2], "ijkl", "klij");
        DT g2 = contract(c, yw, "aijth", Y, "aklth", "ijkl");
        axpy_scale(c, dg[2], &g2, 1.0, nullptr);
    }
    {   // D: sym(dD ysy D) + D dysy D
        DT t = contract(c, dDm, "xijta", K.ysy, "ab", "xijtb");
        dg[3] = contract(c, t, "xijtb", Dm, "xkltb", "ijkl");
        sym_add(c, dg[3], "ijkl", "klij");
        DT t2 = contract(c, Dm, "xijta", dysy, "ab", "xijtb");
        DT g2 = contract(c, t2, "xijtb", Dm, "xkltb", "ijkl");
        axpy_scale(c, dg[3], &g2, 1.0, nullptr);
    }
    const IsoKeep &ik = K.iso;
    const int n = ik.n, cap = ik.cap;
    for (int i = 0; i < 4; ++i) {
        DT V{ik.vec.p + (size_t)i * n * n, {n, n}};
        dg[i].d = {n, n};
        DT p1 = contract(c, V, "pj", dg[i], "pq", "jq");
        DT pm = contract(c, p1, "jq", V, "qi", "ji");
        DT cm = talloc(c, {n, cap});
        hipLaunchKernelGGL(iso_coef_kernel, dim3(g1((long)n * cap)), dim3(256), 0, c.st, pm.p, ik.lam.p + (size_t)i * n,
                           ik.kept[i], n, cap, cm.p);
        TRG_HIP_CHECK(hipGetLastError());
        dU[i] = contract(c, V, "pj", cm, "ji", "pi");
        // null space of the Gram (zero eigenvector columns): (1 - V V^T) dG U / lam
        DT ul = talloc(c, {n, cap});
        hipLaunchKernelGGL(kept_over_lam_kernel, dim3(g1((long)n * cap)), dim3(256), 0, c.st, V.p,
                           ik.lam.p + (size_t)i * n, ik.kept[i], n, cap, ul.p);
        TRG_HIP_CHECK(hipGetLastError());
        DT y1 = contract(c, dg[i], "pq", ul, "qi", "pi");
        DT vy = contract(c, V, "qj", y1, "qi", "ji");
        DT vvy = contract(c, V, "pj", vy, "ji", "pi");
        axpy_scale(c, y1, &vvy, -1.0, nullptr);
        axpy_scale(c, dU[i], &y1, 1.0, nullptr);
        scale_cols(dU[i].p, n, cap, cap, ik.sg[i], c.st);
        dU[i].d = {ik.d1, ik.d2, cap};
    }
}

// One triad step of an impurity tangent (dPhi, dPsi) of the state: the pure
// step's squeezers and norm are held; the re-split and bond-swap tangents live
// in the tangent space of the rank-chi matrices (re-split gauge A^T dA = 0,
// D^T dD = 0; bond swap d(X sigma) = dM Y, dY = (1 - Y Y^T) dM^T X sigma^+);
// the triad isometries move with their Grams (iso_tangents) where they
// truncate.  Returns the new tangent in step order [x, k1, k2, k3, g].
void triad_tangent(Step &T, const Split &sp, const Swap &sw, const TriadKeep &K, const double *dphi_p,
                   const double *dpsi_p, const std::vector<int> &order, DT &dphi_out, DT &dpsi_out) {
    trg_state *S = T.S;
    Ctx &c = T.c;
    const int d = (int)S->dims.size();
    const int chi = S->chi;
    long F = 1;
    for (int v : S->dims) F *= v;
    DT phi, psi, dphi, dpsi;
    phi.p = S->phi;
    psi.p = S->psi;
    dphi.p = const_cast<double *>(dphi_p);
    dpsi.p = const_cast<double *>(dpsi_p);
    phi.d = psi.d = dphi.d = dpsi.d = {(int)F, chi};
    const DT &a = sp.a_nat, &dm = sp.dm_nat;
    const double *cdev = S->dscal + 6;
    // re-split: Z1 = (dT/c) D, Z2 = (dT/c)^T A
    DT w1 = contract(c, psi, "Fg", dm, "Fb", "gb");
    DT w2 = contract(c, dpsi, "Fg", dm, "Fb", "gb");
    DT z1 = contract(c, dphi, "Fg", w1, "gb", "Fb");
    DT z1b = contract(c, phi, "Fg", w2, "gb", "Fb");
    axpy_scale(c, z1, &z1b, 1.0, cdev);
    DT v1 = contract(c, dphi, "Fg", a, "Fa", "ga");
    DT v2 = contract(c, phi, "Fg", a, "Fa", "ga");
    DT z2 = contract(c, psi, "Fg", v1, "ga", "Fa");
    DT z2b = contract(c, dpsi, "Fg", v2, "ga", "Fa");
    axpy_scale(c, z2, &z2b, 1.0, cdev);
    DT spp = talloc(c, {chi, chi});
    hipLaunchKernelGGL(sprime_inv_kernel, dim3(g1((long)chi * chi)), dim3(256), 0, c.st, sp.rot.p, sp.s.p, chi, spp.p);
    // dA = (1 - A A^T) Z1 S'^+, dD = (1 - D D^T) Z2 S'^+, dC = Z1, dB = Z2
    DT p1 = contract(c, a, "Fa", z1, "Fb", "ab");
    DT q1 = contract(c, a, "Fa", p1, "ab", "Fb");
    DT r1 = talloc(c, {(int)F, chi});
    copy(r1.p, z1.p, r1.n(), c.st);
    axpy_scale(c, r1, &q1, -1.0, nullptr);
    DT da = contract(c, r1, "Fb", spp, "bc", "Fc");
    DT p2 = contract(c, dm, "Fa", z2, "Fb", "ab");
    DT q2 = contract(c, dm, "Fa", p2, "ab", "Fb");
    DT r2 = talloc(c, {(int)F, chi});
    copy(r2.p, z2.p, r2.n(), c.st);
    axpy_scale(c, r2, &q2, -1.0, nullptr);
    DT ddm = contract(c, r2, "Fb", spp, "bc", "Fc");
    std::string nat, stp;
    for (int i = 0; i < d; ++i) nat += (char)('a' + i);
    for (int i = 0; i < d; ++i) stp += (char)('a' + order[i]);
    nat += 'z';
    stp += 'z';
    std::vector<int> fd(S->dims.begin(), S->dims.end());
    fd.push_back(chi);
    da.d = ddm.d = z1.d = z2.d = fd;
    DT dA = permuted(c, da, nat, stp), dDm = permuted(c, ddm, nat, stp);
    DT dB = permuted(c, z2, nat, stp), dC = permuted(c, z1, nat, stp);
    // bond swap: dM = dB C + B dC over the shared leg x
    const DT &B = sp.B, &C = sp.C, &X = sw.X, &Y = sw.Y;
    DT by = contract(c, B, "xijka", Y, "bijkh", "xabh");
    DT dby = contract(c, dB, "xijka", Y, "bijkh", "xabh");
    DT dxs = contract(c, C, "xuvwb", dby, "xabh", "auvwh");
    DT dxs2 = contract(c, dC, "xuvwb", by, "xabh", "auvwh");
    axpy_scale(c, dxs, &dxs2, 1.0, nullptr);                            // d(X sigma) = dM Y
    DT cx = contract(c, C, "xuvwb", X, "auvwg", "xabg");
    DT dcx = contract(c, dC, "xuvwb", X, "auvwg", "xabg");
    DT dmx = contract(c, dB, "xijka", cx, "xabg", "bijkg");
    DT dmx2 = contract(c, B, "xijka", dcx, "xabg", "bijkg");
    axpy_scale(c, dmx, &dmx2, 1.0, nullptr);                            // dM^T X
    const int ng = sw.sig.d[0];
    DT sinv = talloc(c, {ng});
    hipLaunchKernelGGL(inv_pos_kernel, dim3(g1(ng)), dim3(256), 0, c.st, sw.sig.p, sinv.p, ng);
    scale_axis(dmx.p, dmx.d, 4, sinv.p, 1, c.st);
    DT yty = contract(c, Y, "bijkh", dmx, "bijkg", "hg");
    DT yyty = contract(c, Y, "bijkh", yty, "hg", "bijkg");
    axpy_scale(c, dmx, &yyty, -1.0, nullptr);                           // dY = (1 - Y Y^T) dM^T X sigma^+
    // triad tensors and makeMG / makeMH, one factor at a time
    DT de = contract(c, dA, "xijta", K.UA, "ijk", "xkta");
    DT df = contract(c, dxs, "aijtg", K.UX, "ijk", "aktg");
    DT dg = contract(c, dmx, "bijtg", K.UY, "ijk", "bktg");
    DT dh = contract(c, dDm, "xijtb", K.UD, "ijk", "xktb");
    DT dijmm, dklnn;
    if (K.iso.truncated) {
        // the isometries' kept subspaces move with the triad Grams (see iso_tangent)
        DT dU[4];
        iso_tangents(T, K, sp.A, sw, sp.Dm, dA, dxs, dmx, dDm, dU);
        DT xs = talloc(c, X.d);
        copy(xs.p, X.p, X.n(), c.st);
        scale_axis(xs.p, xs.d, 4, sw.sig.p, 1, c.st);
        DT de2 = contract(c, sp.A, "xijta", dU[0], "ijk", "xkta");
        DT df2 = contract(c, xs, "aijtg", dU[1], "ijk", "aktg");
        DT dg2 = contract(c, Y, "bijtg", dU[2], "ijk", "bktg");
        DT dh2 = contract(c, sp.Dm, "xijtb", dU[3], "ijk", "xktb");
        axpy_scale(c, de, &de2, 1.0, nullptr);
        axpy_scale(c, df, &df2, 1.0, nullptr);
        axpy_scale(c, dg, &dg2, 1.0, nullptr);
        axpy_scale(c, dh, &dh2, 1.0, nullptr);
        // and so do the triad tensors I..L inside T23 (makeMG) and its makeMH counterpart
        auto t23 = [&](const DT &u1, const DT &m0, const DT &m1, const DT &u2, const char *out) {
            DT im = contract(c, u1, "ijA", m0, "ipk", "jApk");
            DT imm = contract(c, im, "jApk", m1, "jql", "Apkql");
            return contract(c, imm, "Apkql", u2, "pqX", out);
        };
        dijmm = t23(dU[0], K.M0, K.M1, K.UX, "AXkl");
        DT dijmm2 = t23(K.UA, K.M0, K.M1, dU[1], "AXkl");
        axpy_scale(c, dijmm, &dijmm2, 1.0, nullptr);
        dklnn = t23(dU[2], K.N0, K.N1, K.UD, "XAkl");          // [kD, kY, k1, k2] as klnn
        DT dklnn2 = t23(K.UY, K.N0, K.N1, dU[3], "XAkl");
        axpy_scale(c, dklnn, &dklnn2, 1.0, nullptr);
    }
    DT dem = contract(c, de, "xAta", K.M2, "tsc", "xAcas");
    DT dfp = permuted(c, df, "aXsg", "asXg");
    dphi_out = coarse_half(T, dem, K.fp, K.ijmm, &K.em, &dfp);
    if (K.iso.truncated) {
        DT t4 = coarse_half(T, K.em, K.fp, dijmm);
        axpy_scale(c, dphi_out, &t4, 1.0, nullptr);
    }
    DT dhn = contract(c, dh, "xDsb", K.N2, "tsc", "xDcbt");
    DT dgp = permuted(c, dg, "bYtg", "btYg");
    dpsi_out = coarse_half(T, dhn, K.gp, K.klnn, &K.hn, &dgp);
    if (K.iso.truncated) {
        DT t5 = coarse_half(T, K.hn, K.gp, dklnn);
        axpy_scale(c, dpsi_out, &t5, 1.0, nullptr);
    }
}

// numerical status flag (dint[0]) -> error
void check_status(int status) {
    TRG_REQUIRE(status != 1, TRG_E_NUMERICAL, "non-positive or non-finite norm at a re-split");
    TRG_REQUIRE(status != 2, TRG_E_MULTIPLET,
                "a truncation cut falls in a multiplet of more than 32 values (canonical basis not formed); "
                "change tau_deg or D");
    TRG_REQUIRE(status != 3, TRG_E_NUMERICAL,
                "Jacobi SVD of a replayed step not converged within the sweeps allowed at capture");
    TRG_REQUIRE(status != 5, TRG_E_NUMERICAL, "Jacobi SVD of a replayed step met non-finite entries");
    TRG_REQUIRE(status != 4, TRG_E_NUMERICAL, "pivoted Cholesky of a replayed step met a non-finite pivot");
    TRG_REQUIRE(status == 0, TRG_E_NUMERICAL, "numerical status flag set");
}

__global__ void step_inc_kernel(int *k) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *k += 1;
}

__global__ void step_begin_kernel(double *dscal, int *dint) {
    if (threadIdx.x || blockIdx.x) return;
    dscal[3] = dscal[0];
    dint[1] = dint[0];
    dint[3] = dint[2];
}

// a failed step's rollback of the device scalars (accumulator, status, step index)
__global__ void step_undo_kernel(double *dscal, int *dint) {
    if (threadIdx.x || blockIdx.x) return;
    dscal[0] = dscal[3];
    dint[0] = dint[1];
    dint[2] = dint[3];
}

// ---------------------------------------------------------------- one step
void do_step(trg_state *S, int axis, bool triad) {
    TRG_REQUIRE(S->init, -2, "step before tensor_init");
    const int d = S->opt.dim;
    TRG_REQUIRE(axis >= 0 && axis < d, -1, "axis out of range");
    TRG_REQUIRE(d == 4, -6, "the GPU path implements d = 4");
    TRG_REQUIRE(triad || S->ntan == 0, TRG_E_UNSUPPORTED,
                "impurity tangents are carried by triad_atrg_step only (atrg_step: create the state without tangents)");
    S->ar.reset();
    Step T(S);
    // accumulator, status and step index before the step (dscal[3], dint[1], dint[3]);
    // restored if the step fails
    hipLaunchKernelGGL(step_begin_kernel, dim3(1), dim3(1), 0, S->st, S->dscal, S->dint);
    TRG_HIP_CHECK(hipGetLastError());
    if (T.c.capture) {
        // a recorded step also keeps the state and spectra it starts from
        long n = S->chi;
        for (int v : S->dims) n *= v;
        TRG_REQUIRE(S->bak && S->bak_cap >= (size_t)(2 + 2 * S->ntan) * S->cap_state, TRG_E_STATE,
                    "graph capture: no backup buffer");
        copy(S->bak, S->phi, n, S->st);
        copy(S->bak + S->cap_state, S->psi, n, S->st);
        for (int t = 0; t < S->ntan; ++t) {
            copy(S->bak + (2 + 2 * t) * S->cap_state, S->dphi[t], n, S->st);
            copy(S->bak + (3 + 2 * t) * S->cap_state, S->dpsi[t], n, S->st);
        }
        copy(S->dspec + 2048, S->dspec, 2048, S->st);
    }
    std::vector<int> order(d);
    for (int i = 0; i < d; ++i) order[i] = (axis + i) % d;
    Split sp = resplit(T, order);
    Swap sw = bond_swap(T, sp);
    DT phi, psi;
    TriadKeep keep;
    if (triad) triad_coarse(T, sp, sw, phi, psi, S->ntan ? &keep : nullptr);
    else atrg_coarse(T, sp, sw, phi, psi);
    DT dphi[2], dpsi[2];
    for (int t = 0; t < S->ntan; ++t) triad_tangent(T, sp, sw, keep, S->dphi[t], S->dpsi[t], order, dphi[t], dpsi[t]);
    // back to natural axis order
    std::string stp, nat;
    for (int i = 0; i < d; ++i) stp += (char)('a' + order[i]);
    for (int i = 0; i < d; ++i) nat += (char)('a' + i);
    stp += 'z';
    nat += 'z';
    TRG_REQUIRE((size_t)phi.n() <= S->cap_state && (size_t)psi.n() <= S->cap_state, -6, "state exceeds D^5");
    const size_t nsig = sw.sig.d[0], nrsv = sp.s.d[0];
    TRG_REQUIRE(nsig <= 1024 && nrsv <= 1024, -6, "spectra longer than 1024");
    copy(S->dspec, sw.sig.p, nsig, S->st);
    copy(S->dspec + 1024, sp.s.p, nrsv, S->st);
    std::vector<double> sig(nsig, 0.0), rsv(nrsv, 0.0);
    if (!T.c.capture) {
        // numerical status of the step (norm, multiplet sizes) before the state is overwritten
        int status = 0;
        TRG_HIP_CHECK(hipMemcpyAsync(sig.data(), sw.sig.p, sizeof(double) * nsig, hipMemcpyDeviceToHost, S->st));
        TRG_HIP_CHECK(hipMemcpyAsync(rsv.data(), sp.s.p, sizeof(double) * nrsv, hipMemcpyDeviceToHost, S->st));
        TRG_HIP_CHECK(hipMemcpyAsync(&status, S->dint, sizeof(int), hipMemcpyDeviceToHost, S->st));
        TRG_HIP_CHECK(hipStreamSynchronize(S->st));
        check_status(status);
    }
    std::vector<int> perm(d + 1);
    for (int i = 0; i <= d; ++i) perm[i] = (int)stp.find(nat[i]);
    permute(phi.p, S->phi, phi.d, perm, S->st);
    permute(psi.p, S->psi, psi.d, perm, S->st);
    for (int t = 0; t < S->ntan; ++t) {
        permute(dphi[t].p, S->dphi[t], dphi[t].d, perm, S->st);
        permute(dpsi[t].p, S->dpsi[t], dpsi[t].d, perm, S->st);
    }
    std::vector<int> nd(d);
    for (int i = 0; i < d; ++i) nd[i] = phi.d[perm[i]];
    hipLaunchKernelGGL(step_inc_kernel, dim3(1), dim3(1), 0, S->st, S->dint + 2);
    TRG_HIP_CHECK(hipGetLastError());
    S->dims = nd;
    S->chi = phi.d[d];
    S->nsig = nsig;
    S->nrsv = nrsv;
    if (T.c.capture) return;   // the recorded step's host side ends here
    S->sigma_last = sig;
    S->resplit_last = rsv;
    S->spec_stale = false;
    TRG_HIP_CHECK(hipStreamSynchronize(S->st));
    for (auto &t : T.c.timed) {
        float ms = 0.0f;
        TRG_HIP_CHECK(hipEventElapsedTime(&ms, t.a, t.b));
        S->t_ms += ms;
        S->t_flops += t.flops;
        S->t_launch += 1;
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    T.c.timed.clear();
    S->k += 1;
}

}  // namespace
}  // namespace trg

// ====================================================================== C ABI
using trg::Error;

namespace {
int fail(trg_state *s, const Error &e) {
    if (s) s->err = e.what();
    return e.code;
}
int fail_std(trg_state *s, const std::exception &e) {
    if (s) s->err = e.what();
    return TRG_E_HIP;
}
struct DevGuard {
    int prev = -1;
    explicit DevGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (hipSetDevice(dev) != hipSuccess) throw Error(TRG_E_HIP, "hipSetDevice failed");
    }
    ~DevGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};
thread_local std::string g_err;
}  // namespace

extern "C" {

void trg_default_options(trg_options *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->dim = 4;
    o->r = 7;
    o->sketch_mult = 2;
    o->power_iters = 1;
    o->precision = TRG_FP64;
    o->bond_svd = TRG_SVD_SKETCH;
    o->max_sweeps = 300;
    o->tau_deg = trg::TAU_DEG_DEFAULT;
    o->r_bond = 1;
}

int trg_create(const trg_options *opt, trg_state **out) {
    if (!out) return TRG_E_INVALID;
    *out = nullptr;
    if (!opt) return TRG_E_INVALID;
    if (opt->dim != 4 || opt->r < 1 || opt->sketch_mult < 1 || opt->power_iters < 0 ||
        (opt->precision < 0 || opt->precision > 3) || (opt->bond_svd != 0 && opt->bond_svd != 1))
        return TRG_E_INVALID;
    if (!(opt->tau_deg >= 0.0 && opt->tau_deg < 1.0)) return TRG_E_INVALID;
    if (opt->r_bond < 1 || opt->sketch_mult < opt->r_bond) return TRG_E_INVALID;
    if (opt->tangents < 0 || opt->tangents > (TRG_TAN_BETA | TRG_TAN_H)) return TRG_E_INVALID;
    trg_state *s = new (std::nothrow) trg_state();
    if (!s) return TRG_E_NOMEM;
    s->opt = *opt;
    if (s->opt.tau_deg == 0.0) s->opt.tau_deg = trg::TAU_DEG_DEFAULT;
    try {
        DevGuard g(opt->device);
        s->st = static_cast<hipStream_t>(opt->stream);
        s->ar.set_cap(opt->workspace_cap);
        TRG_HIP_CHECK(hipMalloc(&s->dscal, 2048 * sizeof(double)));
        TRG_HIP_CHECK(hipMalloc(&s->dint, 256 * sizeof(int)));
        TRG_HIP_CHECK(hipMalloc(&s->dspec, 4096 * sizeof(double)));
    } catch (const Error &e) {
        g_err = e.what();
        trg_destroy(s);
        return e.code;
    }
    *out = s;
    return TRG_OK;
}

int trg_destroy(trg_state *s) {
    if (!s) return TRG_OK;
    (void)hipSetDevice(s->opt.device);
    if (s->st) (void)hipStreamSynchronize(s->st);
    else (void)hipDeviceSynchronize();
    if (s->phi) (void)hipFree(s->phi);
    if (s->psi) (void)hipFree(s->psi);
    for (int t = 0; t < 2; ++t) {
        if (s->dphi[t]) (void)hipFree(s->dphi[t]);
        if (s->dpsi[t]) (void)hipFree(s->dpsi[t]);
    }
    if (s->dscal) (void)hipFree(s->dscal);
    if (s->dint) (void)hipFree(s->dint);
    if (s->dspec) (void)hipFree(s->dspec);
    if (s->bak) (void)hipFree(s->bak);
    delete s;
    return TRG_OK;
}

int tensor_init(trg_state *s, int model, double beta, double h, int D) {
    if (!s) return TRG_E_INVALID;
    if (model != TRG_MODEL_ISING || !(beta >= 0.0) || !std::isfinite(beta) || !std::isfinite(h) || D < 2)
        return TRG_E_INVALID;
    try {
        DevGuard g(s->opt.device);
        const int d = s->opt.dim;
        // legs D^d, bond r_bond D (ILO keeps r_bond D bond values)
        size_t cap = (size_t)std::max(s->opt.r_bond * D, 2);
        for (int i = 0; i < d; ++i) cap *= (size_t)std::max(D, 2);
        // the sketch's Philox counter packs the bond index in 8 bits; QRs are at most 512 wide
        TRG_REQUIRE((long)s->opt.r_bond * D <= 256 && (long)s->opt.sketch_mult * D <= 512, TRG_E_UNSUPPORTED,
                    "tensor_init: needs r_bond * D <= 256 and sketch_mult * D <= 512");
        const int ntan = ((s->opt.tangents & TRG_TAN_BETA) ? 1 : 0) + ((s->opt.tangents & TRG_TAN_H) ? 1 : 0);
        TRG_REQUIRE(!(s->opt.tangents & TRG_TAN_BETA) || beta > 0.0, TRG_E_INVALID,
                    "tensor_init: the beta tangent needs beta > 0 (the CP factor sqrt(sinh beta) is not "
                    "differentiable at 0)");
        s->init = false;   // set again only once the new state is complete
        if (ntan > 0 && (cap > s->cap_tan || !s->dphi[ntan - 1])) {
            if (s->st) (void)hipStreamSynchronize(s->st);
            for (int t = 0; t < 2; ++t) {
                if (s->dphi[t]) (void)hipFree(s->dphi[t]);
                if (s->dpsi[t]) (void)hipFree(s->dpsi[t]);
                s->dphi[t] = s->dpsi[t] = nullptr;
            }
            s->cap_tan = 0;
            for (int t = 0; t < ntan; ++t) {
                if (hipMalloc(&s->dphi[t], cap * sizeof(double)) != hipSuccess ||
                    hipMalloc(&s->dpsi[t], cap * sizeof(double)) != hipSuccess) {
                    (void)hipGetLastError();
                    for (int u = 0; u < 2; ++u) {
                        if (s->dphi[u]) (void)hipFree(s->dphi[u]);
                        if (s->dpsi[u]) (void)hipFree(s->dpsi[u]);
                        s->dphi[u] = s->dpsi[u] = nullptr;
                    }
                    throw Error(TRG_E_NOMEM, "tensor_init: cannot allocate the impurity tangents");
                }
            }
            s->cap_tan = cap;
        }
        if (cap > s->cap_state) {
            if (s->st) (void)hipStreamSynchronize(s->st);
            if (s->phi) (void)hipFree(s->phi);
            if (s->psi) (void)hipFree(s->psi);
            s->phi = s->psi = nullptr;
            s->cap_state = 0;
            s->dims.clear();
            s->chi = 0;
            if (hipMalloc(&s->phi, cap * sizeof(double)) != hipSuccess ||
                hipMalloc(&s->psi, cap * sizeof(double)) != hipSuccess) {
                (void)hipGetLastError();
                if (s->phi) (void)hipFree(s->phi);
                if (s->psi) (void)hipFree(s->psi);
                s->phi = s->psi = nullptr;
                throw Error(TRG_E_NOMEM, "tensor_init: cannot allocate the D^5 state tensors");
            }
            s->cap_state = cap;
        }
        // CP form: Phi[i_1..i_d, a] = e^{h s_a} prod W[a, i_mu], Psi = prod W[a, j_mu]
        const double cb = std::sqrt(std::cosh(beta)), sb = std::sqrt(std::sinh(beta));
        const double w[2][2] = {{cb, sb}, {cb, -sb}};
        const int F = 1 << d;
        std::vector<double> phi(F * 2), psi(F * 2);
        for (int a = 0; a < 2; ++a) {
            double fa = std::exp(h * (a == 0 ? 1.0 : -1.0));
            for (int idx = 0; idx < F; ++idx) {
                double prod = 1.0;
                for (int mu = 0; mu < d; ++mu) prod *= w[a][(idx >> (d - 1 - mu)) & 1];
                psi[idx * 2 + a] = prod;
                phi[idx * 2 + a] = fa * prod;
            }
        }
        hipStream_t st = s->st;
        TRG_HIP_CHECK(hipMemcpyAsync(s->phi, phi.data(), phi.size() * sizeof(double), hipMemcpyHostToDevice, st));
        TRG_HIP_CHECK(hipMemcpyAsync(s->psi, psi.data(), psi.size() * sizeof(double), hipMemcpyHostToDevice, st));
        // impurity tangents of the CP factors: d/dbeta differentiates every W (product
        // rule over the legs), d/dh brings down s_a in Phi
        std::vector<std::vector<double>> tphi, tpsi;
        int kinds[2], nk = 0;
        if (s->opt.tangents & TRG_TAN_BETA) kinds[nk++] = TRG_TAN_BETA;
        if (s->opt.tangents & TRG_TAN_H) kinds[nk++] = TRG_TAN_H;
        for (int t = 0; t < nk; ++t) {
            std::vector<double> dp(F * 2, 0.0), dq(F * 2, 0.0);
            for (int a = 0; a < 2; ++a) {
                const double sa = a == 0 ? 1.0 : -1.0, fa = std::exp(h * sa);
                for (int idx = 0; idx < F; ++idx) {
                    double prod = 1.0, dprod = 0.0;
                    for (int mu = 0; mu < d; ++mu) {
                        const int i = (idx >> (d - 1 - mu)) & 1;
                        if (kinds[t] == TRG_TAN_BETA) {
                            const double dw = i == 0 ? std::sinh(beta) / (2.0 * cb)
                                                     : (a == 0 ? 1.0 : -1.0) * std::cosh(beta) / (2.0 * sb);
                            dprod = dprod * w[a][i] + prod * dw;
                        }
                        prod *= w[a][i];
                    }
                    if (kinds[t] == TRG_TAN_BETA) {
                        dp[idx * 2 + a] = fa * dprod;
                        dq[idx * 2 + a] = dprod;
                    } else {
                        dp[idx * 2 + a] = sa * fa * prod;
                    }
                }
            }
            tphi.push_back(dp);
            tpsi.push_back(dq);
            s->tan_kind[t] = kinds[t];
        }
        for (int t = 0; t < nk; ++t) {
            TRG_HIP_CHECK(hipMemcpyAsync(s->dphi[t], tphi[t].data(), tphi[t].size() * sizeof(double),
                                         hipMemcpyHostToDevice, st));
            TRG_HIP_CHECK(hipMemcpyAsync(s->dpsi[t], tpsi[t].data(), tpsi[t].size() * sizeof(double),
                                         hipMemcpyHostToDevice, st));
        }
        double zero[2] = {0.0, 0.0};
        int izero[4] = {0, 0, 0, 0};   // status, saved status, step index
        TRG_HIP_CHECK(hipMemcpyAsync(s->dscal, zero, sizeof(zero), hipMemcpyHostToDevice, st));
        TRG_HIP_CHECK(hipMemcpyAsync(s->dint, izero, sizeof(izero), hipMemcpyHostToDevice, st));
        TRG_HIP_CHECK(hipStreamSynchronize(st));
        s->dims.assign(d, 2);
        s->chi = 2;
        s->D = D;
        s->beta = beta;
        s->h = h;
        s->k = 0;
        s->ntan = nk;
        s->init = true;
        s->sigma_last.clear();
        s->resplit_last.clear();
        s->spec_stale = false;
        s->sweep_log.clear();
        s->gen += 1;   // graphs captured before hold the old state's buffers and shapes
    } catch (const Error &e) {
        return fail(s, e);
    } catch (const std::exception &e) {
        return fail_std(s, e);
    }
    return TRG_OK;
}

// A failed step leaves phi, psi and k as they were; the log-norm accumulator and
// the status flag are put back to their values before the step (a step adds its
// 2^-k log c_k at the re-split, before any later part can fail).
static void rollback(trg_state *s) {
    if (hipSetDevice(s->opt.device) != hipSuccess) return;
    (void)hipStreamSynchronize(s->st);
    (void)hipGetLastError();
    bool ok = hipMemcpyAsync(s->dscal, s->dscal + 3, sizeof(double), hipMemcpyDeviceToDevice, s->st) == hipSuccess &&
              hipMemcpyAsync(s->dint, s->dint + 1, sizeof(int), hipMemcpyDeviceToDevice, s->st) == hipSuccess &&
              hipStreamSynchronize(s->st) == hipSuccess;
    if (!ok) {
        // the accumulator could not be restored: the state needs a new tensor_init
        (void)hipGetLastError();
        s->init = false;
        s->err += " (state invalidated; call tensor_init)";
    }
}

static int step_common(trg_state *s, int axis, bool triad) {
    if (!s) return TRG_E_INVALID;
    if (!s->init) {
        s->err = "step before tensor_init";
        return TRG_E_STATE;
    }
    if (axis < 0 || axis >= s->opt.dim) {
        s->err = "axis out of range";
        return TRG_E_INVALID;
    }
    if (triad && s->opt.dim != 4) {
        s->err = "triad-ATRG needs dim 4";
        return TRG_E_INVALID;
    }
    int rc = TRG_OK;
    try {
        DevGuard g(s->opt.device);
        trg::do_step(s, axis, triad);
    } catch (const Error &e) {
        rc = fail(s, e);
    } catch (const std::exception &e) {
        rc = fail_std(s, e);
    }
    if (rc != TRG_OK) rollback(s);
    return rc;
}

int atrg_step(trg_state *s, int axis) { return step_common(s, axis, false); }
int triad_atrg_step(trg_state *s, int axis) { return step_common(s, axis, true); }

// ---------------------------------------------------------------- captured steps
struct trg_graph {
    trg_state *s = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    unsigned long gen = 0;
    std::vector<int> dims_in, dims_out;
    int chi_in = 0, chi_out = 0;
    size_t nsig = 0, nrsv = 0;
    long nstate = 0;   // elements of phi (and psi) when the step starts
};

int trg_graph_destroy(trg_graph *g) {
    if (!g) return TRG_OK;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    return TRG_OK;
}

// The step is recorded on a private stream (a capture cannot use the null
// stream) with the host state put back afterwards: recording runs nothing, so
// the tensors, k and the spectra stay those before the step.
int trg_graph_capture(trg_state *s, int method, int axis, trg_graph **out) {
    if (!s || !out || (method != TRG_METHOD_ATRG && method != TRG_METHOD_TRIAD)) return TRG_E_INVALID;
    *out = nullptr;
    if (!s->init) {
        s->err = "capture before tensor_init";
        return TRG_E_STATE;
    }
    if (axis < 0 || axis >= s->opt.dim) {
        s->err = "axis out of range";
        return TRG_E_INVALID;
    }
    trg_graph *g = new (std::nothrow) trg_graph();
    if (!g) return TRG_E_NOMEM;
    g->s = s;
    g->gen = s->gen;
    g->dims_in = s->dims;
    g->chi_in = s->chi;
    const hipStream_t user = s->st;
    hipStream_t cs = nullptr;
    bool capturing = false;
    int rc = TRG_OK;
    try {
        DevGuard dg(s->opt.device);
        TRG_HIP_CHECK(hipStreamSynchronize(user));
        g->nstate = s->chi;
        for (int v : s->dims) g->nstate *= v;
        const size_t need = (size_t)(2 + 2 * s->ntan) * s->cap_state;
        if (s->bak_cap < need) {
            if (s->bak) (void)hipFree(s->bak);
            s->bak = nullptr;
            s->bak_cap = 0;
            if (hipMalloc(&s->bak, need * sizeof(double)) != hipSuccess) {
                (void)hipGetLastError();
                throw Error(TRG_E_NOMEM, "graph capture: backup of the state could not be allocated");
            }
            s->bak_cap = need;
        }
        TRG_HIP_CHECK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        s->st = cs;
        s->capture_on = true;
        s->ar.freeze(true);
        TRG_HIP_CHECK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        capturing = true;
        trg::do_step(s, axis, method == TRG_METHOD_TRIAD);
        capturing = false;
        TRG_HIP_CHECK(hipStreamEndCapture(cs, &g->graph));
        g->dims_out = s->dims;
        g->chi_out = s->chi;
        g->nsig = s->nsig;
        g->nrsv = s->nrsv;
        TRG_HIP_CHECK(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
    } catch (const Error &e) {
        rc = fail(s, e);
    } catch (const std::exception &e) {
        rc = fail_std(s, e);
    }
    if (capturing) {
        hipGraph_t partial = nullptr;
        if (hipStreamEndCapture(cs, &partial) == hipSuccess && partial) (void)hipGraphDestroy(partial);
        (void)hipGetLastError();
    }
    s->capture_on = false;
    s->ar.freeze(false);
    s->st = user;
    s->dims = g->dims_in;
    s->chi = g->chi_in;
    if (cs) (void)hipStreamDestroy(cs);
    if (rc != TRG_OK) {
        trg_graph_destroy(g);
        return rc;
    }
    *out = g;
    return TRG_OK;
}

int trg_graph_launch(trg_graph *g, int check) {
    if (!g || !g->s || !g->exec) return TRG_E_INVALID;
    trg_state *s = g->s;
    if (!s->init || s->gen != g->gen) {
        s->err = "graph recorded before the last tensor_init or trg_release_workspace";
        return TRG_E_STATE;
    }
    if (s->dims != g->dims_in || s->chi != g->chi_in) {
        s->err = "graph recorded at other shapes";
        return TRG_E_STATE;
    }
    if (s->k >= 0xFFFF) {
        s->err = "step index past the sketch counter's 16 bits";
        return TRG_E_UNSUPPORTED;
    }
    const size_t nsig0 = s->nsig, nrsv0 = s->nrsv;
    const bool stale0 = s->spec_stale;
    try {
        DevGuard dg(s->opt.device);
        TRG_HIP_CHECK(hipGraphLaunch(g->exec, s->st));
        if (check) {
            int status = 0;
            TRG_HIP_CHECK(hipMemcpyAsync(&status, s->dint, sizeof(int), hipMemcpyDeviceToHost, s->st));
            TRG_HIP_CHECK(hipStreamSynchronize(s->st));
            if (status != 0) {
                // back to the state the step started from (it kept a copy)
                const size_t n = (size_t)g->nstate;
                trg::copy(s->phi, s->bak, n, s->st);
                trg::copy(s->psi, s->bak + s->cap_state, n, s->st);
                for (int t = 0; t < s->ntan; ++t) {
                    trg::copy(s->dphi[t], s->bak + (2 + 2 * t) * s->cap_state, n, s->st);
                    trg::copy(s->dpsi[t], s->bak + (3 + 2 * t) * s->cap_state, n, s->st);
                }
                trg::copy(s->dspec, s->dspec + 2048, 2048, s->st);
                hipLaunchKernelGGL(trg::step_undo_kernel, dim3(1), dim3(1), 0, s->st, s->dscal, s->dint);
                TRG_HIP_CHECK(hipGetLastError());
                TRG_HIP_CHECK(hipStreamSynchronize(s->st));
                trg::check_status(status);
            }
        }
    } catch (const Error &e) {
        s->nsig = nsig0;
        s->nrsv = nrsv0;
        s->spec_stale = stale0;
        return fail(s, e);
    }
    s->k += 1;
    s->dims = g->dims_out;
    s->chi = g->chi_out;
    s->nsig = g->nsig;
    s->nrsv = g->nrsv;
    s->spec_stale = true;
    return TRG_OK;
}

int log_z_per_site(trg_state *s, double *out) {
    if (!s || !out) return TRG_E_INVALID;
    if (!s->init) return TRG_E_STATE;
    try {
        DevGuard g(s->opt.device);
        long n = (long)s->chi;
        for (int v : s->dims) n *= v;
        double *part = s->dscal + 1024;
        hipLaunchKernelGGL(trg::dot_partial_kernel, dim3(1024), dim3(256), 0, s->st, s->phi, s->psi, n, part);
        hipLaunchKernelGGL(trg::sum_kernel, dim3(1), dim3(256), 0, s->st, part, 1024, s->dscal + 1);
        double hs[2];
        int status = 0;
        TRG_HIP_CHECK(hipMemcpyAsync(hs, s->dscal, sizeof(hs), hipMemcpyDeviceToHost, s->st));
        TRG_HIP_CHECK(hipMemcpyAsync(&status, s->dint, sizeof(int), hipMemcpyDeviceToHost, s->st));
        TRG_HIP_CHECK(hipStreamSynchronize(s->st));
        trg::check_status(status);
        if (!(hs[1] > 0.0) || !std::isfinite(hs[1])) throw Error(TRG_E_NUMERICAL, "final trace is not positive");
        *out = hs[0] + std::ldexp(std::log(hs[1]), -s->k);
    } catch (const Error &e) {
        return fail(s, e);
    } catch (const std::exception &e) {
        return fail_std(s, e);
    }
    return TRG_OK;
}

int impurity_derivatives(trg_state *s, double *dbeta, double *dh) {
    if (!s) return TRG_E_INVALID;
    if (!s->init) return TRG_E_STATE;
    if (s->ntan == 0) {
        s->err = "impurity_derivatives: the state carries no tangents (trg_options.tangents)";
        return TRG_E_STATE;
    }
    try {
        DevGuard g(s->opt.device);
        long n = (long)s->chi;
        for (int v : s->dims) n *= v;
        // Tr T and Tr dT = sum dPhi Psi + Phi dPsi, fixed-order partial sums
        double *part = s->dscal + 1024;
        double tr[3] = {0.0, 0.0, 0.0};
        hipLaunchKernelGGL(trg::dot_partial_kernel, dim3(1024), dim3(256), 0, s->st, s->phi, s->psi, n, part);
        hipLaunchKernelGGL(trg::sum_kernel, dim3(1), dim3(256), 0, s->st, part, 1024, s->dscal + 8);
        for (int t = 0; t < s->ntan; ++t) {
            hipLaunchKernelGGL(trg::dot_partial_kernel, dim3(512), dim3(256), 0, s->st, s->dphi[t], s->psi, n, part);
            hipLaunchKernelGGL(trg::dot_partial_kernel, dim3(512), dim3(256), 0, s->st, s->phi, s->dpsi[t], n,
                               part + 512);
            hipLaunchKernelGGL(trg::sum_kernel, dim3(1), dim3(256), 0, s->st, part, 1024, s->dscal + 9 + t);
        }
        TRG_HIP_CHECK(hipGetLastError());
        TRG_HIP_CHECK(hipMemcpyAsync(tr, s->dscal + 8, sizeof(tr), hipMemcpyDeviceToHost, s->st));
        TRG_HIP_CHECK(hipStreamSynchronize(s->st));
        if (!(tr[0] > 0.0) || !std::isfinite(tr[0])) throw Error(TRG_E_NUMERICAL, "final trace is not positive");
        const double nan = std::nan("");
        if (dbeta) *dbeta = nan;
        if (dh) *dh = nan;
        for (int t = 0; t < s->ntan; ++t) {
            const double v = std::ldexp(tr[1 + t] / tr[0], -s->k);
            if (s->tan_kind[t] == TRG_TAN_BETA && dbeta) *dbeta = v;
            if (s->tan_kind[t] == TRG_TAN_H && dh) *dh = v;
        }
    } catch (const Error &e) {
        return fail(s, e);
    } catch (const std::exception &e) {
        return fail_std(s, e);
    }
    return TRG_OK;
}

int gu_wen_x(trg_state *s, int axis, double *out) {
    if (!s || !out) return TRG_E_INVALID;
    if (!s->init) return TRG_E_STATE;
    if (axis < 0 || axis >= (int)s->dims.size()) {
        s->err = "gu_wen_x: axis out of range";
        return TRG_E_INVALID;
    }
    trg::Arena::Mark mk = s->ar.mark();
    try {
        DevGuard g(s->opt.device);
        trg::Ctx c;
        c.st = s->st;
        c.ar = &s->ar;
        c.prec = trg::P_FP64;
        trg::DT phi, psi;
        phi.p = s->phi;
        psi.p = s->psi;
        phi.d = s->dims;
        phi.d.push_back(s->chi);
        psi.d = phi.d;
        // A[k, l] = sum over the other legs and the bond of Phi[.., k, .., g] Psi[.., l, .., g]
        std::string la, lb;
        for (int i = 0; i < (int)s->dims.size(); ++i) {
            la += i == axis ? 'k' : (char)('a' + i);
            lb += i == axis ? 'l' : (char)('a' + i);
        }
        la += 'g';
        lb += 'g';
        trg::DT A = trg::contract(c, phi, la, psi, lb, "kl");
        const int n = s->dims[axis];
        hipLaunchKernelGGL(trg::gu_wen_kernel, dim3(1), dim3(256), 0, s->st, A.p, n, s->dscal + 4);
        TRG_HIP_CHECK(hipGetLastError());
        double tr[2];
        TRG_HIP_CHECK(hipMemcpyAsync(tr, s->dscal + 4, sizeof(tr), hipMemcpyDeviceToHost, s->st));
        TRG_HIP_CHECK(hipStreamSynchronize(s->st));
        s->ar.release(mk);
        if (!(tr[1] > 0.0) || !std::isfinite(tr[0]) || !std::isfinite(tr[1]))
            throw Error(TRG_E_NUMERICAL, "gu_wen_x: Tr(A A) is not positive and finite");
        *out = tr[0] * tr[0] / tr[1];
    } catch (const Error &e) {
        (void)hipStreamSynchronize(s->st);
        s->ar.release(mk);
        return fail(s, e);
    } catch (const std::exception &e) {
        (void)hipStreamSynchronize(s->st);
        s->ar.release(mk);
        return fail_std(s, e);
    }
    return TRG_OK;
}

int trg_release_workspace(trg_state *s) {
    if (!s) return TRG_E_INVALID;
    try {
        DevGuard g(s->opt.device);
        TRG_HIP_CHECK(hipStreamSynchronize(s->st));
        s->ar.trim();
        s->gen += 1;   // captured graphs held workspace addresses
    } catch (const Error &e) {
        return fail(s, e);
    }
    return TRG_OK;
}

int trg_shape(trg_state *s, int *dims, int *chi, int *steps) {
    if (!s) return TRG_E_INVALID;
    if (!s->init) return TRG_E_STATE;
    if (dims)
        for (size_t i = 0; i < s->dims.size(); ++i) dims[i] = s->dims[i];
    if (chi) *chi = s->chi;
    if (steps) *steps = s->k;
    return TRG_OK;
}

size_t trg_export_size(trg_state *s, int which) {
    if (!s || !s->init) return 0;
    size_t n = (size_t)s->chi;
    for (int v : s->dims) n *= v;
    if (which == TRG_T_PHI || which == TRG_T_PSI) return n * sizeof(double);
    if (which == TRG_T_SIGMA) return (s->spec_stale ? s->nsig : s->sigma_last.size()) * sizeof(double);
    if (which == TRG_T_RESPLIT) return (s->spec_stale ? s->nrsv : s->resplit_last.size()) * sizeof(double);
    return 0;
}

int trg_export(trg_state *s, int which, void *dst, size_t bytes) {
    if (!s || !dst) return TRG_E_INVALID;
    if (!s->init) return TRG_E_STATE;
    size_t need = trg_export_size(s, which);
    if (need == 0 || bytes != need) return TRG_E_INVALID;
    try {
        DevGuard g(s->opt.device);
        if ((which == TRG_T_SIGMA || which == TRG_T_RESPLIT) && s->spec_stale) {
            // spectra of a replayed step: from the device copies
            std::vector<double> sig(s->nsig), rsv(s->nrsv);
            TRG_HIP_CHECK(hipMemcpyAsync(sig.data(), s->dspec, sizeof(double) * s->nsig, hipMemcpyDeviceToHost, s->st));
            TRG_HIP_CHECK(hipMemcpyAsync(rsv.data(), s->dspec + 1024, sizeof(double) * s->nrsv, hipMemcpyDeviceToHost,
                                         s->st));
            TRG_HIP_CHECK(hipStreamSynchronize(s->st));
            s->sigma_last = sig;
            s->resplit_last = rsv;
            s->spec_stale = false;
        }
        if (which == TRG_T_SIGMA) {
            std::memcpy(dst, s->sigma_last.data(), need);
            return TRG_OK;
        }
        if (which == TRG_T_RESPLIT) {
            std::memcpy(dst, s->resplit_last.data(), need);
            return TRG_OK;
        }
        const double *src = which == TRG_T_PHI ? s->phi : s->psi;
        TRG_HIP_CHECK(hipMemcpyAsync(dst, src, need, hipMemcpyDeviceToHost, s->st));
        TRG_HIP_CHECK(hipStreamSynchronize(s->st));
    } catch (const Error &e) {
        return fail(s, e);
    }
    return TRG_OK;
}

int trg_set_timing(trg_state *s, int enable) {
    if (!s) return TRG_E_INVALID;
    s->timing = enable != 0;
    return TRG_OK;
}

int trg_kernel_time(trg_state *s, double *ms, double *flops, int *launches) {
    if (!s) return TRG_E_INVALID;
    if (ms) *ms = s->t_ms;
    if (flops) *flops = s->t_flops;
    if (launches) *launches = s->t_launch;
    s->t_ms = s->t_flops = 0.0;
    s->t_launch = 0;
    return TRG_OK;
}

const char *trg_strerror(int code) {
    switch (code) {
        case TRG_OK: return "ok";
        case TRG_E_INVALID: return "invalid argument";
        case TRG_E_STATE: return "state not initialised";
        case TRG_E_NOMEM: return "out of device memory or workspace cap";
        case TRG_E_NUMERICAL: return "numerical failure";
        case TRG_E_HIP: return "HIP runtime error";
        case TRG_E_UNSUPPORTED: return "unsupported shape";
        case TRG_E_MULTIPLET: return "truncation cut inside a multiplet too large for the canonical basis";
        default: return "unknown error";
    }
}

const char *trg_last_error(trg_state *s) { return s ? s->err.c_str() : g_err.c_str(); }

int trg_qr(const double *A, int64_t m, int n, double *Q, double *R, void *stream) {
    if (!A || !Q || !R || n < 1 || n > 64 || m < n) {
        g_err = "trg_qr: needs non-NULL A, Q, R, 1 <= n <= 64 and m >= n";
        return TRG_E_INVALID;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    double *ws = nullptr;
    if (hipMalloc(&ws, trg::tsqr_ws_doubles(m, n) * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        g_err = "trg_qr: cannot allocate the QR scratch";
        return TRG_E_NOMEM;
    }
    int rc = TRG_OK;
    try {
        trg::tsqr(A, m, n, Q, R, ws, st);
        TRG_HIP_CHECK(hipStreamSynchronize(st));
    } catch (const Error &e) {
        g_err = e.what();
        rc = e.code;
        (void)hipStreamSynchronize(st);
    }
    (void)hipFree(ws);
    return rc;
}

}  // extern "C"

// ------------------------------------------------- allocation-free thin QR
namespace {
// Scratch of trg_qr_noalloc: 8 Mi doubles (64 MiB) in the code object's device
// globals, one copy per GPU the library runs on, held until the process ends.
// Host code never passes the array's name to a kernel (on the host it is only
// a stand-in symbol); it uses the device address that hipGetSymbolAddress
// returns, fetched once per device and kept in qr_scratch_dev.
constexpr size_t kQrScratchDoubles = size_t(8) << 20;
static __device__ __align__(256) double qr_scratch[kQrScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_qr_scratch_mu;
double *qr_scratch_dev[kMaxDevices] = {};

// Device address of qr_scratch on the current device (looked up on the first
// call on that device); nullptr with g_err set on failure.
double *qr_scratch_ptr() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        g_err = "trg_qr_noalloc: no usable current HIP device";
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_qr_scratch_mu);
    if (!qr_scratch_dev[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(qr_scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            g_err = std::string("trg_qr_noalloc: hipGetSymbolAddress of the scratch failed: ") +
                    hipGetErrorString(e);
            return nullptr;
        }
        qr_scratch_dev[dev] = static_cast<double *>(p);
    }
    return qr_scratch_dev[dev];
}
}  // namespace

extern "C" {

int trg_qr_noalloc(const double *A, int64_t m, int n, double *Q, double *R, void *stream) {
    if (!A || !Q || !R || n < 1 || n > 64 || m < n) {
        g_err = "trg_qr_noalloc: needs non-NULL A, Q, R, 1 <= n <= 64 and m >= n";
        return TRG_E_INVALID;
    }
    const size_t need = trg::tsqr_ws_doubles(m, n);
    if (need > kQrScratchDoubles) {
        g_err = "trg_qr_noalloc: an m x n QR needs " + std::to_string(need) +
                " doubles of scratch, above the fixed " + std::to_string(kQrScratchDoubles) +
                " (every m * n <= 2097152 fits); use trg_qr";
        return TRG_E_UNSUPPORTED;
    }
    double *ws = qr_scratch_ptr();
    if (!ws) return TRG_E_HIP;
    try {
        // every scratch element the kernels read is written earlier in the
        // same call, so the previous call's contents need no clearing
        trg::tsqr(A, m, n, Q, R, ws, static_cast<hipStream_t>(stream));
    } catch (const Error &e) {
        g_err = e.what();
        return e.code;
    }
    return TRG_OK;
}

}  // extern "C"

// ====================================================================== self-tests
namespace {
struct Scratch {
    trg::Arena ar;
    trg::Ctx c;
    Scratch() {
        c.st = nullptr;
        c.ar = &ar;
        c.prec = trg::P_FP64;
    }
    double *up(const double *h, size_t n) {
        double *d = ar.dalloc(n);
        TRG_HIP_CHECK(hipMemcpy(d, h, n * sizeof(double), hipMemcpyHostToDevice));
        return d;
    }
    void down(double *h, const double *d, size_t n) {
        TRG_HIP_CHECK(hipMemcpy(h, d, n * sizeof(double), hipMemcpyDeviceToHost));
    }
};
}  // namespace

extern "C" {

int trg_selftest_gemm(int precision, int ta, int tb, int M, int N, int K, int batch, const double *A,
                      const double *B, double *C) {
    if (!A || !B || !C || M < 1 || N < 1 || K < 0 || batch < 1 || precision < 0 || precision > 3)
        return TRG_E_INVALID;
    try {
        Scratch s;
        size_t na = (size_t)M * K * batch, nb = (size_t)K * N * batch, nc = (size_t)M * N * batch;
        double *a = s.up(A, std::max<size_t>(na, 1)), *b = s.up(B, std::max<size_t>(nb, 1));
        double *c = s.ar.dalloc(nc);
        trg::GemmArgs g{};
        g.M = M; g.N = N; g.K = K; g.batch = batch;
        g.A = a; g.sAr = ta ? 1 : K; g.sAk = ta ? M : 1; g.sAb = (long)M * K;
        g.B = b; g.sBk = tb ? 1 : N; g.sBn = tb ? K : 1; g.sBb = (long)K * N;
        g.C = c; g.sCr = N; g.sCn = 1; g.sCb = (long)M * N;
        g.alpha = 1.0; g.beta = 0.0;
        if (K == 0) {
            trg::fill(c, nc, 0.0, nullptr);
        } else if (precision == trg::P_BF16X6) {
            // the coarse-graining path of BF16X6: both operands split into planes, then
            // gemm_planes with K split in slices of at least 64
            const int Kp = (K + 31) / 32 * 32;
            void *ap = s.ar.alloc(trg::bf16_planes_elems(M, Kp, batch) * 2);
            void *bp = s.ar.alloc(trg::bf16_planes_elems(N, Kp, batch) * 2);
            trg::split_bf16x3(a, g.sAr, g.sAk, g.sAb, M, K, batch, Kp, ap, nullptr);
            trg::split_bf16x3(b, g.sBn, g.sBk, g.sBb, N, K, batch, Kp, bp, nullptr);
            trg::PlaneGemm h{};
            h.A = ap; h.sAp = (long)batch * M * Kp; h.sAb = (long)M * Kp;
            h.B = bp; h.sBp = (long)batch * N * Kp; h.sBb = (long)N * Kp;
            h.M = M; h.N = N; h.Kp = Kp; h.batch = batch;
            h.inner = Kp >= 128 ? 2 : 1;
            h.kslice = (Kp / h.inner + 31) / 32 * 32;
            h.inner = (Kp + h.kslice - 1) / h.kslice;
            double *w = s.ar.dalloc(nc * h.inner);
            h.C = w; h.sCr = N; h.sCn = 1; h.sCb = (long)h.inner * M * N; h.sCi = (long)M * N;
            h.alpha = 1.0; h.beta = 0.0;
            trg::gemm_planes(h, nullptr);
            for (int bt = 0; bt < batch; ++bt)
                trg::sum_slices(w + (long)bt * h.inner * M * N, h.inner, M, N, c + (long)bt * M * N, N, 1, nullptr);
        } else {
            trg::gemm(g, (trg::Prec)precision, nullptr);
        }
        s.down(C, c, nc);
    } catch (const Error &e) {
        g_err = e.what();
        return e.code;
    }
    return TRG_OK;
}

int trg_selftest_permute(int nd, const int *dims, const int *perm, const double *src, double *dst) {
    if (!dims || !perm || !src || !dst || nd < 1 || nd > 8) return TRG_E_INVALID;
    std::vector<int> dv(dims, dims + nd), pv(perm, perm + nd), seen(nd, 0);
    size_t total = 1;
    for (int i = 0; i < nd; ++i) {
        if (dv[i] < 1 || pv[i] < 0 || pv[i] >= nd || seen[pv[i]]++) return TRG_E_INVALID;
        total *= (size_t)dv[i];
    }
    try {
        Scratch s;
        double *a = s.up(src, total);
        double *b = s.ar.dalloc(total);
        trg::permute(a, b, dv, pv, nullptr);
        s.down(dst, b, total);
    } catch (const Error &e) {
        g_err = e.what();
        return e.code;
    }
    return TRG_OK;
}

int trg_selftest_tsqr(int m, int n, const double *A, double *Q, double *R) {
    if (!A || !Q || !R || n < 1 || m < n) return TRG_E_INVALID;
    try {
        Scratch s;
        double *a = s.up(A, (size_t)m * n);
        double *q = s.ar.dalloc((size_t)m * n), *r = s.ar.dalloc((size_t)n * n);
        double *ws = s.ar.dalloc(trg::tsqr_ws_doubles(m, n));
        trg::tsqr(a, m, n, q, r, ws, nullptr);
        s.down(Q, q, (size_t)m * n);
        s.down(R, r, (size_t)n * n);
    } catch (const Error &e) {
        g_err = e.what();
        return e.code;
    }
    return TRG_OK;
}

int trg_selftest_svd(int m, int n, const double *A, double *U, double *S, double *V, int *sweeps) {
    if (!A || !U || !S || !V || n < 1 || m < n) return TRG_E_INVALID;
    try {
        Scratch s;
        std::vector<double> at((size_t)m * n);
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < n; ++j) at[(size_t)j * m + i] = A[(size_t)i * n + j];
        double *ut = s.up(at.data(), at.size());
        double *vt = s.ar.dalloc((size_t)n * n), *work = s.ar.dalloc((size_t)n + 1);
        double *sv = s.ar.dalloc(n), *us = s.ar.dalloc((size_t)m * n), *vs = s.ar.dalloc((size_t)n * n);
        int *flags = static_cast<int *>(s.ar.alloc(64 * sizeof(int)));
        trg::JacobiBatch jb{1, m, n, ut, vt, (long)m * n, (long)n * n};
        int sw = trg::jacobi_svd(jb, 80, flags, work, nullptr);
        trg::jacobi_finish(jb, sv, us, vs, work, nullptr);
        s.down(U, us, (size_t)m * n);
        s.down(S, sv, n);
        s.down(V, vs, (size_t)n * n);
        if (sweeps) *sweeps = sw;
    } catch (const Error &e) {
        g_err = e.what();
        return e.code;
    }
    return TRG_OK;
}

int trg_selftest_eigh(int count, int n, const double *K, double *lam, double *V, int *sweeps) {
    if (!K || !lam || !V || n < 1 || count < 1) return TRG_E_INVALID;
    try {
        Scratch s;
        const size_t nn = (size_t)count * n * n;
        double *k = s.up(K, nn);
        double *l = s.ar.dalloc((size_t)count * n), *v = s.ar.dalloc(nn);
        double *ws = s.ar.dalloc(trg::eigh_ws_doubles(count, n));
        int *iws = static_cast<int *>(s.ar.alloc(trg::eigh_iws_ints(count, n) * sizeof(int)));
        int sw = trg::eigh_sym(k, count, n, l, v, ws, iws, 100, nullptr);
        s.down(lam, l, (size_t)count * n);
        s.down(V, v, nn);
        if (sweeps) *sweeps = sw;
    } catch (const Error &e) {
        g_err = e.what();
        return e.code;
    }
    return TRG_OK;
}

int trg_selftest_pchol(int count, int n, const double *K, double tol, double *X, int *rank) {
    if (!K || !X || !rank || n < 1 || count < 1 || !(tol >= 0.0 && tol < 1.0)) return TRG_E_INVALID;
    if (n > 1024) return TRG_E_UNSUPPORTED;
    try {
        Scratch s;
        const size_t nn = (size_t)count * n * n;
        double *k = s.up(K, nn), *x = s.ar.dalloc(nn);
        int *iws = reinterpret_cast<int *>(s.ar.dalloc((trg::pchol_iws_ints(count, n) + 1) / 2));
        if (!trg::pivoted_cholesky_batched(k, count, n, x, iws, nullptr, tol, rank)) {
            g_err = "pivoted Cholesky: pivot not finite (or not positive with tol = 0)";
            return TRG_E_NUMERICAL;
        }
        s.down(X, x, nn);
    } catch (const Error &e) {
        g_err = e.what();
        return e.code;
    }
    return TRG_OK;
}

int trg_selftest_gram_eig(int count, int n, const double *K, double *lam, double *V, int *sweeps) {
    if (!K || !lam || !V || n < 1 || count < 1) return TRG_E_INVALID;
    if (n > 1024) return TRG_E_UNSUPPORTED;
    try {
        Scratch s;
        const size_t nn = (size_t)count * n * n;
        double *k = s.up(K, nn);
        double *l = s.ar.dalloc((size_t)count * n), *v = s.ar.dalloc(nn);
        int sw = 0;
        if (!trg::gram_eig_pchol(s.c, k, count, n, 100, l, v, &sw)) {
            g_err = "gram eigen-decomposition: pivot not finite";
            return TRG_E_NUMERICAL;
        }
        s.down(lam, l, (size_t)count * n);
        s.down(V, v, nn);
        if (sweeps) *sweeps = sw;
    } catch (const Error &e) {
        g_err = e.what();
        return e.code;
    }
    return TRG_OK;
}

int trg_selftest_sketch(uint64_t seed, int step, uint32_t instance, int chi, int j1, int j2, int j3, int m,
                        double *out) {
    if (!out || chi < 1 || j1 < 1 || j2 < 1 || j3 < 1 || m < 1) return TRG_E_INVALID;
    try {
        Scratch s;
        size_t n = (size_t)chi * j1 * j2 * j3 * m;
        double *o = s.ar.dalloc(n);
        trg::philox_sketch(o, seed, step, instance, {j1, j2, j3}, chi, m, 0, nullptr);
        s.down(out, o, n);
    } catch (const Error &e) {
        g_err = e.what();
        return e.code;
    }
    return TRG_OK;
}

}  // extern "C"
