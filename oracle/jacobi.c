/* The oracle's own Jacobi eigensolver and SVD, in plain C (FP64).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the Python oracle through ctypes; the
 * product path never links or calls it.  Shares no code with the HIP path.
 *
 * oracle_jacobi_eigh: cyclic two-sided Jacobi for a symmetric n x n matrix
 *   (Rutishauser's rotation formulas).  Each sweep visits every pair (p, q)
 *   once, in the round-robin order of the circle method; the disjoint pairs
 *   of one round are rotated simultaneously.  A pair is skipped when
 *   |a_pq| <= n eps sqrt|a_pp| sqrt|a_qq|; the iteration ends after the first
 *   sweep without a rotation.
 *
 * oracle_jacobi_svd: one-sided (Hestenes) Jacobi on the columns of an m x n
 *   matrix stored column by column (ut[j*m + i] = A[i][j]); the accumulated
 *   right rotations go to vt (row j = column j of V).  A pair is rotated
 *   while |u_p . u_q| > sqrt(m) eps |u_p| |u_q|; a column whose squared norm
 *   is below 1e-280 (the caller scales the matrix to unit max) counts as zero.
 *
 * Both return the number of sweeps used, or -1 without convergence.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define EPS 2.220446049250313e-16

/* circle-method schedule: player 0 stays at position 0, the others rotate by
 * one position per round; position i meets position m-1-i. */
static int player_at(int m, int i, int r) { return i == 0 ? 0 : 1 + ((i - 1 + r) % (m - 1)); }

static void round_pairs(int m, int r, int *ps, int *qs, int *np, int n) {
    int cnt = 0;
    for (int i = 0; i < m / 2; ++i) {
        int a = player_at(m, i, r), b = player_at(m, m - 1 - i, r);
        if (a < n && b < n) {
            ps[cnt] = a < b ? a : b;
            qs[cnt] = a < b ? b : a;
            ++cnt;
        }
    }
    *np = cnt;
}

int oracle_jacobi_eigh(int n, double *a, double *v, int max_sweeps) {
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) v[(size_t)i * n + j] = (i == j) ? 1.0 : 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            double s = 0.5 * (a[(size_t)i * n + j] + a[(size_t)j * n + i]);
            a[(size_t)i * n + j] = s;
            a[(size_t)j * n + i] = s;
        }
    if (n < 2) return 0;
    int m = n + (n & 1);
    int *ps = malloc(sizeof(int) * m), *qs = malloc(sizeof(int) * m);
    double *cs = malloc(sizeof(double) * m), *sn = malloc(sizeof(double) * m);
    double *tt = malloc(sizeof(double) * m);
    double tol = n * EPS;
    int sweep;
    for (sweep = 0; sweep < max_sweeps; ++sweep) {
        int rotated = 0;
        for (int r = 0; r < m - 1; ++r) {
            int np;
            round_pairs(m, r, ps, qs, &np, n);
            int act = 0;
            for (int k = 0; k < np; ++k) {
                int p = ps[k], q = qs[k];
                double app = a[(size_t)p * n + p], aqq = a[(size_t)q * n + q], apq = a[(size_t)p * n + q];
                if (fabs(apq) <= tol * sqrt(fabs(app)) * sqrt(fabs(aqq)) || fabs(apq) < 1e-300) {
                    cs[k] = 1.0; sn[k] = 0.0; tt[k] = 0.0;
                    continue;
                }
                double theta = (aqq - app) / (2.0 * apq);
                double t = (theta == 0.0) ? 1.0
                         : copysign(1.0, theta) / (fabs(theta) + hypot(theta, 1.0));
                double c = 1.0 / sqrt(t * t + 1.0);
                cs[k] = c; sn[k] = t * c; tt[k] = t;
                act = 1;
            }
            if (!act) continue;
            rotated = 1;
            /* rows */
#pragma omp parallel for schedule(static) if (n >= 128)
            for (int k = 0; k < np; ++k) {
                if (sn[k] == 0.0) continue;
                double c = cs[k], s = sn[k];
                double *rp = a + (size_t)ps[k] * n, *rq = a + (size_t)qs[k] * n;
                for (int j = 0; j < n; ++j) {
                    double x = rp[j], y = rq[j];
                    rp[j] = c * x - s * y;
                    rq[j] = s * x + c * y;
                }
            }
            /* columns, one row at a time; eigenvector rows likewise */
#pragma omp parallel for schedule(static) if (n >= 128)
            for (int i = 0; i < n; ++i) {
                double *ri = a + (size_t)i * n, *vi = v + (size_t)i * n;
                for (int k = 0; k < np; ++k) {
                    if (sn[k] == 0.0) continue;
                    double c = cs[k], s = sn[k];
                    int p = ps[k], q = qs[k];
                    double x = ri[p], y = ri[q];
                    ri[p] = c * x - s * y;
                    ri[q] = s * x + c * y;
                    x = vi[p]; y = vi[q];
                    vi[p] = c * x - s * y;
                    vi[q] = s * x + c * y;
                }
            }
            for (int k = 0; k < np; ++k) {
                if (sn[k] == 0.0) continue;
                int p = ps[k], q = qs[k];
                a[(size_t)p * n + q] = 0.0;
                a[(size_t)q * n + p] = 0.0;
            }
        }
        if (!rotated) break;
    }
    free(ps); free(qs); free(cs); free(sn); free(tt);
    return sweep < max_sweeps ? sweep : -1;
}

int oracle_jacobi_svd(int m, int n, double *ut, double *vt, int max_sweeps) {
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) vt[(size_t)i * n + j] = (i == j) ? 1.0 : 0.0;
    if (n < 2) return 0;
    int mm = n + (n & 1);
    int *ps = malloc(sizeof(int) * mm), *qs = malloc(sizeof(int) * mm);
    double tol = sqrt((double)m) * EPS;
    int sweep;
    for (sweep = 0; sweep < max_sweeps; ++sweep) {
        int rotated = 0;
        for (int r = 0; r < mm - 1; ++r) {
            int np;
            round_pairs(mm, r, ps, qs, &np, n);
#pragma omp parallel for schedule(dynamic, 1) reduction(| : rotated) if (n >= 128)
            for (int k = 0; k < np; ++k) {
                double *up = ut + (size_t)ps[k] * m, *uq = ut + (size_t)qs[k] * m;
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int i = 0; i < m; ++i) {
                    al += up[i] * up[i];
                    be += uq[i] * uq[i];
                    ga += up[i] * uq[i];
                }
                if (al < 1e-280 || be < 1e-280 || fabs(ga) <= tol * sqrt(al) * sqrt(be)) continue;
                double zeta = (be - al) / (2.0 * ga);
                double t = (zeta == 0.0) ? 1.0
                         : copysign(1.0, zeta) / (fabs(zeta) + hypot(zeta, 1.0));
                double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
                for (int i = 0; i < m; ++i) {
                    double x = up[i], y = uq[i];
                    up[i] = c * x - s * y;
                    uq[i] = s * x + c * y;
                }
                double *vp = vt + (size_t)ps[k] * n, *vq = vt + (size_t)qs[k] * n;
                for (int i = 0; i < n; ++i) {
                    double x = vp[i], y = vq[i];
                    vp[i] = c * x - s * y;
                    vq[i] = s * x + c * y;
                }
                rotated = 1;
            }
        }
        if (!rotated) break;
    }
    free(ps); free(qs);
    return sweep < max_sweeps ? sweep : -1;
}
