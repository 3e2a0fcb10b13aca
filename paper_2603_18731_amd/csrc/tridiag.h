// Lowest eigenpair of a symmetric tridiagonal matrix on the device: Sturm-count
// multisection (kTriThreads points per round) for the eigenvalue, then inverse iteration with
// partial pivoting for its vector.  Shared by the single and the batched Lanczos.
#pragma once

#include <hip/hip_runtime.h>

namespace qsd {

constexpr int kTriThreads = 256;

// Number of eigenvalues of the symmetric tridiagonal (a, b) below x (Sturm sequence).
__device__ int sturm_count(const double *a, const double *b, int m, double x, double pivmin) {
    int c = 0;
    double q = a[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0) ++c;
    for (int i = 1; i < m; ++i) {
        q = a[i] - x - b[i - 1] * b[i - 1] / q;
        if (fabs(q) < pivmin) q = -pivmin;
        if (q < 0) ++c;
    }
    return c;
}

struct TridiagLds {
    double a[1024], b[1024];
    double lu_d[1024], lu_du[1024], lu_du2[1024], lu_dl[1024];
    int lu_piv[1024];
    double lo_s, hi_s;
    int cnt_s[kTriThreads];
};

// Lowest eigenpair of T_m (alpha[0..m), beta[0..m-1)), m <= 1024, computed by one block of
// kTriThreads threads.  tri[0] = theta, tri[1] = beta[m-1] * |s[m-1]|, tri[3 + i] = s[i].
__device__ void tridiag_lowest(const double *__restrict__ alpha, const double *__restrict__ beta, int m,
                               double *__restrict__ tri, TridiagLds &L) {
    double *a = L.a, *b = L.b;
    double &lo_s = L.lo_s, &hi_s = L.hi_s;
    int *cnt_s = L.cnt_s;
    double *lu_d = L.lu_d, *lu_du = L.lu_du, *lu_du2 = L.lu_du2, *lu_dl = L.lu_dl;
    int *lu_piv = L.lu_piv;
    for (int i = threadIdx.x; i < m; i += kTriThreads) {
        a[i] = alpha[i];
        b[i] = beta[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double lo = a[0], hi = a[0];
        double bmax = 0.0;
        for (int i = 0; i < m; ++i) {
            const double r = (i > 0 ? fabs(b[i - 1]) : 0.0) + (i + 1 < m ? fabs(b[i]) : 0.0);
            lo = fmin(lo, a[i] - r);
            hi = fmax(hi, a[i] + r);
            bmax = fmax(bmax, fabs(a[i]) + r);
        }
        const double pad = 2.2e-16 * fmax(bmax, 1e-300) * 4 + 1e-300;
        lo_s = lo - pad;
        hi_s = hi + pad;
    }
    __syncthreads();
    double bnorm = fmax(fabs(lo_s), fabs(hi_s));
    const double pivmin = 1e-290 * fmax(bnorm, 1.0);
    // multisection: each round splits [lo, hi] into kTriThreads + 1 pieces
    for (int round = 0; round < 12; ++round) {
        const double lo = lo_s, hi = hi_s;
        if (!(hi - lo > 4.4e-16 * fmax(fabs(lo), fabs(hi)) + 1e-300)) break;
        const double x = lo + (hi - lo) * (double)(threadIdx.x + 1) / (double)(kTriThreads + 1);
        cnt_s[threadIdx.x] = sturm_count(a, b, m, x, pivmin);
        __syncthreads();
        if (threadIdx.x == 0) {
            double nlo = lo, nhi = hi;
            for (int t = 0; t < kTriThreads; ++t) {
                const double xt = lo + (hi - lo) * (double)(t + 1) / (double)(kTriThreads + 1);
                if (cnt_s[t] >= 1) {
                    nhi = xt;
                    break;
                }
                nlo = xt;
            }
            lo_s = nlo;
            hi_s = nhi;
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double theta = 0.5 * (lo_s + hi_s);
    // inverse iteration on (T - theta I) with partial pivoting (one thread; m <= 1024)
    double *s = tri + 3;
    double *d = lu_d, *du = lu_du, *du2 = lu_du2, *dl = lu_dl;
    int *piv = lu_piv;
    // LU of tridiagonal T - theta I with row interchanges (as in LAPACK dgttrf)
    for (int i = 0; i < m; ++i) {
        d[i] = a[i] - theta;
        if (i + 1 < m) {
            dl[i] = b[i];
            du[i] = b[i];
        }
        du2[i] = 0.0;
    }
    const double tiny = 1e-300 + 2.2e-16 * bnorm;
    for (int i = 0; i + 1 < m; ++i) {
        if (fabs(d[i]) >= fabs(dl[i])) {
            piv[i] = i;
            if (fabs(d[i]) < tiny) d[i] = tiny;
            const double f = dl[i] / d[i];
            dl[i] = f;
            d[i + 1] -= f * du[i];
        } else {
            piv[i] = i + 1;
            const double f = d[i] / dl[i];
            d[i] = dl[i];
            dl[i] = f;
            const double t = du[i];
            du[i] = d[i + 1];
            d[i + 1] = t - f * d[i + 1];
            if (i + 2 < m) {
                du2[i] = du[i + 1];
                du[i + 1] = -f * du[i + 1];
            }
        }
    }
    if (fabs(d[m - 1]) < tiny) d[m - 1] = tiny;
    for (int i = 0; i < m; ++i) s[i] = 1.0;
    for (int it = 0; it < 4; ++it) {
        // forward: L z = P s
        for (int i = 0; i + 1 < m; ++i) {
            if (piv[i] == i) {
                s[i + 1] -= dl[i] * s[i];
            } else {
                const double t = s[i];
                s[i] = s[i + 1];
                s[i + 1] = t - dl[i] * s[i];
            }
        }
        // backward: U x = z
        s[m - 1] /= d[m - 1];
        if (m > 1) s[m - 2] = (s[m - 2] - du[m - 2] * s[m - 1]) / d[m - 2];
        for (int i = m - 3; i >= 0; --i) s[i] = (s[i] - du[i] * s[i + 1] - du2[i] * s[i + 2]) / d[i];
        double nrm = 0.0;
        for (int i = 0; i < m; ++i) nrm += s[i] * s[i];
        nrm = sqrt(nrm);
        for (int i = 0; i < m; ++i) s[i] /= nrm;
    }
    tri[0] = theta;
    tri[1] = fabs(beta[m - 1] * s[m - 1]);
}


}  // namespace qsd
