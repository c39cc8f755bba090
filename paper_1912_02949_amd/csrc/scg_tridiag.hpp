// FP64 minimum eigenpair of a symmetric tridiagonal matrix (the MinEvec step
// of alg:rand-lanczos), computed by one wave64:
//   * eigenvalue: multisection on Sturm counts (each lane evaluates the
//     LDL^T inertia count at one of 64 points; the interval shrinks 65-fold
//     per round) until it is a few ulps wide;
//   * eigenvector: inverse iteration with the tridiagonal LU factorisation
//     with partial pivoting (row interchanges as in LAPACK's gttrf).
#pragma once
#include <hip/hip_runtime.h>
#include <float.h>

namespace scg {

// 1/q for |q| >= pivmin (normal range): hardware reciprocal estimate refined by
// two Newton steps, r <- r (2 - q r), which reach full double precision; the
// chain is much shorter than an IEEE division.
__device__ __forceinline__ double rcp_refined(double q) {
    double r = __builtin_amdgcn_rcp(q);
    r = fma(r, fma(-q, r, 1.0), r);
    r = fma(r, fma(-q, r, 1.0), r);
    return r;
}

// Number of eigenvalues of tridiag(e, d, e) (size k) smaller than x: the
// number of negative pivots of the LDL^T factorisation of T - x I.
__device__ inline int sturm_count(const double* d, const double* e2, int k, double x, double pivmin) {
    int cnt = 0;
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += (q < 0.0);
    for (int i = 1; i < k; ++i) {
        q = (d[i] - x) - e2[i - 1] * rcp_refined(q);
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += (q < 0.0);
    }
    return cnt;
}

// d[k], e[k-1] in LDS (read-only), work: e2[k], lu arrays 4*k doubles, x[k].
// Must be called by all 64 threads of the first wave; returns xi in every
// lane and the unit eigenvector in x (sign: largest-magnitude entry > 0).
__device__ void tridiag_min_eig(const double* d, const double* e, int k, double* e2, double* wa, double* wb,
                                double* wc, double* wf, int* piv, double* x, double* xi_out) {
    const int lane = threadIdx.x & 63;
    if (k == 1) {
        if (lane == 0) { x[0] = 1.0; *xi_out = d[0]; }
        __syncthreads();
        return;
    }
    // Gershgorin interval and |T| estimate
    double lo = 1e308, hi = -1e308, emax2 = 0.0, tnorm = 0.0;
    for (int i = lane; i < k; i += 64) {
        const double el = (i > 0) ? fabs(e[i - 1]) : 0.0;
        const double er = (i < k - 1) ? fabs(e[i]) : 0.0;
        lo = fmin(lo, d[i] - el - er);
        hi = fmax(hi, d[i] + el + er);
        tnorm = fmax(tnorm, fabs(d[i]) + el + er);
        if (i < k - 1) { e2[i] = e[i] * e[i]; emax2 = fmax(emax2, e2[i]); }
    }
    for (int off = 32; off > 0; off >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, off, 64));
        hi = fmax(hi, __shfl_xor(hi, off, 64));
        emax2 = fmax(emax2, __shfl_xor(emax2, off, 64));
        tnorm = fmax(tnorm, __shfl_xor(tnorm, off, 64));
    }
    __syncthreads();
    const double pivmin = DBL_MIN * fmax(1.0, emax2);
    const double pad = 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + 2.0 * pivmin;
    lo -= pad;
    hi += pad;
    for (int it = 0; it < 64; ++it) {
        const double width = hi - lo;
        if (width <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + 4.0 * pivmin) break;
        const double xpt = lo + width * (double)(lane + 1) / 65.0;
        const int c = sturm_count(d, e2, k, xpt, pivmin);
        // smallest lane whose point has at least one eigenvalue below it
        const unsigned long long ballot = __ballot(c >= 1);
        double nlo, nhi;
        if (ballot == 0ull) {
            nlo = __shfl(xpt, 63, 64);
            nhi = hi;
        } else {
            const int j = __ffsll((long long)ballot) - 1;
            nhi = __shfl(xpt, j, 64);
            nlo = (j == 0) ? lo : __shfl(xpt, j - 1, 64);
        }
        if (!(nhi - nlo < width)) break;   // no progress at this precision
        lo = nlo;
        hi = nhi;
    }
    const double xi = 0.5 * (lo + hi);
    if (lane == 0) {
        // LU with partial pivoting of T - xi I: diag a, super b, sub c, 2nd super f
        const double tiny = DBL_EPSILON * fmax(tnorm, DBL_MIN);
        for (int i = 0; i < k; ++i) {
            wa[i] = d[i] - xi;
            if (i < k - 1) { wb[i] = e[i]; wc[i] = e[i]; }
            wf[i] = 0.0;
        }
        for (int i = 0; i < k - 1; ++i) {
            if (fabs(wa[i]) >= fabs(wc[i])) {
                if (fabs(wa[i]) < tiny) wa[i] = (wa[i] < 0.0) ? -tiny : tiny;
                const double m = wc[i] * rcp_refined(wa[i]);
                wc[i] = m;
                piv[i] = 0;
                wa[i + 1] -= m * wb[i];
            } else {
                const double m = wa[i] * rcp_refined(wc[i]);
                wa[i] = wc[i];
                wc[i] = m;
                piv[i] = 1;
                const double t = wa[i + 1];
                wa[i + 1] = wb[i] - m * t;
                wb[i] = t;
                if (i < k - 2) {
                    wf[i] = wb[i + 1];
                    wb[i + 1] = -m * wb[i + 1];
                }
            }
        }
        for (int i = 0; i < k; ++i) {
            if (fabs(wa[i]) < tiny) wa[i] = (wa[i] < 0.0) ? -tiny : tiny;
            wa[i] = rcp_refined(wa[i]);   // keep reciprocals of the pivots
        }
        // deterministic start vector with no special structure (golden-ratio sequence)
        for (int i = 0; i < k; ++i) {
            const double f = 0.6180339887498949 * (double)(i + 1);
            x[i] = 1.0 + 0.5 * (f - floor(f));
        }
        for (int rep = 0; rep < 3; ++rep) {
            // forward: apply row interchanges and multipliers
            for (int i = 0; i < k - 1; ++i) {
                if (piv[i] == 0) {
                    x[i + 1] -= wc[i] * x[i];
                } else {
                    const double t = x[i];
                    x[i] = x[i + 1];
                    x[i + 1] = t - wc[i] * x[i + 1];
                }
            }
            // backward substitution with U (diag a, super b, second super f)
            x[k - 1] *= wa[k - 1];
            if (k >= 2) x[k - 2] = (x[k - 2] - wb[k - 2] * x[k - 1]) * wa[k - 2];
            for (int i = k - 3; i >= 0; --i) x[i] = (x[i] - wb[i] * x[i + 1] - wf[i] * x[i + 2]) * wa[i];
            double nrm = 0.0, big = 0.0;
            for (int i = 0; i < k; ++i) {
                nrm += x[i] * x[i];
                if (fabs(x[i]) > fabs(big)) big = x[i];
            }
            const double sc = (big < 0.0 ? -1.0 : 1.0) * rsqrt(nrm);
            for (int i = 0; i < k; ++i) x[i] *= sc;
        }
        *xi_out = xi;
    }
    __syncthreads();
}

}  // namespace scg
