// FP64 minimum eigenpair of a symmetric tridiagonal matrix (the MinEvec step
// of alg:rand-lanczos), computed by one wave64:
//   * eigenvalue: multisection on Sturm counts (each lane evaluates the
//     LDL^T inertia count at one of 64 points; the interval shrinks 65-fold
//     per round) until it is a few ulps wide;
//   * eigenvector: twisted factorisation of T - xi I (Dhillon and Parlett,
//     "Multiple representations to compute orthogonal eigenvectors of
//     symmetric tridiagonal matrices", LAA 387, 2004): the top-down LDL^T and
//     bottom-up UDU^T pivots D+ and D- run on two lanes at once, the twist
//     index r minimises |gamma_r| = |D+_r + D-_r - (d_r - xi)|, and the
//     vector follows from u_r = 1 by the two one-sided recurrences.
#pragma once
#include <hip/hip_runtime.h>
#include <float.h>

#include "scg_device.hpp"

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
// The entries of each block of eight steps are read before the block's
// recurrence runs, so the LDS latency is paid once per block instead of once
// per step; the arithmetic and its order are those of the plain loop.
__device__ inline int sturm_count(const double* d, const double* e2, int k, double x, double pivmin) {
    int cnt = 0;
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += (q < 0.0);
    int i = 1;
    for (; i + 8 <= k; i += 8) {
        double dd[8], ee[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            dd[j] = d[i + j];
            ee[j] = e2[i + j - 1];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            q = (dd[j] - x) - ee[j] * rcp_refined(q);
            if (fabs(q) < pivmin) q = -pivmin;
            cnt += (q < 0.0);
        }
    }
    for (; i < k; ++i) {
        q = (d[i] - x) - e2[i - 1] * rcp_refined(q);
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += (q < 0.0);
    }
    return cnt;
}

// d[k], e[k-1] in LDS (read-only); work arrays e2, dp, dm, x of length k.
// Must be called by all 64 threads of exactly one wave (no workgroup barrier inside); returns xi in every lane and
// the unit eigenvector in x (sign: largest-magnitude entry positive).
__device__ void tridiag_min_eig(const double* d, const double* e, int k, double* e2, double* dp, double* dm,
                                double* x, double* xi_out) {
    const int lane = threadIdx.x & 63;
    if (k == 1) {
        if (lane == 0) { x[0] = 1.0; *xi_out = d[0]; }
        wave_sync();
        return;
    }
    // Gershgorin interval
    double lo = 1e308, hi = -1e308, emax2 = 0.0;
    for (int i = lane; i < k; i += 64) {
        const double el = (i > 0) ? fabs(e[i - 1]) : 0.0;
        const double er = (i < k - 1) ? fabs(e[i]) : 0.0;
        lo = fmin(lo, d[i] - el - er);
        hi = fmax(hi, d[i] + el + er);
        if (i < k - 1) { e2[i] = e[i] * e[i]; emax2 = fmax(emax2, e2[i]); }
    }
    for (int off = 32; off > 0; off >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, off, 64));
        hi = fmax(hi, __shfl_xor(hi, off, 64));
        emax2 = fmax(emax2, __shfl_xor(emax2, off, 64));
    }
    wave_sync();
    const double pivmin = DBL_MIN * fmax(1.0, emax2);
    const double pad = 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + 2.0 * pivmin;
    lo -= pad;
    hi += pad;
    for (int it = 0; it < 64; ++it) {
        const double width = hi - lo;
        if (width <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + 4.0 * pivmin) break;
        const double xpt = lo + width * (double)(lane + 1) * (1.0 / 65.0);
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
    // pivots of the two factorisations, lane 0 top-down, lane 1 bottom-up
    if (lane < 2) {
        const bool down = (lane == 0);
        int i = down ? 0 : k - 1;
        double q = d[i] - xi;
        if (fabs(q) < pivmin) q = -pivmin;
        (down ? dp : dm)[i] = q;
        for (int st = 1; st < k; ++st) {
            i = down ? st : k - 1 - st;
            const double ee = down ? e2[i - 1] : e2[i];
            q = (d[i] - xi) - ee * rcp_refined(q);
            if (fabs(q) < pivmin) q = -pivmin;
            (down ? dp : dm)[i] = q;
        }
    }
    wave_sync();
    // twist index: argmin |gamma_i|, lowest index on ties
    double best = 1e308;
    int bi = 0;
    for (int i = lane; i < k; i += 64) {
        const double g = fabs(dp[i] + dm[i] - (d[i] - xi));
        if (g < best) { best = g; bi = i; }
    }
    for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (ob < best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    const int r = bi;
    if (lane < 2) {
        const bool up = (lane == 0);   // lane 0: rows r-1 .. 0, lane 1: rows r+1 .. k-1
        double u = 1.0;
        if (up) x[r] = 1.0;
        const int len = up ? r : k - 1 - r;
        const int lmax = (r > k - 1 - r) ? r : k - 1 - r;
        for (int st = 1; st <= lmax; ++st) {
            if (st <= len) {
                const int i = up ? r - st : r + st;
                u = up ? -(e[i] * rcp_refined(dp[i])) * u : -(e[i - 1] * rcp_refined(dm[i])) * u;
                x[i] = u;
            }
        }
    }
    wave_sync();
    double nrm = 0.0, big = 0.0;
    for (int i = lane; i < k; i += 64) {
        nrm += x[i] * x[i];
        if (fabs(x[i]) > fabs(big)) big = x[i];
    }
    for (int off = 32; off > 0; off >>= 1) {
        nrm += __shfl_xor(nrm, off, 64);
        const double ob = __shfl_xor(big, off, 64);
        if (fabs(ob) > fabs(big) || (fabs(ob) == fabs(big) && ob > big)) big = ob;
    }
    const double sc = (big < 0.0 ? -1.0 : 1.0) / sqrt(nrm);
    wave_sync();
    for (int i = lane; i < k; i += 64) x[i] *= sc;
    if (lane == 0) *xi_out = xi;
    wave_sync();
}

}  // namespace scg
