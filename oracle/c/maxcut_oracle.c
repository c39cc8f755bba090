/*
 * Plain FP64 SketchyCGAL iteration for the MaxCut SDP, in C with OpenMP
 * (test infrastructure only: the multi-core CPU timing baseline and a second
 * oracle checked against oracle/sketchycgal.py by the CPU tests).
 *
 * It runs the loop body of alg:sketchy-cgal on an already scaled problem
 * (Section 7.1.1, eqn problem-scaling: C <- C / ||C||_F, b <- b / alpha,
 * alpha <- 1; the caller scales), with the readings the Python oracle takes:
 *   q_t = ceil(t^(1/4) ln n), at least 1, at most n - 1 (or a fixed q);
 *   randomized Lanczos (alg:rand-lanczos) with the basis stored, rho_i the
 *   norm of the new vector, breakdown when rho_i <= 64 eps (|omega_i| +
 *   rho_{i-1}), the Ritz vector renormalised;
 *   the minimum eigenpair of the tridiagonal by cyclic Jacobi rotations on the
 *   dense k x k matrix;
 *   objective tracker from an explicit product C v;
 *   dual step gamma = min(beta0, 4 alpha^2 beta0 / ((t+1)^(3/2) ||z - b||^2)),
 *   beta0 when ||z - b|| = 0 (eqn sketchy-cgal-dual-step, ||A|| = 1), no K guard;
 *   sketch S <- (1 - eta) S + eta alpha v (v^T Omega), tau likewise
 *   (NystromSketch.RankOneUpdate).
 * Start vectors come from Philox4x64-10 (Salmon et al., SC'11) with key
 * (seed, 0) and counter (block, t, instance, 0), Box-Muller on 53-bit
 * uniforms, as the Python oracle draws them.
 *
 * Sums over the n rows are taken in fixed blocks of kBlk rows, each block
 * summed in row order and the block sums added in block order, so results do
 * not depend on the number of threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define kBlk 4096

static const uint64_t kM0 = 0xD2E7470EE14C6C93ULL, kM1 = 0xCA5A826395121157ULL;
static const uint64_t kW0 = 0x9E3779B97F4A7C15ULL, kW1 = 0xBB67AE8584CAA73BULL;

static void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
    for (int r = 0; r < 10; ++r) {
        const unsigned __int128 p0 = (unsigned __int128)kM0 * c[0];
        const unsigned __int128 p1 = (unsigned __int128)kM1 * c[2];
        const uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        const uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        const uint64_t x0 = hi1 ^ c[1] ^ k0, x1 = lo1, x2 = hi0 ^ c[3] ^ k1, x3 = lo0;
        c[0] = x0; c[1] = x1; c[2] = x2; c[3] = x3;
        if (r < 9) { k0 += kW0; k1 += kW1; }
    }
}

/* n standard normals of the stream (seed; index, instance, purpose) */
static void normal_stream(int64_t n, uint64_t seed, uint64_t index, uint64_t instance, uint64_t purpose,
                          double* out) {
    const int64_t nb = (n + 3) / 4;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < nb; ++j) {
        uint64_t c[4] = {(uint64_t)j, index, instance, purpose};
        philox4x64_10(c, seed, 0);
        for (int h = 0; h < 2; ++h) {
            const double u1 = ((double)(c[2 * h] >> 11) + 1.0) * 0x1p-53;
            const double u2 = (double)(c[2 * h + 1] >> 11) * 0x1p-53;
            const double r = sqrt(-2.0 * log(u1)), th = (2.0 * M_PI) * u2;
            const int64_t i0 = 4 * j + 2 * h;
            if (i0 < n) out[i0] = r * cos(th);
            if (i0 + 1 < n) out[i0 + 1] = r * sin(th);
        }
    }
}

/* sum_i a_i b_i in fixed blocks */
static double dot(int64_t n, const double* a, const double* b, double* part) {
    const int64_t nb = (n + kBlk - 1) / kBlk;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nb; ++k) {
        double s = 0.0;
        const int64_t hi = (k + 1) * kBlk < n ? (k + 1) * kBlk : n;
        for (int64_t i = k * kBlk; i < hi; ++i) s += a[i] * b[i];
        part[k] = s;
    }
    double s = 0.0;
    for (int64_t k = 0; k < nb; ++k) s += part[k];
    return s;
}

/* y = C x + w .* x (w may be NULL) */
static void matvec(int64_t n, const int64_t* rp, const int32_t* col, const double* val, const double* w,
                   const double* x, double* y) {
#pragma omp parallel for schedule(static, 1024)
    for (int64_t r = 0; r < n; ++r) {
        double s = 0.0;
        for (int64_t e = rp[r]; e < rp[r + 1]; ++e) s += val[e] * x[col[e]];
        y[r] = (w ? s + w[r] * x[r] : s);
    }
}

/* minimum eigenpair of the symmetric tridiagonal matrix (diagonal d[k],
 * off-diagonal e[k-1]) by cyclic Jacobi on its dense form */
static double tridiag_min(int k, const double* d, const double* e, double* u) {
    double* A = calloc((size_t)k * k, sizeof(double));
    double* V = calloc((size_t)k * k, sizeof(double));
    for (int i = 0; i < k; ++i) {
        A[i * k + i] = d[i];
        V[i * k + i] = 1.0;
        if (i + 1 < k) A[i * k + i + 1] = A[(i + 1) * k + i] = e[i];
    }
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < k; ++j) {
                tot += A[i * k + j] * A[i * k + j];
                if (i != j) off += A[i * k + j] * A[i * k + j];
            }
        if (off <= 1e-32 * tot) break;
        for (int p = 0; p < k - 1; ++p)
            for (int q = p + 1; q < k; ++q) {
                const double apq = A[p * k + q];
                if (apq == 0.0) continue;
                const double theta = (A[q * k + q] - A[p * k + p]) / (2.0 * apq);
                const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int r = 0; r < k; ++r) {   /* columns p, q */
                    const double arp = A[r * k + p], arq = A[r * k + q];
                    A[r * k + p] = c * arp - s * arq;
                    A[r * k + q] = s * arp + c * arq;
                }
                for (int r = 0; r < k; ++r) {   /* rows p, q */
                    const double apr = A[p * k + r], aqr = A[q * k + r];
                    A[p * k + r] = c * apr - s * aqr;
                    A[q * k + r] = s * apr + c * aqr;
                }
                for (int r = 0; r < k; ++r) {
                    const double vrp = V[r * k + p], vrq = V[r * k + q];
                    V[r * k + p] = c * vrp - s * vrq;
                    V[r * k + q] = s * vrp + c * vrq;
                }
            }
    }
    int m = 0;
    for (int i = 1; i < k; ++i)
        if (A[i * k + i] < A[m * k + m]) m = i;
    const double lam = A[m * k + m];
    for (int i = 0; i < k; ++i) u[i] = V[i * k + m];
    free(A);
    free(V);
    return lam;
}

static int lanczos_q(int t, int64_t n, int q_mode, int q_fixed) {
    int q = q_mode == 1 ? q_fixed : (n > 1 ? (int)ceil(pow((double)t, 0.25) * log((double)n)) : 1);
    if (q > n - 1) q = (int)(n - 1);
    return q < 1 ? 1 : q;
}

/*
 * Iterations t_first .. t_last of alg:sketchy-cgal on the scaled problem
 * (C with its diagonal in CSR, b), from the state (z, y, S, *p, *tau), which
 * is updated in place; S and Omega are n x R row-major.  log (may be NULL)
 * receives per iteration: k, xi, v^T C v, p, ||z - b||, gamma.  Returns 0, or
 * -1 when memory runs out.
 */
int scgal_maxcut_iterate(int64_t n, const int64_t* rp, const int32_t* col, const double* val, const double* b,
                         double alpha, int R, const double* Omega, uint64_t seed, int instance, int q_mode,
                         int q_fixed, double beta0, int t_first, int t_last, double* z, double* y, double* S,
                         double* p, double* tau, double* log, int nthreads) {
    if (nthreads > 0) omp_set_num_threads(nthreads);
    int qmax = 1;
    for (int t = t_first; t <= t_last; ++t) {
        const int q = lanczos_q(t, n, q_mode, q_fixed);
        if (q > qmax) qmax = q;
    }
    const int64_t nb = (n + kBlk - 1) / kBlk;
    double* basis = malloc(sizeof(double) * (size_t)n * (size_t)(qmax + 1));
    double *w = malloc(sizeof(double) * n), *u = malloc(sizeof(double) * n), *v = malloc(sizeof(double) * n);
    double* part = malloc(sizeof(double) * (nb > 0 ? nb : 1));
    double* c = malloc(sizeof(double) * R);
    double *om = malloc(sizeof(double) * qmax), *rh = malloc(sizeof(double) * qmax), *co = malloc(sizeof(double) * qmax);
    if (!basis || !w || !u || !v || !part || !c || !om || !rh || !co) return -1;
    const double eps = 2.220446049250313e-16;
    for (int t = t_first; t <= t_last; ++t) {
        const double beta = beta0 * sqrt(t + 1.0), eta = 2.0 / (t + 1.0);
        const int q = lanczos_q(t, n, q_mode, q_fixed);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) w[i] = y[i] + beta * (z[i] - b[i]);
        /* randomized Lanczos, basis stored */
        double* v0 = basis;
        normal_stream(n, seed, (uint64_t)t, (uint64_t)instance, 0, v0);
        const double g = sqrt(dot(n, v0, v0, part));
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) v0[i] /= g;
        double rho_prev = 0.0;
        int k = 0;
        for (int i = 1; i <= q; ++i) {
            const double* vi = basis + (size_t)(i - 1) * n;
            const double* vm = (i > 1) ? basis + (size_t)(i - 2) * n : NULL;
            matvec(n, rp, col, val, w, vi, u);
            const double o = dot(n, vi, u, part);
#pragma omp parallel for schedule(static)
            for (int64_t r = 0; r < n; ++r) u[r] = u[r] - o * vi[r] - (vm ? rho_prev * vm[r] : 0.0);
            const double rr = sqrt(dot(n, u, u, part));
            om[i - 1] = o;
            k = i;
            if (rr <= 64.0 * eps * (fabs(o) + rho_prev)) break;
            if (i == q) break;
            rh[i - 1] = rr;
            double* vn = basis + (size_t)i * n;
#pragma omp parallel for schedule(static)
            for (int64_t r = 0; r < n; ++r) vn[r] = u[r] / rr;
            rho_prev = rr;
        }
        const double xi = (k == 1) ? om[0] : tridiag_min(k, om, rh, co);
        if (k == 1) co[0] = 1.0;
#pragma omp parallel for schedule(static)
        for (int64_t r = 0; r < n; ++r) {
            double s = 0.0;
            for (int j = 0; j < k; ++j) s += co[j] * basis[(size_t)j * n + r];
            v[r] = s;
        }
        const double vn = sqrt(dot(n, v, v, part));
#pragma omp parallel for schedule(static)
        for (int64_t r = 0; r < n; ++r) v[r] /= vn;
        /* objective tracker, primal update, dual step, sketch */
        matvec(n, rp, col, val, NULL, v, u);
        const double cv = dot(n, v, u, part);
        *p = (1.0 - eta) * (*p) + eta * alpha * cv;
#pragma omp parallel for schedule(static)
        for (int64_t r = 0; r < n; ++r) {
            z[r] = (1.0 - eta) * z[r] + eta * alpha * v[r] * v[r];
            u[r] = z[r] - b[r];
        }
        const double r2 = dot(n, u, u, part);
        const double gamma = (r2 == 0.0) ? beta0 : fmin(beta0, 4.0 * alpha * alpha * beta0 / (pow(t + 1.0, 1.5) * r2));
#pragma omp parallel for schedule(static)
        for (int64_t r = 0; r < n; ++r) y[r] += gamma * u[r];
        for (int j = 0; j < R; ++j) {
            double s = 0.0;
            for (int64_t kk = 0; kk < nb; ++kk) part[kk] = 0.0;
#pragma omp parallel for schedule(static)
            for (int64_t kk = 0; kk < nb; ++kk) {
                double a = 0.0;
                const int64_t hi = (kk + 1) * kBlk < n ? (kk + 1) * kBlk : n;
                for (int64_t r = kk * kBlk; r < hi; ++r) a += v[r] * Omega[(size_t)r * R + j];
                part[kk] = a;
            }
            for (int64_t kk = 0; kk < nb; ++kk) s += part[kk];
            c[j] = s;
        }
#pragma omp parallel for schedule(static)
        for (int64_t r = 0; r < n; ++r)
            for (int j = 0; j < R; ++j) S[(size_t)r * R + j] = (1.0 - eta) * S[(size_t)r * R + j] + eta * alpha * v[r] * c[j];
        *tau = (1.0 - eta) * (*tau) + eta * alpha * dot(n, v, v, part);
        if (log) {
            double* L = log + (size_t)(t - t_first) * 6;
            L[0] = k; L[1] = xi; L[2] = cv; L[3] = *p; L[4] = sqrt(r2); L[5] = gamma;
        }
    }
    free(basis); free(w); free(u); free(v); free(part); free(c); free(om); free(rh); free(co);
    return 0;
}
