// NystromSketch.Reconstruct (alg:nystrom-sketch-supp) in FP64 on the device,
// with the trace correction of alg:sketchy-cgal and the error estimate of
// eqn sketch-err-supp.
//
//   sigma   = sqrt(n) eps(||S||_2)   (eps of the storage precision of S;
//             ||S||_2^2 = lambda_max(S^T S) by Jacobi on the R x R Gram)
//   S_sigma = S + sigma Omega,  B = Omega^T S_sigma (symmetrised) = L_c L_c^T
//             (on failure sigma grows tenfold, at most three times)
//   M       = S_sigma L_c^{-T}                     (row-wise forward substitution)
//   [U, Sigma] = svd(M): shifted CholeskyQR3 (Fukaya, Kannan, Nakatsukasa,
//             Yamamoto, Yanagisawa, SIAM J. Sci. Comput. 2020) gives M = Q Rt
//             with orthonormal Q; one-sided Jacobi (Hestenes) on the R x R
//             triangle Rt gives Rt = U_r Sigma V^T, and U = Q U_r
//   Lambda  = max(0, Sigma^2 - sigma); err_r = tau - sum_{j<=r} Lambda_j
//   trace correction: Lambda += (alpha - tr Lambda) / R
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "scg_device.hpp"
#include "scg_internal.hpp"

using namespace scg;

namespace {

constexpr int kGR = 256;     // workgroups of the n x R passes
constexpr int kTile = 64;    // rows staged per tile

struct Small {               // offsets (in doubles) of the R x R matrices
    int G0, P0, Q0;          // S^T S, Omega^T S, Omega^T Omega
    int Lc, L1, L2, L3, W, G;
    int scal;                // sigma, status, tau, shift
    int total;
};

Small small_layout(int R) {
    Small s;
    const int r2 = R * R;
    s.G0 = 0;
    s.P0 = s.G0 + r2;
    s.Q0 = s.P0 + r2;
    s.Lc = s.Q0 + r2;
    s.L1 = s.Lc + r2;
    s.L2 = s.L1 + r2;
    s.L3 = s.L2 + r2;
    s.W = s.L3 + r2;
    s.G = s.W + r2;
    s.scal = s.G + r2;
    s.total = s.scal + 16;
    return s;
}

// Generic last-workgroup reduction of W partial sums per workgroup
// (values in lds_vals[0..W)); totals to out[0..W).
__device__ void grid_sum_dyn(const double* lds_vals, int W, double* part, unsigned* counter, double* out) {
    __shared__ int is_last;
    for (int p = threadIdx.x; p < W; p += kBlock) part[(size_t)blockIdx.x * W + p] = lds_vals[p];
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        is_last = (atomicAdd(counter, 1u) == gridDim.x - 1);
    }
    __syncthreads();
    if (!is_last) return;
    __threadfence();
    for (int p = threadIdx.x; p < W; p += kBlock) {
        double s = 0.0;
        for (int g = 0; g < (int)gridDim.x; ++g) s += part[(size_t)g * W + p];
        out[p] = s;
    }
    if (threadIdx.x == 0) *counter = 0u;
}

// Pass 0: S^T S, Omega^T S, Omega^T Omega.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gram0(int64_t n, int64_t ld, int R, const T* S, const T* Om, uint64_t seed,
                                                  uint64_t inst, double* part, unsigned* counter, double* small,
                                                  Small L) {
    __shared__ double ts[kTile * kRMax], to[kTile * kRMax];
    __shared__ double acc_l[3 * kRMax * kRMax];
    const int r2 = R * R;
    double acc[12];
    for (int a = 0; a < 12; ++a) acc[a] = 0.0;
    int64_t lo, hi;
    split_range(n, blockIdx.x, gridDim.x, lo, hi);
    for (int64_t t0 = lo; t0 < hi; t0 += kTile) {
        const int rows = (hi - t0 < kTile) ? (int)(hi - t0) : kTile;
        for (int e = threadIdx.x; e < rows * R; e += kBlock) {
            const int c = e / rows, rr = e % rows;   // column-major source
            ts[rr * R + c] = (double)S[(int64_t)c * ld + t0 + rr];
            to[rr * R + c] = Om ? (double)Om[(int64_t)c * ld + t0 + rr] : omega_entry<T>(seed, inst, t0 + rr, c);
        }
        __syncthreads();
        int a = 0;
        for (int p = threadIdx.x; p < 3 * r2; p += kBlock, ++a) {
            const int m = p / r2, ij = p % r2, i = ij / R, j = ij % R;
            const double* X = (m == 0) ? ts : to;
            const double* Y = (m == 2) ? to : ts;
            double s = 0.0;
            for (int r = 0; r < rows; ++r) s += X[r * R + i] * Y[r * R + j];
            acc[a] += s;
        }
        __syncthreads();
    }
    int a = 0;
    for (int p = threadIdx.x; p < 3 * r2; p += kBlock, ++a) acc_l[p] = acc[a];
    __syncthreads();
    grid_sum_dyn(acc_l, 3 * r2, part, counter, small + L.G0);
}

// Pass A (first call, sigma > 0): A_r = solve(Lc, S_r + sigma Om_r)
// Pass B (sigma = 0, S = A in place): A_r = solve(Lk, A_r)
// Both accumulate the Gram A^T A of the result.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_trsm_gram(int64_t n, int64_t ld, int R, const T* S, const T* Om, uint64_t seed,
                                                      uint64_t inst, double* A, int first, double* small, Small L,
                                                      int lsel, double* part, unsigned* counter) {
    __shared__ double tile[kTile * kRMax];
    __shared__ double Lm[kRMax * kRMax];
    __shared__ double acc_l[kRMax * kRMax];
    const int r2 = R * R;
    const double* Lsrc = small + lsel;
    for (int e = threadIdx.x; e < r2; e += kBlock) Lm[e] = Lsrc[e];
    const double sigma = small[L.scal + 0];
    __syncthreads();
    double acc[4] = {0, 0, 0, 0};
    int64_t lo, hi;
    split_range(n, blockIdx.x, gridDim.x, lo, hi);
    for (int64_t t0 = lo; t0 < hi; t0 += kTile) {
        const int rows = (hi - t0 < kTile) ? (int)(hi - t0) : kTile;
        if (threadIdx.x < rows) {
            const int64_t r = t0 + threadIdx.x;
            double x[kRMax];
            for (int c = 0; c < R; ++c)
                x[c] = first ? ((double)S[(int64_t)c * ld + r] +
                                sigma * (Om ? (double)Om[(int64_t)c * ld + r] : omega_entry<T>(seed, inst, r, c)))
                             : A[r * R + c];
            // forward substitution with the lower factor: Lm x_new = x
            for (int i = 0; i < R; ++i) {
                double s = x[i];
                for (int j = 0; j < i; ++j) s -= Lm[i * R + j] * x[j];
                x[i] = s / Lm[i * R + i];
            }
            for (int c = 0; c < R; ++c) {
                A[r * R + c] = x[c];
                tile[threadIdx.x * R + c] = x[c];
            }
        }
        __syncthreads();
        int a = 0;
        for (int p = threadIdx.x; p < r2; p += kBlock, ++a) {
            const int i = p / R, j = p % R;
            double s = 0.0;
            for (int r = 0; r < rows; ++r) s += tile[r * R + i] * tile[r * R + j];
            acc[a] += s;
        }
        __syncthreads();
    }
    int a = 0;
    for (int p = threadIdx.x; p < r2; p += kBlock, ++a) acc_l[p] = acc[a];
    __syncthreads();
    grid_sum_dyn(acc_l, r2, part, counter, small + L.G);
}

// Lower Cholesky of sym(A) + shift I (R x R, row-major).  Returns false on failure.
__device__ bool chol_lower(const double* A, double shift, int R, double* Lo) {
    for (int i = 0; i < R * R; ++i) Lo[i] = 0.0;
    for (int j = 0; j < R; ++j) {
        double d = 0.5 * (A[j * R + j] + A[j * R + j]) + shift;
        for (int k = 0; k < j; ++k) d -= Lo[j * R + k] * Lo[j * R + k];
        if (!(d > 0.0) || !isfinite(d)) return false;
        const double ljj = sqrt(d);
        Lo[j * R + j] = ljj;
        for (int i = j + 1; i < R; ++i) {
            double s = 0.5 * (A[i * R + j] + A[j * R + i]);
            for (int k = 0; k < j; ++k) s -= Lo[i * R + k] * Lo[j * R + k];
            Lo[i * R + j] = s / ljj;
        }
    }
    return true;
}

// Largest eigenvalue of a symmetric R x R matrix by cyclic Jacobi (A: R x R work array).
__device__ double sym_lambda_max(const double* A0, int R, double* A) {
    for (int i = 0; i < R * R; ++i) A[i] = A0[i];
    for (int sweep = 0; sweep < 30; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < R; ++i)
            for (int j = 0; j < R; ++j) {
                tot += A[i * R + j] * A[i * R + j];
                if (i != j) off += A[i * R + j] * A[i * R + j];
            }
        if (off <= 1e-30 * tot) break;
        for (int p = 0; p < R; ++p)
            for (int q = p + 1; q < R; ++q) {
                const double apq = A[p * R + q];
                if (apq == 0.0) continue;
                const double th = (A[q * R + q] - A[p * R + p]) / (2.0 * apq);
                const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < R; ++k) {
                    const double akp = A[k * R + p], akq = A[k * R + q];
                    A[k * R + p] = c * akp - s * akq;
                    A[k * R + q] = s * akp + c * akq;
                }
                for (int k = 0; k < R; ++k) {
                    const double apk = A[p * R + k], aqk = A[q * R + k];
                    A[p * R + k] = c * apk - s * aqk;
                    A[q * R + k] = s * apk + c * aqk;
                }
            }
    }
    double m = A[0];
    for (int i = 1; i < R; ++i) m = fmax(m, A[i * R + i]);
    return m;
}

__device__ double spacing(double x, int fp32) {
    if (!(x > 0.0)) return fp32 ? 1.401298464324817e-45 : 4.9406564584124654e-324;
    int e;
    if (fp32) {
        frexpf((float)x, &e);
        return ldexp(1.0, e - 1 - 23);
    }
    frexp(x, &e);
    return ldexp(1.0, e - 1 - 52);
}

// The R x R work of these one-thread kernels lives in LDS, not in per-lane
// private memory (which the runtime would have to back with scratch for
// every wave the device can hold).
//
// sigma, B = Omega^T S + sigma Omega^T Omega, Cholesky with retries.
__global__ void k_small_sigma(int64_t n, int R, int fp32, double* small, Small L) {
    __shared__ double A[kRMax * kRMax], B[kRMax * kRMax];
    if (threadIdx.x != 0) return;
    const double lmax = sym_lambda_max(small + L.G0, R, A);
    double sigma = sqrt((double)n) * spacing(sqrt(fmax(lmax, 0.0)), fp32);
    bool ok = false;
    for (int attempt = 0; attempt < 4 && !ok; ++attempt) {
        for (int i = 0; i < R * R; ++i) B[i] = small[L.P0 + i] + sigma * small[L.Q0 + i];
        ok = chol_lower(B, 0.0, R, small + L.Lc);
        if (!ok) sigma *= 10.0;
    }
    small[L.scal + 0] = sigma;
    small[L.scal + 1] = ok ? 0.0 : 1.0;
    small[L.scal + 4] = sigma;   // kept: sigma is zeroed for the later passes
}

// Cholesky of the Gram of the current A (with the CholeskyQR3 shift when requested).
__global__ void k_small_chol(int64_t n, int R, double* small, Small L, int dst, int shifted) {
    if (threadIdx.x != 0) return;
    const double* G = small + L.G;
    double shift = 0.0;
    if (shifted) {
        double fro2 = 0.0;
        for (int i = 0; i < R; ++i) fro2 += G[i * R + i];
        shift = 11.0 * ((double)n * R + (double)R * (R + 1)) * 1.1102230246251565e-16 * fro2;
    }
    const bool ok = chol_lower(G, shift, R, small + dst);
    if (!ok) small[L.scal + 1] = 2.0;
    small[L.scal + 0] = 0.0;   // the next passes solve in place, without the sigma term
}

// Rt = L3^T L2^T L1^T (upper); one-sided Jacobi: Rt V = U_r Sigma.
// Writes W = L3^{-T} U_r (sorted by decreasing Sigma), Lambda, err.
__global__ void k_small_svd(int R, double* small, Small L, double tau, double alpha, int trace_correct,
                            double* lambda, double* err) {
    __shared__ double A[kRMax * kRMax], Tm[kRMax * kRMax];
    __shared__ double sv[kRMax], u[kRMax], lam[kRMax];
    __shared__ int order[kRMax];
    if (threadIdx.x != 0) return;
    const double* L1 = small + L.L1;
    const double* L2 = small + L.L2;
    const double* L3 = small + L.L3;
    // Tm = L2^T L1^T = (L1 L2)^T
    for (int i = 0; i < R; ++i)
        for (int j = 0; j < R; ++j) {
            double s = 0.0;
            for (int k = 0; k < R; ++k) s += L2[k * R + i] * L1[j * R + k];
            Tm[i * R + j] = s;
        }
    // A = L3^T Tm
    for (int i = 0; i < R; ++i)
        for (int j = 0; j < R; ++j) {
            double s = 0.0;
            for (int k = 0; k < R; ++k) s += L3[k * R + i] * Tm[k * R + j];
            A[i * R + j] = s;
        }
    // one-sided Jacobi on the columns of A
    for (int sweep = 0; sweep < 40; ++sweep) {
        bool rotated = false;
        for (int p = 0; p < R; ++p)
            for (int q = p + 1; q < R; ++q) {
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int k = 0; k < R; ++k) {
                    al += A[k * R + p] * A[k * R + p];
                    be += A[k * R + q] * A[k * R + q];
                    ga += A[k * R + p] * A[k * R + q];
                }
                if (fabs(ga) <= 1e-15 * sqrt(al * be) || ga == 0.0) continue;
                rotated = true;
                const double zeta = (be - al) / (2.0 * ga);
                const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
                for (int k = 0; k < R; ++k) {
                    const double ap = A[k * R + p], aq = A[k * R + q];
                    A[k * R + p] = c * ap - s * aq;
                    A[k * R + q] = s * ap + c * aq;
                }
            }
        if (!rotated) break;
    }
    for (int j = 0; j < R; ++j) {
        double s = 0.0;
        for (int k = 0; k < R; ++k) s += A[k * R + j] * A[k * R + j];
        sv[j] = sqrt(s);
        order[j] = j;
    }
    for (int i = 1; i < R; ++i) {   // insertion sort, decreasing
        const int o = order[i];
        int j = i - 1;
        while (j >= 0 && sv[order[j]] < sv[o]) { order[j + 1] = order[j]; --j; }
        order[j + 1] = o;
    }
    // U_r columns (normalised), then W = L3^{-T} U_r: solve L3^T w = u (back substitution)
    double* W = small + L.W;
    for (int jj = 0; jj < R; ++jj) {
        const int j = order[jj];
        const double s = sv[j];
        for (int k = 0; k < R; ++k) u[k] = (s > 0.0) ? A[k * R + j] / s : (k == jj ? 1.0 : 0.0);
        for (int i = R - 1; i >= 0; --i) {
            double acc = u[i];
            for (int k = i + 1; k < R; ++k) acc -= L3[k * R + i] * u[k];
            u[i] = acc / L3[i * R + i];
        }
        for (int k = 0; k < R; ++k) W[k * R + jj] = u[k];
    }
    const double sigma = small[L.scal + 4];
    double tr = 0.0, cum = 0.0;
    for (int jj = 0; jj < R; ++jj) {
        const double s = sv[order[jj]];
        lam[jj] = fmax(0.0, s * s - sigma);
        tr += lam[jj];
    }
    for (int jj = 0; jj < R; ++jj) {
        cum += lam[jj];
        if (err) err[jj] = tau - cum;
        lambda[jj] = trace_correct ? lam[jj] + (alpha - tr) / R : lam[jj];
    }
}

__global__ __launch_bounds__(kBlock) void k_out(int64_t n, int R, const double* A, const double* small, Small L,
                                                double* U) {
    __shared__ double W[kRMax * kRMax];
    for (int e = threadIdx.x; e < R * R; e += kBlock) W[e] = small[L.W + e];
    __syncthreads();
    for (int64_t r = blockIdx.x * (int64_t)kBlock + threadIdx.x; r < n; r += (int64_t)gridDim.x * kBlock) {
        double a[kRMax];
        for (int k = 0; k < R; ++k) a[k] = A[r * R + k];
        for (int c = 0; c < R; ++c) {
            double s = 0.0;
            for (int k = 0; k < R; ++k) s += a[k] * W[k * R + c];
            U[(size_t)c * n + r] = s;
        }
    }
}

template <typename T>
scg_status recon_generic(const ReconArgs& a) {
    const int64_t n = a.n;
    const int R = a.R;
    const Small L = small_layout(R);
    double* A = a.scratch;                                  // n x R, FP64
    double* part = a.scratch + (size_t)n * R;               // kGR x 3 R^2
    double* small = part + (size_t)kGR * 3 * kRMax * kRMax;
    const T* S = (const T*)a.S;
    const T* Om = (const T*)a.Om;
    const dim3 g(kGR), b(kBlock);
    hipStream_t st = a.stream;
    hipLaunchKernelGGL((k_gram0<T>), g, b, 0, st, n, a.ld, R, S, Om, a.seed, a.instance, part, a.counter, small, L);
    hipLaunchKernelGGL(k_small_sigma, dim3(1), dim3(64), 0, st, n, R, a.fp32, small, L);
    hipLaunchKernelGGL((k_trsm_gram<T>), g, b, 0, st, n, a.ld, R, S, Om, a.seed, a.instance, A, 1, small, L, L.Lc, part, a.counter);
    hipLaunchKernelGGL(k_small_chol, dim3(1), dim3(64), 0, st, n, R, small, L, L.L1, 1);
    hipLaunchKernelGGL((k_trsm_gram<T>), g, b, 0, st, n, a.ld, R, S, Om, a.seed, a.instance, A, 0, small, L, L.L1, part, a.counter);
    hipLaunchKernelGGL(k_small_chol, dim3(1), dim3(64), 0, st, n, R, small, L, L.L2, 0);
    hipLaunchKernelGGL((k_trsm_gram<T>), g, b, 0, st, n, a.ld, R, S, Om, a.seed, a.instance, A, 0, small, L, L.L2, part, a.counter);
    hipLaunchKernelGGL(k_small_chol, dim3(1), dim3(64), 0, st, n, R, small, L, L.L3, 0);
    hipLaunchKernelGGL(k_small_svd, dim3(1), dim3(64), 0, st, R, small, L, a.tau, a.alpha, a.trace_correct, a.lambda,
                       a.err);
    const int go = (int)std::min<int64_t>(4096, std::max<int64_t>(1, (n + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(k_out, dim3(go), b, 0, st, n, R, A, small, L, a.U);
    if (hipGetLastError() != hipSuccess) return SCG_EHIP;
    double stt[2];
    if (hipMemcpyAsync(stt, small + L.scal, sizeof(stt), hipMemcpyDeviceToHost, st) != hipSuccess) return SCG_EHIP;
    if (hipStreamSynchronize(st) != hipSuccess) return SCG_EHIP;
    return (stt[1] != 0.0) ? SCG_ENUMERIC : SCG_OK;
}

}  // namespace

size_t scg_recon_scratch_doubles(int64_t n, int R) {
    return (size_t)n * R + (size_t)kGR * 3 * kRMax * kRMax + 11 * (size_t)kRMax * kRMax + 64;
}

scg_status scg_reconstruct_generic(const ReconArgs& a) {
    return a.fp32 ? recon_generic<float>(a) : recon_generic<double>(a);
}

scg_status scg_reconstruct_impl(scg_ctx* c, double* U, double* lambda, double* err) {
    DevScalars hsc;
    if (hipMemcpyAsync(&hsc, c->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
        return SCG_EHIP;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return SCG_EHIP;
    ReconArgs a;
    a.n = c->n;
    a.ld = c->ld;
    a.R = c->prm.R;
    a.fp32 = (c->prm.precision == SCG_FP32_STREAM);
    a.S = c->S;
    a.Om = (c->prm.omega_mode == 1) ? nullptr : c->Om;
    a.seed = c->prm.seed;
    a.instance = (uint64_t)c->prm.instance;
    a.tau = hsc.tau;
    a.alpha = (c->prm.trace_mode == 1) ? hsc.tau : c->alpha_s;   // trace target: tr X_T when tr X <= alpha
    a.trace_correct = c->prm.trace_correct;
    a.scratch = c->recon;
    a.counter = c->counter;
    a.stream = c->stream;
    a.U = U;
    a.lambda = lambda;
    a.err = err;
    return scg_reconstruct_generic(a);
}
