// Batched SketchyCGAL: many MaxCut instances of uneven size, one persistent
// launch per iteration (alg:sketchy-cgal loop body for every instance).
//
// The instances' CSR blocks are concatenated (block-diagonal C).  One
// workgroup of 1024 threads owns one instance for the whole iteration: shift
// and start vector, the q_t Lanczos steps (SpMV + three-term recurrence with
// workgroup reductions, no device-wide synchronisation), the FP64 tridiagonal
// MinEvec on one wave, the Ritz vector, the objective product, and the z, y
// and sketch updates.  Workgroups are ordered largest instance first.  Each
// instance carries its own iteration counter on the device, so consecutive
// iterations are identical launches and a run of them is replayed from one
// captured hipGraph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "scg_device.hpp"
#include "scg_internal.hpp"
#include "scg_tridiag.hpp"

using namespace scg;

#define HIP_TRY(expr)                                 \
    do {                                              \
        hipError_t e_ = (expr);                       \
        if (e_ != hipSuccess) return SCG_EHIP;        \
    } while (0)

namespace {

constexpr int kBT = 1024;           // threads per instance workgroup
constexpr int kBW = kBT / 64;       // waves
constexpr int kQB = 128;            // Lanczos steps per call
constexpr int kGraphChunk = 16;     // iterations per captured graph
constexpr int kRedMax = kRMax + 1;  // widest workgroup reduction
constexpr size_t kXLBytes = 128 * 1024;   // LDS for the vector being multiplied

// LDS slots of the workgroup reduction results
enum : int {
    SO_OM = 0, SO_RHO = 1, SO_PREP = 2,          // 6 slots
    SO_OBJ = 8,                                  // 2 slots
    SO_PRIM = 10,                                // 3 slots
    SO_RITZ = 16,                                // kRedMax slots
    SO_N = SO_RITZ + kRedMax
};

struct BatchInst {
    int64_t row0;      // first row in the concatenated numbering
    int64_t off_V;     // element offset of the instance's Lanczos basis
    int64_t off_OS;    // element offset of the instance's Omega and S
    int64_t ld;        // column stride of its basis, Omega, S (n rounded up to 64)
    int n;
    int id;            // Philox counter word of the instance
    double cval;       // common off-diagonal value / magnitude, scaled (compressed formats)
    double alpha_s;    // alpha in scaled units
    double c_F, alpha; // scaling constants
};

struct BatchScal {
    double p, tau, xi;
    int32_t t_next, flags, k, pad;
};

template <typename T, typename CT>
struct BatchArgs {
    const BatchInst* inst;
    BatchScal* scal;
    const int32_t* order;
    const int32_t* qtab;    // q_t per instance: qtab[i * T + t - 1]
    const int32_t* rp;      // off-diagonal row pointers, concatenated rows
    const CT* col;          // instance-local column (sign in the top bit for FMT_SGN)
    const T* val;
    const double* dC;
    const double* b;
    double* z;
    double* y;
    T* s;
    T* u;
    T* v;
    T* V;
    const T* Om;
    T* S;
    scg_iter_log* logs;     // logs[i * T + t - 1]
    int T_iters;
    int R;
    int reorth;             // 2: Gram-Schmidt pass against the whole basis
    double beta0, K;
    uint64_t seed;
};

// Workgroup sums of N values per thread; the totals land in out[0..N) (LDS),
// visible to every thread on return.  Two barriers.
template <int N>
__device__ __forceinline__ void breduce(const double (&v)[N], double* red, double* out) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const double s = wave_sum(v[j]);
        if (lane == 0) red[j * kBW + w] = s;
    }
    __syncthreads();
    constexpr int kThr = (N * kBW + 63) / 64 * 64;
    if (threadIdx.x < kThr) {
        const int j = threadIdx.x / kBW, i = threadIdx.x % kBW;
        double s = (j < N) ? red[j * kBW + i] : 0.0;
#pragma unroll
        for (int off = kBW / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        if (i == 0 && j < N) out[j] = s;
    }
    __syncthreads();
}

template <typename CT>
__device__ __forceinline__ int col_index(CT cw) {
    if (sizeof(CT) == 2) return (int)((unsigned)cw & 0x7fffu);
    return (int)((unsigned)cw & 0x7fffffffu);
}
template <typename CT>
__device__ __forceinline__ bool col_neg(CT cw) {
    if (sizeof(CT) == 2) return ((unsigned)cw & 0x8000u) != 0;
    return (int32_t)cw < 0;
}

// Nonzero e of the off-diagonal part times x (the common value of the
// compressed formats is applied once per row by the caller).
template <typename T, typename CT, int FMT>
__device__ __forceinline__ T nz(CT cw, const T* val, int e, const T* x) {
    if (FMT == FMT_VAL) return val[e] * x[(int)cw];
    if (FMT == FMT_PAT) return x[(int)cw];
    const T xv = x[col_index(cw)];
    return col_neg(cw) ? -xv : xv;
}

// sum_{e in row} C_e x_col(e), four nonzeros in flight per step.
template <typename T, typename CT, int FMT>
__device__ __forceinline__ T row_product(const int32_t* rp, const CT* col, const T* val, int r, const T* x) {
    const int e0 = rp[r], e1 = rp[r + 1];
    T a0 = 0, a1 = 0;
    int e = e0;
    for (; e + 4 <= e1; e += 4) {
        const CT c0 = col[e], c1 = col[e + 1], c2 = col[e + 2], c3 = col[e + 3];
        a0 += nz<T, CT, FMT>(c0, val, e, x) + nz<T, CT, FMT>(c1, val, e + 1, x);
        a1 += nz<T, CT, FMT>(c2, val, e + 2, x) + nz<T, CT, FMT>(c3, val, e + 3, x);
    }
    for (; e < e1; ++e) a0 += nz<T, CT, FMT>(col[e], val, e, x);
    return a0 + a1;
}

// One whole iteration of alg:sketchy-cgal for the instance of this workgroup.
// XL: the vector being multiplied is kept in LDS (dynamic shared memory of
// ld * sizeof(T) bytes), so the SpMV gathers never leave the CU.
template <typename T, typename CT, int FMT, int RB, bool XL>
__global__ __launch_bounds__(kBT) void k_batch_iter(BatchArgs<T, CT> A) {
    extern __shared__ __align__(16) unsigned char dyn_lds[];
    __shared__ double red[kRedMax * kBW];
    __shared__ double so[SO_N];
    __shared__ double s_inv[kQB + 1], s_coef[kQB], s_h[kQB + 8];
    __shared__ double td[kQB], te[kQB], te2[kQB], tdp[kQB], tdm[kQB], tx[kQB];
    __shared__ double s_xi;
    T* xl = reinterpret_cast<T*>(dyn_lds);
    const int ii = A.order[blockIdx.x];
    const BatchInst D = A.inst[ii];
    BatchScal* G = A.scal + ii;
    const int t = G->t_next;
    if (t > A.T_iters) return;
    const int n = D.n;
    const int64_t ld = D.ld;
    const int tid = threadIdx.x;
    const int q = A.qtab[(size_t)ii * A.T_iters + (t - 1)];
    const double beta = A.beta0 * sqrt(t + 1.0);
    const double eta = 2.0 / (t + 1.0);
    const double alpha = D.alpha_s;
    const double cv = (FMT == FMT_VAL) ? 1.0 : D.cval;
    const int32_t* rp = A.rp + D.row0;
    double* z = A.z + D.row0;
    double* y = A.y + D.row0;
    const double* b = A.b + D.row0;
    const double* dC = A.dC + D.row0;
    T* s = A.s + D.row0;
    T* u = A.u + D.row0;
    T* v = A.v + D.row0;
    T* V = A.V + D.off_V;
    const T* Om = A.Om + D.off_OS;
    T* S = A.S + D.off_OS;
    const int R = A.R;

    // shift s = dC + y + beta (z - b), start vector, state dot products
    {
        double a[6] = {0, 0, 0, 0, 0, 0};
        for (int qd = tid; 4 * qd < n; qd += kBT) {
            double g[4];
            normal4(A.seed, (uint64_t)qd, (uint64_t)t, (uint64_t)D.id, 0ull, g);
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int r = 4 * qd + m;
                if (r < n) {
                    const double zr = z[r], yr = y[r], br = b[r];
                    const double zb = zr - br;
                    s[r] = (T)(dC[r] + (yr + beta * zb));
                    const T gt = (T)g[m];
                    V[r] = gt;
                    if (XL) xl[r] = gt;
                    a[0] += g[m] * g[m];
                    a[1] += yr * br;
                    a[2] += zb * (zr + br);
                    a[3] += (yr + beta * zb) * zr;
                    a[4] += zb * zb;
                    a[5] += br * br;
                }
            }
        }
        breduce<6>(a, red, so + SO_PREP);
    }
    if (tid == 0) s_inv[0] = 1.0 / sqrt(so[SO_PREP]);
    __syncthreads();

    // randomized Lanczos (alg:rand-lanczos); the basis is stored unnormalised
    int k = 0;
    double rho_prev = 0.0;
    for (int i = 0; i < q; ++i) {
        T* x = V + (size_t)i * ld;
        const T* xg = XL ? xl : x;
        const double xs = s_inv[i];
        double acc[1] = {0.0};
        for (int r = tid; r < n; r += kBT) {
            const T a = row_product<T, CT, FMT>(rp, A.col, A.val, r, xg);
            const double xr = (double)xg[r];
            const T ut = (T)(((double)a * cv + (double)s[r] * xr) * xs);
            u[r] = ut;
            acc[0] += xr * xs * (double)ut;
        }
        breduce<1>(acc, red, so + SO_OM);
        const double om = so[SO_OM];
        if (tid == 0) {
            td[i] = om;
            if (!isfinite(om)) G->flags |= 2;
        }
        k = i + 1;
        if (i == q - 1) break;
        const T* vm = (i > 0) ? V + (size_t)(i - 1) * ld : x;
        T* w = V + (size_t)(i + 1) * ld;
        const double c1 = om * xs, c2 = (i > 0) ? rho_prev * s_inv[i - 1] : 0.0;
        double acc2[1] = {0.0};
        for (int r = tid; r < n; r += kBT) {
            const T wt = (T)((double)u[r] - c1 * (double)xg[r] - c2 * (double)vm[r]);
            w[r] = wt;
            if (XL) xl[r] = wt;   // own row: no other thread reads it before the barrier
            acc2[0] += (double)wt * (double)wt;
        }
        if (A.reorth == 2) {
            // h_j = v_hat_j^T w for j <= i, eight at a time, then w <- w - sum_j h_j v_hat_j
            for (int jb = 0; jb <= i; jb += 8) {
                double hacc[8];
#pragma unroll
                for (int jj = 0; jj < 8; ++jj) hacc[jj] = 0.0;
                for (int r = tid; r < n; r += kBT) {
                    const double wr = (double)w[r];
#pragma unroll
                    for (int jj = 0; jj < 8; ++jj)
                        if (jb + jj <= i) hacc[jj] += (double)V[(size_t)(jb + jj) * ld + r] * wr;
                }
                breduce<8>(hacc, red, s_h + jb);
            }
            acc2[0] = 0.0;
            for (int r = tid; r < n; r += kBT) {
                double a = 0.0;
                for (int j = 0; j <= i; ++j) a += (s_h[j] * s_inv[j]) * s_inv[j] * (double)V[(size_t)j * ld + r];
                const T wt = (T)((double)w[r] - a);
                w[r] = wt;
                if (XL) xl[r] = wt;
                acc2[0] += (double)wt * (double)wt;
            }
        }
        breduce<1>(acc2, red, so + SO_RHO);
        const double rho = sqrt(so[SO_RHO]);
        if (!(rho > 64.0 * DBL_EPSILON * (fabs(om) + rho_prev))) {   // breakdown
            if (tid == 0) G->flags |= isfinite(rho) ? 1 : 3;
            break;
        }
        if (tid == 0) {
            te[i] = rho;
            s_inv[i + 1] = 1.0 / rho;
        }
        rho_prev = rho;
        __syncthreads();
    }
    __syncthreads();

    // MinEvec of T_k on wave 0, then the Ritz coefficients
    if (tid < 64) tridiag_min_eig(td, te, k, te2, tdp, tdm, tx, &s_xi);
    __syncthreads();
    for (int i = tid; i < k; i += kBT) s_coef[i] = tx[i] * s_inv[i];
    __syncthreads();
    const double xi = s_xi;

    // Ritz vector v = sum_j coef_j V_j, ||v||^2 and v^T Omega
    {
        double racc[RB + 1];
#pragma unroll
        for (int c = 0; c <= RB; ++c) racc[c] = 0.0;
        for (int r = tid; r < n; r += kBT) {
            double a = 0.0;
            for (int j = 0; j < k; ++j) a += s_coef[j] * (double)V[(size_t)j * ld + r];
            const T vt = (T)a;
            v[r] = vt;
            if (XL) xl[r] = vt;
            const double vr = (double)vt;   // the stored value is the one every later step uses
            racc[0] += vr * vr;
#pragma unroll
            for (int c = 0; c < RB; ++c)
                if (c < R) racc[c + 1] += vr * (double)Om[(size_t)c * ld + r];
        }
        breduce<RB + 1>(racc, red, so + SO_RITZ);
    }
    const double vnorm2 = so[SO_RITZ];
    const double iv = 1.0 / sqrt(vnorm2);
    const T* vg = XL ? xl : v;

    // objective v_hat^T C v_hat and the eigen-residual ||D v_hat - xi v_hat||^2
    {
        double oa[2] = {0.0, 0.0};
        for (int r = tid; r < n; r += kBT) {
            const T a = row_product<T, CT, FMT>(rp, A.col, A.val, r, vg);
            const double xr = (double)vg[r] * iv;
            const double off = (double)a * cv * iv;
            const double cvr = off + dC[r] * xr;
            const double rr = (off + (double)s[r] * xr) - xi * xr;
            oa[0] += xr * cvr;
            oa[1] += rr * rr;
        }
        breduce<2>(oa, red, so + SO_OBJ);
    }

    // primal update z <- (1 - eta) z + eta alpha v_hat^2, ||z - b||^2
    const double ea = eta * alpha, keep = 1.0 - eta;
    const bool guard = isfinite(A.K);
    {
        double pa[3] = {0.0, 0.0, 0.0};
        for (int r = tid; r < n; r += kBT) {
            const double vh = (double)vg[r] * iv;
            const double zn = keep * z[r] + ea * (vh * vh);
            z[r] = zn;
            const double dd = zn - b[r];
            pa[0] += dd * dd;
            if (guard) {
                pa[1] += y[r] * y[r];
                pa[2] += y[r] * dd;
            }
        }
        breduce<3>(pa, red, so + SO_PRIM);
    }
    const double r2 = so[SO_PRIM];
    double gamma = (r2 == 0.0) ? A.beta0 : fmin(A.beta0, 4.0 * alpha * alpha * A.beta0 / (pow(t + 1.0, 1.5) * r2));
    if (guard) {
        const double ny2 = so[SO_PRIM + 1] + 2.0 * gamma * so[SO_PRIM + 2] + gamma * gamma * r2;
        if (sqrt(fmax(ny2, 0.0)) > A.K) gamma = 0.0;
    }
    // dual update y <- y + gamma (z - b); sketch S <- (1 - eta) S + eta alpha v_hat (v_hat^T Omega)
    for (int r = tid; r < n; r += kBT) {
        y[r] += gamma * (z[r] - b[r]);
        const double vh = ea * ((double)vg[r] * iv);
        for (int c = 0; c < R; ++c) {
            T* sp = S + (size_t)c * ld + r;
            *sp = (T)(keep * (double)*sp + vh * (so[SO_RITZ + 1 + c] * iv));
        }
    }
    if (tid == 0) {
        const double p_old = G->p;
        const double p_new = keep * p_old + ea * so[SO_OBJ];
        const double* pr = so + SO_PREP;
        scg_iter_log L;
        L.t = t;
        L.q = q;
        L.k = k;
        L.flags = G->flags;
        L.xi = xi;
        L.cv = so[SO_OBJ];
        L.p = p_new;
        L.infeas = sqrt(r2);
        L.gamma = gamma;
        L.gap = p_old + pr[3] - alpha * xi;
        L.stop_obj = (p_old + pr[1] + 0.5 * beta * pr[2] - alpha * xi) / (1.0 + fabs(p_old));
        L.stop_feas = sqrt(pr[4]) / (1.0 + sqrt(pr[5]));
        L.resid = sqrt(so[SO_OBJ + 1]);
        L.beta = beta;
        L.eta = eta;
        A.logs[(size_t)ii * A.T_iters + (t - 1)] = L;
        G->p = p_new;
        G->tau = keep * G->tau + ea * (vnorm2 * iv * iv);
        G->k = k;
        G->xi = xi;
        if (!isfinite(p_new) || !isfinite(r2) || !isfinite(xi)) G->flags |= 2;
        G->t_next = t + 1;
    }
}

// ---------------------------------------------------------------- init kernels
__global__ __launch_bounds__(256) void k_bvalidate(int64_t nrows, const int64_t* rp, const int32_t* col,
                                                   const double* val, const double* b, const int32_t* inst_of_row,
                                                   const int64_t* row0, const int* ninst, int32_t* cnt,
                                                   double* dCraw, double* sumsq, double* mm, int* err_out) {
    int err = 0;
    double vmin = INFINITY, vmax = -INFINITY, amin = INFINITY, amax = -INFINITY;
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < nrows; r += (int64_t)gridDim.x * blockDim.x) {
        const int k = inst_of_row[r];
        const int64_t lo = row0[k], hi = lo + ninst[k];
        int32_t c_off = 0;
        double ds = 0.0, ss = 0.0;
        for (int64_t e = rp[r]; e < rp[r + 1]; ++e) {
            const int32_t j = col[e];
            const double vv = val[e];
            if ((int64_t)j < lo || (int64_t)j >= hi) err |= 1;
            if (!isfinite(vv)) err |= 2;
            ss += vv * vv;
            if ((int64_t)j == r) {
                ds += vv;
            } else {
                ++c_off;
                vmin = fmin(vmin, vv);
                vmax = fmax(vmax, vv);
                amin = fmin(amin, fabs(vv));
                amax = fmax(amax, fabs(vv));
            }
        }
        if (!isfinite(b[r])) err |= 4;
        cnt[r] = c_off;
        dCraw[r] = ds;
        sumsq[r] = ss;
    }
    if (err) atomicOr(err_out, err);
    for (int off = 32; off > 0; off >>= 1) {
        vmin = fmin(vmin, __shfl_xor(vmin, off, 64));
        vmax = fmax(vmax, __shfl_xor(vmax, off, 64));
        amin = fmin(amin, __shfl_xor(amin, off, 64));
        amax = fmax(amax, __shfl_xor(amax, off, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        const size_t w = (size_t)(blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6));
        mm[4 * w + 0] = vmin;
        mm[4 * w + 1] = vmax;
        mm[4 * w + 2] = amin;
        mm[4 * w + 3] = amax;
    }
}

template <typename T, typename CT>
__global__ __launch_bounds__(256) void k_bscatter(int64_t nrows, const int64_t* rp, const int32_t* col,
                                                  const double* val, const double* b_in, const int32_t* inst_of_row,
                                                  const int64_t* row0, const double* inv_cF, const double* inv_alpha,
                                                  const int32_t* rp_off, CT* col_off, T* val_off,
                                                  const double* dCraw, double* dC, double* b_out, int fmt) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < nrows; r += (int64_t)gridDim.x * blockDim.x) {
        const int k = inst_of_row[r];
        const int64_t base = row0[k];
        const double sc = inv_cF[k];
        int32_t o = rp_off[r];
        for (int64_t e = rp[r]; e < rp[r + 1]; ++e) {
            const int32_t j = col[e];
            if ((int64_t)j == r) continue;
            const uint32_t lj = (uint32_t)(j - base);
            const uint32_t sign = (sizeof(CT) == 2) ? 0x8000u : 0x80000000u;
            if (fmt == FMT_VAL) {
                col_off[o] = (CT)lj;
                val_off[o] = (T)(val[e] * sc);
            } else if (fmt == FMT_PAT) {
                col_off[o] = (CT)lj;
            } else {
                col_off[o] = (CT)((val[e] < 0.0) ? (lj | sign) : lj);
            }
            ++o;
        }
        dC[r] = dCraw[r] * sc;
        b_out[r] = b_in[r] * inv_alpha[k];
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_bomega(int n, int64_t ld, int R, uint64_t seed, uint64_t id, T* Om) {
    const int64_t ng = (n + 3) / 4;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < ng * R; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t gi = i % ng;
        const int c = (int)(i / ng);
        double g[4];
        normal4(seed, (uint64_t)gi, (uint64_t)c, id, 1ull, g);
        for (int m = 0; m < 4; ++m) {
            const int64_t r = 4 * gi + m;
            if (r < n) Om[(int64_t)c * ld + r] = (T)g[m];
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_bstate_in(int n, int64_t ld, int R, const double* in, T* S) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (int64_t)n * R; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = i / n, r = i % n;
        S[c * ld + r] = (T)in[r * R + c];
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_bstate_out(int n, int64_t ld, int R, const T* S, double* out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (int64_t)n * R; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = i / n, r = i % n;
        out[r * R + c] = (double)S[c * ld + r];
    }
}

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

int q_of(const scg_params& p, int64_t n, int t) {
    int64_t q = (p.q_mode == 1) ? p.q_fixed
                                : ((n > 1) ? (int64_t)std::ceil(std::pow((double)t, 0.25) * std::log((double)n)) : 1);
    return (int)std::max<int64_t>(1, std::min<int64_t>(q, std::max<int64_t>(n - 1, 1)));
}

struct BLayout {
    size_t inst, scal, order, qtab, rp, col, val, dC, b, z, y, s, u, v, V, Om, S, logs, iorow, row0, ninst, invc, inva,
        mm, err, recon, total;
    int64_t nrows, Vtot, OStot;
};

BLayout blayout(const scg_params& p, int ninst, const int64_t* inst_n, int64_t nnz) {
    BLayout L{};
    const size_t es = (p.precision == SCG_FP32_STREAM) ? 4 : 8;
    int64_t nrows = 0, Vtot = 0, OStot = 0, nmax = 0;
    for (int k = 0; k < ninst; ++k) {
        const int64_t n = inst_n[k];
        const int64_t ld = (n + 63) / 64 * 64;
        int qm = 1;
        for (int t = 1; t <= p.T; ++t) qm = std::max(qm, q_of(p, n, t));
        nrows += n;
        Vtot += (int64_t)(qm + 1) * ld;
        OStot += (int64_t)p.R * ld;
        nmax = std::max(nmax, n);
    }
    L.nrows = nrows;
    L.Vtot = Vtot;
    L.OStot = OStot;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = al256(off + bytes); return o; };
    L.inst = take(sizeof(BatchInst) * ninst);
    L.scal = take(sizeof(BatchScal) * ninst);
    L.order = take(4 * ninst);
    L.qtab = take(4 * (size_t)ninst * p.T);
    L.rp = take(4 * (size_t)(nrows + 1));
    L.col = take(4 * (size_t)nnz);
    L.val = take(es * (size_t)nnz);
    L.dC = take(8 * nrows);
    L.b = take(8 * nrows);
    L.z = take(8 * nrows);
    L.y = take(8 * nrows);
    L.s = take(es * nrows);
    L.u = take(es * nrows);
    L.v = take(es * nrows);
    L.V = take(es * (size_t)Vtot);
    L.Om = take(es * (size_t)OStot);
    L.S = take(es * (size_t)OStot);
    L.logs = take(sizeof(scg_iter_log) * (size_t)ninst * p.T);
    L.iorow = take(4 * (size_t)nrows);
    L.row0 = take(8 * (size_t)ninst);
    L.ninst = take(4 * (size_t)ninst);
    L.invc = take(8 * (size_t)ninst);
    L.inva = take(8 * (size_t)ninst);
    L.mm = take(8 * 4 * (size_t)1024 * 16);
    L.err = take(512);   // validation flags, then the reconstruction's counter at +256
    L.recon = take(8 * scg_recon_scratch_doubles(nmax, p.R));
    L.total = off;
    return L;
}

}  // namespace

struct scg_batch {
    scg_params prm;
    int ninst;
    int64_t nrows, nnz_in, nnz_off;
    hipStream_t stream;
    int fmt;
    bool col16;        // 16-bit column indices (every instance small enough)
    bool xl;           // the multiplied vector kept in LDS
    size_t xl_bytes;   // dynamic LDS per workgroup when xl
    std::vector<BatchInst> hinst;
    std::vector<int64_t> row0;
    BatchInst* inst;
    BatchScal* scal;
    int32_t* order;
    int32_t* qtab;
    int32_t* rp;
    void* col;
    void* val;
    double *dC, *b, *z, *y;
    void *s, *u, *v, *V, *Om, *S;
    scg_iter_log* logs;
    double* recon;
    unsigned* counter;
    std::vector<int> t_host;   // per-instance next iteration, mirrored on the host
    hipGraphExec_t graph;
    bool graph_ready;
};

namespace {

template <typename T, typename CT>
BatchArgs<T, CT> bargs(scg_batch* c) {
    BatchArgs<T, CT> A;
    A.inst = c->inst;
    A.scal = c->scal;
    A.order = c->order;
    A.qtab = c->qtab;
    A.rp = c->rp;
    A.col = (const CT*)c->col;
    A.val = (const T*)c->val;
    A.dC = c->dC;
    A.b = c->b;
    A.z = c->z;
    A.y = c->y;
    A.s = (T*)c->s;
    A.u = (T*)c->u;
    A.v = (T*)c->v;
    A.V = (T*)c->V;
    A.Om = (const T*)c->Om;
    A.S = (T*)c->S;
    A.logs = c->logs;
    A.T_iters = c->prm.T;
    A.R = c->prm.R;
    A.reorth = c->prm.reorth;
    A.beta0 = c->prm.beta0;
    A.K = c->prm.K;
    A.seed = c->prm.seed;
    return A;
}

// Launch one iteration, or (prepare) raise the kernel's dynamic-LDS limit.
template <typename T, typename CT, int FMT, int RB, bool XL>
hipError_t launch_leaf(scg_batch* c, bool prepare) {
    auto* kern = &k_batch_iter<T, CT, FMT, RB, XL>;
    const unsigned lds = XL ? (unsigned)c->xl_bytes : 0u;
    if (prepare) return XL ? hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)
                           : hipSuccess;
    hipLaunchKernelGGL(kern, dim3(c->ninst), dim3(kBT), lds, c->stream, bargs<T, CT>(c));
    return hipGetLastError();
}

template <typename T, typename CT, int FMT>
hipError_t launch_fmt(scg_batch* c, bool prepare) {
    if (c->prm.R <= 8)
        return c->xl ? launch_leaf<T, CT, FMT, 8, true>(c, prepare) : launch_leaf<T, CT, FMT, 8, false>(c, prepare);
    return c->xl ? launch_leaf<T, CT, FMT, kRMax, true>(c, prepare) : launch_leaf<T, CT, FMT, kRMax, false>(c, prepare);
}

template <typename T, typename CT>
hipError_t launch_ct(scg_batch* c, bool prepare) {
    if (c->fmt == FMT_PAT) return launch_fmt<T, CT, FMT_PAT>(c, prepare);
    if (c->fmt == FMT_SGN) return launch_fmt<T, CT, FMT_SGN>(c, prepare);
    return launch_fmt<T, CT, FMT_VAL>(c, prepare);
}

template <typename T>
hipError_t launch_t(scg_batch* c, bool prepare) {
    return c->col16 ? launch_ct<T, uint16_t>(c, prepare) : launch_ct<T, int32_t>(c, prepare);
}

hipError_t enqueue_iter(scg_batch* c, bool prepare = false) {
    return (c->prm.precision == SCG_FP32_STREAM) ? launch_t<float>(c, prepare) : launch_t<double>(c, prepare);
}

template <typename T>
scg_status binit_typed(scg_batch* c, const BLayout& L, char* base, const int64_t* row_ptr, const int32_t* col,
                       const double* val, const double* b) {
    const int64_t nrows = c->nrows;
    const int ninst = c->ninst;
    std::vector<int64_t> hrp(nrows + 1);
    HIP_TRY(hipMemcpyAsync(hrp.data(), row_ptr, 8 * (nrows + 1), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (hrp[0] != 0 || hrp[nrows] != c->nnz_in) return SCG_EINVAL;
    for (int64_t r = 0; r < nrows; ++r)
        if (hrp[r + 1] < hrp[r]) return SCG_EINVAL;
    std::vector<int32_t> iorow(nrows), hn(ninst);
    for (int k = 0; k < ninst; ++k) {
        hn[k] = c->hinst[k].n;
        for (int64_t r = c->row0[k]; r < c->row0[k] + c->hinst[k].n; ++r) iorow[r] = k;
    }
    int32_t* d_iorow = (int32_t*)(base + L.iorow);
    int64_t* d_row0 = (int64_t*)(base + L.row0);
    int* d_ninst = (int*)(base + L.ninst);
    double* d_invc = (double*)(base + L.invc);
    double* d_inva = (double*)(base + L.inva);
    double* d_mm = (double*)(base + L.mm);
    int* d_err = (int*)(base + L.err);
    HIP_TRY(hipMemcpyAsync(d_iorow, iorow.data(), 4 * nrows, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(d_row0, c->row0.data(), 8 * ninst, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(d_ninst, hn.data(), 4 * ninst, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemsetAsync(d_err, 0, 256, c->stream));
    int32_t* cnt = (int32_t*)(base + L.rp);   // scratch before the row pointers are written
    double* dCraw = c->z;
    double* sumsq = c->y;
    const int gv = 1024;
    hipLaunchKernelGGL(k_bvalidate, dim3(gv), dim3(256), 0, c->stream, nrows, row_ptr, col, val, b, d_iorow, d_row0,
                       d_ninst, cnt, dCraw, sumsq, d_mm, d_err);
    HIP_TRY(hipGetLastError());
    std::vector<int32_t> hcnt(nrows);
    std::vector<double> hss(nrows), hb(nrows), hmm((size_t)4 * gv * 4);
    int herr = 0;
    HIP_TRY(hipMemcpyAsync(hcnt.data(), cnt, 4 * nrows, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(hss.data(), sumsq, 8 * nrows, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(hb.data(), b, 8 * nrows, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(hmm.data(), d_mm, 8 * hmm.size(), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(&herr, d_err, 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (herr) return SCG_EINVAL;
    double vmin = INFINITY, vmax = -INFINITY, amin = INFINITY, amax = -INFINITY;
    for (size_t w = 0; w < hmm.size() / 4; ++w) {
        vmin = std::min(vmin, hmm[4 * w]);
        vmax = std::max(vmax, hmm[4 * w + 1]);
        amin = std::min(amin, hmm[4 * w + 2]);
        amax = std::max(amax, hmm[4 * w + 3]);
    }
    c->fmt = FMT_VAL;
    if (c->prm.matrix_format != 1 && std::isfinite(vmin)) {
        if (vmin == vmax) c->fmt = FMT_PAT;
        else if (amin == amax && amin > 0.0) c->fmt = FMT_SGN;
    }
    int64_t nmax = 0, ldmax = 0;
    for (int k = 0; k < ninst; ++k) {
        nmax = std::max<int64_t>(nmax, c->hinst[k].n);
        ldmax = std::max<int64_t>(ldmax, c->hinst[k].ld);
    }
    // column words: 16 bits when every local index (and the sign bit) fits
    c->col16 = (c->prm.matrix_format != 1) && (nmax <= ((c->fmt == FMT_SGN) ? 32768 : 65536));
    c->xl_bytes = (size_t)ldmax * sizeof(T);
    c->xl = c->xl_bytes <= kXLBytes;
    std::vector<double> invc(ninst), inva(ninst);
    for (int k = 0; k < ninst; ++k) {
        double ss = 0.0, sb = 0.0;
        for (int64_t r = c->row0[k]; r < c->row0[k] + c->hinst[k].n; ++r) {
            ss += hss[r];
            sb += hb[r];
        }
        const double alpha = (c->prm.alpha > 0.0) ? c->prm.alpha : sb;
        if (!(alpha > 0.0) || !std::isfinite(alpha)) return SCG_EINVAL;
        double cF = std::sqrt(ss);
        if (!(cF > 0.0)) cF = 1.0;
        BatchInst& I = c->hinst[k];
        I.c_F = c->prm.scale ? cF : 1.0;
        I.alpha = alpha;
        I.alpha_s = c->prm.scale ? 1.0 : alpha;
        invc[k] = 1.0 / I.c_F;
        inva[k] = c->prm.scale ? 1.0 / alpha : 1.0;
        I.cval = (c->fmt == FMT_PAT) ? vmin / I.c_F : (c->fmt == FMT_SGN ? amin / I.c_F : 1.0);
    }
    std::vector<int32_t> hrp_off(nrows + 1);
    int64_t acc = 0;
    for (int64_t r = 0; r < nrows; ++r) {
        hrp_off[r] = (int32_t)acc;
        acc += hcnt[r];
        if (acc > INT32_MAX) return SCG_EINVAL;
    }
    hrp_off[nrows] = (int32_t)acc;
    c->nnz_off = acc;
    HIP_TRY(hipMemcpyAsync(c->rp, hrp_off.data(), 4 * (nrows + 1), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(d_invc, invc.data(), 8 * ninst, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(d_inva, inva.data(), 8 * ninst, hipMemcpyHostToDevice, c->stream));
    if (c->col16)
        hipLaunchKernelGGL((k_bscatter<T, uint16_t>), dim3(gv), dim3(256), 0, c->stream, nrows, row_ptr, col, val, b,
                           d_iorow, d_row0, d_invc, d_inva, c->rp, (uint16_t*)c->col, (T*)c->val, dCraw, c->dC, c->b,
                           c->fmt);
    else
        hipLaunchKernelGGL((k_bscatter<T, int32_t>), dim3(gv), dim3(256), 0, c->stream, nrows, row_ptr, col, val, b,
                           d_iorow, d_row0, d_invc, d_inva, c->rp, (int32_t*)c->col, (T*)c->val, dCraw, c->dC, c->b,
                           c->fmt);
    HIP_TRY(hipGetLastError());
    for (int k = 0; k < ninst; ++k) {
        const BatchInst& I = c->hinst[k];
        const int64_t total = (I.n + 3) / 4 * c->prm.R;
        const int g = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (total + 255) / 256));
        hipLaunchKernelGGL((k_bomega<T>), dim3(g), dim3(256), 0, c->stream, I.n, I.ld, c->prm.R, c->prm.seed,
                           (uint64_t)I.id, (T*)c->Om + I.off_OS);
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(c->stream));   // dCraw / sumsq consumed
    // q schedule, LPT order, state
    std::vector<int32_t> qtab((size_t)ninst * c->prm.T);
    std::vector<double> work(ninst);
    for (int k = 0; k < ninst; ++k) {
        for (int t = 1; t <= c->prm.T; ++t) qtab[(size_t)k * c->prm.T + t - 1] = q_of(c->prm, c->hinst[k].n, t);
        work[k] = (double)(hrp_off[c->row0[k] + c->hinst[k].n] - hrp_off[c->row0[k]]) + 2.0 * c->hinst[k].n;
    }
    std::vector<int32_t> order(ninst);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int bb) { return work[a] > work[bb]; });
    HIP_TRY(hipMemcpyAsync(c->qtab, qtab.data(), 4 * qtab.size(), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->order, order.data(), 4 * ninst, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->inst, c->hinst.data(), sizeof(BatchInst) * ninst, hipMemcpyHostToDevice, c->stream));
    std::vector<BatchScal> hs(ninst);
    std::memset(hs.data(), 0, sizeof(BatchScal) * ninst);
    for (auto& x : hs) x.t_next = 1;
    HIP_TRY(hipMemcpyAsync(c->scal, hs.data(), sizeof(BatchScal) * ninst, hipMemcpyHostToDevice, c->stream));
    const size_t es = (c->prm.precision == SCG_FP32_STREAM) ? 4 : 8;
    HIP_TRY(hipMemsetAsync(c->z, 0, 8 * nrows, c->stream));
    HIP_TRY(hipMemsetAsync(c->y, 0, 8 * nrows, c->stream));
    HIP_TRY(hipMemsetAsync(c->S, 0, es * L.OStot, c->stream));
    HIP_TRY(hipMemsetAsync(c->logs, 0, sizeof(scg_iter_log) * ninst * c->prm.T, c->stream));
    HIP_TRY(hipMemsetAsync(c->counter, 0, 256, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return SCG_OK;
}

bool bparams_ok(const scg_params* p, int ninst, const int64_t* inst_n) {
    if (!p || ninst < 1 || !inst_n) return false;
    if (p->R < 1 || p->R > kRMax || p->T < 1 || !(p->beta0 > 0.0) || !(p->K >= 0.0)) return false;
    if (p->q_mode != 0 && p->q_mode != 1) return false;
    if (p->q_mode == 1 && p->q_fixed < 1) return false;
    if (p->reorth != 0 && p->reorth != 2) return false;
    if (p->precision != SCG_FP64 && p->precision != SCG_FP32_STREAM) return false;
    if (p->matrix_format != 0 && p->matrix_format != 1) return false;
    int64_t total = 0;
    for (int k = 0; k < ninst; ++k) {
        const int64_t n = inst_n[k];
        if (n < 1 || n < p->R) return false;
        int qm = 1;
        for (int t = 1; t <= p->T; ++t) qm = std::max(qm, q_of(*p, n, t));
        if (qm > kQB) return false;
        total += n;
    }
    return total < INT32_MAX;
}

}  // namespace

extern "C" {

scg_status scg_batch_workspace_size(const scg_params* p, int32_t n_inst, const int64_t* inst_n, int64_t nnz,
                                    size_t* bytes) {
    if (!bytes || !bparams_ok(p, n_inst, inst_n) || nnz < 0) return SCG_EINVAL;
    *bytes = blayout(*p, n_inst, inst_n, nnz).total;
    return SCG_OK;
}

scg_status sketchycgal_batch_init(scg_batch** out, const scg_params* p, int32_t n_inst, const int64_t* inst_n,
                                  int64_t nnz, const int64_t* row_ptr, const int32_t* col, const double* val,
                                  const double* b, void* workspace, size_t ws_bytes, void* stream) {
    if (!out) return SCG_EINVAL;
    *out = nullptr;
    if (!bparams_ok(p, n_inst, inst_n) || nnz < 0 || !row_ptr || !b || !workspace) return SCG_EINVAL;
    if (nnz > 0 && (!col || !val)) return SCG_EINVAL;
    if (((uintptr_t)workspace & 255) != 0) return SCG_EINVAL;
    const BLayout L = blayout(*p, n_inst, inst_n, nnz);
    if (ws_bytes < L.total) return SCG_ENOMEM;
    scg_batch* c = new (std::nothrow) scg_batch();
    if (!c) return SCG_ENOMEM;
    c->prm = *p;
    c->ninst = n_inst;
    c->nrows = L.nrows;
    c->nnz_in = nnz;
    c->stream = (hipStream_t)stream;
    c->graph = nullptr;
    c->graph_ready = false;
    char* base = (char*)workspace;
    c->inst = (BatchInst*)(base + L.inst);
    c->scal = (BatchScal*)(base + L.scal);
    c->order = (int32_t*)(base + L.order);
    c->qtab = (int32_t*)(base + L.qtab);
    c->rp = (int32_t*)(base + L.rp);
    c->col = base + L.col;
    c->val = base + L.val;
    c->dC = (double*)(base + L.dC);
    c->b = (double*)(base + L.b);
    c->z = (double*)(base + L.z);
    c->y = (double*)(base + L.y);
    c->s = base + L.s;
    c->u = base + L.u;
    c->v = base + L.v;
    c->V = base + L.V;
    c->Om = base + L.Om;
    c->S = base + L.S;
    c->logs = (scg_iter_log*)(base + L.logs);
    c->recon = (double*)(base + L.recon);
    c->counter = (unsigned*)(base + L.err + 256);
    c->hinst.resize(n_inst);
    c->row0.resize(n_inst);
    int64_t r0 = 0, offV = 0, offOS = 0;
    for (int k = 0; k < n_inst; ++k) {
        BatchInst& I = c->hinst[k];
        const int64_t n = inst_n[k];
        I.row0 = r0;
        I.n = (int)n;
        I.id = p->instance + k;
        I.ld = (n + 63) / 64 * 64;
        int qm = 1;
        for (int t = 1; t <= p->T; ++t) qm = std::max(qm, q_of(*p, n, t));
        I.off_V = offV;
        I.off_OS = offOS;
        c->row0[k] = r0;
        r0 += n;
        offV += (int64_t)(qm + 1) * I.ld;
        offOS += (int64_t)p->R * I.ld;
    }
    scg_status st = (p->precision == SCG_FP32_STREAM) ? binit_typed<float>(c, L, base, row_ptr, col, val, b)
                                                       : binit_typed<double>(c, L, base, row_ptr, col, val, b);
    if (st != SCG_OK) {
        (void)hipStreamSynchronize(c->stream);
        delete c;
        return st;
    }
    if (enqueue_iter(c, true) != hipSuccess) {
        delete c;
        return SCG_EHIP;
    }
    c->t_host.assign(n_inst, 1);
    *out = c;
    return SCG_OK;
}

// One launch per iteration; on a non-null stream, runs of kGraphChunk iterations
// replay one captured graph (the launches are identical: each instance's
// iteration counter lives on the device).
scg_status sketchycgal_batch_step(scg_batch* c, int32_t iters) {
    if (!c || iters < 0) return SCG_EINVAL;
    const int tmax = *std::max_element(c->t_host.begin(), c->t_host.end());
    if ((int64_t)tmax - 1 + iters > c->prm.T) return SCG_ESTATE;
    int left = iters;
    if (left >= kGraphChunk && c->stream != nullptr) {
        if (!c->graph_ready) {
            hipGraph_t g = nullptr;
            HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
            hipError_t e = hipSuccess;
            for (int i = 0; i < kGraphChunk && e == hipSuccess; ++i) e = enqueue_iter(c);
            const hipError_t e2 = hipStreamEndCapture(c->stream, &g);
            if (e != hipSuccess || e2 != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return SCG_EHIP;
            }
            e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) return SCG_EHIP;
            c->graph_ready = true;
        }
        while (left >= kGraphChunk) {
            HIP_TRY(hipGraphLaunch(c->graph, c->stream));
            left -= kGraphChunk;
        }
    }
    for (int i = 0; i < left; ++i) HIP_TRY(enqueue_iter(c));
    for (int& t : c->t_host) t += iters;
    return SCG_OK;
}

scg_status sketchycgal_batch_log(scg_batch* c, int32_t inst, scg_iter_log* host_out, int32_t max, int32_t* count) {
    if (!c || !host_out || !count || inst < 0 || inst >= c->ninst || max < 0) return SCG_EINVAL;
    const int m = std::min(c->t_host[inst] - 1, (int)max);
    if (m > 0)
        HIP_TRY(hipMemcpyAsync(host_out, c->logs + (size_t)inst * c->prm.T, sizeof(scg_iter_log) * m,
                               hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    *count = m;
    return SCG_OK;
}

scg_status sketchycgal_batch_summary(scg_batch* c, int32_t inst, scg_summary* o) {
    if (!c || !o || inst < 0 || inst >= c->ninst) return SCG_EINVAL;
    BatchScal hs;
    HIP_TRY(hipMemcpyAsync(&hs, c->scal + inst, sizeof(BatchScal), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    const BatchInst& I = c->hinst[inst];
    double infeas = 0.0;
    const int done = hs.t_next - 1;
    if (done > 0) {
        scg_iter_log L;
        HIP_TRY(hipMemcpy(&L, c->logs + (size_t)inst * c->prm.T + done - 1, sizeof(L), hipMemcpyDeviceToHost));
        infeas = L.infeas;
    }
    std::memset(o, 0, sizeof(*o));
    o->t_done = done;
    o->status_flags = (hs.flags & 2) ? 1 : 0;
    o->p_scaled = hs.p;
    o->tau_scaled = hs.tau;
    o->c_F = I.c_F;
    o->alpha = I.alpha;
    o->alpha_scaled = I.alpha_s;
    o->objective = I.c_F * I.alpha * hs.p / I.alpha_s;
    o->infeasibility = I.alpha / I.alpha_s * infeas;
    o->matrix_format = c->fmt;
    return (hs.flags & 2) ? SCG_ENUMERIC : SCG_OK;
}

scg_status sketchycgal_batch_get_state(scg_batch* c, int32_t inst, int32_t* t_next, double* z, double* y, double* S,
                                       double* p, double* tau) {
    if (!c || inst < 0 || inst >= c->ninst) return SCG_EINVAL;
    const BatchInst& I = c->hinst[inst];
    if (z) HIP_TRY(hipMemcpyAsync(z, c->z + I.row0, 8 * I.n, hipMemcpyDeviceToDevice, c->stream));
    if (y) HIP_TRY(hipMemcpyAsync(y, c->y + I.row0, 8 * I.n, hipMemcpyDeviceToDevice, c->stream));
    if (S) {
        if (c->prm.precision == SCG_FP32_STREAM)
            hipLaunchKernelGGL((k_bstate_out<float>), dim3(256), dim3(256), 0, c->stream, I.n, I.ld, c->prm.R,
                               (const float*)c->S + I.off_OS, S);
        else
            hipLaunchKernelGGL((k_bstate_out<double>), dim3(256), dim3(256), 0, c->stream, I.n, I.ld, c->prm.R,
                               (const double*)c->S + I.off_OS, S);
    }
    BatchScal hs;
    HIP_TRY(hipMemcpyAsync(&hs, c->scal + inst, sizeof(BatchScal), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (t_next) *t_next = hs.t_next;
    if (p) *p = hs.p;
    if (tau) *tau = hs.tau;
    return SCG_OK;
}

scg_status sketchycgal_batch_set_state(scg_batch* c, int32_t inst, int32_t t_next, const double* z, const double* y,
                                       const double* S, double p, double tau) {
    if (!c || inst < 0 || inst >= c->ninst || t_next < 1 || t_next > c->prm.T + 1 || !z || !y || !S)
        return SCG_EINVAL;
    const BatchInst& I = c->hinst[inst];
    HIP_TRY(hipMemcpyAsync(c->z + I.row0, z, 8 * I.n, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->y + I.row0, y, 8 * I.n, hipMemcpyDeviceToDevice, c->stream));
    if (c->prm.precision == SCG_FP32_STREAM)
        hipLaunchKernelGGL((k_bstate_in<float>), dim3(256), dim3(256), 0, c->stream, I.n, I.ld, c->prm.R, S,
                           (float*)c->S + I.off_OS);
    else
        hipLaunchKernelGGL((k_bstate_in<double>), dim3(256), dim3(256), 0, c->stream, I.n, I.ld, c->prm.R, S,
                           (double*)c->S + I.off_OS);
    HIP_TRY(hipGetLastError());
    BatchScal hs;
    std::memset(&hs, 0, sizeof(hs));
    hs.p = p;
    hs.tau = tau;
    hs.t_next = t_next;
    HIP_TRY(hipMemcpyAsync(c->scal + inst, &hs, sizeof(hs), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->t_host[inst] = t_next;
    return SCG_OK;
}

scg_status sketchycgal_batch_reconstruct(scg_batch* c, int32_t inst, double* U, double* lambda, double* err) {
    if (!c || !U || !lambda || inst < 0 || inst >= c->ninst) return SCG_EINVAL;
    const BatchInst& I = c->hinst[inst];
    BatchScal hs;
    HIP_TRY(hipMemcpyAsync(&hs, c->scal + inst, sizeof(BatchScal), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    const size_t es = (c->prm.precision == SCG_FP32_STREAM) ? 4 : 8;
    ReconArgs a;
    a.n = I.n;
    a.ld = I.ld;
    a.R = c->prm.R;
    a.fp32 = (c->prm.precision == SCG_FP32_STREAM);
    a.S = (const char*)c->S + es * I.off_OS;
    a.Om = (const char*)c->Om + es * I.off_OS;
    a.tau = hs.tau;
    a.alpha = I.alpha_s;
    a.trace_correct = c->prm.trace_correct;
    a.scratch = c->recon;
    a.counter = c->counter;
    a.stream = c->stream;
    a.U = U;
    a.lambda = lambda;
    a.err = err;
    return scg_reconstruct_generic(a);
}

void sketchycgal_batch_destroy(scg_batch* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    if (c->graph_ready) (void)hipGraphExecDestroy(c->graph);
    delete c;
}

}  // extern "C"
