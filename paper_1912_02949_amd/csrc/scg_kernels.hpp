// Kernels of one SketchyCGAL iteration (alg:sketchy-cgal) on gfx950.
//
// Per iteration t the host enqueues, with no synchronisation:
//   k_prep        shift s = dC + y + beta (z - b) (primitive 2), Lanczos start
//                 vector (Philox normals), and the pre-update dot products
//                 for the gap / stopping quantities
//   q_t x { k_spmv<LANCZOS>   u = D v_i (primitives 1+2), omega_i = v_i^T u
//           k_lupdate         v_{i+1} = u - omega_i v_i - rho_{i-1} v_{i-1},
//                             rho_i = ||v_{i+1}||  (three-term recurrence)
//           [k_reorth_dot, k_reduce_h, k_reorth_apply: full reorthogonalisation] }
//   k_tridiag     (xi, u) = MinEvec(T_k) in FP64, Ritz coefficients
//   k_ritz        v = sum_j u_j v_j, ||v||, v^T Omega
//   k_spmv<OBJ>   v^T C v (objective tracker), ||D v - xi v||
//   k_primal      z <- (1-eta) z + eta alpha v.v (primitive 3), ||z - b||
//   k_dual_sketch dual step size, y <- y + gamma (z - b),
//                 S <- (1-eta) S + eta alpha v (v^T Omega), p, tau, log record
//
// Reductions: each kernel stores one partial sum per workgroup; the next
// kernel adds them in workgroup order at its start (reduce_partials).  All
// consumer workgroups obtain identical totals, workgroup 0 records them in
// DevScalars.  No fence or atomic is needed, and the results are bitwise
// reproducible.  Lanczos vectors are stored unnormalised; the factor 1/rho
// is applied by the kernel that reads them.
#pragma once
#include <float.h>

#include "scg_device.hpp"
#include "scg_internal.hpp"
#include "scg_tridiag.hpp"

namespace scg {

enum SpmvMode { SPMV_LANCZOS = 0, SPMV_OBJ = 1, SPMV_APPLY = 2 };

// Partial-sum widths of the producers.
constexpr int kWPrep = 6, kWSpmv = 1, kWUpd = 1, kWObj = 2, kWPrimal = 3;

struct IterArgs {
    int t;
    int q;
    double beta, eta, alpha, beta0, K;
    uint64_t seed;
    uint64_t instance;
};

template <int LANES, typename A>
__device__ __forceinline__ A group_sum(A v) {
#pragma unroll
    for (int off = LANES / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Breakdown test of the Lanczos recurrence (reading R3 of the paper's listing).
__device__ __forceinline__ bool lanczos_breakdown(double rho, double om, double rho_prev) {
    return !(rho > 64.0 * DBL_EPSILON * (fabs(om) + rho_prev));
}

// y_r = (sum_{j != r} C_rj x_j + shift_r x_r) * xs over LDS-staged row blocks.
// LANCZOS step i: xs = 1/||v_0|| (i = 0, from k_prep's partials) or 1/rho_{i-1}
//   (from k_lupdate's partials, with the breakdown test); writes u and the
//   partial sums of x_hat^T u.
// OBJ: x = Ritz vector, xs = 1/||v|| (from k_ritz_fin); partial sums of
//   x_hat^T C x_hat and ||D x_hat - xi x_hat||^2.
// APPLY: u = D x, no scaling or reduction.
template <typename T, int LANES, int MODE, int RB>
__global__ __launch_bounds__(kBlock) void k_spmv(Prob<T> P, const T* __restrict__ x, int step) {
    __shared__ T stage[kNB];
    __shared__ T xrow[kRowsCap], srow[kRowsCap], rsum[kRowsCap];
    __shared__ int rbeg[kRowsCap + 1];
    DevScalars* sc = P.sc;
    double xs = 1.0;
    if (MODE == SPMV_LANCZOS) {
        if (sc->done) return;
        if (step == 0) {
            double tot[kWPrep];
            reduce_partials<kWPrep>(P.p_prep, P.G, tot);
            xs = 1.0 / sqrt(tot[0]);
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                sc->inv[0] = xs;
                sc->d_yb = tot[1];
                sc->d_zz = tot[2];
                sc->d_gapdot = tot[3];
                sc->d_zb2 = tot[4];
                sc->b2 = tot[5];
                sc->k = 0;
                if (!isfinite(xs)) sc->flags |= 2;
            }
        } else {
            double tot[kWUpd];
            reduce_partials<kWUpd>(P.p_upd, P.G, tot);
            const double rho = sqrt(tot[0]);
            const double om = sc->omega[step - 1];
            const double rp = (step > 1) ? sc->rho[step - 2] : 0.0;
            if (lanczos_breakdown(rho, om, rp)) {
                if (blockIdx.x == 0 && threadIdx.x == 0) {
                    sc->done = 1;
                    sc->flags |= isfinite(rho) ? 1 : 3;
                }
                return;
            }
            xs = 1.0 / rho;
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                sc->rho[step - 1] = rho;
                sc->inv[step] = xs;
            }
        }
    } else if (MODE == SPMV_OBJ) {
        xs = sc->inv_vnorm;
    }
    const double xi = (MODE == SPMV_OBJ) ? sc->xi : 0.0;
    double acc0 = 0.0, acc1 = 0.0;
    int64_t blo, bhi;
    split_range(P.nrb, xcd_lid(), gridDim.x, blo, bhi);
    const int tid = threadIdx.x;
    auto finish_row = [&](int r, double off, double xr, double sr) {
        if (MODE == SPMV_LANCZOS) {
            const double uu = (off + sr * xr) * xs;
            const T ut = (T)uu;
            P.u[r] = ut;
            acc0 += xr * xs * (double)ut;
        } else if (MODE == SPMV_OBJ) {
            const double cvr = (off + P.dC[r] * xr) * xs;
            const double dvr = (off + sr * xr) * xs;
            acc0 += xr * xs * cvr;
            const double rr = dvr - xi * xr * xs;
            acc1 += rr * rr;
        } else {
            P.u[r] = (T)(off + sr * xr);
        }
    };
    for (int64_t rbk = blo; rbk < bhi; ++rbk) {
        const int r0 = P.rb[rbk], r1 = P.rb[rbk + 1];
        const int e0 = P.rp[r0], e1 = P.rp[r1];
        if (r1 - r0 == 1 && e1 - e0 > kNB) {
            // one long row: the whole workgroup strides over it
            T a = 0;
            for (int e = e0 + tid; e < e1; e += kBlock) a += P.val[e] * x[P.col[e]];
            __shared__ double red[kWaves];
            const double tot = block_sum((double)a, red);
            if (tid == 0) finish_row(r0, tot, (double)x[r0], (double)P.s[r0]);
            __syncthreads();
            continue;
        }
        // phase A: every global load of the row block, issued together
        const int cnt = e1 - e0, nrows = r1 - r0;
        for (int e = tid; e < cnt; e += kBlock) stage[e] = P.val[e0 + e] * x[P.col[e0 + e]];
        for (int i = tid; i < nrows; i += kBlock) {
            xrow[i] = x[r0 + i];
            srow[i] = P.s[r0 + i];
            rbeg[i] = P.rp[r0 + i] - e0;
        }
        if (tid == 0) rbeg[nrows] = cnt;
        __syncthreads();
        // phase B: LANES lanes per row reduce the staged products (LDS only)
        const int g = tid / LANES, lane = tid % LANES;
        for (int base = 0; base < nrows; base += kBlock / LANES) {
            const int i = base + g;
            T a = 0;
            if (i < nrows) {
                const int a0 = rbeg[i], a1 = rbeg[i + 1];
                for (int e = a0 + lane; e < a1; e += LANES) a += stage[e];
            }
            a = group_sum<LANES>(a);
            if (i < nrows && lane == 0) rsum[i] = a;
        }
        __syncthreads();
        // phase C: one thread per row, coalesced stores
        for (int i = tid; i < nrows; i += kBlock) finish_row(r0 + i, (double)rsum[i], (double)xrow[i], (double)srow[i]);
        __syncthreads();
    }
    if (MODE == SPMV_LANCZOS) {
        double v[1] = {acc0};
        write_partials<1>(v, P.p_spmv);
    } else if (MODE == SPMV_OBJ) {
        double v[2] = {acc0, acc1};
        write_partials<2>(v, P.p_obj);
    }
}

// omega_step from the SpMV partials; w = u - omega v_step - rho v_{step-1}
// stored as V[step+1]; partial sums of ||w||^2 (unless reorthogonalising).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_lupdate(Prob<T> P, int step, int with_norm) {
    DevScalars* sc = P.sc;
    if (sc->done) return;
    double tot[kWSpmv];
    reduce_partials<kWSpmv>(P.p_spmv, P.Gs, tot);
    const double om = tot[0];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->omega[step] = om;
        sc->k = step + 1;
        if (!isfinite(om)) sc->flags |= 2;
    }
    const double si = sc->inv[step];
    const double rp = (step > 0) ? sc->rho[step - 1] : 0.0;
    const double sp = (step > 0) ? sc->inv[step - 1] : 0.0;
    const int64_t n = P.n;
    const T* vi = P.V + (size_t)step * n;
    const T* vm = (step > 0) ? P.V + (size_t)(step - 1) * n : vi;
    T* out = P.V + (size_t)(step + 1) * n;
    int64_t lo, hi;
    split_range(n, xcd_lid(), gridDim.x, lo, hi);
    double acc = 0.0;
    for (int64_t r = lo + threadIdx.x; r < hi; r += kBlock) {
        double w = (double)P.u[r] - om * ((double)vi[r] * si);
        if (step > 0) w -= rp * ((double)vm[r] * sp);
        const T wt = (T)w;
        out[r] = wt;
        acc += (double)wt * (double)wt;
    }
    if (with_norm) {
        double v[1] = {acc};
        write_partials<1>(v, P.p_upd);
    }
}

// Full reorthogonalisation, part 1: per-workgroup partials of v_j^T w, j <= step.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_reorth_dot(Prob<T> P, int step) {
    DevScalars* sc = P.sc;
    if (sc->done) return;
    const int64_t n = P.n;
    const int nj = step + 1;
    const T* w = P.V + (size_t)(step + 1) * n;
    int64_t lo, hi;
    split_range(n, xcd_lid(), gridDim.x, lo, hi);
    __shared__ double red[kWaves];
    for (int j = 0; j < nj; ++j) {
        const T* vj = P.V + (size_t)j * n;
        double acc = 0.0;
        for (int64_t r = lo + threadIdx.x; r < hi; r += kBlock) acc += (double)vj[r] * (double)w[r];
        const double bs = block_sum(acc, red);
        if (threadIdx.x == 0) P.p_h[(size_t)blockIdx.x * nj + j] = bs;
    }
}

// Part 2 (one workgroup): h_j = inv_j * sum of the partials.
__global__ __launch_bounds__(kBlock) void k_reduce_h(DevScalars* sc, const double* p_h, int G, int step) {
    if (sc->done) return;
    __shared__ double red[kWaves];
    const int nj = step + 1;
    for (int j = 0; j < nj; ++j) {
        double s = 0.0;
        for (int g = threadIdx.x; g < G; g += kBlock) s += p_h[(size_t)g * nj + j];
        s = block_sum(s, red);
        if (threadIdx.x == 0) sc->h[j] = s * sc->inv[j];
    }
}

// Part 3: w <- w - sum_j h_j v_hat_j; partial sums of ||w||^2.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_reorth_apply(Prob<T> P, int step) {
    DevScalars* sc = P.sc;
    if (sc->done) return;
    __shared__ double hc[kQCap];
    const int nj = step + 1;
    for (int j = threadIdx.x; j < nj; j += kBlock) hc[j] = sc->h[j] * sc->inv[j];
    __syncthreads();
    const int64_t n = P.n;
    T* w = P.V + (size_t)(step + 1) * n;
    int64_t lo, hi;
    split_range(n, xcd_lid(), gridDim.x, lo, hi);
    double acc = 0.0;
    for (int64_t r = lo + threadIdx.x; r < hi; r += kBlock) {
        double a = 0.0;
        for (int j = 0; j < nj; ++j) a += hc[j] * (double)P.V[(size_t)j * n + r];
        const T wt = (T)((double)w[r] - a);
        w[r] = wt;
        acc += (double)wt * (double)wt;
    }
    double v[1] = {acc};
    write_partials<1>(v, P.p_upd);
}

// MinEvec of T_k and the Ritz coefficients coef_j = u_j inv_j.  One wave64.
// Without breakdown the last SpMV's omega partials are still pending.
template <typename T>
__global__ __launch_bounds__(64) void k_tridiag(Prob<T> P, int q) {
    __shared__ double d[kQCap], e[kQCap], e2[kQCap], wa[kQCap], wb[kQCap], wc[kQCap], wf[kQCap], x[kQCap];
    __shared__ int piv[kQCap];
    __shared__ double xi;
    DevScalars* sc = P.sc;
    int k;
    if (!sc->done) {
        double tot[kWSpmv];
        reduce_partials<kWSpmv>(P.p_spmv, P.Gs, tot);
        k = q;
        if (threadIdx.x == 0) {
            sc->omega[q - 1] = tot[0];
            sc->k = q;
            if (!isfinite(tot[0])) sc->flags |= 2;
        }
        for (int i = threadIdx.x; i < k; i += 64) {
            d[i] = (i == q - 1) ? tot[0] : sc->omega[i];
            if (i < k - 1) e[i] = sc->rho[i];
        }
    } else {
        k = sc->k;
        for (int i = threadIdx.x; i < k; i += 64) {
            d[i] = sc->omega[i];
            if (i < k - 1) e[i] = sc->rho[i];
        }
    }
    __syncthreads();
    tridiag_min_eig(d, e, k, e2, wa, wb, wc, wf, piv, x, &xi);
    for (int i = threadIdx.x; i < k; i += 64) sc->coef[i] = x[i] * sc->inv[i];
    if (threadIdx.x == 0) {
        sc->xi = xi;
        if (!isfinite(xi)) sc->flags |= 2;
    }
}

// v = sum_j coef_j V[j]; partial sums of ||v||^2 and v^T Omega (RB >= R columns).
template <typename T, int RB>
__global__ __launch_bounds__(kBlock) void k_ritz(Prob<T> P) {
    DevScalars* sc = P.sc;
    __shared__ double coef[kQCap];
    const int k = sc->k;
    for (int j = threadIdx.x; j < k; j += kBlock) coef[j] = sc->coef[j];
    __syncthreads();
    const int64_t n = P.n;
    const int R = P.R;
    int64_t lo, hi;
    split_range(n, xcd_lid(), gridDim.x, lo, hi);
    double acc[RB + 1];
#pragma unroll
    for (int c = 0; c <= RB; ++c) acc[c] = 0.0;
    for (int64_t r = lo + threadIdx.x; r < hi; r += kBlock) {
        double a = 0.0;
        for (int j = 0; j < k; ++j) a += coef[j] * (double)P.V[(size_t)j * n + r];
        const T vt = (T)a;
        P.v[r] = vt;
        const double vr = (double)vt;
        acc[0] += vr * vr;
#pragma unroll
        for (int c = 0; c < RB; ++c)
            if (c < R) acc[c + 1] += vr * (double)P.Om[(size_t)c * n + r];
    }
    write_partials<RB + 1>(acc, P.p_ritz);
}

// One workgroup: ||v||^2 and v_hat^T Omega from k_ritz's partials.
template <int RB>
__global__ __launch_bounds__(kBlock) void k_ritz_fin(DevScalars* sc, const double* p_ritz, int G, int R) {
    double tot[RB + 1];
    reduce_partials<RB + 1>(p_ritz, G, tot);
    if (threadIdx.x == 0) {
        const double iv = 1.0 / sqrt(tot[0]);
        sc->vnorm2 = tot[0];
        sc->inv_vnorm = iv;
        for (int c = 0; c < R; ++c) sc->comega[c] = tot[c + 1] * iv;
        if (!isfinite(iv)) sc->flags |= 2;
    }
}

// Shift, start vector, and partial sums of the state before the update.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_prep(Prob<T> P, IterArgs it) {
    DevScalars* sc = P.sc;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->done = 0;
        sc->k = 0;
    }
    const int64_t n = P.n;
    const int64_t ng = (n + 3) / 4;
    int64_t lo, hi;
    split_range(ng, xcd_lid(), gridDim.x, lo, hi);
    double a[kWPrep] = {0, 0, 0, 0, 0, 0};
    for (int64_t gi = lo + threadIdx.x; gi < hi; gi += kBlock) {
        double g[4];
        normal4(it.seed, (uint64_t)gi, (uint64_t)it.t, it.instance, 0ull, g);
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int64_t r = 4 * gi + m;
            if (r >= n) break;
            const double zr = P.z[r], yr = P.y[r], br = P.b[r];
            const double zb = zr - br;
            P.s[r] = (T)(P.dC[r] + (yr + it.beta * zb));
            const T gt = (T)g[m];
            P.V[r] = gt;
            a[0] += (double)gt * (double)gt;
            a[1] += yr * br;
            a[2] += zb * (zr + br);
            a[3] += (yr + it.beta * zb) * zr;
            a[4] += zb * zb;
            a[5] += br * br;
        }
    }
    write_partials<kWPrep>(a, P.p_prep);
}

// z update; partial sums of ||z - b||^2 (and y^T y, y^T (z - b) for the K guard).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_primal(Prob<T> P, IterArgs it) {
    DevScalars* sc = P.sc;
    double tot[kWObj];
    reduce_partials<kWObj>(P.p_obj, P.Gs, tot);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->cv = tot[0];
        sc->resid2 = tot[1];
        if (!isfinite(tot[0])) sc->flags |= 2;
    }
    const double iv = sc->inv_vnorm;
    const double ea = it.eta * it.alpha;
    const double keep = 1.0 - it.eta;
    const bool guard = isfinite(it.K);
    int64_t lo, hi;
    split_range(P.n, xcd_lid(), gridDim.x, lo, hi);
    double a[kWPrimal] = {0, 0, 0};
    for (int64_t r = lo + threadIdx.x; r < hi; r += kBlock) {
        const double vh = (double)P.v[r] * iv;
        const double zn = keep * P.z[r] + ea * (vh * vh);
        P.z[r] = zn;
        const double d = zn - P.b[r];
        a[0] += d * d;
        if (guard) {
            const double yr = P.y[r];
            a[1] += yr * yr;
            a[2] += yr * d;
        }
    }
    write_partials<kWPrimal>(a, P.p_primal);
}

// Dual step size (eqn sketchy-cgal-dual-step), K guard, trackers and log;
// y <- y + gamma (z - b);  S <- (1-eta) S + eta alpha v_hat (v_hat^T Omega).
template <typename T, int RB>
__global__ __launch_bounds__(kBlock) void k_dual_sketch(Prob<T> P, IterArgs it) {
    DevScalars* sc = P.sc;
    double tot[kWPrimal];
    reduce_partials<kWPrimal>(P.p_primal, P.G, tot);
    const double r2 = tot[0];
    double gamma = (r2 == 0.0) ? it.beta0
                               : fmin(it.beta0, 4.0 * it.alpha * it.alpha * it.beta0 / (pow(it.t + 1.0, 1.5) * r2));
    if (isfinite(it.K)) {
        const double ny2 = tot[1] + 2.0 * gamma * tot[2] + gamma * gamma * r2;
        if (sqrt(fmax(ny2, 0.0)) > it.K) gamma = 0.0;
    }
    const double iv = sc->inv_vnorm;
    const double ea = it.eta * it.alpha;
    const double keep = 1.0 - it.eta;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->gamma_eff = gamma;
        const double p_old = sc->p;
        const double xi = sc->xi;
        const double stop_obj = (p_old + sc->d_yb + 0.5 * it.beta * sc->d_zz - it.alpha * xi) / (1.0 + fabs(p_old));
        const double gap = p_old + sc->d_gapdot - it.alpha * xi;
        const double stop_feas = sqrt(sc->d_zb2) / (1.0 + sqrt(sc->b2));
        const double p_new = keep * p_old + ea * sc->cv;
        sc->p = p_new;
        sc->tau = keep * sc->tau + ea * (sc->vnorm2 * iv * iv);
        if (!isfinite(p_new) || !isfinite(r2)) sc->flags |= 2;
        if (it.t >= 1 && it.t <= P.T_iters) {
            scg_iter_log L;
            L.t = it.t;
            L.q = it.q;
            L.k = sc->k;
            L.flags = sc->flags;
            L.xi = xi;
            L.cv = sc->cv;
            L.p = p_new;
            L.infeas = sqrt(r2);
            L.gamma = gamma;
            L.gap = gap;
            L.stop_obj = stop_obj;
            L.stop_feas = stop_feas;
            L.resid = sqrt(sc->resid2);
            L.beta = it.beta;
            L.eta = it.eta;
            P.logs[it.t - 1] = L;
        }
        sc->t_done = it.t;
    }
    const int R = P.R;
    double cw[RB];
#pragma unroll
    for (int c = 0; c < RB; ++c) cw[c] = (c < R) ? sc->comega[c] : 0.0;
    int64_t lo, hi;
    split_range(P.n, xcd_lid(), gridDim.x, lo, hi);
    const int64_t n = P.n;
    for (int64_t r = lo + threadIdx.x; r < hi; r += kBlock) {
        P.y[r] += gamma * (P.z[r] - P.b[r]);
        const double vh = ea * ((double)P.v[r] * iv);
#pragma unroll
        for (int c = 0; c < RB; ++c)
            if (c < R) {
                T* sp = P.S + (size_t)c * n + r;
                *sp = (T)(keep * (double)*sp + vh * cw[c]);
            }
    }
}

}  // namespace scg
