// Kernels of one SketchyCGAL iteration (alg:sketchy-cgal) on gfx950.
//
// Per iteration t the host enqueues, with no synchronisation:
//   k_prep        shift s = dC + y + beta (z - w) (primitive 2; w = b, or the
//                 slack proj_K(z + y / beta) of a box constraint set), Lanczos
//                 start vector (Philox normals), and the pre-update dot
//                 products for the gap / stopping quantities
//   q_t x { k_spmv<LANCZOS>   u = D v_i (primitives 1+2), omega_i = v_i^T u
//           k_lupdate         v_{i+1} = u - omega_i v_i - rho_{i-1} v_{i-1},
//                             rho_i = ||v_{i+1}||  (three-term recurrence)
//           [k_reorth_dot, k_reduce_h, k_reorth_apply: reorthogonalisation
//            against v_0 .. v_i (full) or v_{i-1}, v_i (local)] }
//   k_tridiag     (xi, u) = MinEvec(T_k) in FP64, Ritz coefficients
//   k_ritz        v = sum_j u_j v_j, ||v||, v^T Omega
//                 (regenerated basis: k_prep and q_t - 1 x {k_spmv, k_lupdate} run
//                 again, identically, with k_lupdate adding u_j v_j into an FP64
//                 accumulator, and k_ritz_regen adds the last term)
//   k_spmv<OBJ>   v^T C v (objective tracker), ||D v - xi v||
//   k_primal      z <- (1-eta) z + eta ha v.v (primitive 3; ha = alpha, or 0 when
//                 tr X <= alpha and xi >= 0), ||z - w_bar||, dist_K(z)
//   k_dual_sketch dual step size, y <- y + gamma (z - w_bar),
//                 S <- (1-eta) S + eta ha v (v^T Omega), p, tau, log record
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

enum SpmvMode { SPMV_LANCZOS = 0, SPMV_OBJ = 1, SPMV_APPLY = 2, SPMV_XPART = 3 };

// Partial-sum widths of the producers.
constexpr int kWPrep = 6, kWSpmv = 1, kWUpd = 1, kWObj = 2, kWPrimal = 4;

struct IterArgs {
    int t;
    int q;
    double beta, eta, alpha, beta0, K;
    double beta_next;     // beta_{t+1} = beta0 sqrt(t + 2), for the slack of the dual update
    uint64_t seed;
    uint64_t instance;
    int dev;              // 1: t (and beta, eta, beta_next) from DevScalars::t_iter, as in a replayed graph
};

// The iteration's scalars, from the device counter when the launch belongs to
// a captured graph (the same formulas as the host's iter_args).
__device__ __forceinline__ IterArgs resolve_iter(IterArgs it, const DevScalars* sc) {
    if (!it.dev) return it;
    const int t = sc->t_iter;
    it.t = t;
    it.beta = it.beta0 * sqrt(t + 1.0);
    it.beta_next = it.beta0 * sqrt(t + 2.0);
    it.eta = 2.0 / (t + 1.0);
    return it;
}

// Graph replays: set the device iteration counter before a run of replays, and
// advance it as the last launch of each replayed iteration.
__global__ void k_set_t(DevScalars* sc, int t) { sc->t_iter = t; }
__global__ void k_advance_t(DevScalars* sc) { sc->t_iter += 1; }

// Matrix entries move as 16-byte vectors.  They are loaded with the default
// cache policy: a nontemporal hint on this stream measured 13% slower on the
// torus workload (random gathers from a 4 MiB vector) and no faster on the
// geometric one.
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef double f64x2_t __attribute__((ext_vector_type(2)));
typedef int i32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void load_vals4(const float* p, float (&v)[4]) {
    const f32x4_t t = *reinterpret_cast<const f32x4_t*>(p);
    v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
}
__device__ __forceinline__ void load_vals4(const double* p, double (&v)[4]) {
    const f64x2_t a = reinterpret_cast<const f64x2_t*>(p)[0];
    const f64x2_t b = reinterpret_cast<const f64x2_t*>(p)[1];
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}
__device__ __forceinline__ int4 load_cols4(const int* p) {
    const i32x4_t t = *reinterpret_cast<const i32x4_t*>(p);
    return make_int4(t.x, t.y, t.z, t.w);
}

// Rows of the quad starting at row r (the last quad of a vector may be partial).
__device__ __forceinline__ int quad_rows(int64_t r, int64_t n) { return (int)((n - r < 4) ? (n - r) : 4); }

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
//
// Work unit: a row block of at most kNB nonzeros and kRowsCap rows, owned by
// one wave64 with its own LDS slice, so waves never wait on each other:
//   (A) lanes load values and columns as aligned 16-byte quads, gather x,
//       stage the products in LDS, and load x_r, s_r and the row offsets;
//   (B) LANES lanes per row add the staged products (LDS only);
//   (C) one lane per row applies the shift and stores u (coalesced).
// A row with more than kNB nonzeros is a row block of its own; the wave
// strides over it.  The waves of a workgroup own consecutive row-block
// ranges; the XCD-aware renumbering keeps each XCD on a contiguous eighth
// of the rows.
template <typename T>
__device__ __forceinline__ T stream_load(const T* p) { return *p; }

// Product of nonzero e (column word cw) with x, by storage format; the
// common value of FMT_PAT / FMT_SGN is applied once per row instead.
template <typename T, int FMT>
__device__ __forceinline__ T nz_product(const Prob<T>& P, const T* __restrict__ x, int e, int cw) {
    if (FMT == FMT_VAL) return stream_load(P.val + e) * x[cw];
    if (FMT == FMT_PAT) return x[cw];
    const T xv = x[cw & 0x7fffffff];
    return (cw < 0) ? -xv : xv;
}

// Values and column words of one row block, a few 16-byte quads per lane.
constexpr int kQW = (kNB / 4 + 1 + 63) / 64;

template <typename T, int FMT>
struct BlockRegs {
    int4 c[kQW];
    T v[(FMT == FMT_VAL) ? kQW : 1][4];
};

template <typename T, int FMT>
__device__ __forceinline__ void fetch_block(const Prob<T>& P, int e0, int e1, int lane, BlockRegs<T, FMT>& B) {
    const int q0 = e0 >> 2, q1 = (e1 + 3) >> 2;
#pragma unroll
    for (int j = 0; j < kQW; ++j) {
        const int qe = q0 + lane + 64 * j;
        if (qe < q1) {
            const int eb = qe << 2;
            if (eb >= e0 && eb + 4 <= e1) {
                B.c[j] = load_cols4(P.col + eb);
                if (FMT == FMT_VAL) load_vals4(P.val + eb, B.v[FMT == FMT_VAL ? j : 0]);
            } else {
                int cc[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int e = eb + i;
                    const bool ok = (e >= e0 && e < e1);
                    cc[i] = ok ? stream_load(P.col + e) : 0;
                    if (FMT == FMT_VAL) B.v[FMT == FMT_VAL ? j : 0][i] = ok ? stream_load(P.val + e) : (T)0;
                }
                B.c[j] = make_int4(cc[0], cc[1], cc[2], cc[3]);
            }
        }
    }
}

template <typename T, int FMT>
__device__ __forceinline__ T column_product(const T* __restrict__ x, int cw, T v) {
    if (FMT == FMT_VAL) return v * x[cw];
    if (FMT == FMT_PAT) return x[cw];
    const T xv = x[cw & 0x7fffffff];
    return (cw < 0) ? -xv : xv;
}

// Products of the block's entries (gathers of x issued together).
template <typename T, int FMT>
__device__ __forceinline__ void gather_block(const T* __restrict__ x, int e0, int e1, int lane,
                                             const BlockRegs<T, FMT>& B, T (&pr)[kQW][4]) {
    const int q0 = e0 >> 2, q1 = (e1 + 3) >> 2;
#pragma unroll
    for (int j = 0; j < kQW; ++j) {
        const int qe = q0 + lane + 64 * j;
        if (qe < q1) {
            const int cc[4] = {B.c[j].x, B.c[j].y, B.c[j].z, B.c[j].w};
#pragma unroll
            for (int i = 0; i < 4; ++i)
                pr[j][i] = column_product<T, FMT>(x, cc[i], FMT == FMT_VAL ? B.v[FMT == FMT_VAL ? j : 0][i] : (T)0);
        }
    }
}

template <typename T>
__device__ __forceinline__ void store_products(int e0, int e1, int lane, const T (&pr)[kQW][4], T* stage) {
    const int q0 = e0 >> 2, q1 = (e1 + 3) >> 2;
#pragma unroll
    for (int j = 0; j < kQW; ++j) {
        const int qe = q0 + lane + 64 * j;
        if (qe < q1) {
            const int eb = qe << 2;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int e = eb + i;
                if (e >= e0 && e < e1) stage[e - e0] = pr[j][i];
            }
        }
    }
}

// One column segment of the product: the off-diagonal entries whose
// columns fall in segment `seg`.  Launches over the segments run in order;
// all but the last store the raw row sums in u, the later ones add them.
// rbd[k] = (first row, first nonzero) of row block k; rbd[nrb] = (n, end).
//
// SPMV_XPART runs all kSegMax segments in one launch: workgroup b works on
// segment b mod 8, i.e. on the XCD that dispatches it, so each XCD's L2 only
// ever holds its own eighth of x; it stores the raw row sums of its segment
// in xpart[seg * xld + r], and k_xcombine adds the eight partials of each row
// and finishes the product.  A Lanczos product (lanczos = 1) returns early
// once the recurrence has ended.
struct SegArgs {
    const int32_t* rp;
    const int2* rbd;
    int nrb;
    int first;
    int last;
    // SPMV_XPART only
    int lanczos;
    const int32_t* xrp[kSegMax];
    const int2* xrbd[kSegMax];
    int xnrb[kSegMax];
    void* xpart;
    int64_t xld;
};

// Scale of the vector being multiplied, shared by both product kernels.
// LANCZOS (last column segment): step 0 takes 1/||v_0|| from k_prep's partials
// (and records the state dot products), step i > 0 takes rho_{i-1} from the
// update's partials and applies the breakdown test (false: the recurrence
// has ended, the caller returns).  OBJ: 1/||v|| of the Ritz vector.
template <int MODE, typename T>
__device__ __forceinline__ bool spmv_scale(const Prob<T>& P, int step, bool last, double& xs) {
    DevScalars* sc = P.sc;
    xs = 1.0;
    if (MODE == SPMV_OBJ) xs = sc->inv_vnorm;
    if (MODE == SPMV_LANCZOS && last) {
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
                return false;
            }
            xs = 1.0 / rho;
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                sc->rho[step - 1] = rho;
                sc->inv[step] = xs;
            }
        }
    }
    return true;
}

template <typename T, int LANES, int MODE, int RB, int FMT>
__global__ __launch_bounds__(kBlock) void k_spmv(Prob<T> P, const T* __restrict__ x, int step, SegArgs sg) {
    __shared__ T stage_all[kWaves][kNB + 4];
    __shared__ T xrow_all[kWaves][kRowsCap], srow_all[kWaves][kRowsCap], rsum_all[kWaves][kRowsCap];
    __shared__ int rbeg_all[kWaves][kRowsCap + 1];
    __shared__ double wred[kWaves][2];
    DevScalars* sc = P.sc;
    if ((MODE == SPMV_LANCZOS || (MODE == SPMV_XPART && sg.lanczos)) && sc->done) return;
    P.rp = sg.rp;
    const int2* rbd = sg.rbd;
    int nrb = sg.nrb, lid = xcd_lid(), ng = gridDim.x, seg = 0;
    if (MODE == SPMV_XPART) {   // segment = the dispatching XCD; the XCD's workgroups split its row blocks
        seg = blockIdx.x % kXcd;
        P.rp = sg.xrp[seg];
        rbd = sg.xrbd[seg];
        nrb = sg.xnrb[seg];
        lid = blockIdx.x / kXcd;
        ng = gridDim.x / kXcd;
    }
    T* xpart = (MODE == SPMV_XPART) ? static_cast<T*>(sg.xpart) + (size_t)seg * sg.xld : nullptr;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    T* stage = stage_all[wv];
    T* xrow = xrow_all[wv];
    T* srow = srow_all[wv];
    T* rsum = rsum_all[wv];
    int* rbeg = rbeg_all[wv];
    int64_t blo, bhi;
    split_range(nrb, lid * kWaves + wv, ng * kWaves, blo, bhi);
    // first block's descriptors and nonzeros are requested before the scale reduction
    int2 dA = make_int2(0, 0), dB = make_int2(0, 0), dC = make_int2(0, 0);
    BlockRegs<T, FMT> cur;
    if (blo < bhi) {
        dA = rbd[blo];
        dB = rbd[blo + 1];
        if (blo + 1 < bhi) dC = rbd[blo + 2];
        if (!(dB.x - dA.x == 1 && dB.y - dA.y > kNB)) fetch_block<T, FMT>(P, dA.y, dB.y, lane, cur);
    }
    double xs = 1.0;
    if (MODE != SPMV_XPART && !spmv_scale<MODE>(P, step, sg.last, xs)) return;
    const double xi = (MODE == SPMV_OBJ) ? sc->xi : 0.0;
    double acc0 = 0.0, acc1 = 0.0;
    const double cv = (FMT == FMT_VAL) ? 1.0 : P.cval;
    auto finish_row = [&](int r, double off_raw, double xr, double sr) {
        if (MODE == SPMV_XPART) {
            xpart[r] = (T)off_raw;
            return;
        }
        if (!sg.first) off_raw += (double)P.u[r];
        if (!sg.last) {
            P.u[r] = (T)off_raw;
            return;
        }
        const double off = (FMT == FMT_VAL) ? off_raw : off_raw * cv;
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
        const int r0 = dA.x, r1 = dB.x, e0 = dA.y, e1 = dB.y;
        const int nrows = r1 - r0;
        const bool has_next = rbk + 1 < bhi;
        const bool next_long = has_next && (dC.x - dB.x == 1 && dC.y - dB.y > kNB);
        int2 dD = dC;
        if (rbk + 2 < bhi) dD = rbd[rbk + 3];
        if (nrows == 1 && e1 - e0 > kNB) {
            if (has_next && !next_long) fetch_block<T, FMT>(P, dB.y, dC.y, lane, cur);
            T a = 0;
            for (int e = e0 + lane; e < e1; e += 64) a += nz_product<T, FMT>(P, x, e, stream_load(P.col + e));
            const double tot = wave_sum((double)a);
            if (lane == 0)
                finish_row(r0, tot, (MODE == SPMV_XPART) ? 0.0 : (double)x[r0],
                           (MODE == SPMV_XPART) ? 0.0 : (double)P.s[r0]);
        } else {
            // (A) the block's row data, its gathers and the next block's entries are
            // all in flight before any of them is consumed
            T xr_r[kRowsCap / 64], sr_r[kRowsCap / 64];
            int rb_r[kRowsCap / 64];
#pragma unroll
            for (int h = 0; h < kRowsCap / 64; ++h) {
                const int i = lane + 64 * h;
                if (i < nrows) {
                    // the segment partials need neither x_r nor the shift
                    xr_r[h] = (MODE == SPMV_XPART) ? (T)0 : x[r0 + i];
                    sr_r[h] = (MODE == SPMV_XPART) ? (T)0 : stream_load(P.s + r0 + i);
                    rb_r[h] = stream_load(P.rp + r0 + i) - e0;
                }
            }
            T pr[kQW][4];
            gather_block<T, FMT>(x, e0, e1, lane, cur, pr);
            if (has_next && !next_long) fetch_block<T, FMT>(P, dB.y, dC.y, lane, cur);
            store_products<T>(e0, e1, lane, pr, stage);
#pragma unroll
            for (int h = 0; h < kRowsCap / 64; ++h) {
                const int i = lane + 64 * h;
                if (i < nrows) {
                    xrow[i] = xr_r[h];
                    srow[i] = sr_r[h];
                    rbeg[i] = rb_r[h];
                }
            }
            if (lane == 0) rbeg[nrows] = e1 - e0;
            wave_sync();
            // (B)
            const int g = lane / LANES, sub = lane % LANES;
            for (int base = 0; base < nrows; base += 64 / LANES) {
                const int i = base + g;
                T a = 0;
                if (i < nrows) {
                    const int a0 = rbeg[i], a1 = rbeg[i + 1];
                    for (int e = a0 + sub; e < a1; e += LANES) a += stage[e];
                }
                a = group_sum<LANES>(a);
                if (i < nrows && sub == 0) rsum[i] = a;
            }
            wave_sync();
            // (C)
            for (int i = lane; i < nrows; i += 64)
                finish_row(r0 + i, (double)rsum[i], (double)xrow[i], (double)srow[i]);
            wave_sync();
        }
        dA = dB;
        dB = dC;
        dC = dD;
    }
    if (MODE == SPMV_APPLY || MODE == SPMV_XPART || !sg.last) return;
    acc0 = wave_sum(acc0);
    acc1 = wave_sum(acc1);
    if (lane == 0) {
        wred[wv][0] = acc0;
        wred[wv][1] = acc1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s0 = 0.0, s1 = 0.0;
        for (int i = 0; i < kWaves; ++i) {
            s0 += wred[i][0];
            s1 += wred[i][1];
        }
        if (MODE == SPMV_LANCZOS) {
            P.p_spmv[blockIdx.x] = s0;
        } else {
            P.p_obj[(size_t)blockIdx.x * 2 + 0] = s0;
            P.p_obj[(size_t)blockIdx.x * 2 + 1] = s1;
        }
    }
}

// Second pass of the concurrent-segment product: row r's off-diagonal sum is
// the sum of its eight segment partials (segment order, FP64), then the shift,
// the scale and the partial sums exactly as the last segment of k_spmv.  Rows
// go four to a lane as 16-byte quads; the first quad's loads are in flight
// before the scale reduction.
template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void k_xcombine(Prob<T> P, const T* __restrict__ x, int step,
                                                     const T* __restrict__ xpart, int64_t xld) {
    __shared__ double wred[kWaves][2];
    DevScalars* sc = P.sc;
    if (MODE == SPMV_LANCZOS && sc->done) return;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t n = P.n;
    int64_t qlo, qhi;
    split_range((n + 3) / 4, xcd_lid(), gridDim.x, qlo, qhi);
    int64_t qd = qlo + threadIdx.x;
    double off[4] = {0.0, 0.0, 0.0, 0.0};
    // the partial vectors have stride xld (a multiple of 64): a quad never leaves them
    auto load_offs = [&](int64_t q) {
        const int64_t r = 4 * q;
        T pv[kSegMax][4];
#pragma unroll
        for (int sgi = 0; sgi < kSegMax; ++sgi) load_vals4(xpart + (size_t)sgi * xld + r, pv[sgi]);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            double a = 0.0;
#pragma unroll
            for (int sgi = 0; sgi < kSegMax; ++sgi) a += (double)pv[sgi][i];
            off[i] = a;
        }
    };
    if (qd < qhi) load_offs(qd);
    double xs = 1.0;
    if (!spmv_scale<MODE>(P, step, true, xs)) return;
    const double xi = (MODE == SPMV_OBJ) ? sc->xi : 0.0;
    const double cv = P.cval;
    double acc0 = 0.0, acc1 = 0.0;
    for (; qd < qhi; qd += kBlock) {
        if (qd != qlo + threadIdx.x) load_offs(qd);
        const int64_t r = 4 * qd;
        const int m = quad_rows(r, n);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (i >= m) break;
            const double xr = (double)x[r + i], sr = (double)P.s[r + i];
            const double o = off[i] * cv;
            if (MODE == SPMV_LANCZOS) {
                const T ut = (T)((o + sr * xr) * xs);
                P.u[r + i] = ut;
                acc0 += xr * xs * (double)ut;
            } else if (MODE == SPMV_OBJ) {
                const double cvr = (o + P.dC[r + i] * xr) * xs;
                const double dvr = (o + sr * xr) * xs;
                acc0 += xr * xs * cvr;
                const double rr = dvr - xi * xr * xs;
                acc1 += rr * rr;
            } else {
                P.u[r + i] = (T)(o + sr * xr);
            }
        }
    }
    if (MODE == SPMV_APPLY) return;
    acc0 = wave_sum(acc0);
    acc1 = wave_sum(acc1);
    if (lane == 0) {
        wred[wv][0] = acc0;
        wred[wv][1] = acc1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s0 = 0.0, s1 = 0.0;
        for (int i = 0; i < kWaves; ++i) {
            s0 += wred[i][0];
            s1 += wred[i][1];
        }
        if (MODE == SPMV_LANCZOS) {
            P.p_spmv[blockIdx.x] = s0;
        } else {
            P.p_obj[(size_t)blockIdx.x * 2 + 0] = s0;
            P.p_obj[(size_t)blockIdx.x * 2 + 1] = s1;
        }
    }
}

// The chunks a wave takes in the chunk products: the XCD that dispatches the
// workgroup owns one contiguous eighth of the chunks, and its waves take them
// round-robin (chunk lo, lo + step, ...), so at any moment they work on
// neighbouring rows and the x entries those rows gather stay in the XCD's L2
// (each wave taking a contiguous range instead spreads them over the whole
// eighth).  The grid is a multiple of the XCD count.
__device__ __forceinline__ void chunk_sweep(int64_t nchunks, int wv, int64_t& lo, int64_t& hi, int64_t& step) {
    int64_t xlo, xhi;
    split_range(nchunks, blockIdx.x % kXcd, kXcd, xlo, xhi);
    lo = xlo + (int64_t)(blockIdx.x / kXcd) * kWaves + wv;
    hi = xhi;
    step = (int64_t)(gridDim.x / kXcd) * kWaves;
}

// The same product over the quad-chunk layout (matrices whose off-diagonal
// values share one magnitude and whose rows hold at most kQRowMax entries).
// Each row's column words are padded to whole 16-byte quads and rows are
// packed, whole, into chunks of 64 quads; P.qc[c] = (first row, quads used).
// Word bits: 31 sign (FMT_SGN), 30 first quad of a row, 29 padding entry,
// 28..0 column.  One wave takes one chunk at a time, one quad per lane: a
// lane's row is the chunk's first row plus the count of row starts at or
// before it (ballot), rows are summed by a segmented scan across the lanes,
// and the row's last lane applies the shift and the scale exactly as k_spmv
// does.  There is no LDS staging and no row-pointer stream, and every lane's
// gathers depend on one load only.  A wave's chunks follow chunk_sweep.
constexpr int kQStart = 1 << 30, kQPad = 1 << 29, kQColMask = (1 << 29) - 1;
constexpr int kQRowMax = 128;   // off-diagonal entries of the longest row the layout takes

template <typename T, int FMT>
__device__ __forceinline__ T quad_term(const T* __restrict__ x, int w) {
    const T xv = (w & kQPad) ? (T)0 : x[w & kQColMask];
    return (FMT == FMT_SGN && w < 0) ? -xv : xv;
}

template <typename T, int MODE, int FMT>
__global__ __launch_bounds__(kBlock) void k_spmvq(Prob<T> P, const T* __restrict__ x, int step) {
    __shared__ double wred[kWaves][2];
    DevScalars* sc = P.sc;
    if (MODE == SPMV_LANCZOS && sc->done) return;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int64_t clo, chi, cstep;
    chunk_sweep(P.nqc, wv, clo, chi, cstep);
    int2 cd = make_int2(0, 0);
    i32x4_t w = {kQPad, kQPad, kQPad, kQPad};
    T tf[4] = {(T)0, (T)0, (T)0, (T)0};
    if (clo < chi) {
        cd = P.qc[clo];
        if (lane < cd.y) w = reinterpret_cast<const i32x4_t*>(P.qw)[(size_t)clo * 64 + lane];
        tf[0] = quad_term<T, FMT>(x, w.x);
        tf[1] = quad_term<T, FMT>(x, w.y);
        tf[2] = quad_term<T, FMT>(x, w.z);
        tf[3] = quad_term<T, FMT>(x, w.w);
    }
    double xs;
    if (!spmv_scale<MODE>(P, step, true, xs)) return;
    const double xi = (MODE == SPMV_OBJ) ? sc->xi : 0.0;
    const double cv = P.cval;
    double acc0 = 0.0, acc1 = 0.0;
    for (int64_t c = clo; c < chi; c += cstep) {
        const bool valid = lane < cd.y;
        const bool start = valid && (w.x & kQStart);
        const unsigned long long bal = __ballot(start);
        const int rid = __popcll(bal & ((2ull << lane) - 1ull)) - 1;
        T a;
        if (c == clo) a = valid ? (tf[0] + tf[1]) + (tf[2] + tf[3]) : (T)0;
        else a = valid ? (quad_term<T, FMT>(x, w.x) + quad_term<T, FMT>(x, w.y)) +
                             (quad_term<T, FMT>(x, w.z) + quad_term<T, FMT>(x, w.w))
                       : (T)0;
        const int r0 = cd.x, nq = cd.y;
        if (c + cstep < chi) {
            cd = P.qc[c + cstep];
            w = (lane < cd.y) ? reinterpret_cast<const i32x4_t*>(P.qw)[(size_t)(c + cstep) * 64 + lane]
                              : i32x4_t{kQPad, kQPad, kQPad, kQPad};
        }
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const T ya = __shfl_up(a, off, 64);
            const int yr = __shfl_up(rid, off, 64);
            if (lane >= off && yr == rid) a += ya;
        }
        const bool next_start = (lane == 63) || ((bal >> (lane + 1)) & 1ull);
        if (valid && (lane == nq - 1 || next_start)) {
            const int r = r0 + rid;
            const double xr = (double)x[r], sr = (double)P.s[r];
            const double off = (double)a * cv;
            if (MODE == SPMV_LANCZOS) {
                const T ut = (T)((off + sr * xr) * xs);
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
        }
    }
    if (MODE == SPMV_APPLY) return;
    acc0 = wave_sum(acc0);
    acc1 = wave_sum(acc1);
    if (lane == 0) {
        wred[wv][0] = acc0;
        wred[wv][1] = acc1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s0 = 0.0, s1 = 0.0;
        for (int i = 0; i < kWaves; ++i) {
            s0 += wred[i][0];
            s1 += wred[i][1];
        }
        if (MODE == SPMV_LANCZOS) {
            P.p_spmv[blockIdx.x] = s0;
        } else {
            P.p_obj[(size_t)blockIdx.x * 2 + 0] = s0;
            P.p_obj[(size_t)blockIdx.x * 2 + 1] = s1;
        }
    }
}

// The product over the entry-chunk layout (off-diagonal values stored, rows of
// at most kERowMax entries).  The CSR entries, column word and value side by
// side, are packed whole rows at a time into chunks of 256 entries (64 lanes x
// one 16-byte quad each).  Rows are not padded: a row may start anywhere in a
// quad, its first word flagged by kQStart; a row with no off-diagonal entry
// holds one padding entry; padding entries (kQPad, value 0) complete the
// chunk's last quad as part of its last row.  P.qc[c] = (first row, quads
// used).  One wave takes one chunk at a time, one quad per lane:
//   - four ballots of the start flags give each entry's row within the chunk
//     and the chunk's row count; the gathers of x are issued, and in FP64 with
//     them the loads of x_r and the shift of the chunk's rows (one row per
//     lane, coalesced);
//   - the lane sums its four products row by row, a segmented scan across the
//     lanes carries the running sum of the row open at each lane's end, and
//     the lane holding a row's last entry stores the row's sum in the wave's
//     LDS slice;
//   - one lane per row applies the shift and the scale exactly as k_spmv does
//     and stores u (coalesced).
// The next chunk's entries load while the current one is summed; a wave's
// chunks follow chunk_sweep.  No row pointer is read.
constexpr int kERowMax = 64;

template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void k_spmve(Prob<T> P, const T* __restrict__ x, int step) {
    // FP64 loads x_r and the shift of the chunk's rows with the gathers (76 VGPRs, 6 waves per SIMD: 157 us
    // on the geometric workload against 160 us the other way); FP32 loads them in the row pass, which leaves
    // it 61 VGPRs and 8 waves (104 us against 108 us)
    constexpr bool EARLY = sizeof(T) == 8;
    __shared__ double wred[kWaves][2];
    __shared__ T rsum_all[kWaves][256];
    DevScalars* sc = P.sc;
    if (MODE == SPMV_LANCZOS && sc->done) return;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    T* rsum = rsum_all[wv];
    // the chunks of the dispatching XCD's eighth, round-robin over its waves
    int64_t clo, chi, cstep;
    chunk_sweep(P.nqc, wv, clo, chi, cstep);
    int2 cd = make_int2(0, 0);
    i32x4_t w = {kQPad, kQPad, kQPad, kQPad};
    T v[4] = {(T)0, (T)0, (T)0, (T)0};
    auto load_chunk = [&](int64_t c) {
        cd = P.qc[c];
        if (lane < cd.y) {
            const size_t q = (size_t)c * 64 + lane;
            w = reinterpret_cast<const i32x4_t*>(P.qw)[q];
            load_vals4(P.qv + 4 * q, v);
        } else {
            w = i32x4_t{kQPad, kQPad, kQPad, kQPad};
        }
    };
    auto term = [&](int wd, T val) { return (wd & kQPad) ? (T)0 : val * x[wd & kQColMask]; };
    T t[4] = {(T)0, (T)0, (T)0, (T)0};
    T xr0 = (T)0, sr0 = (T)0;
    bool s0 = false, s1 = false, s2 = false, s3 = false, e3 = false;
    int pc = 0, r0 = 0, nq = 0, nrows = 0;
    // the current chunk's flags and row numbers, and all of its loads
    auto issue = [&]() {
        r0 = cd.x;
        nq = cd.y;
        const bool valid = lane < nq;
        s0 = valid && (w.x & kQStart);
        s1 = valid && (w.y & kQStart);
        s2 = valid && (w.z & kQStart);
        s3 = valid && (w.w & kQStart);
        const unsigned long long b0 = __ballot(s0), b1 = __ballot(s1), b2 = __ballot(s2), b3 = __ballot(s3);
        const unsigned long long below = (1ull << lane) - 1ull;
        pc = __popcll(b0 & below) + __popcll(b1 & below) + __popcll(b2 & below) + __popcll(b3 & below);
        nrows = __popcll(b0) + __popcll(b1) + __popcll(b2) + __popcll(b3);
        e3 = valid && ((lane == nq - 1) || (lane < 63 && ((b0 >> (lane + 1)) & 1ull)));   // lane ends a row
        t[0] = term(w.x, v[0]);
        t[1] = term(w.y, v[1]);
        t[2] = term(w.z, v[2]);
        t[3] = term(w.w, v[3]);
        if (EARLY && lane < nrows) {
            xr0 = x[r0 + lane];
            sr0 = P.s[r0 + lane];
        }
    };
    if (clo < chi) {   // the first chunk's loads are in flight before the scale reduction
        load_chunk(clo);
        issue();
    }
    double xs;
    if (!spmv_scale<MODE>(P, step, true, xs)) return;
    const double xi = (MODE == SPMV_OBJ) ? sc->xi : 0.0;
    double acc0 = 0.0, acc1 = 0.0;
    for (int64_t c = clo; c < chi; c += cstep) {
        if (c != clo) issue();
        if (c + cstep < chi) load_chunk(c + cstep);
        const bool valid = lane < nq;
        // the lane's sum of the row open at its end (from its last start on)
        T a = t[0];
        a = s1 ? t[1] : a + t[1];
        a = s2 ? t[2] : a + t[2];
        a = s3 ? t[3] : a + t[3];
        if (!valid) a = (T)0;
        const int rid = pc + (int)s0 + (int)s1 + (int)s2 + (int)s3 - 1;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const T ya = __shfl_up(a, off, 64);
            const int yr = __shfl_up(rid, off, 64);
            if (lane >= off && yr == rid) a += ya;
        }
        T in = __shfl_up(a, 1, 64);   // running sum of the row open at this lane's start
        if (lane == 0) in = (T)0;
        if (valid) {
            int id = pc + (int)s0 - 1;
            T f = s0 ? t[0] : in + t[0];
            if (s1) rsum[id] = f;
            id += (int)s1;
            f = s1 ? t[1] : f + t[1];
            if (s2) rsum[id] = f;
            id += (int)s2;
            f = s2 ? t[2] : f + t[2];
            if (s3) rsum[id] = f;
            id += (int)s3;
            f = s3 ? t[3] : f + t[3];
            if (e3) rsum[id] = f;
        }
        wave_sync();
        for (int i = lane; i < nrows; i += 64) {
            const int64_t r = r0 + i;
            const double xr = (EARLY && i == lane) ? (double)xr0 : (double)x[r];
            const double sr = (EARLY && i == lane) ? (double)sr0 : (double)P.s[r];
            const double off = (double)rsum[i];
            if (MODE == SPMV_LANCZOS) {
                const T ut = (T)((off + sr * xr) * xs);
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
        }
        wave_sync();
    }
    if (MODE == SPMV_APPLY) return;
    acc0 = wave_sum(acc0);
    acc1 = wave_sum(acc1);
    if (lane == 0) {
        wred[wv][0] = acc0;
        wred[wv][1] = acc1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s0 = 0.0, s1 = 0.0;
        for (int i = 0; i < kWaves; ++i) {
            s0 += wred[i][0];
            s1 += wred[i][1];
        }
        if (MODE == SPMV_LANCZOS) {
            P.p_spmv[blockIdx.x] = s0;
        } else {
            P.p_obj[(size_t)blockIdx.x * 2 + 0] = s0;
            P.p_obj[(size_t)blockIdx.x * 2 + 1] = s1;
        }
    }
}

// The concurrent column segments over entry chunks (spmv_lanes = 1 with eight
// segments).  The columns are cut into kSegMax slices; for each slice the
// entries of every row that fall in it (its segment) are packed into chunks of
// 256 entries as in the entry-chunk layout, rows in order and whole, a segment
// with no entry or with more than kERowMax entries holding one padding entry.
// Workgroup b works on slice b mod 8, the XCD that dispatches it, so each XCD's
// L2 only holds its own eighth of x; the XCD's waves take its chunks
// round-robin and store each row's raw slice sum in xpart[slice * xld + r].
// The long segments (more than kERowMax entries, stored apart, their
// placeholder marked by column bit 0) are summed by the same waves after their
// chunks, one wave per segment; the chunk pass stores no sum for their rows.
// k_spmvx's launch is followed by k_xcombine, which adds the eight partials of
// each row.
struct XcArgs {
    const int32_t* qw;   // column words, 256 per chunk, flags as in the entry-chunk layout
    const void* qv;      // values beside the words (values stored), else null
    const int2* qc;      // per chunk: (first row, quads used)
    int64_t cb[kSegMax + 1];   // chunks of slice s: [cb[s], cb[s + 1])
    const int4* lseg;    // long segments: (row, first entry, entries, unused)
    int64_t lb[kSegMax + 1];   // long segments of slice s: [lb[s], lb[s + 1])
    const int32_t* lw;   // their column words
    const void* lv;      // and values (values stored), else null
    void* xpart;
    int64_t xld;
    int lanczos;
};

template <typename T, int FMT>
__device__ __forceinline__ T xc_term(const T* __restrict__ x, int w, T v) {
    if (w & kQPad) return (T)0;
    const T xv = x[w & kQColMask];
    if (FMT == FMT_VAL) return v * xv;
    if (FMT == FMT_SGN && w < 0) return -xv;
    return xv;
}

// The long segments of the sliced chunk layout (k0, k0 + step, ... below
// a.lb[seg + 1]): one wave per segment, each segment starting on a 16-byte quad
// (padding words complete its last quad), one quad of four entries per lane at
// a time; the sum is stored for the row, whose placeholder the chunk pass left
// alone.  The next segment's descriptor loads while one is summed.
template <typename T, int FMT>
__device__ __forceinline__ void long_segments(const T* __restrict__ x, const XcArgs& a, int seg, int64_t k0,
                                              int64_t step, T* out, int lane) {
    const T* lv = static_cast<const T*>(a.lv);
    const int64_t k1 = a.lb[seg + 1];
    int4 d = (k0 < k1) ? a.lseg[k0] : make_int4(0, 0, 0, 0);
    for (int64_t k = k0; k < k1; k += step) {
        const int4 cur = d;
        if (k + step < k1) d = a.lseg[k + step];
        const int nq = (cur.z + 3) >> 2;
        T acc = (T)0;
        for (int q = lane; q < nq; q += 64) {
            const int64_t i = (int64_t)cur.y + 4 * q;
            const i32x4_t w = *reinterpret_cast<const i32x4_t*>(a.lw + i);
            T v[4] = {(T)0, (T)0, (T)0, (T)0};
            if (FMT == FMT_VAL) load_vals4(lv + i, v);
            acc += (xc_term<T, FMT>(x, w.x, v[0]) + xc_term<T, FMT>(x, w.y, v[1])) +
                   (xc_term<T, FMT>(x, w.z, v[2]) + xc_term<T, FMT>(x, w.w, v[3]));
        }
        const double tot = wave_sum((double)acc);
        if (lane == 0) out[cur.x] = (T)tot;
    }
}

template <typename T, int FMT>
__global__ __launch_bounds__(kBlock) void k_spmvx(Prob<T> P, const T* __restrict__ x, XcArgs a) {
    __shared__ T rsum_all[kWaves][256];
    __shared__ unsigned char keep_all[kWaves][256];
    if (a.lanczos && P.sc->done) return;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    T* rsum = rsum_all[wv];
    unsigned char* keep = keep_all[wv];
    // a long segment's placeholder (its row's only entry) is not stored: its wave below stores the sum
    auto own = [](int wd) { return (unsigned char)((wd & (kQPad | kQStart | 1)) != (kQPad | kQStart | 1)); };
    const int seg = blockIdx.x % kXcd;
    const int64_t cstep = (int64_t)(gridDim.x / kXcd) * kWaves;
    const int64_t clo = a.cb[seg] + (int64_t)(blockIdx.x / kXcd) * kWaves + wv, chi = a.cb[seg + 1];
    T* out = static_cast<T*>(a.xpart) + (size_t)seg * a.xld;
    const T* qv = static_cast<const T*>(a.qv);
    int2 cd = make_int2(0, 0);
    i32x4_t w = {kQPad, kQPad, kQPad, kQPad};
    T v[4] = {(T)0, (T)0, (T)0, (T)0};
    auto load_chunk = [&](int64_t c) {
        cd = a.qc[c];
        if (lane < cd.y) {
            const size_t q = (size_t)c * 64 + lane;
            w = reinterpret_cast<const i32x4_t*>(a.qw)[q];
            if (FMT == FMT_VAL) load_vals4(qv + 4 * q, v);
        } else {
            w = i32x4_t{kQPad, kQPad, kQPad, kQPad};
        }
    };
    if (clo < chi) load_chunk(clo);
    for (int64_t c = clo; c < chi; c += cstep) {
        const int r0 = cd.x, nq = cd.y;
        const bool valid = lane < nq;
        const bool s0 = valid && (w.x & kQStart), s1 = valid && (w.y & kQStart);
        const bool s2 = valid && (w.z & kQStart), s3 = valid && (w.w & kQStart);
        const unsigned long long b0 = __ballot(s0), b1 = __ballot(s1), b2 = __ballot(s2), b3 = __ballot(s3);
        const unsigned long long below = (1ull << lane) - 1ull;
        const int pc = __popcll(b0 & below) + __popcll(b1 & below) + __popcll(b2 & below) + __popcll(b3 & below);
        const int nrows = __popcll(b0) + __popcll(b1) + __popcll(b2) + __popcll(b3);
        const bool e3 = valid && ((lane == nq - 1) || (lane < 63 && ((b0 >> (lane + 1)) & 1ull)));
        if (valid) {   // each row by its first entry: a long segment's placeholder is not stored
            int id = pc;
            if (s0) keep[id++] = own(w.x);
            if (s1) keep[id++] = own(w.y);
            if (s2) keep[id++] = own(w.z);
            if (s3) keep[id] = own(w.w);
        }
        const T t0 = xc_term<T, FMT>(x, w.x, v[0]), t1 = xc_term<T, FMT>(x, w.y, v[1]);
        const T t2 = xc_term<T, FMT>(x, w.z, v[2]), t3 = xc_term<T, FMT>(x, w.w, v[3]);
        if (c + cstep < chi) load_chunk(c + cstep);
        T s = t0;
        s = s1 ? t1 : s + t1;
        s = s2 ? t2 : s + t2;
        s = s3 ? t3 : s + t3;
        if (!valid) s = (T)0;
        const int rid = pc + (int)s0 + (int)s1 + (int)s2 + (int)s3 - 1;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const T ya = __shfl_up(s, off, 64);
            const int yr = __shfl_up(rid, off, 64);
            if (lane >= off && yr == rid) s += ya;
        }
        T in = __shfl_up(s, 1, 64);
        if (lane == 0) in = (T)0;
        if (valid) {
            int id = pc + (int)s0 - 1;
            T f = s0 ? t0 : in + t0;
            if (s1) rsum[id] = f;
            id += (int)s1;
            f = s1 ? t1 : f + t1;
            if (s2) rsum[id] = f;
            id += (int)s2;
            f = s2 ? t2 : f + t2;
            if (s3) rsum[id] = f;
            id += (int)s3;
            f = s3 ? t3 : f + t3;
            if (e3) rsum[id] = f;
        }
        wave_sync();
        for (int i = lane; i < nrows; i += 64)
            if (keep[i]) out[r0 + i] = rsum[i];
        wave_sync();
    }
    // then the slice's long segments, round-robin over the XCD's waves
    long_segments<T, FMT>(x, a, seg, a.lb[seg] + (int64_t)(blockIdx.x / kXcd) * kWaves + wv, cstep, out, lane);
}

// Rows of the workgroup's share in quads: for (qd...) { r = 4 qd; m = rows in quad }.
#define SCG_FOR_QUADS(n)                                                   \
    int64_t qlo_, qhi_;                                                    \
    split_range(((n) + 3) / 4, xcd_lid(), gridDim.x, qlo_, qhi_);          \
    for (int64_t qd = qlo_ + threadIdx.x; qd < qhi_; qd += kBlock)


// omega_step from the SpMV partials; w = u - omega v_step - rho v_{step-1}
// stored as V[step+1]; partial sums of ||w||^2 (unless reorthogonalising).
// With accum (the second pass of a regenerated basis) it also adds
// coef_step * V[step] into the FP64 Ritz accumulator, in the order and with
// the rounding k_ritz uses.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_lupdate(Prob<T> P, int step, int with_norm, int accum) {
    DevScalars* sc = P.sc;
    if (sc->done) return;
    const int64_t n = P.n;
    const T* vi = vcol(P, step);
    const T* vm = (step > 0) ? vcol(P, step - 1) : vi;
    T* out = vcol(P, step + 1);
    int64_t qlo, qhi;
    split_range((n + 3) / 4, xcd_lid(), gridDim.x, qlo, qhi);
    int64_t qd = qlo + threadIdx.x;
    double u4[4], i4[4], m4[4], a4[4];
    if (qd < qhi) {   // first quad in flight before the omega reduction
        const int64_t r = 4 * qd;
        const int m = quad_rows(r, n);
        ld4(P.u + r, m, u4);
        ld4(vi + r, m, i4);
        ld4(vm + r, m, m4);
        if (accum) {
            if (step > 0) ld4(P.racc + r, m, a4);
            else a4[0] = a4[1] = a4[2] = a4[3] = 0.0;
        }
    }
    const double cj = accum ? sc->coef[step] : 0.0;
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
    const double a1 = om * si, a2 = rp * sp;
    double acc = 0.0;
    while (qd < qhi) {
        const int64_t r = 4 * qd;
        const int m = quad_rows(r, n);
        double w[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) w[j] = u4[j] - a1 * i4[j] - a2 * m4[j];
        st4(out + r, m, w);
#pragma unroll
        for (int j = 0; j < 4; ++j) acc += w[j] * w[j];
        if (accum) {
#pragma unroll
            for (int j = 0; j < 4; ++j) a4[j] += cj * i4[j];
            st4(P.racc + r, m, a4);
        }
        qd += kBlock;
        if (qd < qhi) {
            const int64_t r2 = 4 * qd;
            const int m2 = quad_rows(r2, n);
            ld4(P.u + r2, m2, u4);
            ld4(vi + r2, m2, i4);
            ld4(vm + r2, m2, m4);
            if (accum) {
                if (step > 0) ld4(P.racc + r2, m2, a4);
                else a4[0] = a4[1] = a4[2] = a4[3] = 0.0;
            }
        }
    }
    if (with_norm) {
        double v[1] = {acc};
        write_partials<1>(v, P.p_upd);
    }
}

// Reorthogonalisation, part 1: per-workgroup partials of v_j^T w, j = j0 .. step.
// j0 = 0 for the full pass, step - 1 (or 0) for the local one, which only needs
// the vectors a regenerated basis keeps.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_reorth_dot(Prob<T> P, int step, int j0) {
    DevScalars* sc = P.sc;
    if (sc->done) return;
    const int64_t n = P.n;
    const int nj = step + 1 - j0;
    const T* w = vcol(P, step + 1);
    int64_t lo, hi;
    split_range(n, xcd_lid(), gridDim.x, lo, hi);
    __shared__ double red[kWaves];
    for (int jj = 0; jj < nj; ++jj) {
        const T* vj = vcol(P, j0 + jj);
        double acc = 0.0;
        for (int64_t r = lo + threadIdx.x; r < hi; r += kBlock) acc += (double)vj[r] * (double)w[r];
        const double bs = block_sum(acc, red);
        if (threadIdx.x == 0) P.p_h[(size_t)blockIdx.x * nj + jj] = bs;
    }
}

// Part 2 (one workgroup): h_j = inv_j * sum of the partials, j = j0 .. step.
__global__ __launch_bounds__(kBlock) void k_reduce_h(DevScalars* sc, const double* p_h, int G, int step, int j0) {
    if (sc->done) return;
    __shared__ double red[kWaves];
    const int nj = step + 1 - j0;
    for (int jj = 0; jj < nj; ++jj) {
        double s = 0.0;
        for (int g = threadIdx.x; g < G; g += kBlock) s += p_h[(size_t)g * nj + jj];
        s = block_sum(s, red);
        if (threadIdx.x == 0) sc->h[j0 + jj] = s * sc->inv[j0 + jj];
    }
}

// Part 3: w <- w - sum_j h_j v_hat_j (j = j0 .. step); partial sums of ||w||^2.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_reorth_apply(Prob<T> P, int step, int j0) {
    DevScalars* sc = P.sc;
    if (sc->done) return;
    __shared__ double hc[kQCap];
    const int nj = step + 1 - j0;
    for (int jj = threadIdx.x; jj < nj; jj += kBlock) hc[jj] = sc->h[j0 + jj] * sc->inv[j0 + jj];
    __syncthreads();
    const int64_t n = P.n;
    T* w = vcol(P, step + 1);
    int64_t lo, hi;
    split_range(n, xcd_lid(), gridDim.x, lo, hi);
    double acc = 0.0;
    for (int64_t r = lo + threadIdx.x; r < hi; r += kBlock) {
        double a = 0.0;
        for (int jj = 0; jj < nj; ++jj) a += hc[jj] * (double)vcol(P, j0 + jj)[r];
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
__global__ __launch_bounds__(kBlock) void k_tridiag(Prob<T> P, int q) {
    __shared__ double d[kQCap], e[kQCap], e2[kQCap], dp[kQCap], dm[kQCap], x[kQCap];
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
        for (int i = threadIdx.x; i < k; i += kBlock) {
            d[i] = (i == q - 1) ? tot[0] : sc->omega[i];
            if (i < k - 1) e[i] = sc->rho[i];
        }
    } else {
        k = sc->k;
        for (int i = threadIdx.x; i < k; i += kBlock) {
            d[i] = sc->omega[i];
            if (i < k - 1) e[i] = sc->rho[i];
        }
    }
    __syncthreads();
    if (threadIdx.x < 64) tridiag_min_eig(d, e, k, e2, dp, dm, x, &xi);
    __syncthreads();
    for (int i = threadIdx.x; i < k; i += kBlock) sc->coef[i] = x[i] * sc->inv[i];
    if (threadIdx.x == 0) {
        sc->kr = k;
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
    double acc[RB + 1];
#pragma unroll
    for (int c = 0; c <= RB; ++c) acc[c] = 0.0;
    SCG_FOR_QUADS(n) {
        const int64_t r = 4 * qd;
        const int m = quad_rows(r, n);
        double a[4] = {0, 0, 0, 0};
        for (int j = 0; j < k; ++j) {
            double t[4];
            ld4(P.V + (size_t)j * P.ld + r, m, t);
            const double cj = coef[j];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] += cj * t[i];
        }
        st4(P.v + r, m, a);
        // norm and v^T Omega of the stored (rounded) vector, which every later step uses
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = (double)(T)a[i];
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[0] += a[i] * a[i];
#pragma unroll
        for (int c = 0; c < RB; ++c)
            if (c < R) {
                double o[4];
                if (P.Om) ld4(P.Om + (size_t)c * P.ld + r, m, o);
                else omega_quad<T>(P.seed, P.instance, qd, c, m, o);
                acc[c + 1] += a[0] * o[0] + a[1] * o[1] + a[2] * o[2] + a[3] * o[3];
            }
    }
    write_partials<RB + 1>(acc, P.p_ritz);
}

// Regenerated basis: the second pass ran k_lupdate for steps 0 .. min(k, q-1)-1
// (a breakdown stops it after step k-1; without one the loop ends at q-2), so
// racc holds that many terms and the last one, coef_{k-1} V[k-1], is added here
// when k = q.  Stored, norm and v^T Omega as k_ritz; restores k.
template <typename T, int RB>
__global__ __launch_bounds__(kBlock) void k_ritz_regen(Prob<T> P, int q) {
    DevScalars* sc = P.sc;
    const int k = sc->kr;
    const int na = (k < q - 1) ? k : q - 1;
    const bool add_last = na < k;
    const double cl = sc->coef[k - 1];
    const T* Vl = vcol(P, k - 1);
    if (blockIdx.x == 0 && threadIdx.x == 0) sc->k = k;
    const int64_t n = P.n;
    const int R = P.R;
    double acc[RB + 1];
#pragma unroll
    for (int c = 0; c <= RB; ++c) acc[c] = 0.0;
    SCG_FOR_QUADS(n) {
        const int64_t r = 4 * qd;
        const int m = quad_rows(r, n);
        double a[4] = {0, 0, 0, 0};
        if (na > 0) ld4(P.racc + r, m, a);
        if (add_last) {
            double t[4];
            ld4(Vl + r, m, t);
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] += cl * t[i];
        }
        st4(P.v + r, m, a);
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = (double)(T)a[i];
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[0] += a[i] * a[i];
#pragma unroll
        for (int c = 0; c < RB; ++c)
            if (c < R) {
                double o[4];
                if (P.Om) ld4(P.Om + (size_t)c * P.ld + r, m, o);
                else omega_quad<T>(P.seed, P.instance, qd, c, m, o);
                acc[c + 1] += a[0] * o[0] + a[1] * o[1] + a[2] * o[2] + a[3] * o[3];
            }
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

// Euclidean projection onto the box [lo, hi] (Appendix D.3), entrywise.
__device__ __forceinline__ double box_proj(double u, double lo, double hi) { return fmin(fmax(u, lo), hi); }

// Ball constraint set {||u - b|| <= r}: the projection of u is
// b + (u - b) min(1, r / ||u - b||); ||u - b||^2 comes from k_ball_norm's partials.
template <typename T>
__device__ __forceinline__ double ball_factor(const Prob<T>& P) {
    double tot[1];
    reduce_partials<1>(P.p_ball, P.G, tot);
    const double nd = sqrt(tot[0]);
    return (nd <= P.ball_r) ? 1.0 : P.ball_r / nd;
}

// Partial sums of ||z + y / beta - b||^2 (the point the ball slack projects).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_ball_norm(Prob<T> P, double beta) {
    const int64_t n = P.n;
    double a = 0.0;
    SCG_FOR_QUADS(n) {
        const int64_t r = 4 * qd;
        const int m = quad_rows(r, n);
        double z4[4], y4[4], b4[4];
        ld4(P.z + r, m, z4);
        ld4(P.y + r, m, y4);
        ld4(P.b + r, m, b4);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double d = (j < m) ? (z4[j] + y4[j] / beta) - b4[j] : 0.0;
            a += d * d;
        }
    }
    double v[1] = {a};
    write_partials<1>(v, P.p_ball);
}

// Ball, after the primal update: with w_bar = b + cb (z + y / beta_{t+1} - b),
// partial sums of ||z - w_bar||^2, ||y||^2 and y^T (z - w_bar).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_ball_r2(Prob<T> P, IterArgs it) {
    it = resolve_iter(it, P.sc);
    const int64_t n = P.n;
    const double cb = ball_factor(P);
    double a[3] = {0.0, 0.0, 0.0};
    SCG_FOR_QUADS(n) {
        const int64_t r = 4 * qd;
        const int m = quad_rows(r, n);
        double z4[4], y4[4], b4[4];
        ld4(P.z + r, m, z4);
        ld4(P.y + r, m, y4);
        ld4(P.b + r, m, b4);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (j < m) {
                const double d = z4[j] - (b4[j] + cb * ((z4[j] + y4[j] / it.beta_next) - b4[j]));
                a[0] += d * d;
                a[1] += y4[j] * y4[j];
                a[2] += y4[j] * d;
            }
        }
    }
    write_partials<3>(a, P.p_ball2);
}

// Shift, start vector, and partial sums of the state before the update.
// Box constraint set: the shift uses the slack w = proj_K(z + y / beta) in
// place of b (alg:full-sketchy-cgal-supp).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_prep(Prob<T> P, IterArgs it) {
    it = resolve_iter(it, P.sc);
    DevScalars* sc = P.sc;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->done = 0;
        sc->k = 0;
    }
    const int64_t n = P.n;
    double cb = 0.0;   // ball: the slack is b + cb (z + y / beta - b)
    if (P.ball) cb = ball_factor(P);
    double a[kWPrep] = {0, 0, 0, 0, 0, 0};
    SCG_FOR_QUADS(n) {
        const int64_t r = 4 * qd;
        const int m = quad_rows(r, n);
        double g[4], z4[4], y4[4], b4[4], d4[4], s4[4], lo4[4], hi4[4];
        normal4(it.seed, (uint64_t)qd, (uint64_t)it.t, it.instance, 0ull, g);
        ld4(P.z + r, m, z4);
        ld4(P.y + r, m, y4);
        ld4(P.b + r, m, b4);
        ld4(P.dC + r, m, d4);
        if (P.lo) {
            ld4(P.lo + r, m, lo4);
            ld4(P.hi + r, m, hi4);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double zb = z4[j] - b4[j];
            const double zw = P.lo ? z4[j] - box_proj(z4[j] + y4[j] / it.beta, lo4[j], hi4[j])
                                   : (P.ball ? z4[j] - (b4[j] + cb * ((z4[j] + y4[j] / it.beta) - b4[j])) : zb);
            s4[j] = d4[j] + (y4[j] + it.beta * zw);
            if (j < m) {
                a[1] += y4[j] * b4[j];
                a[2] += zb * (z4[j] + b4[j]);
                a[3] += (y4[j] + it.beta * zw) * z4[j];
                a[4] += zb * zb;
                a[5] += b4[j] * b4[j];
            } else {
                g[j] = 0.0;
            }
        }
        st4(P.s + r, m, s4);
        st4(P.V + r, m, g);
#pragma unroll
        for (int j = 0; j < 4; ++j) a[0] += g[j] * g[j];
    }
    write_partials<kWPrep>(a, P.p_prep);
}

// z update with H = ha v v^T (ha = alpha, or 0 when tr X <= alpha and xi >= 0);
// partial sums of ||z - w_bar||^2 with the slack w_bar = b, or proj_K(z + y / beta_{t+1})
// for a box, (y^T y, y^T (z - w_bar) for the K guard) and dist_K(z)^2 (box).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_primal(Prob<T> P, IterArgs it) {
    it = resolve_iter(it, P.sc);
    DevScalars* sc = P.sc;
    const double iv = sc->inv_vnorm;
    const bool hon = (P.trace_mode == 0) || (sc->xi < 0.0);
    const double ea = hon ? it.eta * it.alpha : 0.0;
    const double keep = 1.0 - it.eta;
    const bool guard = isfinite(it.K);
    const bool box = P.lo != nullptr;
    const int64_t n = P.n;
    double a[kWPrimal] = {0, 0, 0, 0};
    SCG_FOR_QUADS(n) {
        const int64_t r = 4 * qd;
        const int m = quad_rows(r, n);
        double v4[4], z4[4], b4[4], y4[4], lo4[4], hi4[4];
        ld4(P.v + r, m, v4);
        ld4(P.z + r, m, z4);
        ld4(P.b + r, m, b4);
        if (guard || box) ld4(P.y + r, m, y4);
        if (box) {
            ld4(P.lo + r, m, lo4);
            ld4(P.hi + r, m, hi4);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double vh = v4[j] * iv;
            z4[j] = keep * z4[j] + ea * (vh * vh);
            double dd = 0.0;
            if (j < m) {
                if (box) {
                    dd = z4[j] - box_proj(z4[j] + y4[j] / it.beta_next, lo4[j], hi4[j]);
                    const double dk = z4[j] - box_proj(z4[j], lo4[j], hi4[j]);
                    a[3] += dk * dk;
                } else {
                    dd = z4[j] - b4[j];
                }
            }
            a[0] += dd * dd;
            if (guard) {
                a[1] += y4[j] * y4[j];
                a[2] += y4[j] * dd;
            }
        }
        st4(P.z + r, m, z4);
    }
    write_partials<kWPrimal>(a, P.p_primal);
    if (blockIdx.x == 0) {   // v^T C v and the residual, recorded for the log
        double tot[kWObj];
        reduce_partials<kWObj>(P.p_obj, P.Gs, tot);
        if (threadIdx.x == 0) {
            sc->cv = tot[0];
            sc->resid2 = tot[1];
            if (!isfinite(tot[0])) sc->flags |= 2;
        }
    }
}

// Dual step size (eqn sketchy-cgal-dual-step; the same bound in Appendix D.4),
// K guard, trackers and log; y <- y + gamma (z - w_bar) (w_bar as in k_primal);
// S <- (1-eta) S + eta ha v_hat (v_hat^T Omega).
template <typename T, int RB>
__global__ __launch_bounds__(kBlock) void k_dual_sketch(Prob<T> P, IterArgs it) {
    it = resolve_iter(it, P.sc);
    DevScalars* sc = P.sc;
    const int64_t n = P.n;
    const bool box = P.lo != nullptr;
    int64_t qlo, qhi;
    split_range((n + 3) / 4, xcd_lid(), gridDim.x, qlo, qhi);
    int64_t qd = qlo + threadIdx.x;
    double y4[4], z4[4], b4[4], v4[4], lo4[4], hi4[4];
    auto load = [&](int64_t r, int m) {
        ld4(P.y + r, m, y4);
        ld4(P.z + r, m, z4);
        ld4(P.b + r, m, b4);
        ld4(P.v + r, m, v4);
        if (box) {
            ld4(P.lo + r, m, lo4);
            ld4(P.hi + r, m, hi4);
        }
    };
    if (qd < qhi) load(4 * qd, quad_rows(4 * qd, n));   // first quad in flight before the reduction
    double tot[kWPrimal];
    reduce_partials<kWPrimal>(P.p_primal, P.G, tot);
    // ball: ||z - w_bar||^2, ||y||^2, y^T (z - w_bar) from k_ball_r2, and the slack factor
    double cb = 0.0, tb[3] = {0.0, 0.0, 0.0};
    if (P.ball) {
        cb = ball_factor(P);
        reduce_partials<3>(P.p_ball2, P.G, tb);
    }
    const double r2 = P.ball ? tb[0] : tot[0];
    double gamma = (r2 == 0.0) ? it.beta0
                               : fmin(it.beta0, 4.0 * it.alpha * it.alpha * it.beta0 / (pow(it.t + 1.0, 1.5) * r2));
    if (isfinite(it.K)) {
        const double ny2 = P.ball ? tb[1] + 2.0 * gamma * tb[2] + gamma * gamma * r2
                                  : tot[1] + 2.0 * gamma * tot[2] + gamma * gamma * r2;
        if (sqrt(fmax(ny2, 0.0)) > it.K) gamma = 0.0;
    }
    const double iv = sc->inv_vnorm;
    const bool hon = (P.trace_mode == 0) || (sc->xi < 0.0);
    const double ea = hon ? it.eta * it.alpha : 0.0;
    const double keep = 1.0 - it.eta;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->gamma_eff = gamma;
        const double p_old = sc->p;
        const double xi = sc->xi;
        // the stopping quantities are those of the model problem (diag X = b, tr X = alpha)
        const bool model = !box && !P.ball && P.trace_mode == 0;
        const double stop_obj =
            model ? (p_old + sc->d_yb + 0.5 * it.beta * sc->d_zz - it.alpha * xi) / (1.0 + fabs(p_old)) : NAN;
        const double gap = p_old + sc->d_gapdot - (hon ? it.alpha * xi : 0.0);
        const double stop_feas = model ? sqrt(sc->d_zb2) / (1.0 + sqrt(sc->b2)) : NAN;
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
            // dist_K(z_{t+1}): the box from k_primal, the ball in closed form
            L.infeas = box ? sqrt(tot[3]) : (P.ball ? fmax(0.0, sqrt(tot[0]) - P.ball_r) : sqrt(r2));
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
    while (qd < qhi) {
        const int64_t r = 4 * qd;
        const int m = quad_rows(r, n);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double wb = box ? box_proj(z4[j] + y4[j] / it.beta_next, lo4[j], hi4[j])
                                  : (P.ball ? b4[j] + cb * ((z4[j] + y4[j] / it.beta_next) - b4[j]) : b4[j]);
            y4[j] += gamma * (z4[j] - wb);
            v4[j] = ea * (v4[j] * iv);
        }
        st4(P.y + r, m, y4);
        double s4[RB][4];
#pragma unroll
        for (int c = 0; c < RB; ++c)
            if (c < R) ld4(P.S + (size_t)c * P.ld + r, m, s4[c]);
#pragma unroll
        for (int c = 0; c < RB; ++c)
            if (c < R) {
#pragma unroll
                for (int j = 0; j < 4; ++j) s4[c][j] = keep * s4[c][j] + v4[j] * cw[c];
                st4(P.S + (size_t)c * P.ld + r, m, s4[c]);
            }
        qd += kBlock;
        if (qd < qhi) load(4 * qd, quad_rows(4 * qd, n));
    }
}

}  // namespace scg
