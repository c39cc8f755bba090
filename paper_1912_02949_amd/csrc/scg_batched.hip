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
#include <type_traits>
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
constexpr int kLongRow = 64;        // rows with more off-diagonal entries are summed by a whole wave
constexpr size_t kLdsBudget = 136 * 1024;   // dynamic LDS: the vector being multiplied + slice table

// LDS slots of the workgroup reduction results
enum : int {
    SO_OM = 0, SO_RHO = 1, SO_PREP = 2,          // 6 slots
    SO_OBJ = 8,                                  // 2 slots
    SO_PRIM = 10,                                // 3 slots
    SO_RITZ = 16,                                // kRedMax slots
    SO_N = SO_RITZ + kRedMax
};

struct BatchInst {
    int64_t row0;      // first row in the concatenated CSR numbering
    int64_t pos0;      // offset of the instance's vectors (a multiple of 64 elements)
    int64_t off_V;     // element offset of the instance's Lanczos basis
    int64_t off_OS;    // element offset of the instance's Omega and S
    int64_t ld;        // column stride of its basis, Omega, S (n rounded up to 64)
    int64_t sl0;       // first entry of its slices in the slice table
    int n;
    int id;            // Philox counter word of the instance
    int nshort;        // rows stored in slices; the remaining n - nshort rows are long
    int nsl;           // slices
    double cval;       // common off-diagonal value / magnitude, scaled (compressed formats)
    double alpha_s;    // alpha in scaled units
    double c_F, alpha; // scaling constants
    double beta0;      // the instance's initial penalty beta_0 (its schedule beta_t = beta_0 sqrt(t + 1))
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
    const int32_t* rp;      // off-diagonal row pointers, concatenated rows (at row0)
    const CT* col;          // instance-local column (sign in the top bit for FMT_SGN)
    const T* val;
    // per-instance vectors at pos0
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
    // sliced layout (LDS path): positions are short rows by decreasing length, then long rows
    const int32_t* perm;    // position -> local row (at pos0)
    T* s_pos;               // shift in position order (at pos0)
    const double* dC_pos;   // diagonal of C in position order (at pos0)
    const int2* sdesc;      // slice table: element offset of the slice, width (even)
    const CT* scol;         // slice entries: pair p of lane l at offset + 2 (64 p + l)
    const T* sval;
    int desc_lds_off;       // byte offset of the slice table in dynamic LDS
    int tile;               // columns per LDS tile of the two-tile kernel (a multiple of 64)
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

// rows (or positions) of quad qd that exist: 4, or fewer in the tail quad
__device__ __forceinline__ int quad_m(int qd, int n) {
    const int r = 4 * qd;
    return (r >= n) ? 0 : ((n - r >= 4) ? 4 : n - r);
}
__device__ __forceinline__ void ldi4(const int32_t* p, int m, int (&o)[4]) {
    if (m == 4) {
        const int4 t = *reinterpret_cast<const int4*>(p);
        o[0] = t.x; o[1] = t.y; o[2] = t.z; o[3] = t.w;
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) o[j] = (j < m) ? p[j] : 0;
    }
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

// Off-diagonal entry (column word cw, value vv) times x; the common value of
// the compressed formats is applied once per row by the caller.
template <typename T, typename CT, int FMT>
__device__ __forceinline__ T nzv(CT cw, T vv, const T* x) {
    if (FMT == FMT_VAL) return vv * x[(int)cw];
    if (FMT == FMT_PAT) return x[(int)cw];
    const T xv = x[col_index(cw)];
    return col_neg(cw) ? -xv : xv;
}
template <typename T, typename CT, int FMT>
__device__ __forceinline__ T nz(CT cw, const T* val, int e, const T* x) {
    return nzv<T, CT, FMT>(cw, (FMT == FMT_VAL) ? val[e] : (T)0, x);
}
// The same term with x held as the column tile [lo, hi) (x[c - lo]); entries
// of other columns, and the padding index n (hi <= n), contribute 0.  TL =
// false is nzv itself.
template <typename T, typename CT, int FMT, bool TL>
__device__ __forceinline__ T nzt(CT cw, T vv, const T* x, int lo, int hi) {
    if (!TL) return nzv<T, CT, FMT>(cw, vv, x);
    const int c = (FMT == FMT_SGN) ? col_index(cw) : (int)cw;
    if (c < lo || c >= hi) return (T)0;
    const T xv = x[c - lo];
    if (FMT == FMT_VAL) return vv * xv;
    if (FMT == FMT_PAT) return xv;
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

// Two consecutive slice entries of one lane, loaded as one word and split on use.
template <typename CT> struct PairW;
template <> struct PairW<uint16_t> { using type = uint32_t; };
template <> struct PairW<int32_t> { using type = int2; };
template <typename CT>
__device__ __forceinline__ typename PairW<CT>::type load_cw(const CT* p) {
    return *reinterpret_cast<const typename PairW<CT>::type*>(p);
}
__device__ __forceinline__ uint16_t pair_lo(uint32_t w) { return (uint16_t)(w & 0xffffu); }
__device__ __forceinline__ uint16_t pair_hi(uint32_t w) { return (uint16_t)(w >> 16); }
__device__ __forceinline__ int32_t pair_lo(int2 w) { return w.x; }
__device__ __forceinline__ int32_t pair_hi(int2 w) { return w.y; }
template <typename T> struct PairV;
template <> struct PairV<float> { using type = float2; };
template <> struct PairV<double> { using type = double2; };

// Row products over the sliced layout, the vector in LDS (xl, with xl[n] = 0
// for the padding entries).  Wave w owns slices w, w + 16, ...; four of them
// (their entries, rows, shifts and, for the objective, diagonals) are loaded
// before any is consumed.  `fin(p, row, a, shift, diag)` receives each row's
// off-diagonal sum (without the common value of the compressed formats).
// With TL, xl holds only the columns [lo, hi) of the vector (at xl[c - lo])
// and the sums are those of the tile's columns.
template <typename T, typename CT, int FMT, bool OBJ, bool TL = false, typename Fin>
__device__ __forceinline__ void sell_product(const int2* desc, int nsl, int nshort, int n, const int32_t* perm,
                                             const T* sp, const double* dCp, const CT* scol, const T* sval,
                                             const int32_t* rp, const CT* col, const T* val, const T* xl, Fin fin,
                                             int lo = 0, int hi = 0) {
    using PW = typename PairW<CT>::type;
    using PV = typename PairV<T>::type;
    constexpr int PF = (sizeof(CT) == 2 && FMT != FMT_VAL) ? 6 : 4;   // pairs loaded ahead per slice
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    for (int kb = wv; kb < nsl; kb += 4 * kBW) {
        int2 d[4];
        int row[4];
        T sv[4];
        double dg[4];
        PW cw[4][PF];
        PV vw[4][(FMT == FMT_VAL) ? PF : 1];
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int k = kb + g * kBW;
            d[g] = (k < nsl) ? desc[k] : make_int2(0, 0);
            const int p = k * 64 + lane;
            const bool ok = (k < nsl) && (p < nshort);
            row[g] = ok ? perm[p] : -1;
            sv[g] = ok ? sp[p] : (T)0;
            dg[g] = (OBJ && ok) ? dCp[p] : 0.0;
#pragma unroll
            for (int pp = 0; pp < PF; ++pp) {
                const size_t o = (size_t)d[g].x + 2 * (size_t)(pp * 64 + lane);
                if (2 * pp < d[g].y) {
                    cw[g][pp] = load_cw(scol + o);
                    if (FMT == FMT_VAL) vw[g][pp] = *reinterpret_cast<const PV*>(sval + o);
                }
            }
        }
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            T a = 0;
#pragma unroll
            for (int pp = 0; pp < PF; ++pp) {
                if (2 * pp < d[g].y) {
                    const T v0 = (FMT == FMT_VAL) ? (T)vw[g][pp].x : (T)0;
                    const T v1 = (FMT == FMT_VAL) ? (T)vw[g][pp].y : (T)0;
                    a += nzt<T, CT, FMT, TL>((CT)pair_lo(cw[g][pp]), v0, xl, lo, hi) +
                         nzt<T, CT, FMT, TL>((CT)pair_hi(cw[g][pp]), v1, xl, lo, hi);
                }
            }
            for (int pp = PF; 2 * pp < d[g].y; ++pp) {   // wide slices
                const size_t o = (size_t)d[g].x + 2 * (size_t)(pp * 64 + lane);
                const PW w = load_cw(scol + o);
                T v0 = 0, v1 = 0;
                if (FMT == FMT_VAL) {
                    const PV vv = *reinterpret_cast<const PV*>(sval + o);
                    v0 = vv.x;
                    v1 = vv.y;
                }
                a += nzt<T, CT, FMT, TL>((CT)pair_lo(w), v0, xl, lo, hi) + nzt<T, CT, FMT, TL>((CT)pair_hi(w), v1, xl, lo, hi);
            }
            if (row[g] >= 0) fin((kb + g * kBW) * 64 + lane, row[g], (double)a, (double)sv[g], dg[g]);
        }
    }
    // long rows: one wave each
    for (int p = nshort + wv; p < n; p += kBW) {
        const int r = perm[p];
        const int e0 = rp[r], e1 = rp[r + 1];
        T a = 0;
        for (int e = e0 + lane; e < e1; e += 64)
            a += nzt<T, CT, FMT, TL>(col[e], (FMT == FMT_VAL) ? val[e] : (T)0, xl, lo, hi);
        const double tot = wave_sum((double)a);
        if (lane == 0) fin(p, r, tot, (double)sp[p], OBJ ? dCp[p] : 0.0);
    }
}

// Shared end of an iteration (the objective products are already in
// so[SO_OBJ], so[SO_OBJ + 1]; the Ritz vector is vget(r) and v_hat = v iv):
// primal update of z, the dual step size (eqn sketchy-cgal-dual-step) with
// the K guard, the dual and sketch updates, the trackers and the record.
template <typename T, typename CT, typename VG>
__device__ __forceinline__ void iteration_tail(const BatchArgs<T, CT>& A, const BatchInst& D, BatchScal* G, int ii,
                                               int t, int q, int k, double xi, double beta, double eta, double iv,
                                               double vnorm2, VG vget, double* red, double* so) {
    const int tid = threadIdx.x;
    const int n = D.n;
    const int64_t ld = D.ld;
    const double alpha = D.alpha_s;
    double* z = A.z + D.pos0;
    double* y = A.y + D.pos0;
    const double* b = A.b + D.pos0;
    T* S = A.S + D.off_OS;
    const int R = A.R;
    const double ea = eta * alpha, keep = 1.0 - eta;
    const bool guard = isfinite(A.K);
    {
        double pa[3] = {0.0, 0.0, 0.0};
        for (int qd = tid; 4 * qd < n; qd += kBT) {
            const int m = quad_m(qd, n), r = 4 * qd;
            double z4[4], b4[4], y4[4];
            ld4(z + r, m, z4);
            ld4(b + r, m, b4);
            if (guard) ld4(y + r, m, y4);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const double vh = (j < m) ? vget(r + j) * iv : 0.0;
                z4[j] = keep * z4[j] + ea * (vh * vh);
                const double dd = (j < m) ? z4[j] - b4[j] : 0.0;
                pa[0] += dd * dd;
                if (guard) {
                    pa[1] += y4[j] * y4[j];
                    pa[2] += y4[j] * dd;
                }
            }
            st4(z + r, m, z4);
        }
        breduce<3>(pa, red, so + SO_PRIM);
    }
    const double r2 = so[SO_PRIM];
    double gamma = (r2 == 0.0) ? D.beta0 : fmin(D.beta0, 4.0 * alpha * alpha * D.beta0 / (pow(t + 1.0, 1.5) * r2));
    if (guard) {
        const double ny2 = so[SO_PRIM + 1] + 2.0 * gamma * so[SO_PRIM + 2] + gamma * gamma * r2;
        if (sqrt(fmax(ny2, 0.0)) > A.K) gamma = 0.0;
    }
    for (int qd = tid; 4 * qd < n; qd += kBT) {
        const int m = quad_m(qd, n), r = 4 * qd;
        double y4[4], z4[4], b4[4], vh[4];
        ld4(y + r, m, y4);
        ld4(z + r, m, z4);
        ld4(b + r, m, b4);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            y4[j] += gamma * (z4[j] - b4[j]);
            vh[j] = (j < m) ? ea * (vget(r + j) * iv) : 0.0;
        }
        st4(y + r, m, y4);
        for (int c0 = 0; c0 < R; c0 += 4) {
            double s4[4][4];
#pragma unroll
            for (int cc = 0; cc < 4; ++cc)
                if (c0 + cc < R) ld4(S + (size_t)(c0 + cc) * ld + r, m, s4[cc]);
#pragma unroll
            for (int cc = 0; cc < 4; ++cc)
                if (c0 + cc < R) {
                    const double cwv = so[SO_RITZ + 1 + c0 + cc] * iv;
#pragma unroll
                    for (int j = 0; j < 4; ++j) s4[cc][j] = keep * s4[cc][j] + vh[j] * cwv;
                    st4(S + (size_t)(c0 + cc) * ld + r, m, s4[cc]);
                }
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

// Shift s = dC + y + beta (z - b) (primitive 2), the Lanczos start vector of
// iteration t (handed to `put(r, g)`), and the state dot products used by the
// gap and stopping quantities.
template <typename T, typename CT, typename PUT>
__device__ __forceinline__ void prep_shift(const BatchArgs<T, CT>& A, const BatchInst& D, int t, double beta, PUT put,
                                           double* red, double* so) {
    const int n = D.n;
    const double* z = A.z + D.pos0;
    const double* y = A.y + D.pos0;
    const double* b = A.b + D.pos0;
    const double* dC = A.dC + D.pos0;
    T* s = A.s + D.pos0;
    double a[6] = {0, 0, 0, 0, 0, 0};
    for (int qd = threadIdx.x; 4 * qd < n; qd += kBT) {
        const int m = quad_m(qd, n), r = 4 * qd;
        double g[4], z4[4], y4[4], b4[4], d4[4], s4[4];
        normal4(A.seed, (uint64_t)qd, (uint64_t)t, (uint64_t)D.id, 0ull, g);
        ld4(z + r, m, z4);
        ld4(y + r, m, y4);
        ld4(b + r, m, b4);
        ld4(dC + r, m, d4);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double zb = z4[j] - b4[j];
            s4[j] = d4[j] + (y4[j] + beta * zb);
            if (j < m) {
                a[1] += y4[j] * b4[j];
                a[2] += zb * (z4[j] + b4[j]);
                a[3] += (y4[j] + beta * zb) * z4[j];
                a[4] += zb * zb;
                a[5] += b4[j] * b4[j];
            } else {
                g[j] = 0.0;
            }
            a[0] += g[j] * g[j];
        }
        st4(s + r, m, s4);
        put(r, m, g);
    }
    breduce<6>(a, red, so + SO_PREP);
}

// One whole iteration of alg:sketchy-cgal for the instance of this workgroup,
// the vector being multiplied in LDS.  The off-diagonal part is stored in
// slices of 64 rows (rows sorted by length, padded to the slice's even
// width); only the products use that order, every vector stays in row order.
// Row loops move 4 consecutive entries per thread with 16-byte accesses.
//
// NT = 2 is the form for batches whose largest vector does not fit the LDS
// budget: LDS holds one column tile of A.tile entries at a time; each product
// runs twice over the slices, once per tile of the vector (loaded from its
// global copy, the Lanczos basis or the Ritz vector), the first pass storing
// its row sums in u and the second adding them; the update, the Ritz vector
// and the tail read the vectors from global memory.
template <typename T, typename CT, int FMT, int RB, int NT>
__global__ __launch_bounds__(kBT) void k_batch_sell(BatchArgs<T, CT> A) {
    constexpr bool TL = (NT > 1);
    extern __shared__ __align__(16) unsigned char dyn_lds[];
    __shared__ double red[kRedMax * kBW];
    __shared__ double so[SO_N];
    __shared__ double s_inv[kQB + 1], s_coef[kQB], s_h[kQB + 8];
    __shared__ double td[kQB], te[kQB], te2[kQB], tdp[kQB], tdm[kQB], tx[kQB];
    __shared__ double s_xi;
    T* xl = reinterpret_cast<T*>(dyn_lds);
    int2* desc = reinterpret_cast<int2*>(dyn_lds + A.desc_lds_off);
    const int ii = A.order[blockIdx.x];
    const BatchInst D = A.inst[ii];
    BatchScal* G = A.scal + ii;
    const int t = G->t_next;
    if (t > A.T_iters) return;
    const int n = D.n, nshort = D.nshort, nsl = D.nsl;
    const int64_t ld = D.ld;
    const int tid = threadIdx.x;
    const int q = A.qtab[(size_t)ii * A.T_iters + (t - 1)];
    const double beta = D.beta0 * sqrt(t + 1.0);
    const double eta = 2.0 / (t + 1.0);
    const double cv = (FMT == FMT_VAL) ? 1.0 : D.cval;
    const int32_t* rp = A.rp + D.row0;
    const int32_t* perm = A.perm + D.pos0;
    const T* s = A.s + D.pos0;
    T* sp = A.s_pos + D.pos0;
    const double* dCp = A.dC_pos + D.pos0;
    T* u = A.u + D.pos0;
    T* V = A.V + D.off_V;
    T* vg = A.v + D.pos0;   // the Ritz vector's global copy (two-tile form)
    const T* Om = A.Om + D.off_OS;
    const int h = TL ? A.tile : n;
    for (int kk = tid; kk < nsl; kk += kBT) desc[kk] = A.sdesc[D.sl0 + kk];
    if (!TL && tid == 0) xl[n] = (T)0;

    prep_shift<T, CT>(A, D, t, beta, [&](int r, int m, double (&g)[4]) {
        st4(V + r, m, g);   // rounds g to the stored type
        if (!TL)
            for (int j = 0; j < m; ++j) xl[r + j] = (T)g[j];
    }, red, so);
    // off-diagonal row sums of the vector xg (its LDS copy in the one-tile form):
    // fin(p, r, a, shift, diag) gets each row's complete sum
    auto product = [&](auto obj_tag, const T* xg, auto fin) {
        constexpr bool OBJ = decltype(obj_tag)::value;
        if constexpr (!TL) {
            sell_product<T, CT, FMT, OBJ>(desc, nsl, nshort, n, perm, sp, dCp, A.scol, A.sval, rp, A.col, A.val,
                                          xl, fin);
        } else {
            for (int lo = 0; lo < n; lo += h) {
                const int hi = (lo + h < n) ? lo + h : n;
                __syncthreads();   // the previous tile's readers are done
                for (int r = tid; r < hi - lo; r += kBT) xl[r] = xg[lo + r];
                __syncthreads();
                const bool first = (lo == 0), last = (hi == n);
                sell_product<T, CT, FMT, OBJ, true>(
                    desc, nsl, nshort, n, perm, sp, dCp, A.scol, A.sval, rp, A.col, A.val, xl,
                    [&](int p, int r, double a, double sv, double dg) {
                        // the same thread handles row r in every tile
                        if (!first) a += (double)u[r];
                        if (!last) {
                            u[r] = (T)a;
                            return;
                        }
                        fin(p, r, a, sv, dg);
                    },
                    lo, hi);
            }
        }
    };
    // the shift in position order, for the products
    for (int qd = tid; 4 * qd < n; qd += kBT) {
        const int m = quad_m(qd, n), p = 4 * qd;
        int rr[4];
        ldi4(perm + p, m, rr);
        double s4[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) s4[j] = (j < m) ? (double)s[rr[j]] : 0.0;
        st4(sp + p, m, s4);
    }
    if (tid == 0) s_inv[0] = 1.0 / sqrt(so[SO_PREP]);
    __syncthreads();

    // randomized Lanczos (alg:rand-lanczos); the basis is stored unnormalised
    int k = 0;
    double rho_prev = 0.0;
    for (int i = 0; i < q; ++i) {
        const double xs = s_inv[i];
        double acc[1] = {0.0};
        const T* vi = V + (size_t)i * ld;
        product(std::false_type{}, vi, [&](int, int r, double a, double sv, double) {
            const double xr = TL ? (double)vi[r] : (double)xl[r];
            const T ut = (T)((a * cv + sv * xr) * xs);
            u[r] = ut;
            acc[0] += xr * xs * (double)ut;
        });
        breduce<1>(acc, red, so + SO_OM);
        const double om = so[SO_OM];
        if (tid == 0) {
            td[i] = om;
            if (!isfinite(om)) G->flags |= 2;
        }
        k = i + 1;
        if (i == q - 1) break;
        const T* vm = V + (size_t)(i > 0 ? i - 1 : i) * ld;
        T* w = V + (size_t)(i + 1) * ld;
        const double c1 = om * xs, c2 = (i > 0) ? rho_prev * s_inv[i - 1] : 0.0;
        double acc2[1] = {0.0};
        for (int qb = tid; 4 * qb < n; qb += 2 * kBT) {
            int mq[2];
            double uu[2][4], mm[2][4], xx[2][4];
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {
                const int qd = qb + hh * kBT;
                mq[hh] = quad_m(qd, n);
                if (mq[hh] > 0) {
                    ld4(u + 4 * qd, mq[hh], uu[hh]);
                    ld4(vm + 4 * qd, mq[hh], mm[hh]);
                    if (TL) ld4(vi + 4 * qd, mq[hh], xx[hh]);
                }
            }
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {
                if (mq[hh] > 0) {
                    const int r = 4 * (qb + hh * kBT);
                    double w4[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        w4[j] = (j < mq[hh]) ? uu[hh][j] - c1 * (TL ? xx[hh][j] : (double)xl[r + j]) - c2 * mm[hh][j]
                                             : 0.0;
                    st4(w + r, mq[hh], w4);   // rounds w4 to the stored type
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (j < mq[hh]) {
                            if (!TL) xl[r + j] = (T)w4[j];   // own rows: no other thread reads them before the barrier
                            acc2[0] += w4[j] * w4[j];
                        }
                }
            }
        }
        if (A.reorth != 0) {
            __syncthreads();   // w was written quad-wise by other threads
            // h_j = v_hat_j^T w for j0 <= j <= i (j0 = 0: full, i - 1: local), eight at a
            // time, then w <- w - sum_j h_j v_hat_j
            const int j0 = (A.reorth == 2) ? 0 : (i > 0 ? i - 1 : 0);
            for (int jb = j0; jb <= i; jb += 8) {
                double hacc[8];
#pragma unroll
                for (int jj = 0; jj < 8; ++jj) hacc[jj] = 0.0;
                for (int p = tid; p < n; p += kBT) {
                    const double wr = (double)w[p];
#pragma unroll
                    for (int jj = 0; jj < 8; ++jj)
                        if (jb + jj <= i) hacc[jj] += (double)V[(size_t)(jb + jj) * ld + p] * wr;
                }
                breduce<8>(hacc, red, s_h + jb);
            }
            acc2[0] = 0.0;
            for (int p = tid; p < n; p += kBT) {
                double a = 0.0;
                for (int j = j0; j <= i; ++j) a += (s_h[j] * s_inv[j]) * s_inv[j] * (double)V[(size_t)j * ld + p];
                const T wt = (T)((double)w[p] - a);
                w[p] = wt;
                if (!TL) xl[p] = wt;
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

    // Ritz vector v = sum_j coef_j V_j into LDS: basis column outer, four quads
    // of rows per thread, two columns in flight
    for (int qb0 = 0; 4 * qb0 < n; qb0 += 4 * kBT) {
        double a4[4][4];
        int mq[4];
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            mq[h] = quad_m(qb0 + tid + h * kBT, n);
#pragma unroll
            for (int j = 0; j < 4; ++j) a4[h][j] = 0.0;
        }
#pragma unroll 2
        for (int j = 0; j < k; ++j) {
            const double cj = s_coef[j];
            const T* Vj = V + (size_t)j * ld + 4 * (qb0 + tid);
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                if (mq[h] > 0) {
                    double t4[4];
                    ld4(Vj + 4 * h * kBT, mq[h], t4);
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) a4[h][jj] += cj * t4[jj];
                }
            }
        }
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const int r = 4 * (qb0 + tid + h * kBT);
            if (TL) {
                if (mq[h] > 0) st4(vg + r, mq[h], a4[h]);   // rounds to the stored type
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (j < mq[h]) xl[r + j] = (T)a4[h][j];
            }
        }
    }
    __syncthreads();
    auto vat = [&](int r) { return TL ? (double)vg[r] : (double)xl[r]; };
    // ||v||^2 and v^T Omega from the stored (rounded) vector
    {
        double racc[RB + 1];
#pragma unroll
        for (int c = 0; c <= RB; ++c) racc[c] = 0.0;
        for (int qd = tid; 4 * qd < n; qd += kBT) {
            const int m = quad_m(qd, n), r = 4 * qd;
            double v4[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                v4[j] = (j < m) ? vat(r + j) : 0.0;
                racc[0] += v4[j] * v4[j];
            }
#pragma unroll
            for (int c = 0; c < RB; ++c)
                if (c < A.R) {
                    double o4[4];
                    ld4(Om + (size_t)c * ld + r, m, o4);
                    racc[c + 1] += v4[0] * o4[0] + v4[1] * o4[1] + v4[2] * o4[2] + v4[3] * o4[3];
                }
        }
        breduce<RB + 1>(racc, red, so + SO_RITZ);
    }
    const double vnorm2 = so[SO_RITZ];
    const double iv = 1.0 / sqrt(vnorm2);

    // objective v_hat^T C v_hat and the eigen-residual ||D v_hat - xi v_hat||^2
    {
        double oa[2] = {0.0, 0.0};
        product(std::true_type{}, vg, [&](int p, int r, double a, double sv, double dg) {
            const double xr = vat(r) * iv;
            const double off = a * cv * iv;
            const double rr = (off + sv * xr) - xi * xr;
            oa[0] += xr * (off + dg * xr);
            oa[1] += rr * rr;
        });
        breduce<2>(oa, red, so + SO_OBJ);
    }
    iteration_tail<T, CT>(A, D, G, ii, t, q, k, xi, beta, eta, iv, vnorm2, vat, red, so);
}

// The same iteration with the SpMV gathering from global memory (instances
// whose vector does not fit the LDS budget): CSR rows in row order, one
// thread per row.
template <typename T, typename CT, int FMT, int RB>
__global__ __launch_bounds__(kBT) void k_batch_iter(BatchArgs<T, CT> A) {
    __shared__ double red[kRedMax * kBW];
    __shared__ double so[SO_N];
    __shared__ double s_inv[kQB + 1], s_coef[kQB], s_h[kQB + 8];
    __shared__ double td[kQB], te[kQB], te2[kQB], tdp[kQB], tdm[kQB], tx[kQB];
    __shared__ double s_xi;
    const int ii = A.order[blockIdx.x];
    const BatchInst D = A.inst[ii];
    BatchScal* G = A.scal + ii;
    const int t = G->t_next;
    if (t > A.T_iters) return;
    const int n = D.n;
    const int64_t ld = D.ld;
    const int tid = threadIdx.x;
    const int q = A.qtab[(size_t)ii * A.T_iters + (t - 1)];
    const double beta = D.beta0 * sqrt(t + 1.0);
    const double eta = 2.0 / (t + 1.0);
    const double cv = (FMT == FMT_VAL) ? 1.0 : D.cval;
    const int32_t* rp = A.rp + D.row0;
    const double* dC = A.dC + D.pos0;
    T* s = A.s + D.pos0;
    T* u = A.u + D.pos0;
    T* v = A.v + D.pos0;
    T* V = A.V + D.off_V;
    const T* Om = A.Om + D.off_OS;

    prep_shift<T, CT>(A, D, t, beta, [&](int r, int m, double (&g)[4]) { st4(V + r, m, g); }, red, so);
    if (tid == 0) s_inv[0] = 1.0 / sqrt(so[SO_PREP]);
    __syncthreads();

    int k = 0;
    double rho_prev = 0.0;
    for (int i = 0; i < q; ++i) {
        T* x = V + (size_t)i * ld;
        const double xs = s_inv[i];
        double acc[1] = {0.0};
        for (int r = tid; r < n; r += kBT) {
            const T a = row_product<T, CT, FMT>(rp, A.col, A.val, r, x);
            const double xr = (double)x[r];
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
            const T wt = (T)((double)u[r] - c1 * (double)x[r] - c2 * (double)vm[r]);
            w[r] = wt;
            acc2[0] += (double)wt * (double)wt;
        }
        if (A.reorth != 0) {
            const int j0 = (A.reorth == 2) ? 0 : (i > 0 ? i - 1 : 0);   // full or local
            for (int jb = j0; jb <= i; jb += 8) {
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
                for (int j = j0; j <= i; ++j) a += (s_h[j] * s_inv[j]) * s_inv[j] * (double)V[(size_t)j * ld + r];
                const T wt = (T)((double)w[r] - a);
                w[r] = wt;
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

    if (tid < 64) tridiag_min_eig(td, te, k, te2, tdp, tdm, tx, &s_xi);
    __syncthreads();
    for (int i = tid; i < k; i += kBT) s_coef[i] = tx[i] * s_inv[i];
    __syncthreads();
    const double xi = s_xi;

    {
        double racc[RB + 1];
#pragma unroll
        for (int c = 0; c <= RB; ++c) racc[c] = 0.0;
        for (int r = tid; r < n; r += kBT) {
            double a = 0.0;
            for (int j = 0; j < k; ++j) a += s_coef[j] * (double)V[(size_t)j * ld + r];
            const T vt = (T)a;
            v[r] = vt;
            const double vr = (double)vt;   // the stored value is the one every later step uses
            racc[0] += vr * vr;
#pragma unroll
            for (int c = 0; c < RB; ++c)
                if (c < A.R) racc[c + 1] += vr * (double)Om[(size_t)c * ld + r];
        }
        breduce<RB + 1>(racc, red, so + SO_RITZ);
    }
    const double vnorm2 = so[SO_RITZ];
    const double iv = 1.0 / sqrt(vnorm2);
    {
        double oa[2] = {0.0, 0.0};
        for (int r = tid; r < n; r += kBT) {
            const T a = row_product<T, CT, FMT>(rp, A.col, A.val, r, v);
            const double xr = (double)v[r] * iv;
            const double off = (double)a * cv * iv;
            const double rr = (off + (double)s[r] * xr) - xi * xr;
            oa[0] += xr * (off + dC[r] * xr);
            oa[1] += rr * rr;
        }
        breduce<2>(oa, red, so + SO_OBJ);
    }
    iteration_tail<T, CT>(A, D, G, ii, t, q, k, xi, beta, eta, iv, vnorm2, [&](int r) { return (double)v[r]; },
                          red, so);
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
                                                  const int64_t* row0, const int64_t* pos0, const double* inv_cF,
                                                  const double* inv_alpha, const int32_t* rp_off, CT* col_off,
                                                  T* val_off, const double* dCraw, double* dC, double* b_out, int fmt) {
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
        const int64_t pr = pos0[k] + (r - base);
        dC[pr] = dCraw[r] * sc;
        b_out[pr] = b_in[r] * inv_alpha[k];
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

// MaxCut rounding of one instance (Section 7.2, sec:maxcut-rounding): per
// workgroup partial sums of chi_j^T C_off chi_j (j < R, chi_j = sgn U[:, j],
// sgn 0 = +1) and of tr(C), in scaled units.
template <typename T, typename CT, int FMT, int RB>
__global__ __launch_bounds__(256) void k_bcut_forms(int n, const int32_t* rp, const CT* col, const T* val, double cval,
                                                    const double* dC, const double* U, int R, double* part) {
    __shared__ double red[4];
    double acc[RB + 1];
#pragma unroll
    for (int j = 0; j <= RB; ++j) acc[j] = 0.0;
    for (int r = blockIdx.x * 256 + threadIdx.x; r < n; r += gridDim.x * 256) {
        double off[RB];
#pragma unroll
        for (int j = 0; j < RB; ++j) off[j] = 0.0;
        for (int e = rp[r]; e < rp[r + 1]; ++e) {
            const CT cw = col[e];
            const int c = (FMT == FMT_SGN) ? col_index(cw) : (int)cw;
            const double v = (FMT == FMT_VAL) ? (double)val[e] : ((FMT == FMT_SGN && col_neg(cw)) ? -cval : cval);
#pragma unroll
            for (int j = 0; j < RB; ++j)
                if (j < R) off[j] += v * ((U[(int64_t)j * n + c] < 0.0) ? -1.0 : 1.0);
        }
#pragma unroll
        for (int j = 0; j < RB; ++j)
            if (j < R) acc[j] += ((U[(int64_t)j * n + r] < 0.0) ? -1.0 : 1.0) * off[j];
        acc[RB] += dC[r];
    }
#pragma unroll
    for (int j = 0; j <= RB; ++j) {
        double v = wave_sum(acc[j]);
        __syncthreads();
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
        __syncthreads();
        if (threadIdx.x == 0) part[(size_t)blockIdx.x * (RB + 1) + j] = red[0] + red[1] + red[2] + red[3];
    }
}

__global__ __launch_bounds__(256) void k_bcut_indicator(int n, const double* u, int8_t* chi) {
    for (int r = blockIdx.x * 256 + threadIdx.x; r < n; r += gridDim.x * 256) chi[r] = (u[r] < 0.0) ? (int8_t)-1 : (int8_t)1;
}

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

int q_of(const scg_params& p, int64_t n, int t) {
    int64_t q = (p.q_mode == 1) ? p.q_fixed
                                : ((n > 1) ? (int64_t)std::ceil(std::pow((double)t, 0.25) * std::log((double)n)) : 1);
    return (int)std::max<int64_t>(1, std::min<int64_t>(q, std::max<int64_t>(n - 1, 1)));
}

struct BLayout {
    size_t inst, scal, order, qtab, rp, col, val, dC, b, z, y, s, u, v, V, Om, S, logs, iorow, row0, pos0, ninst, invc,
        inva, mm, err, recon, perm, s_pos, dC_pos, sdesc, scol, sval, total;
    int64_t nrows, nvec, Vtot, OStot, sell_cap, nsl_cap;
};

BLayout blayout(const scg_params& p, int ninst, const int64_t* inst_n, int64_t nnz) {
    BLayout L{};
    const size_t es = (p.precision == SCG_FP32_STREAM) ? 4 : 8;
    int64_t nrows = 0, nvec = 0, Vtot = 0, OStot = 0, nmax = 0;
    for (int k = 0; k < ninst; ++k) {
        const int64_t n = inst_n[k];
        const int64_t ld = (n + 63) / 64 * 64;
        int qm = 1;
        for (int t = 1; t <= p.T; ++t) qm = std::max(qm, q_of(p, n, t));
        nrows += n;
        nvec += ld;
        Vtot += (int64_t)(qm + 1) * ld;
        OStot += (int64_t)p.R * ld;
        nmax = std::max(nmax, n);
    }
    L.nrows = nrows;
    L.nvec = nvec;
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
    // per-instance vectors at 64-aligned offsets pos0 (row order; perm, s_pos, dC_pos in slice position order)
    L.dC = take(8 * nvec);
    L.b = take(8 * nvec);
    L.z = take(8 * nvec);
    L.y = take(8 * nvec);
    L.s = take(es * nvec);
    L.u = take(es * nvec);
    L.v = take(es * nvec);
    L.V = take(es * (size_t)Vtot);
    L.Om = take(es * (size_t)OStot);
    L.S = take(es * (size_t)OStot);
    L.logs = take(sizeof(scg_iter_log) * (size_t)ninst * p.T);
    L.iorow = take(4 * (size_t)nrows);
    L.row0 = take(8 * (size_t)ninst);
    L.pos0 = take(8 * (size_t)ninst);
    L.ninst = take(4 * (size_t)ninst);
    L.invc = take(8 * (size_t)ninst);
    L.inva = take(8 * (size_t)ninst);
    L.mm = take(8 * 4 * (size_t)1024 * 16);
    L.err = take(512);   // validation flags, then the reconstruction's counter at +256
    L.recon = take(8 * scg_recon_scratch_doubles(nmax, p.R));
    // sliced layout: padding is at most 64 * kLongRow per instance (rows sorted by length),
    // plus one entry per row (even widths) and the last slice's unused lanes
    L.sell_cap = nnz + nrows + (int64_t)ninst * (64 * kLongRow + 64 + 63 * kLongRow + 64);
    L.nsl_cap = nrows / 64 + ninst;
    L.perm = take(4 * (size_t)nvec);
    L.s_pos = take(es * (size_t)nvec);
    L.dC_pos = take(8 * (size_t)nvec);
    L.sdesc = take(8 * (size_t)L.nsl_cap);
    L.scol = take(4 * (size_t)L.sell_cap);
    L.sval = take(es * (size_t)L.sell_cap);
    L.total = off;
    return L;
}

}  // namespace

struct scg_batch {
    scg_params prm;
    int ninst;
    int64_t nrows, nvec, nnz_in, nnz_off;
    hipStream_t stream;
    int fmt;
    bool col16;        // 16-bit column indices (every instance small enough)
    int xmode;            // iteration kernel: 1 vector in LDS, 2 in two LDS column tiles, 3 global gathers
    bool fits[4];         // forms the LDS budget admits (form 3 always)
    size_t lds_bytes[3];  // dynamic LDS per workgroup of forms 1 and 2
    int desc_off[3];      // byte offset of the slice table in dynamic LDS, forms 1 and 2
    int tile;             // columns per LDS tile of form 2 (a multiple of 64)
    float form_ms[4];     // one timed iteration of each form tried at init (0: not timed)
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
    int32_t* perm;
    void* s_pos;
    double* dC_pos;
    int2* sdesc;
    void* scol;
    void* sval;
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
    A.perm = c->perm;
    A.s_pos = (T*)c->s_pos;
    A.dC_pos = c->dC_pos;
    A.sdesc = c->sdesc;
    A.scol = (const CT*)c->scol;
    A.sval = (const T*)c->sval;
    A.desc_lds_off = c->desc_off[c->xmode == 2 ? 2 : 1];
    A.tile = c->tile;
    A.T_iters = c->prm.T;
    A.R = c->prm.R;
    A.reorth = c->prm.reorth;
    A.beta0 = c->prm.beta0;
    A.K = c->prm.K;
    A.seed = c->prm.seed;
    return A;
}

// Launch one iteration, or (prepare) raise the kernel's dynamic-LDS limit.
template <typename T, typename CT, int FMT, int RB>
hipError_t launch_leaf(scg_batch* c, bool prepare) {
    if (c->xmode == 1 || c->xmode == 2) {
        auto* kern = (c->xmode == 1) ? &k_batch_sell<T, CT, FMT, RB, 1> : &k_batch_sell<T, CT, FMT, RB, 2>;
        const unsigned lds = (unsigned)c->lds_bytes[c->xmode];
        if (prepare) return hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(kern, dim3(c->ninst), dim3(kBT), lds, c->stream, bargs<T, CT>(c));
    } else {
        if (prepare) return hipSuccess;
        hipLaunchKernelGGL((k_batch_iter<T, CT, FMT, RB>), dim3(c->ninst), dim3(kBT), 0, c->stream, bargs<T, CT>(c));
    }
    return hipGetLastError();
}

template <typename T, typename CT, int FMT>
hipError_t launch_fmt(scg_batch* c, bool prepare) {
    if (c->prm.R <= 8) return launch_leaf<T, CT, FMT, 8>(c, prepare);
    return launch_leaf<T, CT, FMT, kRMax>(c, prepare);
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

// Sliced layout of every instance's off-diagonal part (from the scattered CSR):
// rows with at most kLongRow entries sorted by decreasing length (ties by row),
// cut into slices of 64, each padded to its even maximum width with the index
// n (x[n] = 0 in LDS; value 0); longer rows follow in row order and keep CSR.
template <typename T, typename CT>
scg_status build_slices(scg_batch* c, const BLayout& L, const std::vector<int32_t>& hrp_off) {
    const int64_t nvec = c->nvec;
    const int64_t nnz = c->nnz_off;
    const bool vals = (c->fmt == FMT_VAL);
    std::vector<CT> hcol(nnz);
    std::vector<T> hval(vals ? nnz : 0);
    std::vector<double> hdC(nvec);
    if (nnz > 0) HIP_TRY(hipMemcpyAsync(hcol.data(), c->col, sizeof(CT) * nnz, hipMemcpyDeviceToHost, c->stream));
    if (vals && nnz > 0) HIP_TRY(hipMemcpyAsync(hval.data(), c->val, sizeof(T) * nnz, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(hdC.data(), c->dC, 8 * nvec, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    std::vector<int32_t> perm(nvec, 0);
    std::vector<double> dCp(nvec, 0.0);
    std::vector<int2> desc;
    std::vector<CT> scol;
    std::vector<T> sval;
    for (int k = 0; k < c->ninst; ++k) {
        BatchInst& I = c->hinst[k];
        const int64_t r0 = I.row0;
        const int n = I.n;
        auto len = [&](int r) { return hrp_off[r0 + r + 1] - hrp_off[r0 + r]; };
        std::vector<int32_t> order;
        std::vector<int32_t> longs;
        for (int r = 0; r < n; ++r) (len(r) <= kLongRow ? order : longs).push_back(r);
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return len(a) > len(b); });
        I.nshort = (int)order.size();
        I.nsl = (I.nshort + 63) / 64;
        I.sl0 = (int64_t)desc.size();
        order.insert(order.end(), longs.begin(), longs.end());
        for (int p = 0; p < n; ++p) {
            perm[I.pos0 + p] = order[p];
            dCp[I.pos0 + p] = hdC[I.pos0 + order[p]];
        }
        for (int sl = 0; sl < I.nsl; ++sl) {
            const int w = (len(order[64 * sl]) + 1) & ~1;
            const int64_t off = (int64_t)scol.size();
            desc.push_back(make_int2((int)off, w));
            scol.resize(off + 64 * (int64_t)w, (CT)n);
            if (vals) sval.resize(off + 64 * (int64_t)w, (T)0);
            for (int l = 0; l < 64; ++l) {
                const int p = 64 * sl + l;
                if (p >= I.nshort) break;
                const int r = order[p];
                const int32_t e0 = hrp_off[r0 + r];
                for (int j = 0; j < len(r); ++j) {
                    const int64_t o = off + 2 * (int64_t)((j / 2) * 64 + l) + (j & 1);
                    scol[o] = hcol[e0 + j];
                    if (vals) sval[o] = hval[e0 + j];
                }
            }
        }
    }
    if ((int64_t)scol.size() > L.sell_cap || (int64_t)desc.size() > L.nsl_cap || scol.size() > (size_t)INT32_MAX)
        return SCG_EINVAL;
    HIP_TRY(hipMemcpyAsync(c->perm, perm.data(), 4 * nvec, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->dC_pos, dCp.data(), 8 * nvec, hipMemcpyHostToDevice, c->stream));
    if (!desc.empty()) HIP_TRY(hipMemcpyAsync(c->sdesc, desc.data(), 8 * desc.size(), hipMemcpyHostToDevice, c->stream));
    if (!scol.empty()) HIP_TRY(hipMemcpyAsync(c->scol, scol.data(), sizeof(CT) * scol.size(), hipMemcpyHostToDevice, c->stream));
    if (!sval.empty()) HIP_TRY(hipMemcpyAsync(c->sval, sval.data(), sizeof(T) * sval.size(), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return SCG_OK;
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
    int64_t* d_pos0 = (int64_t*)(base + L.pos0);
    std::vector<int64_t> hpos0(ninst);
    for (int k = 0; k < ninst; ++k) hpos0[k] = c->hinst[k].pos0;
    int* d_ninst = (int*)(base + L.ninst);
    double* d_invc = (double*)(base + L.invc);
    double* d_inva = (double*)(base + L.inva);
    double* d_mm = (double*)(base + L.mm);
    int* d_err = (int*)(base + L.err);
    HIP_TRY(hipMemcpyAsync(d_iorow, iorow.data(), 4 * nrows, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(d_row0, c->row0.data(), 8 * ninst, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(d_pos0, hpos0.data(), 8 * ninst, hipMemcpyHostToDevice, c->stream));
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
    // column words: 16 bits when every local index, the padding index n and the sign bit fit
    c->col16 = (c->prm.matrix_format != 1) && (nmax <= ((c->fmt == FMT_SGN) ? 32767 : 65535));
    // LDS forms: the whole vector (plus the zero at index n), or a column tile of
    // half of the longest one, and the slice table within the budget
    {
        int64_t nslmax = 0;
        for (int k = 0; k < ninst; ++k) nslmax = std::max<int64_t>(nslmax, (c->hinst[k].n + 63) / 64);
        const size_t xb1 = al256((size_t)(ldmax + 64) * sizeof(T));
        c->tile = (int)(((ldmax + 1) / 2 + 63) / 64 * 64);
        const size_t xb2 = al256((size_t)c->tile * sizeof(T));
        c->desc_off[1] = (int)xb1;
        c->desc_off[2] = (int)xb2;
        c->lds_bytes[1] = xb1 + 8 * (size_t)nslmax;
        c->lds_bytes[2] = xb2 + 8 * (size_t)nslmax;
        c->fits[1] = c->lds_bytes[1] <= kLdsBudget;
        c->fits[2] = c->lds_bytes[2] <= kLdsBudget;
        c->fits[3] = true;
        const int f = c->prm.batch_kernel;
        if (f != 0 && !c->fits[f]) return SCG_EINVAL;   // a forced form that does not fit
    }
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
                           d_iorow, d_row0, d_pos0, d_invc, d_inva, c->rp, (uint16_t*)c->col, (T*)c->val, dCraw, c->dC, c->b,
                           c->fmt);
    else
        hipLaunchKernelGGL((k_bscatter<T, int32_t>), dim3(gv), dim3(256), 0, c->stream, nrows, row_ptr, col, val, b,
                           d_iorow, d_row0, d_pos0, d_invc, d_inva, c->rp, (int32_t*)c->col, (T*)c->val, dCraw, c->dC, c->b,
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
    if (c->fits[1] || c->fits[2]) {
        const scg_status st = c->col16 ? build_slices<T, uint16_t>(c, L, hrp_off) : build_slices<T, int32_t>(c, L, hrp_off);
        if (st != SCG_OK) return st;
    }
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
    const size_t es = (c->prm.precision == SCG_FP32_STREAM) ? 4 : 8;
    // the state before iteration 1 (also after each form timed below)
    auto reset_state = [&]() -> scg_status {
        std::vector<BatchScal> hs(ninst);
        std::memset(hs.data(), 0, sizeof(BatchScal) * ninst);
        for (auto& x : hs) x.t_next = 1;
        HIP_TRY(hipMemcpyAsync(c->scal, hs.data(), sizeof(BatchScal) * ninst, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(hipMemsetAsync(c->z, 0, 8 * c->nvec, c->stream));
        HIP_TRY(hipMemsetAsync(c->y, 0, 8 * c->nvec, c->stream));
        HIP_TRY(hipMemsetAsync(c->S, 0, es * L.OStot, c->stream));
        HIP_TRY(hipMemsetAsync(c->logs, 0, sizeof(scg_iter_log) * ninst * c->prm.T, c->stream));
        HIP_TRY(hipMemsetAsync(c->counter, 0, 256, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        return SCG_OK;
    };
    scg_status st = reset_state();
    if (st != SCG_OK) return st;
    // the iteration kernel: forced, the first form that fits, or the fastest on one
    // iteration (after a warm-up iteration) in the order 1, 2, 3, a later form
    // replacing an earlier one only when at least 3% faster
    for (int f = 0; f < 4; ++f) c->form_ms[f] = 0.f;
    if (c->prm.batch_kernel != 0) {
        c->xmode = c->prm.batch_kernel;
    } else {
        c->xmode = c->fits[1] ? 1 : (c->fits[2] ? 2 : 3);
        if (c->prm.autotune) {
            hipEvent_t e0, e1;
            HIP_TRY(hipEventCreate(&e0));
            HIP_TRY(hipEventCreate(&e1));
            float best = 1e30f;
            int best_f = c->xmode;
            for (int f = 1; f <= 3; ++f) {
                if (!c->fits[f]) continue;
                c->xmode = f;
                HIP_TRY(enqueue_iter(c, true));
                HIP_TRY(enqueue_iter(c));
                if ((st = reset_state()) != SCG_OK) return st;
                HIP_TRY(hipEventRecord(e0, c->stream));
                HIP_TRY(enqueue_iter(c));
                HIP_TRY(hipEventRecord(e1, c->stream));
                HIP_TRY(hipEventSynchronize(e1));
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                c->form_ms[f] = ms;
                if (ms < best * 0.97f) {
                    best = ms;
                    best_f = f;
                }
                if ((st = reset_state()) != SCG_OK) return st;
            }
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            c->xmode = best_f;
        }
    }
    return SCG_OK;
}

bool bparams_ok(const scg_params* p, int ninst, const int64_t* inst_n) {
    if (!p || ninst < 1 || !inst_n) return false;
    if (p->R < 1 || p->R > kRMax || p->T < 1 || !(p->beta0 > 0.0) || !(p->K >= 0.0)) return false;
    if (p->q_mode != 0 && p->q_mode != 1) return false;
    if (p->q_mode == 1 && p->q_fixed < 1) return false;
    if (p->reorth < 0 || p->reorth > 2) return false;
    if (p->precision != SCG_FP64 && p->precision != SCG_FP32_STREAM) return false;
    if (p->matrix_format != 0 && p->matrix_format != 1) return false;
    if (p->basis_mode != 0 || p->omega_mode != 0) return false;   // the batch keeps both in HBM
    if (p->trace_mode != 0 || p->constraint_set != 0) return false;   // the MaxCut model only
    if (p->batch_kernel < 0 || p->batch_kernel > 3) return false;
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
    c->nvec = L.nvec;
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
    c->perm = (int32_t*)(base + L.perm);
    c->s_pos = base + L.s_pos;
    c->dC_pos = (double*)(base + L.dC_pos);
    c->sdesc = (int2*)(base + L.sdesc);
    c->scol = base + L.scol;
    c->sval = base + L.sval;
    c->hinst.resize(n_inst);
    c->row0.resize(n_inst);
    int64_t r0 = 0, offV = 0, offOS = 0, pv = 0;
    for (int k = 0; k < n_inst; ++k) {
        BatchInst& I = c->hinst[k];
        const int64_t n = inst_n[k];
        I.row0 = r0;
        I.pos0 = pv;
        I.n = (int)n;
        I.id = p->instance + k;
        I.beta0 = p->beta0;
        I.ld = (n + 63) / 64 * 64;
        int qm = 1;
        for (int t = 1; t <= p->T; ++t) qm = std::max(qm, q_of(*p, n, t));
        I.off_V = offV;
        I.off_OS = offOS;
        c->row0[k] = r0;
        r0 += n;
        pv += I.ld;
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
scg_status sketchycgal_batch_set_beta0(scg_batch* c, const double* beta0) {
    if (!c || !beta0) return SCG_EINVAL;
    for (int k = 0; k < c->ninst; ++k)
        if (!(beta0[k] > 0.0) || !std::isfinite(beta0[k])) return SCG_EINVAL;
    for (int k = 0; k < c->ninst; ++k)
        if (c->t_host[k] != 1) return SCG_ESTATE;
    for (int k = 0; k < c->ninst; ++k) c->hinst[k].beta0 = beta0[k];
    HIP_TRY(hipMemcpyAsync(c->inst, c->hinst.data(), sizeof(BatchInst) * c->ninst, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return SCG_OK;
}

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
    o->spmv_grid = c->ninst;
    o->batch_kernel = c->xmode;
    return (hs.flags & 2) ? SCG_ENUMERIC : SCG_OK;
}

scg_status sketchycgal_batch_get_state(scg_batch* c, int32_t inst, int32_t* t_next, double* z, double* y, double* S,
                                       double* p, double* tau) {
    if (!c || inst < 0 || inst >= c->ninst) return SCG_EINVAL;
    const BatchInst& I = c->hinst[inst];
    if (z) HIP_TRY(hipMemcpyAsync(z, c->z + I.pos0, 8 * I.n, hipMemcpyDeviceToDevice, c->stream));
    if (y) HIP_TRY(hipMemcpyAsync(y, c->y + I.pos0, 8 * I.n, hipMemcpyDeviceToDevice, c->stream));
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
    HIP_TRY(hipMemcpyAsync(c->z + I.pos0, z, 8 * I.n, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->y + I.pos0, y, 8 * I.n, hipMemcpyDeviceToDevice, c->stream));
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
    a.seed = c->prm.seed;
    a.instance = (uint64_t)I.id;
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

scg_status sketchycgal_batch_round(scg_batch* c, int32_t inst, const double* U, int8_t* chi, double* weights,
                                   int32_t* best) {
    if (!c || !U || !weights || !best || inst < 0 || inst >= c->ninst) return SCG_EINVAL;
    const BatchInst& I = c->hinst[inst];
    const int R = c->prm.R;
    const int RBs = (R <= 8) ? 8 : kRMax;
    const int G = std::max(1, std::min(1024, (I.n + 255) / 256));
    const int32_t* rp = c->rp + I.row0;
    const double* dC = c->dC + I.pos0;
    double* part = c->recon;
    const dim3 g(G), b(256);
#define SCG_BCUT(T, CT, FMT, RB)                                                                               \
    hipLaunchKernelGGL((k_bcut_forms<T, CT, FMT, RB>), g, b, 0, c->stream, I.n, rp, (const CT*)c->col,          \
                       (const T*)c->val, I.cval, dC, U, R, part)
#define SCG_BCUT_RB(T, CT, FMT) \
    do { if (RBs == 8) SCG_BCUT(T, CT, FMT, 8); else SCG_BCUT(T, CT, FMT, kRMax); } while (0)
#define SCG_BCUT_FMT(T, CT)                                          \
    do {                                                             \
        if (c->fmt == FMT_PAT) SCG_BCUT_RB(T, CT, FMT_PAT);          \
        else if (c->fmt == FMT_SGN) SCG_BCUT_RB(T, CT, FMT_SGN);     \
        else SCG_BCUT_RB(T, CT, FMT_VAL);                            \
    } while (0)
    if (c->prm.precision == SCG_FP32_STREAM) {
        if (c->col16) SCG_BCUT_FMT(float, uint16_t); else SCG_BCUT_FMT(float, int32_t);
    } else {
        if (c->col16) SCG_BCUT_FMT(double, uint16_t); else SCG_BCUT_FMT(double, int32_t);
    }
#undef SCG_BCUT_FMT
#undef SCG_BCUT_RB
#undef SCG_BCUT
    HIP_TRY(hipGetLastError());
    std::vector<double> h((size_t)G * (RBs + 1));
    HIP_TRY(hipMemcpyAsync(h.data(), part, sizeof(double) * h.size(), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    double tr = 0.0;
    std::vector<double> q(R, 0.0);
    for (int gi = 0; gi < G; ++gi) {
        for (int j = 0; j < R; ++j) q[j] += h[(size_t)gi * (RBs + 1) + j];
        tr += h[(size_t)gi * (RBs + 1) + RBs];
    }
    int bi = 0;
    for (int j = 0; j < R; ++j) {
        weights[j] = -I.c_F * (q[j] + tr);
        if (weights[j] > weights[bi]) bi = j;
    }
    *best = bi;
    if (chi) {
        hipLaunchKernelGGL(k_bcut_indicator, g, b, 0, c->stream, I.n, U + (int64_t)bi * I.n, chi);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipStreamSynchronize(c->stream));
    }
    return SCG_OK;
}

void sketchycgal_batch_destroy(scg_batch* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    if (c->graph_ready) (void)hipGraphExecDestroy(c->graph);
    delete c;
}

}  // extern "C"
