// Host runtime and C ABI of the SketchyCGAL library (see include/sketchycgal.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "scg_kernels.hpp"

using namespace scg;

#define HIP_TRY(expr)                                 \
    do {                                              \
        hipError_t e_ = (expr);                       \
        if (e_ != hipSuccess) return SCG_EHIP;        \
    } while (0)

scg_status scg_reconstruct_impl(scg_ctx* c, double* U, double* lambda, double* err);

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int q_for(const scg_params& p, int64_t n, int t) {
    int64_t q;
    if (p.q_mode == 1) {
        q = p.q_fixed;
    } else {
        q = (n > 1) ? (int64_t)std::ceil(std::pow((double)t, 0.25) * std::log((double)n)) : 1;
    }
    const int64_t cap = std::max<int64_t>(n - 1, 1);
    return (int)std::max<int64_t>(1, std::min<int64_t>(q, cap));
}

int qmax_for(const scg_params& p, int64_t n) {
    int m = 1;
    if (p.q_mode == 1) return q_for(p, n, 1);
    return std::max(m, q_for(p, n, p.T));   // q_t is nondecreasing in t
}

size_t elem_size(const scg_params& p) { return p.precision == SCG_FP32_STREAM ? 4 : 8; }

// Chunks of the quad-chunk SpMV layout (column words) to reserve (0: that
// layout is never used with these parameters).  A row takes max(1, ceil(d / 4))
// quads and rows of at most kQRowMax entries (32 quads) are packed whole into
// chunks of 64 quads; a chunk is closed only when the next row does not fit,
// so every chunk but the last holds at least 33 quads.  The sum over rows is
// at most nnz / 4 + n quads.
int64_t quad_chunk_cap(const scg_params& p, int64_t n, int64_t nnz) {
    if (p.matrix_format == 1 || (p.spmv_lanes != 0 && p.spmv_lanes != 1) || p.segments > 1) return 0;
    if (n >= ((int64_t)1 << 29)) return 0;   // columns must fit the 29-bit field
    const int64_t dq = nnz / 4 + n + 1;
    return dq / 33 + 2;
}

// Chunks of the entry-chunk layout (values stored) to reserve.  A row takes
// max(1, d) entries and rows of at most kERowMax entries are packed whole
// into chunks of 256; a chunk is closed only when the next row does not fit,
// so every chunk but the last holds at least 256 - kERowMax + 1 entries.  The
// sum over rows is at most nnz + n entries.
int64_t entry_chunk_cap(const scg_params& p, int64_t n, int64_t nnz) {
    if ((p.spmv_lanes != 0 && p.spmv_lanes != 1) || p.segments > 1) return 0;
    if (n >= ((int64_t)1 << 29)) return 0;
    return (nnz + n) / (256 - kERowMax + 1) + 2;
}

// Column segments the SpMV may use with these parameters: kSegMax when the
// autotuner may try them (or they are forced), else 1.  Sizes the segment row
// pointers, the row-block descriptors and the concurrent-segment partials.
int seg_cap(const scg_params& p, int64_t n, int64_t nnz) {
    if (p.segments > 1) return kSegMax;
    if (p.segments == 0 && p.autotune && n >= (1 << 18) && nnz >= (1 << 20) && p.spmv_lanes != 1) return kSegMax;
    return 1;
}

// Chunks of the sliced entry-chunk layout (the eight concurrent column segments
// over entry chunks; 0: never used with these parameters).  Slice s holds
// max(1, d) entries per row for its d <= kERowMax entries of the row, else one
// (the long segment is stored apart); every chunk of a slice but its last holds
// at least 256 - kERowMax + 1 entries, and the slices hold at most nnz + 8 n.
int64_t xchunk_cap(const scg_params& p, int64_t n, int64_t nnz) {
    if (seg_cap(p, n, nnz) < kSegMax || (p.segments != 0 && p.segments != kSegMax)) return 0;
    if ((p.spmv_lanes != 0 && p.spmv_lanes != 1) || n >= ((int64_t)1 << 29)) return 0;
    return (nnz + kSegMax * n) / (256 - kERowMax + 1) + 2 * kSegMax;
}

struct Layout {
    size_t rp, col, val, dC, b, z, y, s, V, u, v, xp, Om, S, rb, sc, part, counter, logs, recon, racc, lo, hi, qw, qv,
        qc, xqw, xqv, xqc, xlseg, xlw, xlv, total;
    size_t recon_bytes;
};

Layout make_layout(const scg_params& p, int64_t n, int64_t nnz) {
    Layout L{};
    const size_t es = elem_size(p);
    const int qm = qmax_for(p, n);
    const size_t R = (size_t)p.R;
    const size_t ld = (size_t)((n + 63) / 64 * 64);
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    const int nsc = seg_cap(p, n, nnz);
    L.rp = take(sizeof(int32_t) * (size_t)nsc * (n + 1));
    L.col = take(sizeof(int32_t) * (size_t)nnz);
    L.val = take(es * (size_t)nnz);
    L.dC = take(8 * n);
    L.b = take(8 * n);
    L.z = take(8 * n);
    L.y = take(8 * n);
    L.s = take(es * n);
    // the Lanczos basis: all q_t + 1 vectors, or three rotating ones when it is regenerated
    L.V = take(es * ld * (size_t)(p.basis_mode == 1 ? 3 : qm + 1));
    L.u = take(es * n);
    L.v = take(es * n);
    L.xp = take(nsc > 1 ? es * ld * (size_t)kSegMax : 0);   // concurrent-segment row sums
    L.Om = take(p.omega_mode == 1 ? 0 : es * ld * R);   // generated from Philox where used
    L.S = take(es * ld * R);
    L.rb = take(sizeof(int2) * (size_t)nsc * (n + 2));
    L.sc = take(sizeof(DevScalars));
    const size_t pw = 19 + (size_t)kRMax + (size_t)qm + 2;   // slices of Prob (scg_internal.hpp)
    L.part = take(8 * (size_t)kGMax * pw);
    L.counter = take(256);
    L.logs = take(sizeof(scg_iter_log) * (size_t)p.T);
    L.recon_bytes = 8 * scg_recon_scratch_doubles(n, p.R);
    L.recon = take(L.recon_bytes);
    L.racc = take(p.basis_mode == 1 ? 8 * ld : 0);
    L.lo = take(p.constraint_set == 1 ? 8 * (size_t)n : 0);   // box constraint set, scaled
    L.hi = take(p.constraint_set == 1 ? 8 * (size_t)n : 0);
    // the chunk layouts: column words for the larger of the two, values for the entry layout
    const int64_t nqc = quad_chunk_cap(p, n, nnz), nec = entry_chunk_cap(p, n, nnz);
    L.qw = take(sizeof(int32_t) * 256 * (size_t)std::max(nqc, nec));
    L.qv = take(es * 256 * (size_t)nec);
    L.qc = take(sizeof(int2) * (size_t)std::max(nqc, nec));
    const int64_t nxc = xchunk_cap(p, n, nnz);
    L.xqw = take(sizeof(int32_t) * 256 * (size_t)nxc);
    L.xqv = take(es * 256 * (size_t)nxc);
    L.xqc = take(sizeof(int2) * (size_t)nxc);
    L.xlseg = take(nxc > 0 ? sizeof(int4) * (size_t)(nnz / (kERowMax + 1) + kSegMax) : 0);
    // long entries: each segment starts on a 16-byte quad, so at most 3 padding words per segment
    const size_t nlw = (size_t)nnz + 4 * (size_t)(nnz / (kERowMax + 1) + kSegMax);
    L.xlw = take(nxc > 0 ? sizeof(int32_t) * nlw : 0);
    L.xlv = take(nxc > 0 ? es * nlw : 0);
    L.total = off;
    return L;
}

int round8(int64_t x) { return (int)((x + 7) / 8 * 8); }

template <typename T>
Prob<T> prob(scg_ctx* c) {
    Prob<T> P;
    P.n = c->n;
    P.ld = c->ld;
    P.R = c->prm.R;
    P.rp = c->rp;
    P.col = c->col;
    P.val = (const T*)c->val;
    P.cval = c->cval;
    P.dC = c->dC;
    P.b = c->b;
    P.lo = c->lo;
    P.hi = c->hi;
    P.ball = (c->prm.constraint_set == 2) ? 1 : 0;
    P.ball_r = c->ball_r;
    P.trace_mode = c->prm.trace_mode;
    P.z = c->z;
    P.y = c->y;
    P.s = (T*)c->s;
    P.V = (T*)c->V;
    P.u = (T*)c->u;
    P.v = (T*)c->v;
    P.Om = (c->prm.omega_mode == 1) ? nullptr : (const T*)c->Om;
    P.seed = c->prm.seed;
    P.instance = (uint64_t)c->prm.instance;
    P.vmod = (c->prm.basis_mode == 1) ? 3 : 0;
    P.racc = c->racc;
    P.S = (T*)c->S;
    P.rb = c->rb;
    P.nrb = c->nrb;
    P.qw = c->qw;
    P.qv = (const T*)c->qv;
    P.qc = c->qc;
    P.nqc = c->nqc;
    P.sc = c->sc;
    double* pp = c->part;
    P.p_prep = pp;
    P.p_spmv = pp + (size_t)kGMax * 6;
    P.p_upd = pp + (size_t)kGMax * 7;
    P.p_ritz = pp + (size_t)kGMax * 8;
    P.p_obj = pp + (size_t)kGMax * (9 + kRMax);
    P.p_primal = pp + (size_t)kGMax * (11 + kRMax);
    P.p_ball = pp + (size_t)kGMax * (15 + kRMax);
    P.p_ball2 = pp + (size_t)kGMax * (16 + kRMax);
    P.p_h = pp + (size_t)kGMax * (19 + kRMax);
    P.G = c->G;
    P.Gs = c->Gs;
    P.logs = c->logs;
    P.T_iters = c->prm.T;
    return P;
}

template <typename T, int MODE, int RB, int FMT>
void launch_spmv_x(scg_ctx* c, const T* x, int step, int lanes) {
    Prob<T> P = prob<T>(c);
    dim3 g(c->Gs), b(kBlock);
    SegArgs sg{};
    sg.first = 1;
    sg.last = 1;
    sg.lanczos = (MODE == SPMV_LANCZOS) ? 1 : 0;
    for (int s = 0; s < kSegMax; ++s) {
        sg.xrp[s] = c->rp_seg[s];
        sg.xrbd[s] = c->rbd_seg[s];
        sg.xnrb[s] = c->nrb_seg[s];
    }
    sg.xpart = c->xpart;
    sg.xld = c->ld;
    switch (lanes) {
        case 2: hipLaunchKernelGGL((k_spmv<T, 2, SPMV_XPART, RB, FMT>), g, b, 0, c->stream, P, x, step, sg); break;
        case 4: hipLaunchKernelGGL((k_spmv<T, 4, SPMV_XPART, RB, FMT>), g, b, 0, c->stream, P, x, step, sg); break;
        case 8: hipLaunchKernelGGL((k_spmv<T, 8, SPMV_XPART, RB, FMT>), g, b, 0, c->stream, P, x, step, sg); break;
        case 16: hipLaunchKernelGGL((k_spmv<T, 16, SPMV_XPART, RB, FMT>), g, b, 0, c->stream, P, x, step, sg); break;
        default: hipLaunchKernelGGL((k_spmv<T, 32, SPMV_XPART, RB, FMT>), g, b, 0, c->stream, P, x, step, sg); break;
    }
    hipLaunchKernelGGL((k_xcombine<T, MODE>), g, b, 0, c->stream, P, x, step, (const T*)c->xpart, (int64_t)c->ld);
}

template <typename T, int MODE, int RB, int FMT>
void launch_spmv_f(scg_ctx* c, const T* x, int step, int lanes) {
    if (c->xseg) {
        launch_spmv_x<T, MODE, RB, FMT>(c, x, step, lanes);
        return;
    }
    Prob<T> P = prob<T>(c);
    dim3 g(c->Gs), b(kBlock);
    for (int sgi = 0; sgi < c->nseg; ++sgi) {
        SegArgs sg{};
        sg.rp = c->rp_seg[sgi];
        sg.rbd = c->rbd_seg[sgi];
        sg.nrb = c->nrb_seg[sgi];
        sg.first = (sgi == 0);
        sg.last = (sgi == c->nseg - 1);
        switch (lanes) {
            case 2: hipLaunchKernelGGL((k_spmv<T, 2, MODE, RB, FMT>), g, b, 0, c->stream, P, x, step, sg); break;
            case 4: hipLaunchKernelGGL((k_spmv<T, 4, MODE, RB, FMT>), g, b, 0, c->stream, P, x, step, sg); break;
            case 8: hipLaunchKernelGGL((k_spmv<T, 8, MODE, RB, FMT>), g, b, 0, c->stream, P, x, step, sg); break;
            case 16: hipLaunchKernelGGL((k_spmv<T, 16, MODE, RB, FMT>), g, b, 0, c->stream, P, x, step, sg); break;
            default: hipLaunchKernelGGL((k_spmv<T, 32, MODE, RB, FMT>), g, b, 0, c->stream, P, x, step, sg); break;
        }
    }
}

// The eight concurrent column segments over entry chunks: the slice pass (with
// the long segments) and the combining pass.
template <typename T, int MODE>
void launch_spmv_xc(scg_ctx* c, const T* x, int step) {
    const Prob<T> P = prob<T>(c);
    XcArgs a{};
    a.qw = c->xqw;
    a.qv = c->xqv;
    a.qc = c->xqc;
    a.lseg = c->xlseg;
    a.lw = c->xlw;
    a.lv = c->xlv;
    for (int s = 0; s <= kSegMax; ++s) {
        a.cb[s] = c->xcb[s];
        a.lb[s] = c->xlb[s];
    }
    a.xpart = c->xpart;
    a.xld = c->ld;
    a.lanczos = (MODE == SPMV_LANCZOS) ? 1 : 0;
    const dim3 g(c->Gs), b(kBlock);
    if (c->fmt == FMT_PAT) hipLaunchKernelGGL((k_spmvx<T, FMT_PAT>), g, b, 0, c->stream, P, x, a);
    else if (c->fmt == FMT_SGN) hipLaunchKernelGGL((k_spmvx<T, FMT_SGN>), g, b, 0, c->stream, P, x, a);
    else hipLaunchKernelGGL((k_spmvx<T, FMT_VAL>), g, b, 0, c->stream, P, x, a);
    hipLaunchKernelGGL((k_xcombine<T, MODE>), g, b, 0, c->stream, P, x, step, (const T*)c->xpart, (int64_t)c->ld);
}

template <typename T, int MODE>
void launch_spmv(scg_ctx* c, const T* x, int step, int lanes = 0) {
    if (lanes == 0) lanes = c->lanes;
    if (lanes == 1 && c->xseg) {   // the concurrent column segments over entry chunks
        launch_spmv_xc<T, MODE>(c, x, step);
        return;
    }
    if (lanes == 1) {   // the chunk products: padded column-word quads, or entries with values
        const dim3 g(c->Gs), b(kBlock);
        if (c->fmt == FMT_PAT) hipLaunchKernelGGL((k_spmvq<T, MODE, FMT_PAT>), g, b, 0, c->stream, prob<T>(c), x, step);
        else if (c->fmt == FMT_SGN)
            hipLaunchKernelGGL((k_spmvq<T, MODE, FMT_SGN>), g, b, 0, c->stream, prob<T>(c), x, step);
        else hipLaunchKernelGGL((k_spmve<T, MODE>), g, b, 0, c->stream, prob<T>(c), x, step);
        return;
    }
    if (c->fmt == FMT_PAT) launch_spmv_f<T, MODE, 8, FMT_PAT>(c, x, step, lanes);
    else if (c->fmt == FMT_SGN) launch_spmv_f<T, MODE, 8, FMT_SGN>(c, x, step, lanes);
    else launch_spmv_f<T, MODE, 8, FMT_VAL>(c, x, step, lanes);
}

template <typename T, int RB>
void launch_ritz_rb(scg_ctx* c, const Prob<T>& P, int q) {
    const dim3 g(c->G), b(kBlock), one(1);
    if (c->prm.basis_mode == 1) hipLaunchKernelGGL((k_ritz_regen<T, RB>), g, b, 0, c->stream, P, q);
    else hipLaunchKernelGGL((k_ritz<T, RB>), g, b, 0, c->stream, P);
    hipLaunchKernelGGL((k_ritz_fin<RB>), one, b, 0, c->stream, c->sc, P.p_ritz, c->G, c->prm.R);
}

template <typename T>
void launch_ritz(scg_ctx* c, int q) {
    Prob<T> P = prob<T>(c);
    const int R = c->prm.R;
    if (R <= 8) launch_ritz_rb<T, 8>(c, P, q);
    else if (R <= 16) launch_ritz_rb<T, 16>(c, P, q);
    else launch_ritz_rb<T, 32>(c, P, q);
}

// Column i of the Lanczos basis (three rotating columns when it is regenerated).
template <typename T>
const T* basis_col(scg_ctx* c, int i) {
    const int j = (c->prm.basis_mode == 1) ? i % 3 : i;
    return (const T*)c->V + (size_t)j * c->ld;
}

template <typename T>
void launch_dual_sketch(scg_ctx* c, const IterArgs& it) {
    Prob<T> P = prob<T>(c);
    dim3 g(c->G), b(kBlock);
    if (c->prm.R <= 8) hipLaunchKernelGGL((k_dual_sketch<T, 8>), g, b, 0, c->stream, P, it);
    else if (c->prm.R <= 16) hipLaunchKernelGGL((k_dual_sketch<T, 16>), g, b, 0, c->stream, P, it);
    else hipLaunchKernelGGL((k_dual_sketch<T, 32>), g, b, 0, c->stream, P, it);
}

IterArgs iter_args(scg_ctx* c, int t) {
    IterArgs it;
    it.t = t;
    it.q = q_for(c->prm, c->n, t);
    it.beta = c->prm.beta0 * std::sqrt(t + 1.0);
    it.beta_next = c->prm.beta0 * std::sqrt(t + 2.0);
    it.eta = 2.0 / (t + 1.0);
    it.alpha = c->alpha_s;
    it.beta0 = c->prm.beta0;
    it.K = c->prm.K;
    it.seed = c->prm.seed;
    it.instance = (uint64_t)c->prm.instance;
    it.dev = 0;
    return it;
}

template <typename T>
void enqueue_prep(scg_ctx* c, const IterArgs& it) {
    hipLaunchKernelGGL((k_prep<T>), dim3(c->G), dim3(kBlock), 0, c->stream, prob<T>(c), it);
}

// Ball constraint set: partial sums of ||z + y / beta - b||^2 for the slack.
template <typename T>
void enqueue_ball_norm(scg_ctx* c, double beta) {
    hipLaunchKernelGGL((k_ball_norm<T>), dim3(c->G), dim3(kBlock), 0, c->stream, prob<T>(c), beta);
}

// Lanczos step i after its product: three-term update (accumulating the Ritz
// vector in the second sweep of a regenerated basis), then the optional
// reorthogonalisation against v_j0 .. v_i.
template <typename T>
void enqueue_update(scg_ctx* c, const Prob<T>& P, int i, int accum) {
    const dim3 g(c->G), b(kBlock);
    if (c->prm.reorth == 0) {
        hipLaunchKernelGGL((k_lupdate<T>), g, b, 0, c->stream, P, i, 1, accum);
        return;
    }
    const int j0 = (c->prm.reorth == 2) ? 0 : std::max(0, i - 1);
    hipLaunchKernelGGL((k_lupdate<T>), g, b, 0, c->stream, P, i, 0, accum);
    hipLaunchKernelGGL((k_reorth_dot<T>), g, b, 0, c->stream, P, i, j0);
    hipLaunchKernelGGL(k_reduce_h, dim3(1), b, 0, c->stream, c->sc, P.p_h, c->G, i, j0);
    hipLaunchKernelGGL((k_reorth_apply<T>), g, b, 0, c->stream, P, i, j0);
}

// One iteration; with dev the kernels take t, beta and eta from the device
// counter (the form captured into a graph and replayed for every t with the same q).
template <typename T>
void enqueue_iteration(scg_ctx* c, int t, int dev = 0) {
    IterArgs it = iter_args(c, t);
    it.dev = dev;
    Prob<T> P = prob<T>(c);
    if (P.ball) enqueue_ball_norm<T>(c, it.beta);
    enqueue_prep<T>(c, it);
    for (int i = 0; i < it.q; ++i) {
        launch_spmv<T, SPMV_LANCZOS>(c, basis_col<T>(c, i), i);
        if (i == it.q - 1) break;   // rho_q and v_{q+1} are never used
        enqueue_update<T>(c, P, i, 0);
    }
    hipLaunchKernelGGL((k_tridiag<T>), dim3(1), dim3(kBlock), 0, c->stream, P, it.q);
    if (c->prm.basis_mode == 1) {
        // second pass: the same recurrence regenerates v_0 .. v_{k-1} (bitwise, the
        // products are deterministic) and k_lupdate accumulates the Ritz vector
        enqueue_prep<T>(c, it);
        for (int i = 0; i + 1 < it.q; ++i) {
            launch_spmv<T, SPMV_LANCZOS>(c, basis_col<T>(c, i), i);
            enqueue_update<T>(c, P, i, 1);
        }
    }
    launch_ritz<T>(c, it.q);
    launch_spmv<T, SPMV_OBJ>(c, (const T*)c->v, 0);
    hipLaunchKernelGGL((k_primal<T>), dim3(c->G), dim3(kBlock), 0, c->stream, P, it);
    if (P.ball) {
        enqueue_ball_norm<T>(c, it.beta_next);
        hipLaunchKernelGGL((k_ball_r2<T>), dim3(c->G), dim3(kBlock), 0, c->stream, P, it);
    }
    launch_dual_sketch<T>(c, it);
}

// ------------------------------------------------------------- init kernels
// Box constraint set in scaled units; err bit 8 for lo > hi, a NaN bound or an
// empty side (lo = +inf or hi = -inf).
__global__ __launch_bounds__(kBlock) void k_set_box(int64_t n, const double* lo, const double* hi, double inv_alpha,
                                                    double* lo_s, double* hi_s, DevScalars* sc) {
    int err = 0;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const double l = lo ? lo[i] : -INFINITY;
        const double h = hi ? hi[i] : INFINITY;
        if (!(l <= h) || l == INFINITY || h == -INFINITY) err = 8;
        lo_s[i] = l * inv_alpha;
        hi_s[i] = h * inv_alpha;
    }
    if (err) atomicOr(&sc->err, err);
}

__global__ __launch_bounds__(kBlock) void k_validate(int64_t n, const int64_t* rp, const int32_t* col,
                                                     const double* val, const double* b, int32_t* cnt,
                                                     double* dCraw, DevScalars* sc, double* part,
                                                     unsigned* counter, double* mm) {
    int64_t lo, hi;
    split_range(n, xcd_lid(), gridDim.x, lo, hi);
    double a[2] = {0.0, 0.0};
    double vmin = INFINITY, vmax = -INFINITY, amin = INFINITY, amax = -INFINITY;
    int err = 0;
    for (int64_t r = lo + threadIdx.x; r < hi; r += kBlock) {
        int32_t c_off = 0;
        double dsum = 0.0;
        for (int64_t e = rp[r]; e < rp[r + 1]; ++e) {
            const int32_t j = col[e];
            const double v = val[e];
            if (j < 0 || (int64_t)j >= n) err |= 1;
            if (!isfinite(v)) err |= 2;
            a[0] += v * v;
            if ((int64_t)j == r) {
                dsum += v;
            } else {
                ++c_off;
                vmin = fmin(vmin, v);
                vmax = fmax(vmax, v);
                amin = fmin(amin, fabs(v));
                amax = fmax(amax, fabs(v));
            }
        }
        cnt[r] = c_off;
        dCraw[r] = dsum;
        const double br = b[r];
        if (!isfinite(br)) err |= 4;
        a[1] += br;
    }
    if (err) atomicOr(&sc->err, err);
    // per-workgroup extremes of the off-diagonal values (combined on the host)
    {
        __shared__ double red4[4][kWaves];
        double m4[4] = {vmin, -vmax, amin, -amax};
        for (int i = 0; i < 4; ++i) {
            double v = m4[i];
            for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
            if ((threadIdx.x & 63) == 0) red4[i][threadIdx.x >> 6] = v;
        }
        __syncthreads();
        if (threadIdx.x < 4) {
            double v = red4[threadIdx.x][0];
            for (int w = 1; w < kWaves; ++w) v = fmin(v, red4[threadIdx.x][w]);
            mm[(size_t)blockIdx.x * 4 + threadIdx.x] = v;
        }
    }
    double tot[2];
    if (grid_sum<2>(a, part, counter, tot) && threadIdx.x == 0) {
        sc->sum_sq = tot[0];
        sc->sum_b = tot[1];
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_scatter(int64_t n, const int64_t* rp, const int32_t* col,
                                                    const double* val, const double* b_in, const int32_t* rp_off,
                                                    int32_t* col_off, T* val_off, const double* dCraw, double* dC,
                                                    double* b_out, double inv_cF, double inv_alpha, int fmt) {
    int64_t lo, hi;
    split_range(n, xcd_lid(), gridDim.x, lo, hi);
    for (int64_t r = lo + threadIdx.x; r < hi; r += kBlock) {
        int32_t o = rp_off[r];
        for (int64_t e = rp[r]; e < rp[r + 1]; ++e) {
            const int32_t j = col[e];
            if ((int64_t)j == r) continue;
            if (fmt == FMT_VAL) {
                col_off[o] = j;
                val_off[o] = (T)(val[e] * inv_cF);
            } else if (fmt == FMT_PAT) {
                col_off[o] = j;
            } else {
                col_off[o] = (val[e] < 0.0) ? (int32_t)((uint32_t)j | 0x80000000u) : j;
            }
            ++o;
        }
        dC[r] = dCraw[r] * inv_cF;
        b_out[r] = b_in[r] * inv_alpha;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_omega(int64_t n, int64_t ld, int R, uint64_t seed, uint64_t instance,
                                                  T* Om) {
    const int64_t ng = (n + 3) / 4;
    const int64_t total = ng * R;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < total; i += (int64_t)gridDim.x * kBlock) {
        const int64_t gi = i % ng;
        const int c = (int)(i / ng);
        double g[4];
        normal4(seed, (uint64_t)gi, (uint64_t)c, instance, 1ull, g);
        for (int m = 0; m < 4; ++m) {
            const int64_t r = 4 * gi + m;
            if (r < n) Om[(int64_t)c * ld + r] = (T)g[m];
        }
    }
}

template <typename Tin, typename Tout>
__global__ __launch_bounds__(kBlock) void k_cast(int64_t cnt, const Tin* in, Tout* out) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * kBlock)
        out[i] = (Tout)in[i];
}

// out (column-major n x R) <-> in (row-major n x R), with a type change.
template <typename Tin, typename Tout>
__global__ __launch_bounds__(kBlock) void k_transpose_cast(int64_t n, int64_t ld, int R, const Tin* in, Tout* out,
                                                           int to_colmajor) {
    const int64_t cnt = n * R;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * kBlock) {
        if (to_colmajor) {
            const int64_t r = i / R, c = i % R;           // i indexes the row-major input
            out[c * ld + r] = (Tout)in[i];
        } else {
            const int64_t c = i / n, r = i % n;           // i indexes column c, row r
            out[r * R + c] = (Tout)in[c * ld + r];
        }
    }
}

template <typename Tin, typename Tout>
void transpose_cast(scg_ctx* c, const Tin* in, Tout* out, int to_colmajor) {
    const int64_t cnt = c->n * c->prm.R;
    const int g = (int)std::min<int64_t>(4096, std::max<int64_t>(1, (cnt + kBlock - 1) / kBlock));
    hipLaunchKernelGGL((k_transpose_cast<Tin, Tout>), dim3(g), dim3(kBlock), 0, c->stream, c->n, c->ld, c->prm.R,
                       in, out, to_colmajor);
}

template <typename Tin, typename Tout>
void cast(scg_ctx* c, int64_t cnt, const Tin* in, Tout* out) {
    const int g = (int)std::min<int64_t>(4096, std::max<int64_t>(1, (cnt + kBlock - 1) / kBlock));
    hipLaunchKernelGGL((k_cast<Tin, Tout>), dim3(g), dim3(kBlock), 0, c->stream, cnt, in, out);
}

void partition_rows(const std::vector<int32_t>& rp, int64_t n, std::vector<int32_t>& rb);

// Row blocks of at most kNB nonzeros and kRowsCap rows (a longer row is a
// block of its own), as (first row, first nonzero) pairs; the last entry is
// (n, end of the nonzeros).
std::vector<int2> block_descriptors(const std::vector<int32_t>& rp, int64_t n) {
    std::vector<int32_t> rb;
    partition_rows(rp, n, rb);
    std::vector<int2> d(rb.size());
    for (size_t k = 0; k < rb.size(); ++k) d[k] = make_int2(rb[k], rp[rb[k]]);
    return d;
}

void partition_rows(const std::vector<int32_t>& rp, int64_t n, std::vector<int32_t>& rb) {
    rb.clear();
    rb.push_back(0);
    int64_t cur_nnz = 0, cur_rows = 0;
    for (int64_t r = 0; r < n; ++r) {
        const int64_t len = rp[r + 1] - rp[r];
        if (len > kNB) {
            if (cur_rows > 0) rb.push_back((int32_t)r);
            rb.push_back((int32_t)(r + 1));
            cur_nnz = cur_rows = 0;
            continue;
        }
        if (cur_rows > 0 && (cur_nnz + len > kNB || cur_rows >= kRowsCap)) {
            rb.push_back((int32_t)r);
            cur_nnz = cur_rows = 0;
        }
        cur_nnz += len;
        ++cur_rows;
    }
    if (cur_rows > 0) rb.push_back((int32_t)n);
}

int pick_lanes(double mean_len) {
    int l = 2;
    while (l < 32 && 2.0 * l <= mean_len) l *= 2;
    return l;
}

// Per-row counts of off-diagonal entries in each of nseg column segments.
__global__ __launch_bounds__(kBlock) void k_segcount(int64_t n, const int64_t* rp, const int32_t* col, int nseg,
                                                     int64_t seglen, int32_t* cnt) {
    int64_t lo, hi;
    split_range(n, xcd_lid(), gridDim.x, lo, hi);
    for (int64_t r = lo + threadIdx.x; r < hi; r += kBlock) {
        int32_t cs[kSegMax] = {};
        for (int64_t e = rp[r]; e < rp[r + 1]; ++e) {
            const int32_t j = col[e];
            if ((int64_t)j == r) continue;
            cs[(int)(j / seglen)]++;
        }
        for (int s = 0; s < nseg; ++s) cnt[(size_t)s * n + r] = cs[s];
    }
}

// Scatter the off-diagonal entries into the segment layout (rp_s absolute).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_scatter_seg(int64_t n, const int64_t* rp, const int32_t* col,
                                                        const double* val, int nseg, int64_t seglen,
                                                        const int32_t* rps, int64_t rps_stride, int32_t* col_off,
                                                        T* val_off, double inv_cF, int fmt) {
    int64_t lo, hi;
    split_range(n, xcd_lid(), gridDim.x, lo, hi);
    for (int64_t r = lo + threadIdx.x; r < hi; r += kBlock) {
        int32_t o[kSegMax];
        for (int s = 0; s < nseg; ++s) o[s] = rps[(size_t)s * rps_stride + r];
        for (int64_t e = rp[r]; e < rp[r + 1]; ++e) {
            const int32_t j = col[e];
            if ((int64_t)j == r) continue;
            const int s = (int)(j / seglen);
            const int32_t at = o[s]++;
            if (fmt == FMT_VAL) {
                col_off[at] = j;
                val_off[at] = (T)(val[e] * inv_cF);
            } else if (fmt == FMT_PAT) {
                col_off[at] = j;
            } else {
                col_off[at] = (val[e] < 0.0) ? (int32_t)((uint32_t)j | 0x80000000u) : j;
            }
        }
    }
}

// Build the nseg-segment layout of the off-diagonal part from the input CSR.
// The sliced entry-chunk layout from the sliced CSR that build_segments has just
// written (row pointers of slice s at rp + s (n + 1), entries in col / val):
// thread per (slice, row); eoff = the segment's first slot.  The words and
// values of every chunk were filled with padding (kQPad, 0) beforehand.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_scatter_xchunks(int64_t n, const int32_t* rp, const int32_t* col,
                                                            const T* val, const int32_t* eoff, int32_t* qw, T* qv,
                                                            int fmt) {
    const int64_t tot = (int64_t)kSegMax * n;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < tot; i += (int64_t)gridDim.x * kBlock) {
        const int64_t s = i / n, r = i - s * n;
        const int32_t* rps = rp + s * (n + 1);
        const int32_t e0 = rps[r], d = rps[r + 1] - e0;
        const int64_t o = eoff[i];
        if (d == 0 || d > kERowMax) {   // placeholder; column bit 0 marks a long segment
            qw[o] = kQPad | kQStart | (d > kERowMax ? 1 : 0);
            continue;
        }
        for (int k = 0; k < d; ++k) {
            qw[o + k] = (k == 0) ? (col[e0 + k] | kQStart) : col[e0 + k];
            if (fmt == FMT_VAL) qv[o + k] = val[e0 + k];
        }
    }
}

// Entries of the long segments, one wave per segment: (row, first entry, entries, source entry).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_copy_long(int64_t nl, const int4* lseg, const int32_t* col, const T* val,
                                                      int32_t* lw, T* lv, int fmt) {
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int64_t k = (int64_t)blockIdx.x * kWaves + wv; k < nl; k += (int64_t)gridDim.x * kWaves) {
        const int4 d = lseg[k];
        const int64_t src = d.w;
        for (int e = lane; e < d.z; e += 64) {
            lw[(int64_t)d.y + e] = col[src + e];
            if (fmt == FMT_VAL) lv[(int64_t)d.y + e] = val[src + e];
        }
    }
}

template <typename T>
scg_status build_xchunks(scg_ctx* c) {
    c->nxc = 0;
    if (!c->xqw || c->nseg != kSegMax) return SCG_OK;
    const int64_t n = c->n;
    std::vector<int32_t> hrp((size_t)kSegMax * (n + 1)), hc((size_t)kSegMax * n);
    HIP_TRY(hipMemcpyAsync(hrp.data(), c->rp, sizeof(int32_t) * hrp.size(), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (int s = 0; s < kSegMax; ++s)
        for (int64_t r = 0; r < n; ++r)
            hc[(size_t)s * n + r] = hrp[(size_t)s * (n + 1) + r + 1] - hrp[(size_t)s * (n + 1) + r];
    std::vector<int32_t> eoff((size_t)kSegMax * n);
    std::vector<int2> qc;
    std::vector<int4> lseg;
    int64_t loff = 0;
    for (int s = 0; s < kSegMax; ++s) {
        c->xcb[s] = (int64_t)qc.size();
        c->xlb[s] = (int64_t)lseg.size();
        int fill = 256;
        for (int64_t r = 0; r < n; ++r) {
            const int d = hc[(size_t)s * n + r];
            const int slots = (d == 0 || d > kERowMax) ? 1 : d;
            if (fill + slots > 256) {
                qc.push_back(make_int2((int)r, 0));
                fill = 0;
            }
            const int64_t o = (int64_t)(qc.size() - 1) * 256 + fill;
            if (o > INT32_MAX) return SCG_OK;
            eoff[(size_t)s * n + r] = (int32_t)o;
            fill += slots;
            qc.back().y = (fill + 3) / 4;
            if (d > kERowMax) {
                if (loff + d + 3 > INT32_MAX) return SCG_OK;   // entry offsets are int32
                lseg.push_back(make_int4((int)r, (int)loff, d, hrp[(size_t)s * (n + 1) + r]));
                loff += (d + 3) / 4 * 4;
            }
        }
    }
    c->xcb[kSegMax] = (int64_t)qc.size();
    c->xlb[kSegMax] = (int64_t)lseg.size();
    if ((int64_t)qc.size() > c->xqc_cap || (int64_t)lseg.size() > c->xlseg_cap ||
        loff > c->nnz_in + 4 * c->xlseg_cap)
        return SCG_OK;   // cannot happen within the reserved bounds
    // the offsets go through the concurrent-segment partials (8 ld elements of at least 4 bytes), unused yet
    int32_t* deoff = static_cast<int32_t*>(c->xpart);
    const size_t slots = 256 * qc.size();
    HIP_TRY(hipMemcpyAsync(deoff, eoff.data(), sizeof(int32_t) * eoff.size(), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->xqc, qc.data(), sizeof(int2) * qc.size(), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemsetD32Async((hipDeviceptr_t)c->xqw, kQPad, slots, c->stream));
    HIP_TRY(hipMemsetAsync(c->xqv, 0, sizeof(T) * slots, c->stream));
    hipLaunchKernelGGL((k_scatter_xchunks<T>), dim3(c->G), dim3(kBlock), 0, c->stream, n, c->rp, c->col,
                       (const T*)c->val, deoff, c->xqw, (T*)c->xqv, c->fmt);
    HIP_TRY(hipGetLastError());
    if (!lseg.empty()) {
        HIP_TRY(hipMemcpyAsync(c->xlseg, lseg.data(), sizeof(int4) * lseg.size(), hipMemcpyHostToDevice, c->stream));
        HIP_TRY(hipMemsetD32Async((hipDeviceptr_t)c->xlw, kQPad, (size_t)loff, c->stream));
        HIP_TRY(hipMemsetAsync(c->xlv, 0, sizeof(T) * (size_t)loff, c->stream));
        hipLaunchKernelGGL((k_copy_long<T>), dim3(c->G), dim3(kBlock), 0, c->stream, (int64_t)lseg.size(), c->xlseg,
                           c->col, (const T*)c->val, c->xlw, (T*)c->xlv, c->fmt);
        HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->nxc = (int64_t)qc.size();
    return SCG_OK;
}

template <typename T>
scg_status build_segments(scg_ctx* c, int nseg, const int64_t* row_ptr, const int32_t* col, const double* val) {
    const int64_t n = c->n;
    const int64_t seglen = (n + nseg - 1) / nseg;
    int32_t* cnt = c->rb;   // scratch: nseg * n ints fit in the row-block area
    hipLaunchKernelGGL(k_segcount, dim3(c->G), dim3(kBlock), 0, c->stream, n, row_ptr, col, nseg, seglen, cnt);
    std::vector<int32_t> hc((size_t)nseg * n);
    HIP_TRY(hipMemcpyAsync(hc.data(), cnt, sizeof(int32_t) * hc.size(), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    std::vector<int32_t> hrp((size_t)nseg * (n + 1));
    int64_t acc = 0;
    for (int s = 0; s < nseg; ++s) {
        for (int64_t r = 0; r < n; ++r) {
            hrp[(size_t)s * (n + 1) + r] = (int32_t)acc;
            acc += hc[(size_t)s * n + r];
        }
        hrp[(size_t)s * (n + 1) + n] = (int32_t)acc;
    }
    if (acc != c->nnz_off) return SCG_EINVAL;
    int maxnrb = 0;
    std::vector<std::vector<int2>> hrbd(nseg);
    for (int s = 0; s < nseg; ++s) {
        std::vector<int32_t> rps(hrp.begin() + (size_t)s * (n + 1), hrp.begin() + (size_t)(s + 1) * (n + 1));
        hrbd[s] = block_descriptors(rps, n);
        maxnrb = std::max(maxnrb, (int)hrbd[s].size() - 1);
    }
    for (int s = 0; s < nseg; ++s) {
        c->rp_seg[s] = c->rp + (size_t)s * (n + 1);
        c->rbd_seg[s] = reinterpret_cast<int2*>(c->rb) + (size_t)s * (n + 2);
        c->nrb_seg[s] = (int)hrbd[s].size() - 1;
        HIP_TRY(hipMemcpyAsync(c->rp_seg[s], hrp.data() + (size_t)s * (n + 1), sizeof(int32_t) * (n + 1),
                               hipMemcpyHostToDevice, c->stream));
        HIP_TRY(hipMemcpyAsync(c->rbd_seg[s], hrbd[s].data(), sizeof(int2) * hrbd[s].size(), hipMemcpyHostToDevice,
                               c->stream));
    }
    c->nseg = nseg;
    c->seglen = seglen;
    c->nrb = maxnrb;
    c->Gs = std::min(kGMax, std::max(8, round8((maxnrb + kWaves - 1) / kWaves)));
    hipLaunchKernelGGL((k_scatter_seg<T>), dim3(c->G), dim3(kBlock), 0, c->stream, n, row_ptr, col, val, nseg, seglen,
                       c->rp, (int64_t)(n + 1), c->col, (T*)c->val, 1.0 / c->c_F, c->fmt);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(c->stream));
    return SCG_OK;
}

// Column words of the quad-chunk layout: row r's off-diagonal entries (input
// order, diagonal skipped, as k_scatter) from word qoff[r] on, padded to a
// whole quad, the first word flagged as the row's start.
__global__ __launch_bounds__(kBlock) void k_scatter_quad(int64_t n, const int64_t* rp, const int32_t* col,
                                                         const double* val, const int64_t* qoff, int32_t* qw,
                                                         int fmt) {
    int64_t lo, hi;
    split_range(n, xcd_lid(), gridDim.x, lo, hi);
    for (int64_t r = lo + threadIdx.x; r < hi; r += kBlock) {
        const int64_t o = qoff[r];
        int64_t d = 0;
        for (int64_t e = rp[r]; e < rp[r + 1]; ++e) {
            const int32_t j = col[e];
            if ((int64_t)j == r) continue;
            int32_t w = j;
            if (fmt == FMT_SGN && val[e] < 0.0) w = (int32_t)((uint32_t)w | 0x80000000u);
            if (d == 0) w |= kQStart;
            qw[o + d] = w;
            ++d;
        }
        const int64_t end = 4 * ((d > 0) ? (d + 3) / 4 : 1);
        for (int64_t k = d; k < end; ++k) qw[o + k] = kQPad | (k == 0 ? kQStart : 0);
    }
}

// Build the quad-chunk layout when the matrix qualifies (column words only,
// every row at most kQRowMax off-diagonal entries); cnt = off-diagonal
// entries per row.  The word offsets go through the basis area, unused yet.
template <typename T>
scg_status build_quad_chunks(scg_ctx* c, const int64_t* row_ptr, const int32_t* col, const double* val,
                             const std::vector<int32_t>& cnt) {
    c->nqc = 0;
    const int64_t n = c->n;
    if (!c->qw || c->fmt == FMT_VAL) return SCG_OK;
    for (int64_t r = 0; r < n; ++r)
        if (cnt[r] > kQRowMax) return SCG_OK;
    std::vector<int64_t> qoff(n);
    std::vector<int2> qc;
    int fill = 64;
    for (int64_t r = 0; r < n; ++r) {
        const int rq = std::max(1, (cnt[r] + 3) / 4);
        if (fill + rq > 64) {
            qc.push_back(make_int2((int)r, 0));
            fill = 0;
        }
        qoff[r] = (int64_t)(qc.size() - 1) * 256 + 4 * fill;
        fill += rq;
        qc.back().y = fill;
    }
    if ((int64_t)qc.size() > c->qc_cap) return SCG_OK;   // cannot happen within the reserved bound
    int64_t* dqoff = reinterpret_cast<int64_t*>(c->V);
    HIP_TRY(hipMemcpyAsync(dqoff, qoff.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->qc, qc.data(), sizeof(int2) * qc.size(), hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(k_scatter_quad, dim3(c->G), dim3(kBlock), 0, c->stream, n, row_ptr, col, val, dqoff, c->qw,
                       c->fmt);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->nqc = (int64_t)qc.size();
    return SCG_OK;
}

// The entry-chunk layout: row r's off-diagonal entries (input order, diagonal
// skipped, values scaled as k_scatter stores them) from entry eoff[r] on, the
// first word flagged as the row's start; a row without off-diagonal entries
// takes one padding entry flagged as a start.  The words and values of every
// chunk were filled with padding (kQPad, 0) beforehand.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_scatter_entries(int64_t n, const int64_t* rp, const int32_t* col,
                                                            const double* val, const int64_t* eoff, int32_t* qw,
                                                            T* qv, double inv_cF) {
    int64_t lo, hi;
    split_range(n, xcd_lid(), gridDim.x, lo, hi);
    for (int64_t r = lo + threadIdx.x; r < hi; r += kBlock) {
        const int64_t o = eoff[r];
        int64_t d = 0;
        for (int64_t e = rp[r]; e < rp[r + 1]; ++e) {
            const int32_t j = col[e];
            if ((int64_t)j == r) continue;
            qw[o + d] = (d == 0) ? (j | kQStart) : j;
            qv[o + d] = (T)(val[e] * inv_cF);
            ++d;
        }
        if (d == 0) qw[o] = kQPad | kQStart;
    }
}

// Build the entry-chunk layout when the matrix qualifies (values stored, every
// row at most kERowMax off-diagonal entries); cnt = off-diagonal entries per
// row.  The entry offsets go through the basis area, unused yet.
template <typename T>
scg_status build_entry_chunks(scg_ctx* c, const int64_t* row_ptr, const int32_t* col, const double* val,
                              const std::vector<int32_t>& cnt) {
    c->nqc = 0;
    const int64_t n = c->n;
    if (!c->qv || c->fmt != FMT_VAL) return SCG_OK;
    for (int64_t r = 0; r < n; ++r)
        if (cnt[r] > kERowMax) return SCG_OK;
    std::vector<int64_t> eoff(n);
    std::vector<int2> qc;
    int fill = 256;
    for (int64_t r = 0; r < n; ++r) {
        const int d = std::max(1, (int)cnt[r]);
        if (fill + d > 256) {
            qc.push_back(make_int2((int)r, 0));
            fill = 0;
        }
        eoff[r] = (int64_t)(qc.size() - 1) * 256 + fill;
        fill += d;
        qc.back().y = (fill + 3) / 4;
    }
    if ((int64_t)qc.size() > entry_chunk_cap(c->prm, n, c->nnz_in)) return SCG_OK;   // cannot happen (the bound)
    const size_t slots = 256 * qc.size();
    int64_t* deoff = reinterpret_cast<int64_t*>(c->V);
    HIP_TRY(hipMemcpyAsync(deoff, eoff.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->qc, qc.data(), sizeof(int2) * qc.size(), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemsetD32Async((hipDeviceptr_t)c->qw, kQPad, slots, c->stream));
    HIP_TRY(hipMemsetAsync(c->qv, 0, sizeof(T) * slots, c->stream));
    hipLaunchKernelGGL((k_scatter_entries<T>), dim3(c->G), dim3(kBlock), 0, c->stream, n, row_ptr, col, val, deoff,
                       c->qw, (T*)c->qv, 1.0 / c->c_F);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->nqc = (int64_t)qc.size();
    return SCG_OK;
}

// Shift, start vector, the first product and the first update of iteration
// `it` (its partial sums are what the timed step-1 products reduce).
template <typename T>
void time_spmv_setup(scg_ctx* c, const IterArgs& it) {
    enqueue_prep<T>(c, it);
    launch_spmv<T, SPMV_LANCZOS>(c, basis_col<T>(c, 0), 0);
    hipLaunchKernelGGL((k_lupdate<T>), dim3(c->G), dim3(kBlock), 0, c->stream, prob<T>(c), 0, 1, 0);
}

// Workgroups of the chunk product that the device keeps resident at once (its
// occupancy times the compute units), at most kGMax; 0 if the runtime cannot tell.
template <typename T>
int chunk_resident_grid(scg_ctx* c) {
    int per_cu = 0, cus = 0;
    hipError_t e;
    if (c->fmt == FMT_VAL)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_spmve<T, SPMV_LANCZOS>, kBlock, 0);
    else if (c->fmt == FMT_PAT)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_spmvq<T, SPMV_LANCZOS, FMT_PAT>, kBlock, 0);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_spmvq<T, SPMV_LANCZOS, FMT_SGN>, kBlock, 0);
    if (e != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess)
        return 0;
    return std::min(kGMax, per_cu * cus / 8 * 8);
}

// Autotuner: time the Lanczos SpMV on this matrix for each lanes-per-row
// choice, column-segment count and grid, and the quad-chunk product when the
// matrix has that layout, and keep the fastest.  The candidates run the
// product of Lanczos step 1 of iteration 1 (after its shift, start vector,
// first product and update), timed with HIP events on the context stream.
template <typename T>
scg_status autotune_spmv(scg_ctx* c, const int64_t* row_ptr, const int32_t* col, const double* val) {
    const IterArgs it = iter_args(c, 1);
    time_spmv_setup<T>(c, it);   // candidates are timed as the step-1 product a solve repeats
    const T* x1 = basis_col<T>(c, 1);
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    const double mean = c->n > 0 ? (double)c->nnz_off / (double)c->n : 1.0;
    float best = 1e30f;
    int best_l = c->lanes, best_s = 1, best_g = 0;
    // candidates are tried in a fixed order and a later one replaces the best only
    // when it is at least 3% faster, so near-ties do not flip between runs
    auto better = [&](float ms) { return ms < best * 0.97f; };
    // average of five launches after one warm-up, HIP events on the context stream
    auto time_lanes = [&](int l, float& ms) -> hipError_t {
        launch_spmv<T, SPMV_LANCZOS>(c, x1, 1, l);
        hipError_t e = hipEventRecord(e0, c->stream);
        if (e != hipSuccess) return e;
        for (int r = 0; r < 5; ++r) launch_spmv<T, SPMV_LANCZOS>(c, x1, 1, l);
        if ((e = hipEventRecord(e1, c->stream)) != hipSuccess) return e;
        if ((e = hipEventSynchronize(e1)) != hipSuccess) return e;
        return hipEventElapsedTime(&ms, e0, e1);
    };
    const int cap = (int)(c->rb_cap / (size_t)(c->n + 2));   // segments the workspace was sized for
    bool best_x = false;
    for (int nseg : {1, 2, 4}) {
        if (c->prm.segments > 0 && nseg != c->prm.segments) continue;
        if (nseg > 1) {
            if (nseg > cap || (c->prm.segments == 0 && c->n < (1 << 18))) break;
            scg_status st = build_segments<T>(c, nseg, row_ptr, col, val);
            if (st != SCG_OK) return st;
        }
        // grid: one row-block range per wave (natural), or fewer workgroups so that
        // the whole grid is resident and each wave walks a longer range
        const int g_nat = c->Gs;
        for (int gcap : {0, 1536, 1024}) {
            if (c->prm.spmv_grid > 0 && gcap != 0) continue;   // a forced grid is applied afterwards
            if (gcap != 0 && gcap >= g_nat) continue;
            c->Gs = (gcap != 0) ? gcap : g_nat;
            for (int l : {2, 4, 8, 16, 32}) {
                if (c->prm.spmv_lanes > 0 && l != c->prm.spmv_lanes) continue;
                if (c->prm.spmv_lanes == 0 && l > 4 * mean + 4) break;
                float ms = 0.f;
                HIP_TRY(time_lanes(l, ms));
                if (better(ms)) { best = ms; best_l = l; best_s = nseg; best_g = gcap; }
            }
        }
        c->Gs = g_nat;
    }
    // eight segments in one launch, one per XCD, and the combining pass
    if (cap >= kSegMax && c->xpart && (c->prm.segments == kSegMax || (c->prm.segments == 0 && c->n >= (1 << 18))) &&
        c->prm.spmv_lanes != 1) {
        scg_status st = build_segments<T>(c, kSegMax, row_ptr, col, val);
        if (st != SCG_OK) return st;
        const int g_keep = c->Gs;
        c->xseg = true;
        for (int g : {2048, 1024}) {
            if (c->prm.spmv_grid > 0 && g != 2048) continue;   // a forced grid is applied afterwards
            c->Gs = g;
            for (int l : {2, 4, 8}) {
                if (c->prm.spmv_lanes > 0 && l != c->prm.spmv_lanes) continue;
                float ms = 0.f;
                HIP_TRY(time_lanes(l, ms));
                if (better(ms)) { best = ms; best_l = l; best_s = kSegMax; best_g = g; best_x = true; }
            }
        }
        c->xseg = false;
        c->Gs = g_keep;
    }
    // the eight concurrent segments over entry chunks, when the row-block form of the eight segments
    // beat every single-launch shape (slicing the columns pays on this matrix) or they are forced
    if (c->xqw && c->xpart && (best_x || (c->prm.spmv_lanes == 1 && c->prm.segments == kSegMax))) {
        if (c->nseg != kSegMax) {
            scg_status st = build_segments<T>(c, kSegMax, row_ptr, col, val);
            if (st != SCG_OK) return st;
        }
        if (c->nxc == 0) {
            scg_status st = build_xchunks<T>(c);
            if (st != SCG_OK) return st;
        }
        if (c->nxc > 0) {
            const int g_keep = c->Gs;
            c->xseg = true;
            for (int g : {1024, 2048}) {
                if (c->prm.spmv_grid > 0 && g != 1024) continue;   // a forced grid is applied afterwards
                c->Gs = g;
                float ms = 0.f;
                HIP_TRY(time_lanes(1, ms));
                if (better(ms)) { best = ms; best_l = 1; best_s = kSegMax; best_g = g; best_x = true; }
            }
            c->xseg = false;
            c->Gs = g_keep;
        }
    }
    // the chunk product, when the matrix has a chunk layout: 1536 or 2048 workgroups, or as many as
    // the kernel's occupancy keeps resident
    if (c->nqc > 0 && (c->prm.spmv_lanes == 0 || c->prm.spmv_lanes == 1) && c->prm.segments <= 1) {
        c->xseg = false;
        const int g_keep = c->Gs;
        const int cand[3] = {1536, 2048, chunk_resident_grid<T>(c)};
        for (int i = 0; i < 3; ++i) {
            const int g = cand[i];
            if (c->prm.spmv_grid > 0 && g != 1536) continue;   // a forced grid is applied afterwards
            if (i == 2 && (g == 1536 || g == 2048 || g < 8)) continue;   // the resident grid, if another
            c->Gs = g;
            float ms = 0.f;
            HIP_TRY(time_lanes(1, ms));
            if (better(ms)) { best = ms; best_l = 1; best_s = 1; best_g = g; }
        }
        c->Gs = g_keep;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (c->nseg != best_s) {
        scg_status st = build_segments<T>(c, best_s, row_ptr, col, val);
        if (st != SCG_OK) return st;
    }
    c->xseg = best_x;
    if (best_l == 1 || best_x) c->Gs = best_g;
    else if (best_g != 0) c->Gs = std::min(c->Gs, best_g);
    c->lanes = best_l;
    return SCG_OK;
}

template <typename T>
scg_status init_typed(scg_ctx* c, const int64_t* row_ptr, const int32_t* col, const double* val, const double* b,
                      const double* omega) {
    const int64_t n = c->n;
    std::vector<int64_t> hrp(n + 1);
    HIP_TRY(hipMemcpyAsync(hrp.data(), row_ptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (hrp[0] != 0 || hrp[n] != c->nnz_in) return SCG_EINVAL;
    for (int64_t r = 0; r < n; ++r)
        if (hrp[r + 1] < hrp[r]) return SCG_EINVAL;
    int32_t* cnt = c->rb;   // n ints of scratch before the partition is written
    double* dCraw = c->z;   // scratch before the state is zeroed
    HIP_TRY(hipMemsetAsync(c->sc, 0, sizeof(DevScalars), c->stream));
    HIP_TRY(hipMemsetAsync(c->counter, 0, 256, c->stream));
    double* mm = c->part + (size_t)kGMax * 2;
    hipLaunchKernelGGL(k_validate, dim3(c->G), dim3(kBlock), 0, c->stream, n, row_ptr, col, val, b, cnt, dCraw,
                       c->sc, c->part, c->counter, mm);
    HIP_TRY(hipGetLastError());
    std::vector<int32_t> hcnt(n);
    HIP_TRY(hipMemcpyAsync(hcnt.data(), cnt, sizeof(int32_t) * n, hipMemcpyDeviceToHost, c->stream));
    std::vector<double> hmm((size_t)c->G * 4);
    HIP_TRY(hipMemcpyAsync(hmm.data(), mm, sizeof(double) * 4 * c->G, hipMemcpyDeviceToHost, c->stream));
    DevScalars hsc;
    HIP_TRY(hipMemcpyAsync(&hsc, c->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (hsc.err != 0) return SCG_EINVAL;
    const double alpha = (c->prm.alpha > 0.0) ? c->prm.alpha : hsc.sum_b;
    if (!(alpha > 0.0) || !std::isfinite(alpha)) return SCG_EINVAL;
    c->alpha_orig = alpha;
    double cF = std::sqrt(hsc.sum_sq);
    if (!(cF > 0.0)) cF = 1.0;
    c->c_F = c->prm.scale ? cF : 1.0;
    c->alpha_s = c->prm.scale ? 1.0 : alpha;
    // storage format of the off-diagonal values
    double vmin = INFINITY, vmax = -INFINITY, amin = INFINITY, amax = -INFINITY;
    for (int g = 0; g < c->G; ++g) {
        vmin = std::min(vmin, hmm[4 * g + 0]);
        vmax = std::max(vmax, -hmm[4 * g + 1]);
        amin = std::min(amin, hmm[4 * g + 2]);
        amax = std::max(amax, -hmm[4 * g + 3]);
    }
    c->fmt = FMT_VAL;
    c->cval = 1.0;
    if (c->prm.matrix_format != 1 && std::isfinite(vmin)) {   // some off-diagonal entry exists
        if (vmin == vmax) {
            c->fmt = FMT_PAT;
            c->cval = vmin / c->c_F;
        } else if (amin == amax && amin > 0.0) {
            c->fmt = FMT_SGN;
            c->cval = amin / c->c_F;
        }
    }
    std::vector<int32_t> hrp_off(n + 1);
    int64_t acc = 0;
    for (int64_t r = 0; r < n; ++r) {
        hrp_off[r] = (int32_t)acc;
        acc += hcnt[r];
        if (acc > INT32_MAX) return SCG_EINVAL;
    }
    hrp_off[n] = (int32_t)acc;
    c->nnz_off = acc;
    std::vector<int2> hrbd = block_descriptors(hrp_off, n);
    c->nrb = (int)hrbd.size() - 1;
    c->Gs = std::min(kGMax, std::max(8, round8((c->nrb + kWaves - 1) / kWaves)));
    c->nseg = 1;
    c->seglen = n;
    c->rp_seg[0] = c->rp;
    c->rbd_seg[0] = reinterpret_cast<int2*>(c->rb);
    c->nrb_seg[0] = c->nrb;
    c->lanes = pick_lanes(n > 0 ? (double)acc / (double)n : 1.0);
    HIP_TRY(hipMemcpyAsync(c->rp, hrp_off.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->rb, hrbd.data(), sizeof(int2) * hrbd.size(), hipMemcpyHostToDevice, c->stream));
    const double inv_cF = 1.0 / c->c_F;
    const double inv_alpha = c->prm.scale ? 1.0 / alpha : 1.0;
    hipLaunchKernelGGL((k_scatter<T>), dim3(c->G), dim3(kBlock), 0, c->stream, n, row_ptr, col, val, b, c->rp,
                       c->col, (T*)c->val, dCraw, c->dC, c->b, inv_cF, inv_alpha, c->fmt);
    HIP_TRY(hipGetLastError());
    {
        scg_status st = (c->fmt == FMT_VAL) ? build_entry_chunks<T>(c, row_ptr, col, val, hcnt)
                                            : build_quad_chunks<T>(c, row_ptr, col, val, hcnt);
        if (st != SCG_OK) return st;
    }
    if (c->lo) {   // K = {b} until sketchycgal_set_constraints
        HIP_TRY(hipMemcpyAsync(c->lo, c->b, 8 * n, hipMemcpyDeviceToDevice, c->stream));
        HIP_TRY(hipMemcpyAsync(c->hi, c->b, 8 * n, hipMemcpyDeviceToDevice, c->stream));
    }
    if (c->prm.omega_mode == 1) {
        // Omega is generated from Philox wherever it is used
    } else if (omega) {
        transpose_cast<double, T>(c, omega, (T*)c->Om, 1);
    } else {
        const int64_t total = (n + 3) / 4 * c->prm.R;
        const int g = (int)std::min<int64_t>(8192, std::max<int64_t>(1, (total + kBlock - 1) / kBlock));
        hipLaunchKernelGGL((k_omega<T>), dim3(g), dim3(kBlock), 0, c->stream, n, c->ld, c->prm.R, c->prm.seed,
                           (uint64_t)c->prm.instance, (T*)c->Om);
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(c->stream));   // dCraw (in z) is consumed before z is zeroed
    HIP_TRY(hipMemsetAsync(c->z, 0, 8 * n, c->stream));
    HIP_TRY(hipMemsetAsync(c->y, 0, 8 * n, c->stream));
    HIP_TRY(hipMemsetAsync(c->S, 0, elem_size(c->prm) * c->ld * c->prm.R, c->stream));
    HIP_TRY(hipMemsetAsync(c->sc, 0, sizeof(DevScalars), c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (c->prm.autotune && (c->nnz_off >= (1 << 20) || c->prm.segments > 0)) {
        scg_status st = autotune_spmv<T>(c, row_ptr, col, val);
        if (st != SCG_OK) return st;
        HIP_TRY(hipMemsetAsync(c->sc, 0, sizeof(DevScalars), c->stream));
    } else if (c->prm.segments > 1) {
        scg_status st = build_segments<T>(c, c->prm.segments, row_ptr, col, val);
        if (st != SCG_OK) return st;
        if (c->prm.segments == kSegMax) {   // the concurrent form
            c->xseg = true;
            c->Gs = kGMax;
            if (c->prm.spmv_lanes == 1) {   // over entry chunks
                st = build_xchunks<T>(c);
                if (st != SCG_OK) return st;
            }
        }
    }
    // forced SpMV shape (overrides the autotuner); the quad-chunk product needs its layout
    if (c->prm.spmv_lanes == 1 && (c->xseg ? c->nxc == 0 : c->nqc == 0)) return SCG_EINVAL;
    if (c->prm.spmv_lanes > 0) c->lanes = c->prm.spmv_lanes;
    if (c->prm.spmv_grid > 0) c->Gs = std::min(c->Gs, std::max(8, round8(c->prm.spmv_grid)));
    HIP_TRY(hipMemsetAsync(c->logs, 0, sizeof(scg_iter_log) * c->prm.T, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->t_next = 1;
    return SCG_OK;
}

// The captured iteration for Lanczos step count q (instantiated on first use).
template <typename T>
hipError_t graph_for(scg_ctx* c, int t, int q, hipGraphExec_t* out) {
    auto f = c->graphs.find(q);
    if (f != c->graphs.end()) {
        *out = f->second;
        return hipSuccess;
    }
    hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    enqueue_iteration<T>(c, t, 1);
    hipLaunchKernelGGL(k_advance_t, dim3(1), dim3(1), 0, c->stream, c->sc);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(c->stream, &g);
    if (e != hipSuccess) return e;
    hipGraphExec_t ge = nullptr;
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return e;
    c->graphs[q] = ge;
    *out = ge;
    return hipSuccess;
}

// Runs of iterations with the same q_t replay one captured iteration, after a
// one-thread kernel has set the device counter to the run's first t.
template <typename T>
scg_status step_graphs(scg_ctx* c, int32_t iters) {
    int k = 0;
    while (k < iters) {
        const int t = c->t_next;
        const int q = q_for(c->prm, c->n, t);
        int m = 1;
        while (k + m < iters && q_for(c->prm, c->n, t + m) == q) ++m;
        hipGraphExec_t ge = nullptr;
        HIP_TRY(graph_for<T>(c, t, q, &ge));
        hipLaunchKernelGGL(k_set_t, dim3(1), dim3(1), 0, c->stream, c->sc, t);
        HIP_TRY(hipGetLastError());
        for (int j = 0; j < m; ++j) HIP_TRY(hipGraphLaunch(ge, c->stream));
        c->t_next += m;
        k += m;
    }
    return SCG_OK;
}

bool params_ok(const scg_params* p, int64_t n, int64_t nnz) {
    if (!p || n < 1 || nnz < 0 || n >= INT32_MAX) return false;
    if (p->R < 1 || p->R > kRMax || p->R > n) return false;
    if (p->T < 1) return false;
    if (!(p->beta0 > 0.0) || !(p->K >= 0.0)) return false;
    if (p->q_mode != 0 && p->q_mode != 1) return false;
    if (p->q_mode == 1 && p->q_fixed < 1) return false;
    if (p->reorth < 0 || p->reorth > 2) return false;
    if (p->precision != SCG_FP64 && p->precision != SCG_FP32_STREAM) return false;
    if (qmax_for(*p, n) + 1 > kQCap) return false;
    const int l = p->spmv_lanes;
    if (l != 0 && l != 1 && l != 2 && l != 4 && l != 8 && l != 16 && l != 32) return false;
    if (l == 1 && p->segments > 1 && p->segments != kSegMax) return false;   // the chunk products
    if (p->segments != 0 && p->segments != 1 && p->segments != 2 && p->segments != 4 && p->segments != kSegMax)
        return false;
    if (p->spmv_grid < 0 || p->spmv_grid > kGMax) return false;
    if (p->basis_mode != 0 && p->basis_mode != 1) return false;
    if (p->basis_mode == 1 && p->reorth == 2) return false;   // full reorthogonalisation needs the stored basis
    if (p->omega_mode != 0 && p->omega_mode != 1) return false;
    if (p->trace_mode != 0 && p->trace_mode != 1) return false;
    if (p->constraint_set < 0 || p->constraint_set > 2) return false;
    if (p->batch_kernel != 0) return false;   // a batched-engine parameter
    return true;
}

}  // namespace

extern "C" {

void scg_default_params(scg_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->R = 10;
    p->T = 100;
    p->beta0 = 1.0;
    p->K = INFINITY;
    p->alpha = 0.0;
    p->seed = 0;
    p->q_mode = 0;
    p->q_fixed = 0;
    p->scale = 1;
    p->trace_correct = 1;
    p->reorth = 0;
    p->precision = SCG_FP64;
    p->instance = 0;
    p->matrix_format = 0;
    p->autotune = 1;
    p->segments = 0;
    p->spmv_lanes = 0;
    p->spmv_grid = 0;
    p->basis_mode = 0;
    p->omega_mode = 0;
    p->trace_mode = 0;
    p->constraint_set = 0;
}

scg_status scg_workspace_size(const scg_params* p, int64_t n, int64_t nnz, size_t* bytes) {
    if (!bytes || !params_ok(p, n, nnz)) return SCG_EINVAL;
    *bytes = make_layout(*p, n, nnz).total;
    return SCG_OK;
}

scg_status sketchycgal_init(scg_ctx** out, const scg_params* p, int64_t n, int64_t nnz, const int64_t* row_ptr,
                            const int32_t* col, const double* val, const double* b, const double* omega,
                            void* workspace, size_t ws_bytes, void* stream) {
    if (!out) return SCG_EINVAL;
    *out = nullptr;
    if (!params_ok(p, n, nnz) || !row_ptr || !b || !workspace) return SCG_EINVAL;
    if (nnz > 0 && (!col || !val)) return SCG_EINVAL;
    if (((uintptr_t)workspace & 255) != 0) return SCG_EINVAL;
    if (omega && p->omega_mode == 1) return SCG_EINVAL;   // a generated Omega is the Philox one
    const Layout L = make_layout(*p, n, nnz);
    if (ws_bytes < L.total) return SCG_ENOMEM;
    scg_ctx* c = new (std::nothrow) scg_ctx();
    if (!c) return SCG_ENOMEM;
    c->prm = *p;
    c->n = n;
    c->nnz_in = nnz;
    c->stream = (hipStream_t)stream;
    if (hipGetDevice(&c->device) != hipSuccess) { delete c; return SCG_EHIP; }
    c->qmax = qmax_for(*p, n);
    c->ld = (n + 63) / 64 * 64;
    c->G = std::min(kGMax, std::max(8, round8((n + 1023) / 1024)));
    char* base = (char*)workspace;
    c->rp = (int32_t*)(base + L.rp);
    c->col = (int32_t*)(base + L.col);
    c->val = base + L.val;
    c->dC = (double*)(base + L.dC);
    c->b = (double*)(base + L.b);
    c->z = (double*)(base + L.z);
    c->y = (double*)(base + L.y);
    c->s = base + L.s;
    c->V = base + L.V;
    c->u = base + L.u;
    c->v = base + L.v;
    c->Om = base + L.Om;
    c->racc = (p->basis_mode == 1) ? (double*)(base + L.racc) : nullptr;
    c->lo = (p->constraint_set == 1) ? (double*)(base + L.lo) : nullptr;
    c->hi = (p->constraint_set == 1) ? (double*)(base + L.hi) : nullptr;
    c->S = base + L.S;
    c->rb = (int32_t*)(base + L.rb);
    c->rb_cap = (size_t)seg_cap(*p, n, nnz) * (n + 2);
    c->xpart = (seg_cap(*p, n, nnz) > 1) ? (void*)(base + L.xp) : nullptr;
    c->xseg = false;
    c->sc = (DevScalars*)(base + L.sc);
    c->part = (double*)(base + L.part);
    c->counter = (unsigned*)(base + L.counter);
    c->logs = (scg_iter_log*)(base + L.logs);
    c->recon = (double*)(base + L.recon);
    c->recon_bytes = L.recon_bytes;
    const int64_t nec = entry_chunk_cap(*p, n, nnz);
    c->qc_cap = std::max(quad_chunk_cap(*p, n, nnz), nec);
    c->qw = (c->qc_cap > 0) ? (int32_t*)(base + L.qw) : nullptr;
    c->qv = (nec > 0) ? (void*)(base + L.qv) : nullptr;
    c->qc = (c->qc_cap > 0) ? (int2*)(base + L.qc) : nullptr;
    c->nqc = 0;
    c->xqc_cap = xchunk_cap(*p, n, nnz);
    c->xqw = (c->xqc_cap > 0) ? (int32_t*)(base + L.xqw) : nullptr;
    c->xqv = (c->xqc_cap > 0) ? (void*)(base + L.xqv) : nullptr;
    c->xqc = (c->xqc_cap > 0) ? (int2*)(base + L.xqc) : nullptr;
    c->xlseg = (c->xqc_cap > 0) ? (int4*)(base + L.xlseg) : nullptr;
    c->xlseg_cap = (c->xqc_cap > 0) ? nnz / (kERowMax + 1) + kSegMax : 0;
    c->xlw = (c->xqc_cap > 0) ? (int32_t*)(base + L.xlw) : nullptr;
    c->xlv = (c->xqc_cap > 0) ? (void*)(base + L.xlv) : nullptr;
    c->nxc = 0;
    for (int s = 0; s <= kSegMax; ++s) c->xcb[s] = c->xlb[s] = 0;
    scg_status st = (p->precision == SCG_FP32_STREAM) ? init_typed<float>(c, row_ptr, col, val, b, omega)
                                                       : init_typed<double>(c, row_ptr, col, val, b, omega);
    if (st != SCG_OK) {
        (void)hipStreamSynchronize(c->stream);
        delete c;
        return st;
    }
    *out = c;
    return SCG_OK;
}

scg_status sketchycgal_step(scg_ctx* c, int32_t iters) {
    if (!c || iters < 0) return SCG_EINVAL;
    if ((int64_t)c->t_next - 1 + iters > c->prm.T) return SCG_ESTATE;
    // on a non-null stream whole iterations are replayed from captured graphs
    // (not with the ball constraint set, whose norm passes take beta by value)
    if (c->stream != nullptr && c->prm.constraint_set != 2 && iters > 0) {
        return (c->prm.precision == SCG_FP32_STREAM) ? step_graphs<float>(c, iters) : step_graphs<double>(c, iters);
    }
    for (int k = 0; k < iters; ++k) {
        if (c->prm.precision == SCG_FP32_STREAM) enqueue_iteration<float>(c, c->t_next);
        else enqueue_iteration<double>(c, c->t_next);
        c->t_next++;
    }
    HIP_TRY(hipGetLastError());
    return SCG_OK;
}

scg_status sketchycgal_set_constraints(scg_ctx* c, const double* lo, const double* hi) {
    if (!c || c->prm.constraint_set != 1 || !c->lo) return SCG_EINVAL;
    if (c->t_next != 1) return SCG_ESTATE;
    const int64_t n = c->n;
    const double inv_alpha = c->prm.scale ? 1.0 / c->alpha_orig : 1.0;   // as b (k_scatter)
    const int g = (int)std::min<int64_t>(4096, std::max<int64_t>(1, (n + kBlock - 1) / kBlock));
    HIP_TRY(hipMemsetAsync(&c->sc->err, 0, sizeof(int32_t), c->stream));
    hipLaunchKernelGGL(k_set_box, dim3(g), dim3(kBlock), 0, c->stream, n, lo, hi, inv_alpha, c->lo, c->hi, c->sc);
    HIP_TRY(hipGetLastError());
    int32_t err = 0;
    HIP_TRY(hipMemcpyAsync(&err, &c->sc->err, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (err != 0) {   // back to K = {b}
        HIP_TRY(hipMemcpyAsync(c->lo, c->b, 8 * n, hipMemcpyDeviceToDevice, c->stream));
        HIP_TRY(hipMemcpyAsync(c->hi, c->b, 8 * n, hipMemcpyDeviceToDevice, c->stream));
        HIP_TRY(hipMemsetAsync(&c->sc->err, 0, sizeof(int32_t), c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        return SCG_EINVAL;
    }
    return SCG_OK;
}

scg_status sketchycgal_set_ball(scg_ctx* c, double radius) {
    if (!c || c->prm.constraint_set != 2 || !(radius >= 0.0) || !std::isfinite(radius)) return SCG_EINVAL;
    if (c->t_next != 1) return SCG_ESTATE;
    c->ball_r = radius * (c->prm.scale ? 1.0 / c->alpha_orig : 1.0);   // scaled like b (k_scatter)
    return SCG_OK;
}

scg_status sketchycgal_log(scg_ctx* c, scg_iter_log* host_out, int32_t max, int32_t* count) {
    if (!c || !host_out || !count || max < 0) return SCG_EINVAL;
    const int done = c->t_next - 1;
    const int m = std::min(done, (int)max);
    if (m > 0) HIP_TRY(hipMemcpyAsync(host_out, c->logs, sizeof(scg_iter_log) * m, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    *count = m;
    return SCG_OK;
}

scg_status sketchycgal_summary(scg_ctx* c, scg_summary* o) {
    if (!c || !o) return SCG_EINVAL;
    DevScalars hsc;
    HIP_TRY(hipMemcpyAsync(&hsc, c->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    // ||z - b|| after the last update: recomputed from the log of the last iteration
    double infeas_s = 0.0;
    const int done = c->t_next - 1;
    if (done > 0) {
        scg_iter_log L;
        HIP_TRY(hipMemcpy(&L, c->logs + (done - 1), sizeof(L), hipMemcpyDeviceToHost));
        infeas_s = L.infeas;
    }
    o->t_done = done;
    o->status_flags = (hsc.flags & 2) ? 1 : 0;
    o->p_scaled = hsc.p;
    o->tau_scaled = hsc.tau;
    o->c_F = c->c_F;
    o->alpha = c->alpha_orig;
    o->alpha_scaled = c->alpha_s;
    o->objective = c->c_F * c->alpha_orig * hsc.p / c->alpha_s;
    o->infeasibility = c->alpha_orig / c->alpha_s * infeas_s;
    o->spmv_lanes = c->lanes;
    o->spmv_segments = c->nseg;
    o->matrix_format = c->fmt;
    o->spmv_grid = c->Gs;
    return (hsc.flags & 2) ? SCG_ENUMERIC : SCG_OK;
}

scg_status sketchycgal_get_state(scg_ctx* c, int32_t* t_next, double* z, double* y, double* S, double* p,
                                 double* tau) {
    if (!c) return SCG_EINVAL;
    const int64_t n = c->n;
    if (z) HIP_TRY(hipMemcpyAsync(z, c->z, 8 * n, hipMemcpyDeviceToDevice, c->stream));
    if (y) HIP_TRY(hipMemcpyAsync(y, c->y, 8 * n, hipMemcpyDeviceToDevice, c->stream));
    if (S) {
        if (c->prm.precision == SCG_FP32_STREAM) transpose_cast<float, double>(c, (const float*)c->S, S, 0);
        else transpose_cast<double, double>(c, (const double*)c->S, S, 0);
    }
    DevScalars hsc;
    HIP_TRY(hipMemcpyAsync(&hsc, c->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (t_next) *t_next = c->t_next;
    if (p) *p = hsc.p;
    if (tau) *tau = hsc.tau;
    return SCG_OK;
}

scg_status sketchycgal_set_state(scg_ctx* c, int32_t t_next, const double* z, const double* y, const double* S,
                                 double p, double tau) {
    if (!c || t_next < 1 || t_next > c->prm.T + 1 || !z || !y || !S) return SCG_EINVAL;
    const int64_t n = c->n;
    HIP_TRY(hipMemcpyAsync(c->z, z, 8 * n, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->y, y, 8 * n, hipMemcpyDeviceToDevice, c->stream));
    if (c->prm.precision == SCG_FP32_STREAM) transpose_cast<double, float>(c, S, (float*)c->S, 1);
    else transpose_cast<double, double>(c, S, (double*)c->S, 1);
    DevScalars hsc;
    HIP_TRY(hipMemcpyAsync(&hsc, c->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    hsc.p = p;
    hsc.tau = tau;
    HIP_TRY(hipMemcpyAsync(c->sc, &hsc, sizeof(DevScalars), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->t_next = t_next;
    return SCG_OK;
}

scg_status sketchycgal_lanczos_coeffs(scg_ctx* c, double* omega, double* rho, int32_t cap, int32_t* k, double* xi) {
    if (!c || !k) return SCG_EINVAL;
    DevScalars hsc;
    HIP_TRY(hipMemcpyAsync(&hsc, c->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    *k = hsc.k;
    if (xi) *xi = hsc.xi;
    for (int i = 0; i < std::min<int>(hsc.k, cap); ++i) {
        if (omega) omega[i] = hsc.omega[i];
        if (rho && i < hsc.k - 1) rho[i] = hsc.rho[i];
    }
    return SCG_OK;
}

scg_status sketchycgal_apply(scg_ctx* c, const double* x, double* y) {
    if (!c || !x || !y) return SCG_EINVAL;
    if (c->t_next > c->prm.T) return SCG_ESTATE;
    const IterArgs it = iter_args(c, c->t_next);
    const int64_t n = c->n;
    if (c->prm.precision == SCG_FP32_STREAM) {
        enqueue_prep<float>(c, it);
        float* xs = (float*)c->V + c->ld;
        cast<double, float>(c, n, x, xs);
        launch_spmv<float, SPMV_APPLY>(c, xs, 0);
        cast<float, double>(c, n, (const float*)c->u, y);
    } else {
        enqueue_prep<double>(c, it);
        launch_spmv<double, SPMV_APPLY>(c, x, 0);
        HIP_TRY(hipMemcpyAsync(y, c->u, 8 * n, hipMemcpyDeviceToDevice, c->stream));
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(c->stream));
    return SCG_OK;
}

scg_status sketchycgal_time_spmv(scg_ctx* c, int32_t reps, double* avg_ms) {
    if (!c || reps < 1 || !avg_ms) return SCG_EINVAL;
    const IterArgs it = iter_args(c, std::min(c->t_next, c->prm.T));
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    if (c->prm.precision == SCG_FP32_STREAM) time_spmv_setup<float>(c, it);
    else time_spmv_setup<double>(c, it);
    HIP_TRY(hipEventRecord(e0, c->stream));
    for (int r = 0; r < reps; ++r) {
        if (c->prm.precision == SCG_FP32_STREAM) launch_spmv<float, SPMV_LANCZOS>(c, basis_col<float>(c, 1), 1);
        else launch_spmv<double, SPMV_LANCZOS>(c, basis_col<double>(c, 1), 1);
    }
    HIP_TRY(hipEventRecord(e1, c->stream));
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *avg_ms = (double)ms / reps;
    return SCG_OK;
}

scg_status sketchycgal_reconstruct(scg_ctx* c, double* U, double* lambda, double* err) {
    if (!c || !U || !lambda) return SCG_EINVAL;
    return scg_reconstruct_impl(c, U, lambda, err);
}

void sketchycgal_destroy(scg_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    delete c;
}

const char* scg_status_string(scg_status s) {
    switch (s) {
        case SCG_OK: return "ok";
        case SCG_EINVAL: return "invalid argument";
        case SCG_ENOMEM: return "workspace too small";
        case SCG_EHIP: return "HIP runtime error";
        case SCG_ENUMERIC: return "numerical failure (NaN/Inf or Cholesky)";
        case SCG_ESTATE: return "invalid state";
    }
    return "unknown status";
}

}  // extern "C"
