// SketchyCGAL for the phase retrieval SDP (Section 7.3, eqn
// numerics-phase-retrieval-sdp) on coded diffraction measurements
// (Appendix F.1): minimise tr X over complex Hermitian psd X with A X = b and
// tr X <= alpha, (A X)_{j,l} = a_{j,l}^* X a_{j,l}, a_{j,l}^* x the l-th entry
// of DFT_n(conj(psi_j) x).  The loop is alg:sketchy-cgal with the
// trace-bounded set of Appendix D.2 (H = alpha v v^* when xi < 0, else 0), in
// complex FP64 arithmetic.
//
// Operator.  D_t = C + A^*(w) applied to v is
//     v / sqrt(n) + sum_j psi_j * DFT_n^* (c_j * DFT_n (conj(psi_j) * v)),
// c_j = s_j w_j (s_j the per-waveform scaling).  Each length-n DFT is split
// four-step, n = n1 n2 (m = n2 m1 + m2, k = k1 + n1 k2):
//   column pass   Y[k1, m2] = w_n^{k1 m2} DFT_n1(x[n2 m1 + m2])[k1]
//   row pass      X[k1 + n1 k2] = DFT_n2(Y[k1, .])[k2]
// Every measurement-indexed vector (b, z, y, c) is stored in the row pass's
// output order, position k1 n2 + k2, so the forward row DFT, the product
// with c_j and the inverse row DFT run in one kernel on one LDS row, and the
// inverse column pass sums the waveforms.  Three launches per product:
//   k_pr_colfwd  (n2 / tc tiles) x L     load, modulate, column DFT, twiddle
//   k_pr_row     (n1 / rw rows) x L      row DFT, x c_j, inverse row DFT, twiddle
//   k_pr_colinv  (n2 / tc tiles) x G     inverse column DFT, x psi_j, sum over
//                                        the group's waveforms, + v / sqrt(n),
//                                        partial v^* D v
// The DFTs are mixed-radix Stockham passes (radices 8, 4, 2, 5, 3) on a tile
// of at most 4096 complex values in LDS (one padding value after every eight,
// so no pass has bank conflicts), each pass staging its butterflies in
// registers between two barriers (so one buffer suffices), with the stage
// twiddles from a 128-value two-level table in LDS.  The forward passes run
// 512 threads per workgroup (two workgroups per CU), the inverse column pass
// 1024 (its per-thread sums in registers).  Waveforms that take at most 256
// values are stored as one-byte codes, tile by tile, into a dictionary staged
// in LDS.  The forward column pass is one-dimensional and XCD-mapped: all L
// waveforms of a column tile run in a row on one XCD, which keeps that tile of
// the vector in its L2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <map>
#include <vector>

#include "../../include/sketchycgal.h"
#include "scg_device.hpp"
#include "scg_tridiag.hpp"

using namespace scg;

namespace {

constexpr int kFT = 512;              // threads of the DFT kernels (8 wave64)
constexpr int kTile = 4096;           // complex values per LDS tile (64 KiB)
constexpr int kTileP = kTile + kTile / 8;   // the tile with one padding value after every eight
constexpr int kFI = 1024;             // threads of the inverse column pass (its sums stay in registers)
constexpr int kMaxStages = 16;
constexpr int kPQCap = 512;           // Lanczos steps per iteration at most
constexpr int kPRMax = 16;            // sketch size at most
constexpr int kPLMax = 32;            // waveforms at most
constexpr int kTwShift = 12;          // n-point twiddle = high table x low table (4096 entries)
constexpr int kGU = 1024;             // workgroups of the streaming passes (at most)

struct Fft {
    int N, ns;
    int rad[kMaxStages];
    const double2* tw;                // [0, 64): exp(-2 pi i 64 h / N); [64, 128): exp(-2 pi i l / N)
};

// The DFT passes read exp(-2 pi i t / N) as the product of two entries of a
// 128-value table staged in LDS (high part t >> 6, low part t & 63).
constexpr int kTwLds = 128;

__device__ __forceinline__ void load_tw(double2* tws, const Fft& F, int nt) {
    for (int i = threadIdx.x; i < kTwLds; i += nt) tws[i] = F.tw[i];
}

struct PrScalars {
    double omega[kPQCap];
    double nrm[kPQCap + 1];          // nrm[i] = ||V[i]||: V[i] / nrm[i] is the Lanczos vector v_i
    double coef[kPQCap];             // eigenvector of T_k
    double dots[2 * kPRMax];         // v^* Omega of the normalised Ritz vector
    double xi, ha, xnorm, p, tau, gamma, one;
    int k, broken, flags, t_iter;    // t_iter: the iteration counter read by a replayed graph
};

struct PrArgs {
    int64_t n;
    int L, R, n1, n2, tc, ltc, rw, lrw, G, mpg, ntc, nrw;
    Fft f1, f2;
    const double2* twh;
    const double2* twl;
    const double2* psi;       // L x n (when the waveforms are stored whole)
    const uint8_t* psic;      // L x n dictionary codes (when they take at most 256 values)
    const double2* dict;      // the dictionary
    int coded, ndict;
    const double* s;          // L
    const double* b;          // L x n, row-pass order
    double* z;
    double* y;
    double* c;
    double2* Y;               // L x n intermediate
    double2* P;               // G x n group sums
    double2* V;               // Lanczos basis, (qcap + 1) x n
    double2* xr;              // Ritz vector
    const double2* Om;        // R x n
    double2* S;               // R x n
    double* p_col;            // G * ntc partials of v^* P_g
    double* p_upd;            // kGU partials
    double* p_meas;           // L * nrw * 3 partials
    double* p_prep;           // kGU partials
    double* p_sk;             // kGU * 2R partials
    PrScalars* sc;
    scg_iter_log* log;
    double c_scale, alpha_s, beta0, K;
};

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {
    return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscl(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// x times -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ double2 mi(double2 x) {
    return INV ? make_double2(-x.y, x.x) : make_double2(x.y, -x.x);
}

// Iteration t of a launch: the argument, or (t = 0, a replayed graph) the device counter; beta_t and
// eta_t from it as the host computes them.
__device__ __forceinline__ int pr_t(const PrArgs& A, int t) { return t > 0 ? t : A.sc->t_iter; }
__device__ __forceinline__ double pr_beta(const PrArgs& A, int t) { return A.beta0 * sqrt(t + 1.0); }
__device__ __forceinline__ double pr_eta(int t) { return 2.0 / (t + 1.0); }

__global__ void k_pr_set_t(PrScalars* sc, int t) { sc->t_iter = t; }
__global__ void k_pr_advance_t(PrScalars* sc) { sc->t_iter += 1; }

// LDS position of tile value i: one padding value after every eight, so that
// the eight lanes a 16-byte LDS access serves per cycle fall into distinct
// bank groups also when a pass stores its outputs R or Ns values apart.
__device__ __forceinline__ int pad(int i) { return i + (i >> 3); }

// psi_j(m) for tile value idx of column tile `tile`: from the dictionary codes, stored tile by tile
// (codes of waveform j, tile t, value idx = m1 tc + c at j * ntc * n1 * tc + t * n1 * tc + idx, so a
// tile reads whole cache lines; dl: the dictionary staged in LDS), or the stored waveform at j n + m.
__device__ __forceinline__ double2 psi_at(const PrArgs& A, const double2* dl, int j, int tile, int idx, int64_t m) {
    return A.coded ? dl[A.psic[((size_t)j * A.ntc + tile) * ((size_t)A.n1 << A.ltc) + idx]]
                   : A.psi[(size_t)j * A.n + m];
}

__device__ __forceinline__ void load_dict(double2* dl, const PrArgs& A, int nt) {
    if (A.coded)
        for (int i = threadIdx.x; i < A.ndict; i += nt) dl[i] = A.dict[i];
}

// Sum over an NT-thread workgroup (fixed order); red holds NT / 64 doubles.
template <int NT = kFT>
__device__ __forceinline__ double ft_sum(double v, double* red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) s += red[i];
    return s;
}

// exp(-+2 pi i t / n) from the two-level table.
__device__ __forceinline__ double2 twn(const PrArgs& A, int64_t t) {
    return cmul(A.twh[t >> kTwShift], A.twl[t & ((1 << kTwShift) - 1)]);
}

// ------------------------------------------------------------------ radix-R DFTs
// y_p = sum_m x_m exp(-+2 pi i p m / R), written from the factorisations of
// the small DFT matrices (radix 4 = two radix-2 stages, radix 8 = radix 2 on
// two radix-4 halves, radices 3 and 5 from the real and imaginary parts of the
// roots of unity).
template <int R, bool INV>
struct Radix;

template <bool INV>
struct Radix<2, INV> {
    __device__ static void run(double2 (&a)[2]) {
        const double2 t = a[0];
        a[0] = cadd(t, a[1]);
        a[1] = csub(t, a[1]);
    }
};

template <bool INV>
__device__ __forceinline__ void dft4(double2& a0, double2& a1, double2& a2, double2& a3) {
    const double2 s0 = cadd(a0, a2), d0 = csub(a0, a2), s1 = cadd(a1, a3), d1 = mi<INV>(csub(a1, a3));
    a0 = cadd(s0, s1);
    a2 = csub(s0, s1);
    a1 = cadd(d0, d1);
    a3 = csub(d0, d1);
}

template <bool INV>
struct Radix<4, INV> {
    __device__ static void run(double2 (&a)[4]) { dft4<INV>(a[0], a[1], a[2], a[3]); }
};

template <bool INV>
struct Radix<8, INV> {
    __device__ static void run(double2 (&a)[8]) {
        double2 e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
        double2 o0 = a[1], o1 = a[3], o2 = a[5], o3 = a[7];
        dft4<INV>(e0, e1, e2, e3);
        dft4<INV>(o0, o1, o2, o3);
        const double h = 0.70710678118654752440;
        // o_k times exp(-+2 pi i k / 8)
        o1 = INV ? make_double2(h * (o1.x - o1.y), h * (o1.x + o1.y)) : make_double2(h * (o1.x + o1.y), h * (o1.y - o1.x));
        o2 = mi<INV>(o2);
        o3 = INV ? make_double2(-h * (o3.x + o3.y), h * (o3.x - o3.y)) : make_double2(h * (o3.y - o3.x), -h * (o3.x + o3.y));
        a[0] = cadd(e0, o0);
        a[4] = csub(e0, o0);
        a[1] = cadd(e1, o1);
        a[5] = csub(e1, o1);
        a[2] = cadd(e2, o2);
        a[6] = csub(e2, o2);
        a[3] = cadd(e3, o3);
        a[7] = csub(e3, o3);
    }
};

template <bool INV>
struct Radix<3, INV> {
    __device__ static void run(double2 (&a)[3]) {
        const double s3 = 0.86602540378443864676;   // sin(2 pi / 3)
        const double2 t = cadd(a[1], a[2]);
        const double2 m = csub(a[0], cscl(t, 0.5));
        const double2 d = cscl(mi<INV>(csub(a[1], a[2])), s3);
        a[0] = cadd(a[0], t);
        a[1] = cadd(m, d);
        a[2] = csub(m, d);
    }
};

template <bool INV>
struct Radix<5, INV> {
    __device__ static void run(double2 (&a)[5]) {
        const double c1 = 0.30901699437494742410, c2 = -0.80901699437494742410;   // cos(2 pi / 5), cos(4 pi / 5)
        const double s1 = 0.95105651629515357212, s2 = 0.58778525229247312917;    // sin(2 pi / 5), sin(4 pi / 5)
        const double2 t1 = cadd(a[1], a[4]), t2 = cadd(a[2], a[3]);
        const double2 d1 = csub(a[1], a[4]), d2 = csub(a[2], a[3]);
        const double2 b1 = make_double2(a[0].x + c1 * t1.x + c2 * t2.x, a[0].y + c1 * t1.y + c2 * t2.y);
        const double2 b2 = make_double2(a[0].x + c2 * t1.x + c1 * t2.x, a[0].y + c2 * t1.y + c1 * t2.y);
        const double2 e1 = mi<INV>(make_double2(s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y));
        const double2 e2 = mi<INV>(make_double2(s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y));
        a[0] = cadd(a[0], cadd(t1, t2));
        a[1] = cadd(b1, e1);
        a[4] = csub(b1, e1);
        a[2] = cadd(b2, e2);
        a[3] = csub(b2, e2);
    }
};

// One Stockham pass of radix R over nseq = 2^lns interleaved sequences of
// length N held at buf[pad(e * nseq + s)]: butterfly j of sequence s takes the R
// values at j + r N / R, multiplies them by exp(-+2 pi i k r / (Ns R)) with
// k = j mod Ns (Ns the product of the earlier radices), transforms them and
// stores them at (j / Ns) Ns R + k + r Ns.  All butterflies of a thread are
// read before the barrier and written after it.
template <int R, bool INV, int NT>
__device__ __forceinline__ void fft_pass(double2* buf, int N, int lns, int Ns, const double2* tws) {
    // j / Ns as a multiply-high: floor(j m / 2^32) with m = floor(2^32 / Ns) + 1 (2^32 / Ns for a
    // power of two) equals floor(j / Ns) for every j, Ns <= 4096
    const uint32_t mag = (Ns > 1) ? 0xFFFFFFFFu / (uint32_t)Ns + 1u : 0u;
    constexpr int MB = (kTile / NT + R - 1) / R;
    const int nseq = 1 << lns;
    const int nb = N / R;
    const int total = nb << lns;
    const int tstride = N / (Ns * R);
    double2 v[MB][R];
    int ob[MB];
#pragma unroll
    for (int u = 0; u < MB; ++u) {
        const int bb = threadIdx.x + u * NT;
        if (bb < total) {
            const int s = bb & (nseq - 1), j = bb >> lns;
            const int jq = (Ns > 1) ? (int)__umulhi((uint32_t)j, mag) : j;
            const int k = j - jq * Ns;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                double2 x = buf[pad(((j + r * nb) << lns) + s)];
                if (r > 0) {
                    const int t = k * r * tstride;
                    double2 w = cmul(tws[t >> 6], tws[64 + (t & 63)]);
                    if (INV) w.y = -w.y;
                    x = cmul(x, w);
                }
                v[u][r] = x;
            }
            Radix<R, INV>::run(v[u]);
            ob[u] = ((jq * Ns * R + k) << lns) + s;
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < MB; ++u) {
        const int bb = threadIdx.x + u * NT;
        if (bb < total) {
#pragma unroll
            for (int r = 0; r < R; ++r) buf[pad(ob[u] + ((r * Ns) << lns))] = v[u][r];
        }
    }
    __syncthreads();
}

// In-place DFT (natural order in and out) of the nseq interleaved sequences.
// The caller has made the tile visible to the workgroup (barrier).
template <bool INV, int NT>
__device__ void fft_tile(double2* buf, const Fft& F, int lns, const double2* tws) {
    int Ns = 1;
    for (int st = 0; st < F.ns; ++st) {
        const int R = F.rad[st];
        if (R == 8) fft_pass<8, INV, NT>(buf, F.N, lns, Ns, tws);
        else if (R == 4) fft_pass<4, INV, NT>(buf, F.N, lns, Ns, tws);
        else if (R == 2) fft_pass<2, INV, NT>(buf, F.N, lns, Ns, tws);
        else if (R == 5) fft_pass<5, INV, NT>(buf, F.N, lns, Ns, tws);
        else fft_pass<3, INV, NT>(buf, F.N, lns, Ns, tws);
        Ns *= R;
    }
}

// ------------------------------------------------------------------ operator kernels
// Column pass of DFT_n(conj(psi_j) x) for x = src / *dv, tile of tc columns.
__global__ __launch_bounds__(kFT) void k_pr_colfwd(PrArgs A, const double2* __restrict__ src, const double* dv,
                                                  int lanczos) {
    __shared__ double2 buf[kTileP];
    __shared__ double2 tws[kTwLds];
    __shared__ double2 dl[256];
    if (lanczos && A.sc->broken) return;
    // one-dimensional grid of ntc * L work items (padded to a multiple of 8): XCD x takes a contiguous
    // range of them, all L waveforms of a column tile in a row, so the tile of x stays in its L2
    const int wi = xcd_lid();
    if (wi >= A.ntc * A.L) return;
    const int tile = wi / A.L, j = wi - tile * A.L;
    const int m20 = tile * A.tc;
    const double d = *dv;
    const int tot = A.n1 << A.ltc;
    load_tw(tws, A.f1, kFT);
    load_dict(dl, A, kFT);
    __syncthreads();
    for (int idx = threadIdx.x; idx < tot; idx += kFT) {
        const int m1 = idx >> A.ltc, m2 = m20 + (idx & (A.tc - 1));
        double2 val = make_double2(0.0, 0.0);
        if (m2 < A.n2) {
            const int64_t m = (int64_t)m1 * A.n2 + m2;
            double2 x = src[m];
            x.x /= d;
            x.y /= d;
            val = cmulc(x, psi_at(A, dl, j, tile, idx, m));
        }
        buf[pad(idx)] = val;
    }
    __syncthreads();
    fft_tile<false, kFT>(buf, A.f1, A.ltc, tws);
    double2* Yj = A.Y + (size_t)j * A.n;
    // this thread's outputs share m2 and step k1 by kFT / tc: w_n^{k1 m2} = w_n^{k1_0 m2} (w_n^{(kFT / tc) m2})^u
    const int m2 = m20 + (threadIdx.x & (A.tc - 1));
    const int k1_0 = threadIdx.x >> A.ltc;
    if (m2 < A.n2 && k1_0 < A.n1) {
        double2 w = twn(A, (int64_t)k1_0 * m2);
        const double2 ws = twn(A, ((int64_t)(kFT >> A.ltc) * m2) % A.n);
        for (int idx = threadIdx.x; idx < tot; idx += kFT) {
            Yj[(int64_t)(idx >> A.ltc) * A.n2 + m2] = cmul(buf[pad(idx)], w);
            w = cmul(w, ws);
        }
    }
}

// Row pass.  MODE 0: X = DFT_n2(row), X *= c_j, inverse DFT, conjugate twiddle,
// back in place (the input of the inverse column pass).  MODE 1: the measured
// values m = s_j |X|^2 update z <- (1 - eta) z + eta ha m, with partial sums of
// ||z - b||^2, <y, z - b>, ||y||^2.  MODE 2: m written to out in natural order.
template <int MODE>
__global__ __launch_bounds__(kFT) void k_pr_row(PrArgs A, int lanczos, int tt, double* out) {
    __shared__ double2 buf[kTileP];
    __shared__ double2 tws[kTwLds];
    __shared__ double red[kFT / 64];
    if (lanczos && A.sc->broken) return;
    const int j = blockIdx.y;
    const int k10 = blockIdx.x * A.rw;
    double2* Yj = A.Y + (size_t)j * A.n;
    load_tw(tws, A.f2, kFT);
    for (int r = 0; r < A.rw; ++r) {
        const int k1 = k10 + r;
        for (int e = threadIdx.x; e < A.n2; e += kFT)
            buf[pad((e << A.lrw) + r)] = (k1 < A.n1) ? Yj[(int64_t)k1 * A.n2 + e] : make_double2(0.0, 0.0);
    }
    // the dual weights of this thread's tile positions p = tid + kFT u (row p & (rw - 1), entry
    // p >> lrw), loaded before the forward transform so their latency overlaps it
    constexpr int kPT = kTile / kFT;
    double cw[kPT];
    if (MODE == 0) {
        const double* cj = A.c + (size_t)j * A.n;
#pragma unroll
        for (int u = 0; u < kPT; ++u) {
            const int p = threadIdx.x + u * kFT;
            const int k1 = k10 + (p & (A.rw - 1));
            cw[u] = (p < (A.n2 << A.lrw) && k1 < A.n1) ? cj[(int64_t)k1 * A.n2 + (p >> A.lrw)] : 0.0;
        }
    }
    __syncthreads();
    fft_tile<false, kFT>(buf, A.f2, A.lrw, tws);
    if (MODE == 0) {
#pragma unroll
        for (int u = 0; u < kPT; ++u) {
            const int p = threadIdx.x + u * kFT;
            if (p < (A.n2 << A.lrw)) buf[pad(p)] = cscl(buf[pad(p)], cw[u]);
        }
        __syncthreads();
        fft_tile<true, kFT>(buf, A.f2, A.lrw, tws);
        for (int r = 0; r < A.rw; ++r) {
            const int k1 = k10 + r;
            if (k1 >= A.n1 || (int)threadIdx.x >= A.n2) continue;
            // conj(w_n^{k1 e}) for e = tid + kFT u: the first one times conj(w_n^{k1 kFT})^u
            double2 w = twn(A, (int64_t)k1 * threadIdx.x);
            double2 ws = twn(A, ((int64_t)k1 * kFT) % A.n);
            w.y = -w.y;
            ws.y = -ws.y;
            for (int e = threadIdx.x; e < A.n2; e += kFT) {
                Yj[(int64_t)k1 * A.n2 + e] = cmul(buf[pad((e << A.lrw) + r)], w);
                w = cmul(w, ws);
            }
        }
    } else if (MODE == 1) {
        const double eta = pr_eta(pr_t(A, tt));
        const double sj = A.s[j];
        const double eh = eta * A.sc->ha;
        const double keep = 1.0 - eta;
        double a_r2 = 0.0, a_yzb = 0.0, a_yy = 0.0;
        for (int r = 0; r < A.rw; ++r) {
            const int k1 = k10 + r;
            if (k1 >= A.n1) continue;
            for (int e = threadIdx.x; e < A.n2; e += kFT) {
                const double2 X = buf[pad((e << A.lrw) + r)];
                const double m = sj * (X.x * X.x + X.y * X.y);
                const size_t pos = (size_t)j * A.n + (size_t)k1 * A.n2 + e;
                const double zn = keep * A.z[pos] + eh * m;
                A.z[pos] = zn;
                const double dd = zn - A.b[pos];
                const double yo = A.y[pos];
                a_r2 += dd * dd;
                a_yzb += yo * dd;
                a_yy += yo * yo;
            }
        }
        const int wg = blockIdx.y * gridDim.x + blockIdx.x;
        a_r2 = ft_sum(a_r2, red);
        a_yzb = ft_sum(a_yzb, red);
        a_yy = ft_sum(a_yy, red);
        if (threadIdx.x == 0) {
            A.p_meas[3 * wg + 0] = a_r2;
            A.p_meas[3 * wg + 1] = a_yzb;
            A.p_meas[3 * wg + 2] = a_yy;
        }
    } else {
        const double sj = A.s[j];
        for (int r = 0; r < A.rw; ++r) {
            const int k1 = k10 + r;
            if (k1 >= A.n1) continue;
            for (int e = threadIdx.x; e < A.n2; e += kFT) {
                const double2 X = buf[pad((e << A.lrw) + r)];
                out[(size_t)j * A.n + k1 + (size_t)A.n1 * e] = sj * (X.x * X.x + X.y * X.y);
            }
        }
    }
}

// Inverse column pass summed over the waveforms of group g; group 0 adds the
// C term x / sqrt(n) (x = src / *dv).  Writes P_g and the partial Re(x^* P_g).
__global__ __launch_bounds__(kFI) void k_pr_colinv(PrArgs A, const double2* __restrict__ src, const double* dv,
                                                  int lanczos) {
    __shared__ double2 buf[kTileP];
    __shared__ double2 tws[kTwLds];
    __shared__ double2 dl[256];
    __shared__ double red[kFI / 64];
    if (lanczos && A.sc->broken) return;
    load_tw(tws, A.f1, kFI);
    load_dict(dl, A, kFI);
    const int g = blockIdx.y;
    const int m20 = blockIdx.x * A.tc;
    const int tot = A.n1 << A.ltc;
    double2 acc[kTile / kFI];
#pragma unroll
    for (int u = 0; u < kTile / kFI; ++u) acc[u] = make_double2(0.0, 0.0);
    const int j0 = g * A.mpg, j1 = min(A.L, j0 + A.mpg);
    for (int j = j0; j < j1; ++j) {
        const double2* Zj = A.Y + (size_t)j * A.n;
        const size_t jn = (size_t)j * A.n;
        int code[kTile / kFI];   // the waveform codes of this thread's outputs, loaded with the tile
#pragma unroll
        for (int u = 0; u < kTile / kFI; ++u) {
            const int idx = threadIdx.x + u * kFI;
            code[u] = 0;
            if (idx < tot) {
                const int k1 = idx >> A.ltc, m2 = m20 + (idx & (A.tc - 1));
                buf[pad(idx)] = (m2 < A.n2) ? Zj[(int64_t)k1 * A.n2 + m2] : make_double2(0.0, 0.0);
                if (A.coded && m2 < A.n2)
                    code[u] = A.psic[((size_t)j * A.ntc + blockIdx.x) * ((size_t)A.n1 << A.ltc) + idx];
            }
        }
        __syncthreads();
        fft_tile<true, kFI>(buf, A.f1, A.ltc, tws);
#pragma unroll
        for (int u = 0; u < kTile / kFI; ++u) {
            const int idx = threadIdx.x + u * kFI;
            if (idx < tot) {
                const int m1 = idx >> A.ltc, m2 = m20 + (idx & (A.tc - 1));
                if (m2 < A.n2) {
                    const double2 ps = A.coded ? dl[code[u]] : A.psi[jn + (int64_t)m1 * A.n2 + m2];
                    acc[u] = cadd(acc[u], cmul(ps, buf[pad(idx)]));
                }
            }
        }
        __syncthreads();
    }
    const double d = *dv;
    double dot = 0.0;
    double2* Pg = A.P + (size_t)g * A.n;
#pragma unroll
    for (int u = 0; u < kTile / kFI; ++u) {
        const int idx = threadIdx.x + u * kFI;
        if (idx < tot) {
            const int m1 = idx >> A.ltc, m2 = m20 + (idx & (A.tc - 1));
            if (m2 < A.n2) {
                const int64_t m = (int64_t)m1 * A.n2 + m2;
                double2 x = src[m];
                x.x /= d;
                x.y /= d;
                double2 a = acc[u];
                if (g == 0) a = cadd(cscl(x, A.c_scale), a);
                Pg[m] = a;
                dot += x.x * a.x + x.y * a.y;
            }
        }
    }
    dot = ft_sum<kFI>(dot, red);
    if (threadIdx.x == 0) A.p_col[(size_t)g * gridDim.x + blockIdx.x] = dot;
}

// ------------------------------------------------------------------ Lanczos
// Start vector of iteration t: complex element m is the Box-Muller pair
// (2m, 2m + 1) of the Philox stream (seed; t, instance, purpose 2).
__global__ __launch_bounds__(kBlock) void k_pr_start(PrArgs A, uint64_t seed, int tt, uint64_t inst, int q) {
    const uint64_t t = (uint64_t)pr_t(A, tt);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        A.sc->broken = 0;
        A.sc->k = q;
    }
    double acc = 0.0;
    for (int64_t h = blockIdx.x * (int64_t)kBlock + threadIdx.x; 2 * h < A.n; h += (int64_t)gridDim.x * kBlock) {
        double g[4];
        normal4(seed, (uint64_t)h, t, inst, 2ull, g);
        A.V[2 * h] = make_double2(g[0], g[1]);
        acc += g[0] * g[0] + g[1] * g[1];
        if (2 * h + 1 < A.n) {
            A.V[2 * h + 1] = make_double2(g[2], g[3]);
            acc += g[2] * g[2] + g[3] * g[3];
        }
    }
    const double v[1] = {acc};
    write_partials<1>(v, A.p_upd);
}

// nrm[i1] = sqrt(sum of partials); with check, the breakdown test of the step
// that produced V[i1]: rho <= 64 eps (|omega| + rho_prev).
__global__ __launch_bounds__(kBlock) void k_pr_norm(PrArgs A, int i1, int nparts, int check) {
    if (A.sc->broken) return;
    double s[1];
    reduce_partials<1>(A.p_upd, nparts, s);
    if (threadIdx.x == 0) {
        const double r = sqrt(s[0]);
        if (check) {
            const int i = i1 - 1;
            const double rprev = (i > 0) ? A.sc->nrm[i] : 0.0;
            if (r <= 64.0 * 2.220446049250313e-16 * (fabs(A.sc->omega[i]) + rprev)) {
                A.sc->broken = 1;
                A.sc->k = i + 1;
                return;
            }
        }
        A.sc->nrm[i1] = r;
    }
}

// omega_i = sum of the v^* P_g partials; V[i+1] = sum_g P_g - omega_i v_i - rho_{i-1} v_{i-1}.
__global__ __launch_bounds__(kBlock) void k_pr_update(PrArgs A, int i) {
    if (A.sc->broken) return;
    double om[1];
    reduce_partials<1>(A.p_col, A.G * A.ntc, om);
    const double w = om[0];
    if (blockIdx.x == 0 && threadIdx.x == 0) A.sc->omega[i] = w;
    const double di = A.sc->nrm[i];
    const double rprev = (i > 0) ? A.sc->nrm[i] : 0.0;
    const double dp = (i > 0) ? A.sc->nrm[i - 1] : 1.0;
    const double2* vi = A.V + (size_t)i * A.n;
    const double2* vp = A.V + (size_t)(i > 0 ? i - 1 : 0) * A.n;
    double2* vo = A.V + (size_t)(i + 1) * A.n;
    double acc = 0.0;
    for (int64_t m = blockIdx.x * (int64_t)kBlock + threadIdx.x; m < A.n; m += (int64_t)gridDim.x * kBlock) {
        double2 dv = A.P[m];
        for (int g = 1; g < A.G; ++g) dv = cadd(dv, A.P[(size_t)g * A.n + m]);
        double2 x = vi[m];
        x.x /= di;
        x.y /= di;
        double2 u = csub(dv, cscl(x, w));
        if (i > 0) {
            double2 xp = vp[m];
            xp.x /= dp;
            xp.y /= dp;
            u = csub(u, cscl(xp, rprev));
        }
        vo[m] = u;
        acc += u.x * u.x + u.y * u.y;
    }
    const double v[1] = {acc};
    write_partials<1>(v, A.p_upd);
}

// MinEvec of T_k; without breakdown the last step's omega partials are still pending.
__global__ __launch_bounds__(kBlock) void k_pr_tridiag(PrArgs A, int q) {
    __shared__ double d[kPQCap], e[kPQCap], e2[kPQCap], dp[kPQCap], dm[kPQCap], x[kPQCap];
    __shared__ double xi;
    PrScalars* sc = A.sc;
    const bool broken = sc->broken != 0;
    double tot[1];
    if (!broken) reduce_partials<1>(A.p_col, A.G * A.ntc, tot);
    const int k = broken ? sc->k : q;
    for (int i = threadIdx.x; i < k; i += kBlock) {
        d[i] = (!broken && i == q - 1) ? tot[0] : sc->omega[i];
        if (i < k - 1) e[i] = sc->nrm[i + 1];
    }
    __syncthreads();
    if (threadIdx.x < 64) tridiag_min_eig(d, e, k, e2, dp, dm, x, &xi);
    __syncthreads();
    for (int i = threadIdx.x; i < k; i += kBlock) sc->coef[i] = x[i];
    if (threadIdx.x == 0) {
        if (!broken) {
            sc->omega[q - 1] = tot[0];
            sc->k = q;
        }
        sc->xi = xi;
        sc->ha = (xi < 0.0) ? A.alpha_s : 0.0;
        if (!isfinite(xi)) sc->flags |= 1;
    }
}

// Ritz vector sum_j u_j v_j and partials of its squared norm.
__global__ __launch_bounds__(kBlock) void k_pr_ritz(PrArgs A) {
    __shared__ double cf[kPQCap], dn[kPQCap];
    const int k = A.sc->k;
    for (int j = threadIdx.x; j < k; j += kBlock) {
        cf[j] = A.sc->coef[j];
        dn[j] = A.sc->nrm[j];
    }
    __syncthreads();
    double acc = 0.0;
    for (int64_t m = blockIdx.x * (int64_t)kBlock + threadIdx.x; m < A.n; m += (int64_t)gridDim.x * kBlock) {
        double2 x = make_double2(0.0, 0.0);
        for (int j = 0; j < k; ++j) {
            double2 v = A.V[(size_t)j * A.n + m];
            v.x /= dn[j];
            v.y /= dn[j];
            x = cadd(x, cscl(v, cf[j]));
        }
        A.xr[m] = x;
        acc += x.x * x.x + x.y * x.y;
    }
    const double v[1] = {acc};
    write_partials<1>(v, A.p_upd);
}

__global__ __launch_bounds__(kBlock) void k_pr_xnorm(PrArgs A, int nparts) {
    double s[1];
    reduce_partials<1>(A.p_upd, nparts, s);
    if (threadIdx.x == 0) A.sc->xnorm = sqrt(s[0]);
}

// ------------------------------------------------------------------ state updates
// Start of iteration t: c = s_j (y + beta (z - b)) and partials of <w, z>.
__global__ __launch_bounds__(kBlock) void k_pr_prep(PrArgs A, int tt) {
    const double beta = pr_beta(A, pr_t(A, tt));
    double acc = 0.0;
    const int64_t tot = (int64_t)A.L * A.n;
    for (int64_t pos = blockIdx.x * (int64_t)kBlock + threadIdx.x; pos < tot; pos += (int64_t)gridDim.x * kBlock) {
        const int j = (int)(pos / A.n);
        const double zz = A.z[pos];
        const double w = A.y[pos] + beta * (zz - A.b[pos]);
        A.c[pos] = A.s[j] * w;
        acc += w * zz;
    }
    const double v[1] = {acc};
    write_partials<1>(v, A.p_prep);
}

// Scalars of the iteration: gap, p, tau, gamma (dual step size, eqn
// sketchy-cgal-dual-step with ||A|| = 1, the K guard), and the log record.
__global__ __launch_bounds__(kBlock) void k_pr_scalars(PrArgs A, int tt, int q, int nmeas, int nprep) {
    const int t = pr_t(A, tt);
    const double beta = pr_beta(A, t), eta = pr_eta(t);
    double m3[3], wz[1];
    reduce_partials<3>(A.p_meas, nmeas, m3);
    reduce_partials<1>(A.p_prep, nprep, wz);
    if (threadIdx.x != 0) return;
    PrScalars* sc = A.sc;
    const double r2 = m3[0], yzb = m3[1], yy = m3[2];
    const double xi = sc->xi, ha = sc->ha;
    const double gap = sc->p + wz[0] - ha * xi;
    const double cv = A.c_scale;
    sc->p = (1.0 - eta) * sc->p + eta * ha * cv;
    sc->tau = (1.0 - eta) * sc->tau + eta * ha;
    const double a = A.alpha_s;
    double gamma = (r2 == 0.0) ? A.beta0
                               : fmin(A.beta0, 4.0 * a * a * A.beta0 / (pow(t + 1.0, 1.5) * r2));
    if (isfinite(A.K)) {
        const double ny2 = yy + 2.0 * gamma * yzb + gamma * gamma * r2;
        if (sqrt(fmax(ny2, 0.0)) > A.K) gamma = 0.0;
    }
    sc->gamma = gamma;
    if (!isfinite(r2) || !isfinite(xi)) sc->flags |= 1;
    scg_iter_log& L = A.log[t - 1];
    L.t = t;
    L.q = q;
    L.k = sc->k;
    L.flags = sc->broken ? 1 : 0;
    L.xi = xi;
    L.cv = cv;
    L.p = sc->p;
    L.infeas = sqrt(r2);
    L.gamma = gamma;
    L.gap = gap;
    L.stop_obj = __builtin_nan("");
    L.stop_feas = __builtin_nan("");
    L.resid = __builtin_nan("");
    L.beta = beta;
    L.eta = eta;
}

__global__ __launch_bounds__(kBlock) void k_pr_dual(PrArgs A) {
    const double gamma = A.sc->gamma;
    if (gamma == 0.0) return;
    const int64_t tot = (int64_t)A.L * A.n;
    for (int64_t pos = blockIdx.x * (int64_t)kBlock + threadIdx.x; pos < tot; pos += (int64_t)gridDim.x * kBlock)
        A.y[pos] = A.y[pos] + gamma * (A.z[pos] - A.b[pos]);
}

// Partials of v^* Omega_c (v = xr / xnorm), 2R doubles per workgroup (RB >= R).
template <int RB>
__global__ __launch_bounds__(kBlock) void k_pr_skdot(PrArgs A) {
    __shared__ double red[kWaves];
    const double d = A.sc->xnorm;
    double acc[2 * RB];
#pragma unroll
    for (int c = 0; c < 2 * RB; ++c) acc[c] = 0.0;
    for (int64_t m = blockIdx.x * (int64_t)kBlock + threadIdx.x; m < A.n; m += (int64_t)gridDim.x * kBlock) {
        double2 v = A.xr[m];
        v.x /= d;
        v.y /= d;
#pragma unroll
        for (int c = 0; c < RB; ++c) {
            if (c < A.R) {
                const double2 o = A.Om[(size_t)c * A.n + m];
                acc[2 * c] += v.x * o.x + v.y * o.y;       // conj(v) o
                acc[2 * c + 1] += v.x * o.y - v.y * o.x;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 2 * RB; ++c) {
        if (c < 2 * A.R) {
            const double s = block_sum(acc[c], red);
            if (threadIdx.x == 0) A.p_sk[(size_t)blockIdx.x * 2 * A.R + c] = s;
        }
    }
}

// v^* Omega from the partials (fixed order), into the scalars.
__global__ __launch_bounds__(kBlock) void k_pr_skred(PrArgs A, int nparts) {
    __shared__ double red[kWaves];
    for (int c = 0; c < 2 * A.R; ++c) {
        double s = 0.0;
        for (int g = threadIdx.x; g < nparts; g += kBlock) s += A.p_sk[(size_t)g * 2 * A.R + c];
        s = block_sum(s, red);
        if (threadIdx.x == 0) A.sc->dots[c] = s;
    }
}

// S <- (1 - eta) S + eta ha v (v^* Omega).
template <int RB>
__global__ __launch_bounds__(kBlock) void k_pr_skupd(PrArgs A, int tt) {
    const double eta = pr_eta(pr_t(A, tt));
    double2 dt[RB];
#pragma unroll
    for (int c = 0; c < RB; ++c) dt[c] = (c < A.R) ? make_double2(A.sc->dots[2 * c], A.sc->dots[2 * c + 1])
                                                   : make_double2(0.0, 0.0);
    const double d = A.sc->xnorm;
    const double eh = eta * A.sc->ha, keep = 1.0 - eta;
    for (int64_t m = blockIdx.x * (int64_t)kBlock + threadIdx.x; m < A.n; m += (int64_t)gridDim.x * kBlock) {
        double2 v = A.xr[m];
        v.x /= d;
        v.y /= d;
#pragma unroll
        for (int c = 0; c < RB; ++c) {
            if (c < A.R) {
                const double2 o = cmul(v, dt[c]);
                double2& s = A.S[(size_t)c * A.n + m];
                s = make_double2(keep * s.x + eh * o.x, keep * s.y + eh * o.y);
            }
        }
    }
}

// ------------------------------------------------------------------ data movement
// Natural order (j, l) <-> row-pass order (j, k1, k2) with l = k1 + n1 k2.
__global__ __launch_bounds__(kBlock) void k_pr_to_rowpass(PrArgs A, const double* src, double* dst, int scale_s,
                                                         double div) {
    const int64_t tot = (int64_t)A.L * A.n;
    for (int64_t pos = blockIdx.x * (int64_t)kBlock + threadIdx.x; pos < tot; pos += (int64_t)gridDim.x * kBlock) {
        const int j = (int)(pos / A.n);
        const int64_t r = pos - (int64_t)j * A.n;
        const int64_t k1 = r / A.n2, k2 = r - k1 * A.n2;
        const double v = src[(size_t)j * A.n + k1 + (int64_t)A.n1 * k2];
        dst[pos] = (scale_s ? A.s[j] * v : v) / div;
    }
}
__global__ __launch_bounds__(kBlock) void k_pr_from_rowpass(PrArgs A, const double* src, double* dst) {
    const int64_t tot = (int64_t)A.L * A.n;
    for (int64_t pos = blockIdx.x * (int64_t)kBlock + threadIdx.x; pos < tot; pos += (int64_t)gridDim.x * kBlock) {
        const int j = (int)(pos / A.n);
        const int64_t r = pos - (int64_t)j * A.n;
        const int64_t k1 = r / A.n2, k2 = r - k1 * A.n2;
        dst[(size_t)j * A.n + k1 + (int64_t)A.n1 * k2] = src[pos];
    }
}
__global__ __launch_bounds__(kBlock) void k_pr_sum_groups(PrArgs A, double2* out) {
    for (int64_t m = blockIdx.x * (int64_t)kBlock + threadIdx.x; m < A.n; m += (int64_t)gridDim.x * kBlock) {
        double2 v = A.P[m];
        for (int g = 1; g < A.G; ++g) v = cadd(v, A.P[(size_t)g * A.n + m]);
        out[m] = v;
    }
}
// Column c of Omega: the Box-Muller pairs of the stream (seed; c, instance, purpose 3).
__global__ __launch_bounds__(kBlock) void k_pr_omega(PrArgs A, double2* Om, uint64_t seed, uint64_t inst) {
    const int c = blockIdx.y;
    for (int64_t h = blockIdx.x * (int64_t)kBlock + threadIdx.x; 2 * h < A.n; h += (int64_t)gridDim.x * kBlock) {
        double g[4];
        normal4(seed, (uint64_t)h, (uint64_t)c, inst, 3ull, g);
        Om[(size_t)c * A.n + 2 * h] = make_double2(g[0], g[1]);
        if (2 * h + 1 < A.n) Om[(size_t)c * A.n + 2 * h + 1] = make_double2(g[2], g[3]);
    }
}
// Per-waveform sums: pass 0 ||psi_j||^2 (L values), pass 1 the upper triangle
// of sum_m w_j w_k |psi_j(m)|^2 |psi_k(m)|^2 with w = 1 / ||psi||^2.
__global__ __launch_bounds__(kBlock) void k_pr_maskstats(PrArgs A, const double* w, int pass, double* part) {
    __shared__ double red[kWaves];
    const int L = A.L;
    const int nv = pass == 0 ? L : L * (L + 1) / 2;
    for (int o = 0; o < nv; ++o) {
        int j = o, k = o;
        if (pass == 1) {   // o -> (j, k), j <= k
            j = 0;
            int rem = o;
            while (rem >= L - j) { rem -= L - j; ++j; }
            k = j + rem;
        }
        double acc = 0.0;
        for (int64_t m = blockIdx.x * (int64_t)kBlock + threadIdx.x; m < A.n; m += (int64_t)gridDim.x * kBlock) {
            const double2 a = A.psi[(size_t)j * A.n + m];
            const double pa = a.x * a.x + a.y * a.y;
            if (pass == 0) {
                acc += pa;
            } else {
                const double2 bb = A.psi[(size_t)k * A.n + m];
                acc += (w[j] * pa) * (w[k] * (bb.x * bb.x + bb.y * bb.y));
            }
        }
        const double s = block_sum(acc, red);
        if (threadIdx.x == 0) part[(size_t)blockIdx.x * nv + o] = s;
    }
}
// Partials of ||(z - b) / s_j||^2 (infeasibility in the original scaling).
__global__ __launch_bounds__(kBlock) void k_pr_infeas(PrArgs A, double* part) {
    __shared__ double red[kWaves];
    double acc = 0.0;
    const int64_t tot = (int64_t)A.L * A.n;
    for (int64_t pos = blockIdx.x * (int64_t)kBlock + threadIdx.x; pos < tot; pos += (int64_t)gridDim.x * kBlock) {
        const int j = (int)(pos / A.n);
        const double d = (A.z[pos] - A.b[pos]) / A.s[j];
        acc += d * d;
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// ------------------------------------------------------------------ reconstruction kernels
// Partials of X1^* X2 (R x R complex, entry (a, b) = sum_m conj(X1[a][m]) X2[b][m]).
__global__ __launch_bounds__(kBlock) void k_pr_gram(int64_t n, int R, const double2* X1, const double2* X2,
                                                   double* part) {
    __shared__ double red[kWaves];
    for (int a = 0; a < R; ++a)
        for (int b = 0; b < R; ++b) {
            double re = 0.0, im = 0.0;
            for (int64_t m = blockIdx.x * (int64_t)kBlock + threadIdx.x; m < n; m += (int64_t)gridDim.x * kBlock) {
                const double2 u = X1[(size_t)a * n + m], v = X2[(size_t)b * n + m];
                re += u.x * v.x + u.y * v.y;
                im += u.x * v.y - u.y * v.x;
            }
            re = block_sum(re, red);
            im = block_sum(im, red);
            if (threadIdx.x == 0) {
                part[((size_t)blockIdx.x * R * R + a * R + b) * 2] = re;
                part[((size_t)blockIdx.x * R * R + a * R + b) * 2 + 1] = im;
            }
        }
}
// Row-wise: x L^* = a with a = S + sigma Omega (first) or the current row of Wk,
// L lower triangular (R x R complex, row-major in Lm).  x_c = (a_c - sum_{k<c} x_k conj(L[c][k])) / L[c][c].
__global__ __launch_bounds__(kBlock) void k_pr_trsm(int64_t n, int R, const double2* S, const double2* Om,
                                                   double sigma, int first, const double2* Lm, double2* Wk) {
    __shared__ double2 Ls[kPRMax * kPRMax];
    for (int e = threadIdx.x; e < R * R; e += kBlock) Ls[e] = Lm[e];
    __syncthreads();
    for (int64_t m = blockIdx.x * (int64_t)kBlock + threadIdx.x; m < n; m += (int64_t)gridDim.x * kBlock) {
        double2 x[kPRMax];
        for (int c = 0; c < R; ++c) {
            double2 a = first ? cadd(S[(size_t)c * n + m], cscl(Om[(size_t)c * n + m], sigma)) : Wk[(size_t)c * n + m];
            for (int k = 0; k < c; ++k) a = csub(a, cmulc(x[k], Ls[c * R + k]));
            x[c] = cscl(a, 1.0 / Ls[c * R + c].x);
        }
        for (int c = 0; c < R; ++c) Wk[(size_t)c * n + m] = x[c];
    }
}
// out[c][m] = sum_k Wk[k][m] M[k][c]  (M row-major R x R complex).
__global__ __launch_bounds__(kBlock) void k_pr_rmul(int64_t n, int R, const double2* Wk, const double2* Mm,
                                                   double2* out) {
    __shared__ double2 Ms[kPRMax * kPRMax];
    for (int e = threadIdx.x; e < R * R; e += kBlock) Ms[e] = Mm[e];
    __syncthreads();
    for (int64_t m = blockIdx.x * (int64_t)kBlock + threadIdx.x; m < n; m += (int64_t)gridDim.x * kBlock) {
        double2 a[kPRMax];
        for (int k = 0; k < R; ++k) a[k] = Wk[(size_t)k * n + m];
        for (int c = 0; c < R; ++c) {
            double2 s = make_double2(0.0, 0.0);
            for (int k = 0; k < R; ++k) s = cadd(s, cmul(a[k], Ms[k * R + c]));
            out[(size_t)c * n + m] = s;
        }
    }
}
// Rounding: chi = f u_0 (f = sqrt(alpha lambda_1) on the chosen column), partials
// of ||chi||^2, chi^* chi_nat, ||chi_nat||^2.
__global__ __launch_bounds__(kBlock) void k_pr_round(int64_t n, const double2* u, double f, const double2* chit,
                                                    double2* chi, double* part) {
    __shared__ double red[kWaves];
    double a = 0.0, cr = 0.0, ci = 0.0, tt = 0.0;
    for (int64_t m = blockIdx.x * (int64_t)kBlock + threadIdx.x; m < n; m += (int64_t)gridDim.x * kBlock) {
        const double2 x = cscl(u[m], f);
        if (chi) chi[m] = x;
        a += x.x * x.x + x.y * x.y;
        if (chit) {
            const double2 y = chit[m];
            cr += x.x * y.x + x.y * y.y;
            ci += x.x * y.y - x.y * y.x;
            tt += y.x * y.x + y.y * y.y;
        }
    }
    a = block_sum(a, red);
    cr = block_sum(cr, red);
    ci = block_sum(ci, red);
    tt = block_sum(tt, red);
    if (threadIdx.x == 0) {
        part[4 * blockIdx.x] = a;
        part[4 * blockIdx.x + 1] = cr;
        part[4 * blockIdx.x + 2] = ci;
        part[4 * blockIdx.x + 3] = tt;
    }
}

// ------------------------------------------------------------------ host helpers
using cd = std::complex<double>;

// Workgroups of the column pass: ntc * L work items, rounded up to a multiple of 8 (XCD renumbering).
int colfwd_grid(const PrArgs& A) { return ((A.ntc * A.L + kXcd - 1) / kXcd) * kXcd; }

// Radices of a 2,3,5-smooth N (8 first, then 4, 2, 5, 3); false if N has another factor.
bool radix_plan(int N, std::vector<int>& r) {
    r.clear();
    for (int f : {8, 4, 2, 5, 3})
        while (N % f == 0) {
            r.push_back(f);
            N /= f;
        }
    return N == 1 && (int)r.size() <= kMaxStages;
}

bool smooth(int64_t N) {
    for (int f : {2, 3, 5})
        while (N % f == 0) N /= f;
    return N == 1;
}

// Cholesky of a Hermitian R x R matrix (row-major), lower factor; false if not positive definite.
bool chol_c(const std::vector<cd>& B, int R, std::vector<cd>& Lo) {
    Lo.assign((size_t)R * R, cd(0.0, 0.0));
    for (int j = 0; j < R; ++j) {
        double d = B[j * R + j].real();
        for (int k = 0; k < j; ++k) d -= std::norm(Lo[j * R + k]);
        if (!(d > 0.0)) return false;
        const double l = std::sqrt(d);
        Lo[j * R + j] = l;
        for (int i = j + 1; i < R; ++i) {
            cd s = B[i * R + j];
            for (int k = 0; k < j; ++k) s -= Lo[i * R + k] * std::conj(Lo[j * R + k]);
            Lo[i * R + j] = s / l;
        }
    }
    return true;
}

// One-sided Jacobi (Hestenes) on the columns of A (R x R complex, row-major):
// on return the columns are mutually orthogonal; their norms are the
// singular values and the normalised columns the left singular vectors.
void jacobi_columns(std::vector<cd>& A, int R) {
    for (int sweep = 0; sweep < 60; ++sweep) {
        bool rotated = false;
        for (int p = 0; p < R; ++p)
            for (int q = p + 1; q < R; ++q) {
                double al = 0.0, be = 0.0;
                cd ga(0.0, 0.0);
                for (int k = 0; k < R; ++k) {
                    al += std::norm(A[k * R + p]);
                    be += std::norm(A[k * R + q]);
                    ga += std::conj(A[k * R + p]) * A[k * R + q];
                }
                const double ag = std::abs(ga);
                if (ag == 0.0 || ag <= 1e-15 * std::sqrt(al * be)) continue;
                rotated = true;
                const cd ph = ga / ag;   // a_q <- conj(ph) a_q makes the inner product real
                const double zeta = (be - al) / (2.0 * ag);
                const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
                for (int k = 0; k < R; ++k) {
                    const cd ap = A[k * R + p], aq = A[k * R + q] * std::conj(ph);
                    A[k * R + p] = c * ap - s * aq;
                    A[k * R + q] = s * ap + c * aq;
                }
            }
        if (!rotated) break;
    }
}

double max_singular(std::vector<cd> A, int R) {
    jacobi_columns(A, R);
    double m = 0.0;
    for (int j = 0; j < R; ++j) {
        double s = 0.0;
        for (int k = 0; k < R; ++k) s += std::norm(A[k * R + j]);
        m = std::max(m, std::sqrt(s));
    }
    return m;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

// ------------------------------------------------------------------ context
struct scg_pr_ctx {
    scg_pr_params prm;
    int64_t n;
    int L, qcap;
    PrArgs A;
    hipStream_t stream;
    double alpha0, c_F, opnorm;
    std::vector<double> s;
    int t_next;
    double2* Wk;                     // R x n reconstruction work array
    double2* small;                  // R x R matrices for the reconstruction
    double* p_red;                   // host-reduced partials
    std::map<int, hipGraphExec_t> graphs;   // captured iterations by Lanczos step count (non-null streams)
};

namespace {

struct Layout {
    size_t psi, psic, dict, s, b, z, y, c, Y, P, V, xr, Om, S, Wk, small, tw1, tw2, twh, twl, p_col, p_upd, p_meas,
        p_prep, p_sk, p_red, sc, log, total;
};

struct Shape {
    int n1, n2, tc, ltc, rw, lrw, G, mpg, ntc, nrw, ntwh;
    int Gmax;   // the most waveform groups the workspace holds (every candidate of the init tuner)
};

int ilog2(int x) {
    int l = 0;
    while ((1 << l) < x) ++l;
    return l;
}

bool choose_shape(int64_t n, int L, int groups, int tile_cols, Shape& sh) {
    if (n < 2 || n > (int64_t)kTile * kTile || !smooth(n)) return false;
    int64_t n1 = -1;
    for (int64_t d = 1; d <= kTile; ++d) {
        if (n % d) continue;
        const int64_t e = n / d;
        if (e <= kTile && smooth(d) && smooth(e)) {
            n1 = d;
            break;
        }
    }
    if (n1 < 0) return false;
    sh.n1 = (int)n1;
    sh.n2 = (int)(n / n1);
    int tc = 1;
    while (tc * 2 <= 64 && (int64_t)sh.n1 * tc * 2 <= kTile) tc *= 2;
    if (tile_cols > 0) {
        if ((tile_cols & (tile_cols - 1)) || (int64_t)sh.n1 * tile_cols > kTile) return false;
        tc = tile_cols;
    }
    sh.tc = tc;
    sh.ltc = ilog2(tc);
    int rw = 1;
    while ((int64_t)sh.n2 * rw * 2 <= kTile && rw * 2 <= 64) rw *= 2;
    sh.rw = rw;
    sh.lrw = ilog2(rw);
    sh.ntc = (sh.n2 + tc - 1) / tc;
    sh.nrw = (sh.n1 + rw - 1) / rw;
    // one group (every waveform summed in one workgroup) unless forced or tuned at init: at n = 10^6 one
    // group takes 130 us, four 157, twelve 215 (fewer groups write and re-read fewer sums)
    int G = groups > 0 ? std::min(groups, L) : 1;
    sh.mpg = (L + G - 1) / G;
    sh.G = (L + sh.mpg - 1) / sh.mpg;
    sh.Gmax = groups > 0 ? sh.G : L;
    sh.ntwh = (int)((n >> kTwShift) + 1);
    return true;
}

int qmax_for(const scg_pr_params* p, int64_t n) {
    int q = 1;
    if (p->q_mode == 1) q = p->q_fixed;
    else q = (int)std::ceil(std::pow((double)p->T, 0.25) * std::log((double)n));
    q = (int)std::max<int64_t>(1, std::min<int64_t>(q, n - 1));
    return q;
}

Layout layout(const scg_pr_params* p, int64_t n, int L, const Shape& sh, int qcap) {
    Layout l;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    const size_t cn = sizeof(double2) * (size_t)n, rn = sizeof(double) * (size_t)n;
    l.psi = take(cn * L);
    l.psic = take((size_t)sh.ntc * sh.n1 * sh.tc * L);
    l.dict = take(sizeof(double2) * 256);
    l.s = take(sizeof(double) * kPLMax);
    l.b = take(rn * L);
    l.z = take(rn * L);
    l.y = take(rn * L);
    l.c = take(rn * L);
    l.Y = take(cn * L);
    l.P = take(cn * sh.Gmax);
    l.V = take(cn * (size_t)(qcap + 1));
    l.xr = take(cn);
    l.Om = take(cn * p->R);
    l.S = take(cn * p->R);
    l.Wk = take(cn * p->R);
    l.small = take(sizeof(double2) * kPRMax * kPRMax);
    l.tw1 = take(sizeof(double2) * kTwLds);
    l.tw2 = take(sizeof(double2) * kTwLds);
    l.twh = take(sizeof(double2) * sh.ntwh);
    l.twl = take(sizeof(double2) * (1 << kTwShift));
    l.p_col = take(sizeof(double) * (size_t)sh.Gmax * sh.ntc);
    l.p_upd = take(sizeof(double) * kGU);
    l.p_meas = take(sizeof(double) * 3 * (size_t)L * sh.nrw);
    l.p_prep = take(sizeof(double) * kGU);
    l.p_sk = take(sizeof(double) * kGU * 2 * kPRMax);
    l.p_red = take(sizeof(double) * kGU * std::max(2 * kPRMax * kPRMax, kPLMax * (kPLMax + 1) / 2));
    l.sc = take(sizeof(PrScalars));
    l.log = take(sizeof(scg_iter_log) * (size_t)p->T);
    l.total = o;
    return l;
}

bool params_ok(const scg_pr_params* p, int64_t n, int L) {
    if (!p) return false;
    if (p->R < 1 || p->R > kPRMax || p->R > n) return false;
    if (p->T < 1) return false;
    if (!(p->beta0 > 0.0) || !std::isfinite(p->beta0)) return false;
    if (!(p->K >= 0.0)) return false;
    if (!(p->alpha > 0.0) && p->alpha != 0.0) return false;
    if (!std::isfinite(p->alpha)) return false;
    if (p->q_mode != 0 && p->q_mode != 1) return false;
    if (p->q_mode == 1 && (p->q_fixed < 1)) return false;
    if (p->scale != 0 && p->scale != 1) return false;
    if (p->trace_correct != 0 && p->trace_correct != 1) return false;
    if (p->mask_groups < 0 || p->mask_groups > L) return false;
    if (p->tile_cols < 0) return false;
    if (p->mask_format != 0 && p->mask_format != 1) return false;
    if (p->autotune != 0 && p->autotune != 1) return false;
    if (L < 1 || L > kPLMax) return false;
    if (qmax_for(p, n) > kPQCap) return false;
    return true;
}

int grid_for(int64_t items) { return (int)std::max<int64_t>(1, std::min<int64_t>(kGU, (items + kBlock - 1) / kBlock)); }

std::vector<double2> twiddles(int64_t N, int64_t count, int64_t step) {
    std::vector<double2> t((size_t)count);
    for (int64_t i = 0; i < count; ++i) {
        const long double a = -2.0L * 3.14159265358979323846264338327950288L * (long double)((i * step) % N) /
                              (long double)N;
        t[(size_t)i] = make_double2((double)cosl(a), (double)sinl(a));
    }
    return t;
}

#define PR_HIP(x)                                  \
    do {                                           \
        if ((x) != hipSuccess) return SCG_EHIP;    \
    } while (0)

// Sum `parts` partial records of `w` doubles each (fixed order) on the host.
scg_status host_reduce(scg_pr_ctx* c, const double* dev, int parts, int w, std::vector<double>& out) {
    std::vector<double> h((size_t)parts * w);
    PR_HIP(hipMemcpyAsync(h.data(), dev, sizeof(double) * h.size(), hipMemcpyDeviceToHost, c->stream));
    PR_HIP(hipStreamSynchronize(c->stream));
    out.assign(w, 0.0);
    for (int g = 0; g < parts; ++g)
        for (int k = 0; k < w; ++k) out[k] += h[(size_t)g * w + k];
    return SCG_OK;
}

// D v for the stored w (in c) applied to src / *dv; the group sums land in P and
// the partials of v^* D v in p_col.
void enqueue_apply(scg_pr_ctx* c, const double2* src, const double* dv, int lanczos) {
    PrArgs& A = c->A;
    hipLaunchKernelGGL(k_pr_colfwd, dim3(colfwd_grid(A)), dim3(kFT), 0, c->stream, A, src, dv, lanczos);
    hipLaunchKernelGGL(k_pr_row<0>, dim3(A.nrw, A.L), dim3(kFT), 0, c->stream, A, lanczos, 0, (double*)nullptr);
    hipLaunchKernelGGL(k_pr_colinv, dim3(A.ntc, A.G), dim3(kFI), 0, c->stream, A, src, dv, lanczos);
}

int q_of(const scg_pr_ctx* c, int t) {
    int q;
    if (c->prm.q_mode == 1) q = c->prm.q_fixed;
    else q = (int)std::ceil(std::pow((double)t, 0.25) * std::log((double)c->n));
    return (int)std::max<int64_t>(1, std::min<int64_t>(q, std::min<int64_t>(c->n - 1, c->qcap)));
}

// One iteration with q Lanczos steps.  With dev the kernels take t (and beta_t, eta_t) from the device
// counter: the form captured into a graph and replayed for every iteration with the same q; otherwise t
// is the launch argument.
void enqueue_iteration(scg_pr_ctx* c, int t_host, int q, bool dev) {
    PrArgs& A = c->A;
    hipStream_t st = c->stream;
    const int t = dev ? 0 : t_host;
    const int gL = grid_for((int64_t)A.L * A.n), gn = grid_for(A.n), gh = grid_for((A.n + 1) / 2);
    hipLaunchKernelGGL(k_pr_prep, dim3(gL), dim3(kBlock), 0, st, A, t);
    hipLaunchKernelGGL(k_pr_start, dim3(gh), dim3(kBlock), 0, st, A, (uint64_t)c->prm.seed, t,
                       (uint64_t)c->prm.instance, q);
    hipLaunchKernelGGL(k_pr_norm, dim3(1), dim3(kBlock), 0, st, A, 0, gh, 0);
    for (int i = 0; i < q; ++i) {
        const double2* vi = A.V + (size_t)i * A.n;
        enqueue_apply(c, vi, &A.sc->nrm[i], 1);
        if (i == q - 1) break;
        hipLaunchKernelGGL(k_pr_update, dim3(gn), dim3(kBlock), 0, st, A, i);
        hipLaunchKernelGGL(k_pr_norm, dim3(1), dim3(kBlock), 0, st, A, i + 1, gn, 1);
    }
    hipLaunchKernelGGL(k_pr_tridiag, dim3(1), dim3(kBlock), 0, st, A, q);
    hipLaunchKernelGGL(k_pr_ritz, dim3(gn), dim3(kBlock), 0, st, A);
    hipLaunchKernelGGL(k_pr_xnorm, dim3(1), dim3(kBlock), 0, st, A, gn);
    hipLaunchKernelGGL(k_pr_colfwd, dim3(colfwd_grid(A)), dim3(kFT), 0, st, A, (const double2*)A.xr, &A.sc->xnorm, 0);
    hipLaunchKernelGGL(k_pr_row<1>, dim3(A.nrw, A.L), dim3(kFT), 0, st, A, 0, t, (double*)nullptr);
    hipLaunchKernelGGL(k_pr_scalars, dim3(1), dim3(kBlock), 0, st, A, t, q, A.nrw * A.L, gL);
    hipLaunchKernelGGL(k_pr_dual, dim3(gL), dim3(kBlock), 0, st, A);
    const int R = A.R;
    if (R <= 1) hipLaunchKernelGGL(k_pr_skdot<1>, dim3(gn), dim3(kBlock), 0, st, A);
    else if (R <= 2) hipLaunchKernelGGL(k_pr_skdot<2>, dim3(gn), dim3(kBlock), 0, st, A);
    else if (R <= 4) hipLaunchKernelGGL(k_pr_skdot<4>, dim3(gn), dim3(kBlock), 0, st, A);
    else if (R <= 8) hipLaunchKernelGGL(k_pr_skdot<8>, dim3(gn), dim3(kBlock), 0, st, A);
    else hipLaunchKernelGGL(k_pr_skdot<16>, dim3(gn), dim3(kBlock), 0, st, A);
    hipLaunchKernelGGL(k_pr_skred, dim3(1), dim3(kBlock), 0, st, A, gn);
    if (R <= 1) hipLaunchKernelGGL(k_pr_skupd<1>, dim3(gn), dim3(kBlock), 0, st, A, t);
    else if (R <= 2) hipLaunchKernelGGL(k_pr_skupd<2>, dim3(gn), dim3(kBlock), 0, st, A, t);
    else if (R <= 4) hipLaunchKernelGGL(k_pr_skupd<4>, dim3(gn), dim3(kBlock), 0, st, A, t);
    else if (R <= 8) hipLaunchKernelGGL(k_pr_skupd<8>, dim3(gn), dim3(kBlock), 0, st, A, t);
    else hipLaunchKernelGGL(k_pr_skupd<16>, dim3(gn), dim3(kBlock), 0, st, A, t);
}

// The captured iteration for Lanczos step count q (instantiated on first use, cached in the context).
hipError_t graph_for(scg_pr_ctx* c, int q, hipGraphExec_t* out) {
    auto f = c->graphs.find(q);
    if (f != c->graphs.end()) {
        *out = f->second;
        return hipSuccess;
    }
    hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    enqueue_iteration(c, 0, q, true);
    hipLaunchKernelGGL(k_pr_advance_t, dim3(1), dim3(1), 0, c->stream, c->A.sc);
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

// Runs of iterations with the same q_t replay one captured iteration, after a one-thread kernel has set
// the device counter to the run's first t.
scg_status step_graphs(scg_pr_ctx* c, int32_t iters) {
    int k = 0;
    while (k < iters) {
        const int t = c->t_next;
        const int q = q_of(c, t);
        int m = 1;
        while (k + m < iters && q_of(c, t + m) == q) ++m;
        hipGraphExec_t ge = nullptr;
        PR_HIP(graph_for(c, q, &ge));
        hipLaunchKernelGGL(k_pr_set_t, dim3(1), dim3(1), 0, c->stream, c->A.sc, t);
        PR_HIP(hipGetLastError());
        for (int j = 0; j < m; ++j) PR_HIP(hipGraphLaunch(ge, c->stream));
        c->t_next += m;
        k += m;
    }
    return SCG_OK;
}

// Waveform groups of the inverse column pass, chosen at init: one product D v (after a warm-up one)
// timed with HIP events for G in {1, 2, 3, 4, 6, 12, L} (as far as they differ and fit L), the fastest
// kept; a later candidate replaces the best so far only when at least 3% faster.  The operands are the
// first iteration's dual weights and start vector, which the first iteration forms again.
scg_status tune_groups(scg_pr_ctx* c) {
    PrArgs& A = c->A;
    hipStream_t st = c->stream;
    hipLaunchKernelGGL(k_pr_prep, dim3(grid_for((int64_t)A.L * A.n)), dim3(kBlock), 0, st, A, 1);
    const int gh = grid_for((A.n + 1) / 2);
    hipLaunchKernelGGL(k_pr_start, dim3(gh), dim3(kBlock), 0, st, A, (uint64_t)c->prm.seed, 1,
                       (uint64_t)c->prm.instance, 1);
    hipLaunchKernelGGL(k_pr_norm, dim3(1), dim3(kBlock), 0, st, A, 0, gh, 0);
    hipEvent_t e0, e1;
    PR_HIP(hipEventCreate(&e0));
    PR_HIP(hipEventCreate(&e1));
    int best_g = -1, best_mpg = 0;
    float best_ms = 0.f;
    std::vector<int> seen;
    for (int cand : {1, 2, 3, 4, 6, 12, A.L}) {
        if (cand > A.L) continue;
        const int mpg = (A.L + cand - 1) / cand;
        const int G = (A.L + mpg - 1) / mpg;
        if (std::find(seen.begin(), seen.end(), G) != seen.end()) continue;
        seen.push_back(G);
        A.G = G;
        A.mpg = mpg;
        enqueue_apply(c, A.V, &A.sc->nrm[0], 0);
        PR_HIP(hipEventRecord(e0, st));
        enqueue_apply(c, A.V, &A.sc->nrm[0], 0);
        PR_HIP(hipEventRecord(e1, st));
        PR_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        PR_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (best_g < 0 || ms < 0.97f * best_ms) {
            best_g = G;
            best_mpg = mpg;
            best_ms = ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    A.G = best_g;
    A.mpg = best_mpg;
    return hipGetLastError() == hipSuccess ? SCG_OK : SCG_EHIP;
}

}  // namespace

extern "C" {

void scg_pr_default_params(scg_pr_params* p) {
    std::memset(p, 0, sizeof(*p));
    p->R = 5;
    p->T = 100;
    p->beta0 = 1.0;
    p->K = INFINITY;
    p->alpha = 0.0;
    p->seed = 0;
    p->q_mode = 0;
    p->q_fixed = 0;
    p->scale = 1;
    p->trace_correct = 1;
    p->instance = 0;
    p->mask_groups = 0;
    p->tile_cols = 0;
    p->mask_format = 0;
    p->autotune = 1;
}

scg_status scg_pr_workspace_size(const scg_pr_params* p, int64_t n, int32_t L, size_t* bytes) {
    if (!bytes || !params_ok(p, n, L)) return SCG_EINVAL;
    Shape sh;
    if (!choose_shape(n, L, p->mask_groups, p->tile_cols, sh)) return SCG_EINVAL;
    *bytes = layout(p, n, L, sh, qmax_for(p, n)).total;
    return SCG_OK;
}

scg_status scg_pr_init(scg_pr_ctx** out, const scg_pr_params* p, int64_t n, int32_t L, const double* psi,
                       const double* b, const double* omega, void* workspace, size_t ws_bytes, void* stream) {
    if (!out) return SCG_EINVAL;
    *out = nullptr;
    if (!params_ok(p, n, L) || !psi || !b || !workspace) return SCG_EINVAL;
    if (((uintptr_t)workspace) & 255) return SCG_EINVAL;
    Shape sh;
    if (!choose_shape(n, L, p->mask_groups, p->tile_cols, sh)) return SCG_EINVAL;
    const int qcap = qmax_for(p, n);
    const Layout l = layout(p, n, L, sh, qcap);
    if (ws_bytes < l.total) return SCG_ENOMEM;
    std::vector<int> r1, r2;
    if (!radix_plan(sh.n1, r1) || !radix_plan(sh.n2, r2)) return SCG_EINVAL;

    const double2* psi_in = (const double2*)psi;
    scg_pr_ctx* c = new scg_pr_ctx();
    c->prm = *p;
    c->n = n;
    c->L = L;
    c->qcap = qcap;
    c->stream = (hipStream_t)stream;
    c->t_next = 1;
    char* w = (char*)workspace;
    PrArgs& A = c->A;
    A.n = n;
    A.L = L;
    A.R = p->R;
    A.n1 = sh.n1;
    A.n2 = sh.n2;
    A.tc = sh.tc;
    A.ltc = sh.ltc;
    A.rw = sh.rw;
    A.lrw = sh.lrw;
    A.G = sh.G;
    A.mpg = sh.mpg;
    A.ntc = sh.ntc;
    A.nrw = sh.nrw;
    A.psi = psi_in;   // the caller's copy until the waveforms are stored below
    A.psic = (const uint8_t*)(w + l.psic);
    A.dict = (const double2*)(w + l.dict);
    A.coded = 0;
    A.ndict = 0;
    A.s = (const double*)(w + l.s);
    A.b = (const double*)(w + l.b);
    A.z = (double*)(w + l.z);
    A.y = (double*)(w + l.y);
    A.c = (double*)(w + l.c);
    A.Y = (double2*)(w + l.Y);
    A.P = (double2*)(w + l.P);
    A.V = (double2*)(w + l.V);
    A.xr = (double2*)(w + l.xr);
    A.Om = (const double2*)(w + l.Om);
    A.S = (double2*)(w + l.S);
    A.p_col = (double*)(w + l.p_col);
    A.p_upd = (double*)(w + l.p_upd);
    A.p_meas = (double*)(w + l.p_meas);
    A.p_prep = (double*)(w + l.p_prep);
    A.p_sk = (double*)(w + l.p_sk);
    A.sc = (PrScalars*)(w + l.sc);
    A.log = (scg_iter_log*)(w + l.log);
    c->Wk = (double2*)(w + l.Wk);
    c->small = (double2*)(w + l.small);
    c->p_red = (double*)(w + l.p_red);
    A.f1.N = sh.n1;
    A.f1.ns = (int)r1.size();
    for (size_t i = 0; i < r1.size(); ++i) A.f1.rad[i] = r1[i];
    A.f1.tw = (const double2*)(w + l.tw1);
    A.f2.N = sh.n2;
    A.f2.ns = (int)r2.size();
    for (size_t i = 0; i < r2.size(); ++i) A.f2.rad[i] = r2[i];
    A.f2.tw = (const double2*)(w + l.tw2);
    A.twh = (const double2*)(w + l.twh);
    A.twl = (const double2*)(w + l.twl);
    A.beta0 = p->beta0;
    A.K = p->K;
    c->alpha0 = (p->alpha > 0.0) ? p->alpha : 3.0 * (double)n;

    auto fail = [&](scg_status s) {
        delete c;
        return s;
    };
    hipStream_t st = c->stream;
    {
        std::vector<double2> t1 = twiddles(sh.n1, 64, 64), t2 = twiddles(sh.n2, 64, 64);
        const std::vector<double2> l1 = twiddles(sh.n1, 64, 1), l2 = twiddles(sh.n2, 64, 1);
        t1.insert(t1.end(), l1.begin(), l1.end());
        t2.insert(t2.end(), l2.begin(), l2.end());
        const std::vector<double2> th = twiddles(n, sh.ntwh, (int64_t)1 << kTwShift), tl = twiddles(n, 1 << kTwShift, 1);
        if (hipMemcpyAsync((void*)A.f1.tw, t1.data(), sizeof(double2) * t1.size(), hipMemcpyHostToDevice, st) ||
            hipMemcpyAsync((void*)A.f2.tw, t2.data(), sizeof(double2) * t2.size(), hipMemcpyHostToDevice, st) ||
            hipMemcpyAsync((void*)A.twh, th.data(), sizeof(double2) * th.size(), hipMemcpyHostToDevice, st) ||
            hipMemcpyAsync((void*)A.twl, tl.data(), sizeof(double2) * tl.size(), hipMemcpyHostToDevice, st) ||
            hipStreamSynchronize(st))
            return fail(SCG_EHIP);
    }
    // scaling (eqn problem-scaling): s_j = 1 / (||psi_j||^2 N), N = sqrt(n lambda_max(Q Q^T))
    const int gn = grid_for(n);
    std::vector<double> s0(L, 1.0), sv(L, 1.0);
    c->opnorm = 1.0;
    if (p->scale) {
        std::vector<double> nr;
        hipLaunchKernelGGL(k_pr_maskstats, dim3(gn), dim3(kBlock), 0, st, A, (const double*)nullptr, 0, c->p_red);
        if (host_reduce(c, c->p_red, gn, L, nr) != SCG_OK) return fail(SCG_EHIP);
        for (int j = 0; j < L; ++j) {
            if (!(nr[j] > 0.0) || !std::isfinite(nr[j])) return fail(SCG_EINVAL);
            s0[j] = 1.0 / nr[j];
        }
        if (hipMemcpyAsync((void*)A.s, s0.data(), sizeof(double) * L, hipMemcpyHostToDevice, st))
            return fail(SCG_EHIP);
        std::vector<double> qq;
        hipLaunchKernelGGL(k_pr_maskstats, dim3(gn), dim3(kBlock), 0, st, A, A.s, 1, c->p_red);
        if (host_reduce(c, c->p_red, gn, L * (L + 1) / 2, qq) != SCG_OK) return fail(SCG_EHIP);
        std::vector<cd> Q((size_t)L * L);
        int o = 0;
        for (int j = 0; j < L; ++j)
            for (int k = j; k < L; ++k, ++o) Q[j * L + k] = Q[k * L + j] = cd(qq[o], 0.0);
        const double lmax = max_singular(Q, L);   // symmetric psd: singular values = eigenvalues
        c->opnorm = std::sqrt((double)n * lmax);
        for (int j = 0; j < L; ++j) sv[j] = s0[j] / c->opnorm;
    }
    // store the waveforms: as one-byte codes into a dictionary when they take at most 256 values
    // (compared bitwise), else whole
    {
        bool coded = false;
        int ndict = 0;
        if (p->mask_format == 0) {
            std::vector<double2> h((size_t)n * L);
            if (hipMemcpyAsync(h.data(), psi, sizeof(double2) * h.size(), hipMemcpyDeviceToHost, st) ||
                hipStreamSynchronize(st))
                return fail(SCG_EHIP);
            std::vector<double2> dict;
            const size_t tile_vals = (size_t)sh.n1 * sh.tc;
            std::vector<uint8_t> codes((size_t)L * sh.ntc * tile_vals, 0);
            coded = true;
            for (size_t i = 0; i < h.size() && coded; ++i) {
                int k = 0;
                const int nd = (int)dict.size();
                for (; k < nd; ++k)
                    if (std::memcmp(&dict[k], &h[i], sizeof(double2)) == 0) break;
                if (k == nd) {
                    if (nd == 256) {
                        coded = false;
                        break;
                    }
                    dict.push_back(h[i]);
                }
                {   // waveform j, m = m1 n2 + m2 -> tile m2 / tc, value m1 tc + m2 % tc
                    const size_t jj = i / (size_t)n, m = i - jj * (size_t)n;
                    const size_t m1 = m / (size_t)sh.n2, m2 = m - m1 * (size_t)sh.n2;
                    codes[(jj * sh.ntc + m2 / sh.tc) * tile_vals + m1 * sh.tc + (m2 % sh.tc)] = (uint8_t)k;
                }
            }
            ndict = (int)dict.size();
            if (coded) {
                if (hipMemcpyAsync((void*)A.psic, codes.data(), codes.size(), hipMemcpyHostToDevice, st) ||
                    hipMemcpyAsync((void*)A.dict, dict.data(), sizeof(double2) * dict.size(), hipMemcpyHostToDevice,
                                   st) ||
                    hipStreamSynchronize(st))
                    return fail(SCG_EHIP);
            }
        }
        A.psi = (const double2*)(w + l.psi);
        A.coded = coded ? 1 : 0;
        A.ndict = coded ? ndict : 0;
        if (!coded && hipMemcpyAsync((void*)A.psi, psi, sizeof(double2) * (size_t)n * L, hipMemcpyDeviceToDevice, st))
            return fail(SCG_EHIP);
    }
    c->s = sv;
    if (hipMemcpyAsync((void*)A.s, sv.data(), sizeof(double) * L, hipMemcpyHostToDevice, st)) return fail(SCG_EHIP);
    c->c_F = p->scale ? std::sqrt((double)n) : 1.0;
    A.c_scale = 1.0 / c->c_F;
    A.alpha_s = p->scale ? 1.0 : c->alpha0;
    const int gL = grid_for((int64_t)L * n);
    hipLaunchKernelGGL(k_pr_to_rowpass, dim3(gL), dim3(kBlock), 0, st, A, b, (double*)A.b, 1,
                       p->scale ? c->alpha0 : 1.0);
    if (hipMemsetAsync(A.z, 0, sizeof(double) * (size_t)L * n, st) ||
        hipMemsetAsync(A.y, 0, sizeof(double) * (size_t)L * n, st) ||
        hipMemsetAsync(A.S, 0, sizeof(double2) * (size_t)n * p->R, st) ||
        hipMemsetAsync(A.sc, 0, sizeof(PrScalars), st) ||
        hipMemsetAsync(A.log, 0, sizeof(scg_iter_log) * (size_t)p->T, st))
        return fail(SCG_EHIP);
    {
        const double one = 1.0;
        if (hipMemcpyAsync(&A.sc->one, &one, sizeof(double), hipMemcpyHostToDevice, st)) return fail(SCG_EHIP);
    }
    if (omega) {
        if (hipMemcpyAsync((void*)A.Om, omega, sizeof(double2) * (size_t)n * p->R, hipMemcpyDeviceToDevice, st))
            return fail(SCG_EHIP);
    } else {
        hipLaunchKernelGGL(k_pr_omega, dim3(grid_for((n + 1) / 2), p->R), dim3(kBlock), 0, st, A, (double2*)A.Om,
                           (uint64_t)p->seed, (uint64_t)p->instance);
    }
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) return fail(SCG_EHIP);
    if (p->mask_groups == 0 && p->autotune && L > 1) {
        const scg_status ts = tune_groups(c);
        if (ts != SCG_OK) return fail(ts);
    }
    *out = c;
    return SCG_OK;
}

scg_status scg_pr_destroy(scg_pr_ctx* c) {
    if (!c) return SCG_EINVAL;
    (void)hipStreamSynchronize(c->stream);
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    delete c;
    return SCG_OK;
}

scg_status scg_pr_step(scg_pr_ctx* c, int32_t iters) {
    if (!c || iters < 0) return SCG_EINVAL;
    if (c->t_next + iters - 1 > c->prm.T) return SCG_ESTATE;
    if (c->stream != nullptr) return step_graphs(c, iters);
    for (int i = 0; i < iters; ++i) {
        enqueue_iteration(c, c->t_next, q_of(c, c->t_next), false);
        ++c->t_next;
    }
    return hipGetLastError() == hipSuccess ? SCG_OK : SCG_EHIP;
}

scg_status scg_pr_apply(scg_pr_ctx* c, const double* w, const double* x, double* y) {
    if (!c || !w || !x || !y) return SCG_EINVAL;
    PrArgs& A = c->A;
    hipLaunchKernelGGL(k_pr_to_rowpass, dim3(grid_for((int64_t)A.L * A.n)), dim3(kBlock), 0, c->stream, A, w, A.c, 1,
                       1.0);
    enqueue_apply(c, (const double2*)x, &A.sc->one, 0);
    hipLaunchKernelGGL(k_pr_sum_groups, dim3(grid_for(A.n)), dim3(kBlock), 0, c->stream, A, (double2*)y);
    PR_HIP(hipGetLastError());
    PR_HIP(hipStreamSynchronize(c->stream));
    return SCG_OK;
}

scg_status scg_pr_measure(scg_pr_ctx* c, const double* x, double* m) {
    if (!c || !x || !m) return SCG_EINVAL;
    PrArgs& A = c->A;
    hipLaunchKernelGGL(k_pr_colfwd, dim3(colfwd_grid(A)), dim3(kFT), 0, c->stream, A, (const double2*)x, &A.sc->one, 0);
    hipLaunchKernelGGL(k_pr_row<2>, dim3(A.nrw, A.L), dim3(kFT), 0, c->stream, A, 0, 0, m);
    PR_HIP(hipGetLastError());
    PR_HIP(hipStreamSynchronize(c->stream));
    return SCG_OK;
}

scg_status scg_pr_log(scg_pr_ctx* c, scg_iter_log* host_out, int32_t max, int32_t* count) {
    if (!c || !host_out || max < 0 || !count) return SCG_EINVAL;
    const int cnt = std::min(max, c->t_next - 1);
    if (cnt > 0) {
        PR_HIP(hipMemcpyAsync(host_out, c->A.log, sizeof(scg_iter_log) * cnt, hipMemcpyDeviceToHost, c->stream));
    }
    PR_HIP(hipStreamSynchronize(c->stream));
    *count = cnt;
    return SCG_OK;
}

scg_status scg_pr_summary(scg_pr_ctx* c, scg_pr_info* o, int32_t check_numeric) {
    if (!c || !o) return SCG_EINVAL;
    PrScalars hs;
    PR_HIP(hipMemcpyAsync(&hs, c->A.sc, sizeof(PrScalars), hipMemcpyDeviceToHost, c->stream));
    const int g = grid_for((int64_t)c->L * c->n);
    hipLaunchKernelGGL(k_pr_infeas, dim3(g), dim3(kBlock), 0, c->stream, c->A, c->p_red);
    std::vector<double> inf;
    if (host_reduce(c, c->p_red, g, 1, inf) != SCG_OK) return SCG_EHIP;
    std::memset(o, 0, sizeof(*o));
    o->t_done = c->t_next - 1;
    o->status_flags = hs.flags;
    o->objective = c->c_F * c->alpha0 * hs.p / c->A.alpha_s;
    o->infeasibility = c->alpha0 / c->A.alpha_s * std::sqrt(inf[0]);
    o->p_scaled = hs.p;
    o->tau_scaled = hs.tau;
    o->alpha = c->alpha0;
    o->alpha_scaled = c->A.alpha_s;
    o->c_F = c->c_F;
    o->op_norm = c->opnorm;
    o->n1 = c->A.n1;
    o->n2 = c->A.n2;
    o->tile_cols = c->A.tc;
    o->row_tile = c->A.rw;
    o->mask_groups = c->A.G;
    o->mask_codes = c->A.coded;
    if (check_numeric && (hs.flags & 1)) return SCG_ENUMERIC;
    return SCG_OK;
}

scg_status scg_pr_get_state(scg_pr_ctx* c, int32_t* t_next, double* z, double* y, double* S, double* p,
                            double* tau) {
    if (!c) return SCG_EINVAL;
    PrArgs& A = c->A;
    const int g = grid_for((int64_t)A.L * A.n);
    if (z) hipLaunchKernelGGL(k_pr_from_rowpass, dim3(g), dim3(kBlock), 0, c->stream, A, (const double*)A.z, z);
    if (y) hipLaunchKernelGGL(k_pr_from_rowpass, dim3(g), dim3(kBlock), 0, c->stream, A, (const double*)A.y, y);
    if (S) PR_HIP(hipMemcpyAsync(S, A.S, sizeof(double2) * (size_t)A.n * A.R, hipMemcpyDeviceToDevice, c->stream));
    PrScalars hs;
    PR_HIP(hipMemcpyAsync(&hs, A.sc, sizeof(PrScalars), hipMemcpyDeviceToHost, c->stream));
    PR_HIP(hipGetLastError());
    PR_HIP(hipStreamSynchronize(c->stream));
    if (t_next) *t_next = c->t_next;
    if (p) *p = hs.p;
    if (tau) *tau = hs.tau;
    return SCG_OK;
}

scg_status scg_pr_set_state(scg_pr_ctx* c, int32_t t_next, const double* z, const double* y, const double* S,
                            double p, double tau) {
    if (!c || !z || !y || !S) return SCG_EINVAL;
    if (t_next < 1 || t_next > c->prm.T + 1 || !std::isfinite(p) || !std::isfinite(tau)) return SCG_EINVAL;
    PrArgs& A = c->A;
    const int g = grid_for((int64_t)A.L * A.n);
    hipLaunchKernelGGL(k_pr_to_rowpass, dim3(g), dim3(kBlock), 0, c->stream, A, z, A.z, 0, 1.0);
    hipLaunchKernelGGL(k_pr_to_rowpass, dim3(g), dim3(kBlock), 0, c->stream, A, y, A.y, 0, 1.0);
    PR_HIP(hipMemcpyAsync(A.S, S, sizeof(double2) * (size_t)A.n * A.R, hipMemcpyDeviceToDevice, c->stream));
    double pt[2] = {p, tau};
    PR_HIP(hipMemcpyAsync(&A.sc->p, &pt[0], sizeof(double), hipMemcpyHostToDevice, c->stream));
    PR_HIP(hipMemcpyAsync(&A.sc->tau, &pt[1], sizeof(double), hipMemcpyHostToDevice, c->stream));
    PR_HIP(hipGetLastError());
    PR_HIP(hipStreamSynchronize(c->stream));
    c->t_next = t_next;
    return SCG_OK;
}

scg_status scg_pr_reconstruct(scg_pr_ctx* c, double* U, double* lambda, double* err) {
    if (!c || !U || !lambda) return SCG_EINVAL;
    PrArgs& A = c->A;
    const int R = A.R;
    const int64_t n = A.n;
    hipStream_t st = c->stream;
    const int g = std::min(256, grid_for(n));
    PrScalars hs;
    PR_HIP(hipMemcpyAsync(&hs, A.sc, sizeof(PrScalars), hipMemcpyDeviceToHost, st));
    auto gram = [&](const double2* X1, const double2* X2, std::vector<cd>& Gm) -> scg_status {
        hipLaunchKernelGGL(k_pr_gram, dim3(g), dim3(kBlock), 0, st, n, R, X1, X2, c->p_red);
        std::vector<double> h;
        if (host_reduce(c, c->p_red, g, 2 * R * R, h) != SCG_OK) return SCG_EHIP;
        Gm.resize((size_t)R * R);
        for (int e = 0; e < R * R; ++e) Gm[e] = cd(h[2 * e], h[2 * e + 1]);
        return SCG_OK;
    };
    auto upload = [&](const std::vector<cd>& M) -> scg_status {
        std::vector<double2> h((size_t)R * R);
        for (int e = 0; e < R * R; ++e) h[e] = make_double2(M[e].real(), M[e].imag());
        PR_HIP(hipMemcpyAsync(c->small, h.data(), sizeof(double2) * h.size(), hipMemcpyHostToDevice, st));
        PR_HIP(hipStreamSynchronize(st));
        return SCG_OK;
    };
    std::vector<cd> G0, P0, Q0;
    if (gram(A.S, A.S, G0) || gram(A.Om, A.S, P0) || gram(A.Om, A.Om, Q0)) return SCG_EHIP;
    // sigma = sqrt(n) eps(||S||_2), ||S||_2^2 = lambda_max(S^* S)
    const double snorm = std::sqrt(max_singular(G0, R));
    double sigma = std::sqrt((double)n) * (std::nextafter(snorm, INFINITY) - snorm);
    std::vector<cd> Lc;
    bool ok = false;
    for (int attempt = 0; attempt < 4 && !ok; ++attempt) {
        std::vector<cd> B((size_t)R * R), H((size_t)R * R);
        for (int e = 0; e < R * R; ++e) B[e] = P0[e] + sigma * Q0[e];
        for (int i = 0; i < R; ++i)
            for (int j = 0; j < R; ++j) H[i * R + j] = 0.5 * (B[i * R + j] + std::conj(B[j * R + i]));
        ok = chol_c(H, R, Lc);
        if (!ok) sigma *= 10.0;
    }
    if (!ok) return SCG_ENUMERIC;
    // M = S_sigma Lc^{-*}
    if (upload(Lc)) return SCG_EHIP;
    hipLaunchKernelGGL(k_pr_trsm, dim3(g), dim3(kBlock), 0, st, n, R, (const double2*)A.S, A.Om, sigma, 1,
                       (const double2*)c->small, c->Wk);
    // shifted CholeskyQR3: M = Q R_tot, R_tot = L3^* L2^* L1^*
    std::vector<cd> Rt((size_t)R * R, cd(0.0, 0.0));
    for (int i = 0; i < R; ++i) Rt[i * R + i] = 1.0;
    for (int pass = 0; pass < 3; ++pass) {
        std::vector<cd> Gm, Lk;
        if (gram(c->Wk, c->Wk, Gm)) return SCG_EHIP;
        if (pass == 0) {
            double fro2 = 0.0;
            for (int i = 0; i < R; ++i) fro2 += Gm[i * R + i].real();
            const double shift = 11.0 * ((double)n * R + (double)R * (R + 1)) * 1.1102230246251565e-16 * fro2;
            for (int i = 0; i < R; ++i) Gm[i * R + i] += shift;
        }
        if (!chol_c(Gm, R, Lk)) return SCG_ENUMERIC;
        if (upload(Lk)) return SCG_EHIP;
        hipLaunchKernelGGL(k_pr_trsm, dim3(g), dim3(kBlock), 0, st, n, R, (const double2*)nullptr,
                           (const double2*)nullptr, 0.0, 0, (const double2*)c->small, c->Wk);
        // Rt <- Lk^* Rt
        std::vector<cd> Nt((size_t)R * R, cd(0.0, 0.0));
        for (int i = 0; i < R; ++i)
            for (int j = 0; j < R; ++j) {
                cd s(0.0, 0.0);
                for (int k = 0; k < R; ++k) s += std::conj(Lk[k * R + i]) * Rt[k * R + j];
                Nt[i * R + j] = s;
            }
        Rt = Nt;
    }
    jacobi_columns(Rt, R);
    std::vector<double> svals(R);
    std::vector<int> order(R);
    for (int j = 0; j < R; ++j) {
        double s = 0.0;
        for (int k = 0; k < R; ++k) s += std::norm(Rt[k * R + j]);
        svals[j] = std::sqrt(s);
        order[j] = j;
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b2) { return svals[a] > svals[b2]; });
    std::vector<cd> Ur((size_t)R * R);
    for (int jj = 0; jj < R; ++jj) {
        const int j = order[jj];
        for (int k = 0; k < R; ++k)
            Ur[k * R + jj] = (svals[j] > 0.0) ? Rt[k * R + j] / svals[j] : cd(k == jj ? 1.0 : 0.0, 0.0);
    }
    if (upload(Ur)) return SCG_EHIP;
    hipLaunchKernelGGL(k_pr_rmul, dim3(g), dim3(kBlock), 0, st, n, R, (const double2*)c->Wk,
                       (const double2*)c->small, (double2*)U);
    std::vector<double> lam(R), er(R);
    double tr = 0.0, cum = 0.0;
    for (int jj = 0; jj < R; ++jj) {
        const double sv = svals[order[jj]];
        lam[jj] = std::max(0.0, sv * sv - sigma);
        tr += lam[jj];
    }
    for (int jj = 0; jj < R; ++jj) {
        cum += lam[jj];
        er[jj] = hs.tau - cum;
    }
    if (c->prm.trace_correct)
        for (int jj = 0; jj < R; ++jj) lam[jj] += (hs.tau - tr) / R;
    PR_HIP(hipMemcpyAsync(lambda, lam.data(), sizeof(double) * R, hipMemcpyHostToDevice, st));
    if (err) PR_HIP(hipMemcpyAsync(err, er.data(), sizeof(double) * R, hipMemcpyHostToDevice, st));
    PR_HIP(hipGetLastError());
    PR_HIP(hipStreamSynchronize(st));
    return SCG_OK;
}

scg_status scg_pr_round(scg_pr_ctx* c, const double* U, const double* lambda, const double* chi_true, double* chi,
                        double* rel_err) {
    if (!c || !U || !lambda) return SCG_EINVAL;
    if (rel_err && !chi_true) return SCG_EINVAL;
    PrArgs& A = c->A;
    const int R = A.R;
    std::vector<double> lam(R);
    PR_HIP(hipMemcpyAsync(lam.data(), lambda, sizeof(double) * R, hipMemcpyDeviceToHost, c->stream));
    PR_HIP(hipStreamSynchronize(c->stream));
    int best = 0;
    for (int j = 1; j < R; ++j)
        if (lam[j] > lam[best]) best = j;
    // original units: X = alpha X_scaled
    const double f = std::sqrt(std::max(0.0, lam[best]) * c->alpha0 / A.alpha_s);
    const int g = std::min(256, grid_for(A.n));
    hipLaunchKernelGGL(k_pr_round, dim3(g), dim3(kBlock), 0, c->stream, A.n, (const double2*)U + (size_t)best * A.n,
                       f, (const double2*)chi_true, (double2*)chi, c->p_red);
    std::vector<double> r;
    if (host_reduce(c, c->p_red, g, 4, r) != SCG_OK) return SCG_EHIP;
    if (rel_err) {
        const double m = std::hypot(r[1], r[2]);
        *rel_err = std::sqrt(std::max(0.0, r[0] + r[3] - 2.0 * m)) / std::sqrt(r[3]);
    }
    return SCG_OK;
}

scg_status scg_pr_time_apply(scg_pr_ctx* c, int32_t reps, double* ms) {
    if (!c || reps < 1 || !ms) return SCG_EINVAL;
    PrArgs& A = c->A;
    hipStream_t st = c->stream;
    const int t = std::min(c->t_next, c->prm.T);
    // valid operands: the dual weights of iteration t and its start vector in V[0]
    hipLaunchKernelGGL(k_pr_prep, dim3(grid_for((int64_t)A.L * A.n)), dim3(kBlock), 0, st, A, t);
    const int gh = grid_for((A.n + 1) / 2);
    hipLaunchKernelGGL(k_pr_start, dim3(gh), dim3(kBlock), 0, st, A, (uint64_t)c->prm.seed, t,
                       (uint64_t)c->prm.instance, 1);
    hipLaunchKernelGGL(k_pr_norm, dim3(1), dim3(kBlock), 0, st, A, 0, gh, 0);
    const double2* v = A.V;
    const double* dv = &A.sc->nrm[0];
    hipEvent_t ev[5];
    for (auto& e : ev) PR_HIP(hipEventCreate(&e));
    enqueue_apply(c, v, dv, 0);   // warm-up
    PR_HIP(hipEventRecord(ev[0], st));
    for (int r = 0; r < reps; ++r)
        hipLaunchKernelGGL(k_pr_colfwd, dim3(colfwd_grid(A)), dim3(kFT), 0, st, A, v, dv, 0);
    PR_HIP(hipEventRecord(ev[1], st));
    for (int r = 0; r < reps; ++r)
        hipLaunchKernelGGL(k_pr_row<0>, dim3(A.nrw, A.L), dim3(kFT), 0, st, A, 0, 0, (double*)nullptr);
    PR_HIP(hipEventRecord(ev[2], st));
    for (int r = 0; r < reps; ++r)
        hipLaunchKernelGGL(k_pr_colinv, dim3(A.ntc, A.G), dim3(kFI), 0, st, A, v, dv, 0);
    PR_HIP(hipEventRecord(ev[3], st));
    for (int r = 0; r < reps; ++r) enqueue_apply(c, v, dv, 0);
    PR_HIP(hipEventRecord(ev[4], st));
    PR_HIP(hipEventSynchronize(ev[4]));
    for (int i = 0; i < 4; ++i) {
        float f = 0.f;
        PR_HIP(hipEventElapsedTime(&f, ev[i], ev[i + 1]));
        ms[i] = (double)f / reps;
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    return hipGetLastError() == hipSuccess ? SCG_OK : SCG_EHIP;
}

}  // extern "C"
