// MaxCut rounding of a reconstructed solution (Section 7.2, sec:maxcut-rounding).
//
// X_hat = U Lambda U^T with U (n x R) orthonormal.  The entrywise signs of the
// R columns of U are signed indicators of R cuts (sgn 0 taken as +1); the
// weight of cut chi is -chi^T C chi, which for the MaxCut data C = -L/4
// (eqn:comb-laplacian) is (1/4) chi^T L chi, the total weight of the cut edges.
// One pass over the stored off-diagonal matrix evaluates all R quadratic forms
// at once; the diagonal contributes tr(C) to each.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "scg_device.hpp"
#include "scg_internal.hpp"

using namespace scg;

namespace {

__device__ __forceinline__ double sgn1(double u) { return (u < 0.0) ? -1.0 : 1.0; }

// Partials per workgroup: [0, R) sum_r chi_j(r) (C_off chi_j)_r in scaled units, [R] sum_r diag_r.
template <typename T, int FMT, int RB>
__global__ __launch_bounds__(kBlock) void k_cut_forms(int64_t n, int nseg, const int32_t* rp0, const int32_t* rp1,
                                                      const int32_t* rp2, const int32_t* rp3, const int32_t* col,
                                                      const T* val, double cval, const double* dC, const double* U,
                                                      int R, double* part) {
    __shared__ double red[kWaves];
    const int32_t* rps[4] = {rp0, rp1, rp2, rp3};
    double acc[RB + 1];
#pragma unroll
    for (int j = 0; j <= RB; ++j) acc[j] = 0.0;
    for (int64_t r = blockIdx.x * (int64_t)kBlock + threadIdx.x; r < n; r += (int64_t)gridDim.x * kBlock) {
        double off[RB];
#pragma unroll
        for (int j = 0; j < RB; ++j) off[j] = 0.0;
        for (int sg = 0; sg < nseg; ++sg) {
            const int32_t* rp = rps[sg];
            for (int e = rp[r]; e < rp[r + 1]; ++e) {
                const int cw = col[e];
                const int c = (FMT == FMT_SGN) ? (cw & 0x7fffffff) : cw;
                const double v = (FMT == FMT_VAL) ? (double)val[e] : ((FMT == FMT_SGN && cw < 0) ? -cval : cval);
#pragma unroll
                for (int j = 0; j < RB; ++j)
                    if (j < R) off[j] += v * sgn1(U[(int64_t)j * n + c]);
            }
        }
#pragma unroll
        for (int j = 0; j < RB; ++j)
            if (j < R) acc[j] += sgn1(U[(int64_t)j * n + r]) * off[j];
        acc[RB] += dC[r];
    }
#pragma unroll
    for (int j = 0; j <= RB; ++j) {
        const double s = block_sum(acc[j], red);
        if (threadIdx.x == 0) part[(size_t)blockIdx.x * (RB + 1) + j] = s;
    }
}

__global__ __launch_bounds__(kBlock) void k_cut_indicator(int64_t n, const double* u, int8_t* chi) {
    for (int64_t r = blockIdx.x * (int64_t)kBlock + threadIdx.x; r < n; r += (int64_t)gridDim.x * kBlock)
        chi[r] = (u[r] < 0.0) ? (int8_t)-1 : (int8_t)1;
}

template <typename T, int FMT>
void launch_forms(scg_ctx* c, const double* U, int RBsel) {
    const int32_t* rp[4] = {c->rp_seg[0], c->rp_seg[0], c->rp_seg[0], c->rp_seg[0]};
    for (int s = 0; s < c->nseg; ++s) rp[s] = c->rp_seg[s];
    const dim3 g(c->G), b(kBlock);
    if (RBsel == 8)
        hipLaunchKernelGGL((k_cut_forms<T, FMT, 8>), g, b, 0, c->stream, (int64_t)c->n, c->nseg, rp[0], rp[1], rp[2],
                           rp[3], c->col, (const T*)c->val, c->cval, c->dC, U, c->prm.R, c->part);
    else
        hipLaunchKernelGGL((k_cut_forms<T, FMT, kRMax>), g, b, 0, c->stream, (int64_t)c->n, c->nseg, rp[0], rp[1],
                           rp[2], rp[3], c->col, (const T*)c->val, c->cval, c->dC, U, c->prm.R, c->part);
}

template <typename T>
void launch_forms_t(scg_ctx* c, const double* U, int RBsel) {
    if (c->fmt == FMT_PAT) launch_forms<T, FMT_PAT>(c, U, RBsel);
    else if (c->fmt == FMT_SGN) launch_forms<T, FMT_SGN>(c, U, RBsel);
    else launch_forms<T, FMT_VAL>(c, U, RBsel);
}

}  // namespace

extern "C" scg_status sketchycgal_round(scg_ctx* c, const double* U, int8_t* chi, double* weights, int32_t* best) {
    if (!c || !U || !weights || !best) return SCG_EINVAL;
    const int R = c->prm.R;
    const int RBsel = (R <= 8) ? 8 : kRMax;
    if (c->prm.precision == SCG_FP32_STREAM) launch_forms_t<float>(c, U, RBsel);
    else launch_forms_t<double>(c, U, RBsel);
    if (hipGetLastError() != hipSuccess) return SCG_EHIP;
    std::vector<double> h((size_t)c->G * (RBsel + 1));
    if (hipMemcpyAsync(h.data(), c->part, sizeof(double) * h.size(), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
        return SCG_EHIP;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return SCG_EHIP;
    double tr = 0.0;
    std::vector<double> q(R, 0.0);
    for (int g = 0; g < c->G; ++g) {
        for (int j = 0; j < R; ++j) q[j] += h[(size_t)g * (RBsel + 1) + j];
        tr += h[(size_t)g * (RBsel + 1) + RBsel];
    }
    int bi = 0;
    for (int j = 0; j < R; ++j) {
        weights[j] = -c->c_F * (q[j] + tr);   // original units
        if (weights[j] > weights[bi]) bi = j;
    }
    *best = bi;
    if (chi) {
        hipLaunchKernelGGL(k_cut_indicator, dim3(c->G), dim3(kBlock), 0, c->stream, (int64_t)c->n,
                           U + (int64_t)bi * c->n, chi);
        if (hipGetLastError() != hipSuccess) return SCG_EHIP;
        if (hipStreamSynchronize(c->stream) != hipSuccess) return SCG_EHIP;
    }
    return SCG_OK;
}
