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
#include <mutex>
#include <vector>

#include "scg_device.hpp"
#include "scg_internal.hpp"

using namespace scg;

namespace {

__device__ __forceinline__ double sgn1(double u) { return (u < 0.0) ? -1.0 : 1.0; }

// Row pointers of the column segments the stored matrix is split into.
struct SegRows {
    const int32_t* rp[kSegMax];
};

// Partials per workgroup: [0, R) sum_r chi_j(r) (C_off chi_j)_r in scaled units, [R] sum_r diag_r.
template <typename T, int FMT, int RB>
__global__ __launch_bounds__(kBlock) void k_cut_forms(int64_t n, int nseg, SegRows sr, const int32_t* col,
                                                      const T* val, double cval, const double* dC, const double* U,
                                                      int R, double* part) {
    __shared__ double red[kWaves];
    double acc[RB + 1];
#pragma unroll
    for (int j = 0; j <= RB; ++j) acc[j] = 0.0;
    for (int64_t r = blockIdx.x * (int64_t)kBlock + threadIdx.x; r < n; r += (int64_t)gridDim.x * kBlock) {
        double off[RB];
#pragma unroll
        for (int j = 0; j < RB; ++j) off[j] = 0.0;
        for (int sg = 0; sg < nseg; ++sg) {
            const int32_t* rp = sr.rp[sg];
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
    SegRows sr{};
    for (int s = 0; s < kSegMax; ++s) sr.rp[s] = c->rp_seg[(s < c->nseg) ? s : 0];
    const dim3 g(c->G), b(kBlock);
    if (RBsel == 8)
        hipLaunchKernelGGL((k_cut_forms<T, FMT, 8>), g, b, 0, c->stream, (int64_t)c->n, c->nseg, sr, c->col,
                           (const T*)c->val, c->cval, c->dC, U, c->prm.R, c->part);
    else
        hipLaunchKernelGGL((k_cut_forms<T, FMT, kRMax>), g, b, 0, c->stream, (int64_t)c->n, c->nseg, sr, c->col,
                           (const T*)c->val, c->cval, c->dC, U, c->prm.R, c->part);
}

template <typename T>
void launch_forms_t(scg_ctx* c, const double* U, int RBsel) {
    if (c->fmt == FMT_PAT) launch_forms<T, FMT_PAT>(c, U, RBsel);
    else if (c->fmt == FMT_SGN) launch_forms<T, FMT_SGN>(c, U, RBsel);
    else launch_forms<T, FMT_VAL>(c, U, RBsel);
}

// ---------------------------------------------------------------------------
// The same rounding without a context or workspace (scg_round_csr): the cut
// forms are evaluated on the caller's CSR in FP64 (diagonal included), and the
// per-workgroup partial sums go to `scratch`, a static device array the
// library holds on every device it runs on until the process ends.  Host code
// reaches it only through the address hipGetSymbolAddress returns for the
// current device; the array's name is not a device address on the host.
constexpr int kRoundG = 1024;                          // workgroups of the scratch launch (at most)
constexpr int kRoundW = kRMax + 1;                     // partials per workgroup: R forms + bounds flag
constexpr size_t kRoundScratch = (size_t)kRoundG * kRoundW;   // doubles (264 KiB)
static __device__ __align__(256) double scratch[kRoundScratch];

// Partials per workgroup g: part[g * kRoundW + j] = sum over its rows r of
// chi_j(r) (C chi_j)_r for j < R (C with its diagonal), part[g * kRoundW + kRMax]
// = 1 if a row pointer or a column index of its rows is out of range (those
// entries are skipped, never read), else 0.  Every slot the host reads is
// written by this launch, so nothing needs clearing between calls.
template <int RB>
__global__ __launch_bounds__(kBlock) void k_cut_forms_csr(int64_t n, int64_t nnz, const int64_t* rp,
                                                          const int32_t* col, const double* val, const double* U,
                                                          int R, double* part) {
    __shared__ double red[kWaves];
    double acc[RB];
#pragma unroll
    for (int j = 0; j < RB; ++j) acc[j] = 0.0;
    double bad = 0.0;
    for (int64_t r = blockIdx.x * (int64_t)kBlock + threadIdx.x; r < n; r += (int64_t)gridDim.x * kBlock) {
        int64_t e0 = rp[r], e1 = rp[r + 1];
        if (e0 < 0 || e1 < e0 || e1 > nnz) {
            bad = 1.0;
            e1 = e0;
        }
        double row[RB];
#pragma unroll
        for (int j = 0; j < RB; ++j) row[j] = 0.0;
        for (int64_t e = e0; e < e1; ++e) {
            const int32_t c = col[e];
            if (c < 0 || (int64_t)c >= n) {
                bad = 1.0;
                continue;
            }
            const double v = val[e];
#pragma unroll
            for (int j = 0; j < RB; ++j)
                if (j < R) row[j] += v * sgn1(U[(int64_t)j * n + c]);
        }
#pragma unroll
        for (int j = 0; j < RB; ++j)
            if (j < R) acc[j] += sgn1(U[(int64_t)j * n + r]) * row[j];
    }
#pragma unroll
    for (int j = 0; j < RB; ++j) {
        const double s = block_sum(acc[j], red);
        if (threadIdx.x == 0) part[(size_t)blockIdx.x * kRoundW + j] = s;
    }
    const double sb = block_sum(bad, red);
    if (threadIdx.x == 0) part[(size_t)blockIdx.x * kRoundW + kRMax] = sb;
}

// Device address of `scratch` on each device, taken once per device with that
// device current.
double* scratch_address(int dev) {
    static std::mutex mu;
    static std::vector<double*> addr;
    std::lock_guard<std::mutex> lock(mu);
    if (dev < 0) return nullptr;
    if ((size_t)dev >= addr.size()) addr.resize((size_t)dev + 1, nullptr);
    if (!addr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        addr[dev] = static_cast<double*>(ptr);
    }
    return addr[dev];
}

}  // namespace

extern "C" scg_status scg_round_csr(int64_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col,
                                    const double* val, int32_t R, const double* U, int8_t* chi, double* weights,
                                    int32_t* best, void* stream) {
    if (n < 1 || nnz < 0 || R < 1 || R > kRMax || R > n || !row_ptr || (nnz > 0 && (!col || !val)) || !U ||
        !weights || !best)
        return SCG_EINVAL;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return SCG_EHIP;
    double* part = scratch_address(dev);
    if (!part) return SCG_EHIP;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int G = (int)std::min<int64_t>(kRoundG, std::max<int64_t>(1, (n + kBlock - 1) / kBlock));
    if (R <= 8)
        hipLaunchKernelGGL((k_cut_forms_csr<8>), dim3(G), dim3(kBlock), 0, st, n, nnz, row_ptr, col, val, U, R, part);
    else
        hipLaunchKernelGGL((k_cut_forms_csr<kRMax>), dim3(G), dim3(kBlock), 0, st, n, nnz, row_ptr, col, val, U, R,
                           part);
    if (hipGetLastError() != hipSuccess) return SCG_EHIP;
    std::vector<double> h((size_t)G * kRoundW);
    if (hipMemcpyAsync(h.data(), part, sizeof(double) * h.size(), hipMemcpyDeviceToHost, st) != hipSuccess)
        return SCG_EHIP;
    if (hipStreamSynchronize(st) != hipSuccess) return SCG_EHIP;
    std::vector<double> q(R, 0.0);
    for (int g = 0; g < G; ++g) {
        if (h[(size_t)g * kRoundW + kRMax] != 0.0) return SCG_EINVAL;
        for (int j = 0; j < R; ++j) q[j] += h[(size_t)g * kRoundW + j];
    }
    int bi = 0;
    for (int j = 0; j < R; ++j) {
        weights[j] = -q[j];
        if (weights[j] > weights[bi]) bi = j;
    }
    *best = bi;
    if (chi) {
        const int Gi = (int)std::min<int64_t>(2048, std::max<int64_t>(1, (n + kBlock - 1) / kBlock));
        hipLaunchKernelGGL(k_cut_indicator, dim3(Gi), dim3(kBlock), 0, st, n, U + (int64_t)bi * n, chi);
        if (hipGetLastError() != hipSuccess) return SCG_EHIP;
        if (hipStreamSynchronize(st) != hipSuccess) return SCG_EHIP;
    }
    return SCG_OK;
}

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
