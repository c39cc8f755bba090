/*
 * A plain C consumer of the phase retrieval ABI (scg_pr_*, include/sketchycgal.h):
 * a 64-dimensional complex signal measured through 12 coded diffraction waveforms
 * (Appendix F.1: entries uniform in {1, i, -1, -i} times sqrt(2)/2 with probability
 * 0.8, else sqrt(3); b_{j,l} = |DFT_n(conj(psi_j) chi)_l|^2, taken here by a direct
 * DFT), recovered by SketchyCGAL (alg:sketchy-cgal over tr X <= alpha), the Nystrom
 * reconstruction and the rounding of Section 7.3.2, all through the C ABI with
 * caller-owned device buffers.  Checks:
 *   - the adjoint identity <A(x x^*), w> = Re(x^* (C + A^*(w)) x) - ||x||^2 / sqrt(n)
 *     between scg_pr_measure and scg_pr_apply (scaled units, C = I / sqrt(n));
 *   - after 600 iterations the rounded signal's relative error (Section 7.3.3) is
 *     below 1e-2, the paper's success criterion, and tr X is within 1% of ||chi||^2.
 * The signal and waveforms come from a 64-bit linear congruential generator
 * (Knuth's MMIX constants).  Exit status 0 on success.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>

#include <hip/hip_runtime_api.h>

#include "sketchycgal.h"

#define N 64
#define L 12
#define NR 4
#define NT 600

#define CHECK(x)                                                                   \
    do {                                                                           \
        scg_status s_ = (x);                                                       \
        if (s_ != SCG_OK) {                                                        \
            fprintf(stderr, "%s: %s\n", #x, scg_status_string(s_));                \
            return 1;                                                              \
        }                                                                          \
    } while (0)
#define HCHECK(x)                                                                  \
    do {                                                                           \
        if ((x) != hipSuccess) {                                                   \
            fprintf(stderr, "%s failed\n", #x);                                    \
            return 1;                                                              \
        }                                                                          \
    } while (0)

static uint64_t lcg_state = 0x2545F4914F6CDD1Dull;

static double uniform(void) {   /* 53-bit uniform in [0, 1) */
    lcg_state = lcg_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg_state >> 11) * 0x1p-53;
}

int main(void) {
    const double pi = 3.14159265358979323846;
    static double chi[2 * N], psi[2 * L * N], b[L * N], w[L * N], m[L * N], y[2 * N];
    double energy = 0.0;
    for (int k = 0; k < N; ++k) {   /* complex standard normal by Box-Muller */
        const double u1 = 1.0 - uniform(), u2 = uniform();
        const double r = sqrt(-2.0 * log(u1)), th = 2.0 * pi * u2;
        chi[2 * k] = r * cos(th) / sqrt(2.0);
        chi[2 * k + 1] = r * sin(th) / sqrt(2.0);
        energy += chi[2 * k] * chi[2 * k] + chi[2 * k + 1] * chi[2 * k + 1];
    }
    for (int j = 0; j < L; ++j)
        for (int k = 0; k < N; ++k) {
            const int ph = (int)(uniform() * 4.0) % 4;
            const double mag = (uniform() < 0.8) ? sqrt(2.0) / 2.0 : sqrt(3.0);
            const double re[4] = {1.0, 0.0, -1.0, 0.0}, im[4] = {0.0, 1.0, 0.0, -1.0};
            psi[2 * (j * N + k)] = re[ph] * mag;
            psi[2 * (j * N + k) + 1] = im[ph] * mag;
        }
    for (int j = 0; j < L; ++j)   /* b_{j,l} = |sum_k e^{-2 pi i l k / N} conj(psi_j(k)) chi(k)|^2 */
        for (int l = 0; l < N; ++l) {
            double ar = 0.0, ai = 0.0;
            for (int k = 0; k < N; ++k) {
                const double pr = psi[2 * (j * N + k)], pim = -psi[2 * (j * N + k) + 1];
                const double xr = pr * chi[2 * k] - pim * chi[2 * k + 1];
                const double xi = pr * chi[2 * k + 1] + pim * chi[2 * k];
                const double a = -2.0 * pi * (double)((l * k) % N) / N;
                ar += cos(a) * xr - sin(a) * xi;
                ai += cos(a) * xi + sin(a) * xr;
            }
            b[j * N + l] = ar * ar + ai * ai;
        }
    for (int i = 0; i < L * N; ++i) w[i] = uniform() - 0.5;

    double *d_psi, *d_b, *d_x, *d_y, *d_w, *d_m, *d_U, *d_lam, *d_err, *d_chi;
    void* d_ws;
    HCHECK(hipMalloc((void**)&d_psi, sizeof(psi)));
    HCHECK(hipMalloc((void**)&d_b, sizeof(b)));
    HCHECK(hipMalloc((void**)&d_x, sizeof(chi)));
    HCHECK(hipMalloc((void**)&d_y, sizeof(y)));
    HCHECK(hipMalloc((void**)&d_w, sizeof(w)));
    HCHECK(hipMalloc((void**)&d_m, sizeof(m)));
    HCHECK(hipMalloc((void**)&d_U, sizeof(double) * 2 * NR * N));
    HCHECK(hipMalloc((void**)&d_lam, sizeof(double) * NR));
    HCHECK(hipMalloc((void**)&d_err, sizeof(double) * NR));
    HCHECK(hipMalloc((void**)&d_chi, sizeof(chi)));
    HCHECK(hipMemcpy(d_psi, psi, sizeof(psi), hipMemcpyHostToDevice));
    HCHECK(hipMemcpy(d_b, b, sizeof(b), hipMemcpyHostToDevice));
    HCHECK(hipMemcpy(d_x, chi, sizeof(chi), hipMemcpyHostToDevice));
    HCHECK(hipMemcpy(d_w, w, sizeof(w), hipMemcpyHostToDevice));

    scg_pr_params p;
    scg_pr_default_params(&p);
    p.R = NR;
    p.T = NT;
    p.seed = 3;
    size_t bytes = 0;
    CHECK(scg_pr_workspace_size(&p, N, L, &bytes));
    HCHECK(hipMalloc(&d_ws, bytes));
    scg_pr_ctx* ctx = NULL;
    CHECK(scg_pr_init(&ctx, &p, N, L, d_psi, d_b, NULL, d_ws, bytes, NULL));

    /* adjoint identity between the measurement and the operator */
    CHECK(scg_pr_measure(ctx, d_x, d_m));
    CHECK(scg_pr_apply(ctx, d_w, d_x, d_y));
    HCHECK(hipMemcpy(m, d_m, sizeof(m), hipMemcpyDeviceToHost));
    HCHECK(hipMemcpy(y, d_y, sizeof(y), hipMemcpyDeviceToHost));
    double lhs = 0.0, rhs = 0.0, scale = 0.0;
    for (int i = 0; i < L * N; ++i) {
        lhs += w[i] * m[i];
        scale += fabs(w[i] * m[i]);
    }
    for (int k = 0; k < N; ++k) rhs += chi[2 * k] * y[2 * k] + chi[2 * k + 1] * y[2 * k + 1];
    rhs -= energy / sqrt((double)N);
    const double adj = fabs(lhs - rhs) / scale;

    CHECK(scg_pr_step(ctx, NT));
    scg_pr_info info;
    CHECK(scg_pr_summary(ctx, &info, 1));
    CHECK(scg_pr_reconstruct(ctx, d_U, d_lam, d_err));
    double rel = -1.0;
    CHECK(scg_pr_round(ctx, d_U, d_lam, d_x, d_chi, &rel));
    printf("abi_phase: adjoint identity %.2e, relative error %.3e, tr X / ||chi||^2 %.6f\n", adj, rel,
           info.objective / energy);
    CHECK(scg_pr_destroy(ctx));
    HCHECK(hipFree(d_ws));
    HCHECK(hipFree(d_psi));
    HCHECK(hipFree(d_b));
    HCHECK(hipFree(d_x));
    HCHECK(hipFree(d_y));
    HCHECK(hipFree(d_w));
    HCHECK(hipFree(d_m));
    HCHECK(hipFree(d_U));
    HCHECK(hipFree(d_lam));
    HCHECK(hipFree(d_err));
    HCHECK(hipFree(d_chi));
    if (!(adj < 1e-12)) return 2;
    if (!(rel >= 0.0 && rel < 1e-2)) return 3;
    if (!(fabs(info.objective / energy - 1.0) < 1e-2)) return 4;
    return 0;
}
