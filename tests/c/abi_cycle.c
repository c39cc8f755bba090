/*
 * A plain C consumer of include/sketchycgal.h: the MaxCut SDP of the 9-cycle,
 * whose value is (9/2)(1 + cos(pi/9)) (odd cycles, Delorme and Poljak), solved
 * by SketchyCGAL (alg:sketchy-cgal), reconstructed (alg:nystrom-sketch-supp)
 * and rounded to cuts (Section 7.2) through the C ABI alone: the caller owns
 * every device buffer, including the workspace.  Exit status 0 on success.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>

#include <hip/hip_runtime_api.h>

#include "sketchycgal.h"

#define N 9
#define NNZ (3 * N)

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

int main(void) {
    /* C = -L/4 of the unit-weight cycle: -1/2 on the diagonal, +1/4 between neighbours */
    int64_t rp[N + 1];
    int32_t col[NNZ];
    double val[NNZ], b[N];
    int64_t e = 0;
    for (int i = 0; i < N; ++i) {
        int nb[3] = {(i + N - 1) % N, i, (i + 1) % N};
        for (int a = 0; a < 3; ++a)   /* columns in increasing order */
            for (int c = a + 1; c < 3; ++c)
                if (nb[c] < nb[a]) { int t = nb[a]; nb[a] = nb[c]; nb[c] = t; }
        rp[i] = e;
        for (int a = 0; a < 3; ++a) {
            col[e] = nb[a];
            val[e] = (nb[a] == i) ? -0.5 : 0.25;
            ++e;
        }
        b[i] = 1.0;
    }
    rp[N] = e;

    int64_t* d_rp;
    int32_t* d_col;
    double *d_val, *d_b, *d_U, *d_lam, *d_err;
    int8_t* d_chi;
    HCHECK(hipMalloc((void**)&d_rp, sizeof(rp)));
    HCHECK(hipMalloc((void**)&d_col, sizeof(col)));
    HCHECK(hipMalloc((void**)&d_val, sizeof(val)));
    HCHECK(hipMalloc((void**)&d_b, sizeof(b)));
    HCHECK(hipMemcpy(d_rp, rp, sizeof(rp), hipMemcpyHostToDevice));
    HCHECK(hipMemcpy(d_col, col, sizeof(col), hipMemcpyHostToDevice));
    HCHECK(hipMemcpy(d_val, val, sizeof(val), hipMemcpyHostToDevice));
    HCHECK(hipMemcpy(d_b, b, sizeof(b), hipMemcpyHostToDevice));

    scg_params p;
    scg_default_params(&p);
    p.R = 4;
    p.T = 2000;
    p.seed = 1;
    size_t ws = 0;
    CHECK(scg_workspace_size(&p, N, NNZ, &ws));
    void* work;
    HCHECK(hipMalloc(&work, ws));   /* hipMalloc memory is 256-byte aligned */

    scg_ctx* ctx = NULL;
    CHECK(sketchycgal_init(&ctx, &p, N, NNZ, d_rp, d_col, d_val, d_b, NULL, work, ws, NULL));
    CHECK(sketchycgal_step(ctx, p.T));
    scg_summary s;
    CHECK(sketchycgal_summary(ctx, &s));

    HCHECK(hipMalloc((void**)&d_U, sizeof(double) * N * 4));
    HCHECK(hipMalloc((void**)&d_lam, sizeof(double) * 4));
    HCHECK(hipMalloc((void**)&d_err, sizeof(double) * 4));
    HCHECK(hipMalloc((void**)&d_chi, N));
    CHECK(sketchycgal_reconstruct(ctx, d_U, d_lam, d_err));
    double weights[4];
    int32_t best = -1;
    CHECK(sketchycgal_round(ctx, d_U, d_chi, weights, &best));
    double lam[4];
    HCHECK(hipMemcpy(lam, d_lam, sizeof(lam), hipMemcpyDeviceToHost));
    sketchycgal_destroy(ctx);

    const double sdp = 4.5 * (1.0 + cos(acos(-1.0) / 9.0));
    const double cut = -s.objective;
    const double lam_sum = lam[0] + lam[1] + lam[2] + lam[3];
    printf("abi_cycle: SDP value %.6f (closed form %.6f), t_done %d, lambda sum %.12f, best rounded cut %.1f\n",
           cut, sdp, s.t_done, lam_sum, weights[best]);
    int ok = fabs(cut - sdp) / sdp < 2e-3 && s.t_done == p.T && fabs(lam_sum - 1.0) < 1e-12 && best >= 0 &&
             best < 4 && weights[best] <= 8.0 + 1e-9 && weights[best] >= 0.878 * sdp;

    hipFree(work);
    hipFree(d_rp);
    hipFree(d_col);
    hipFree(d_val);
    hipFree(d_b);
    hipFree(d_U);
    hipFree(d_lam);
    hipFree(d_err);
    hipFree(d_chi);
    return ok ? 0 : 1;
}
