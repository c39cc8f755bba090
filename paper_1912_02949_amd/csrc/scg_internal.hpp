// Internal layout shared by the SketchyCGAL host runtime and its kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>

#include "../../include/sketchycgal.h"

namespace scg {

constexpr int kQCap = 512;     // maximum Lanczos steps per call
constexpr int kRMax = 32;      // maximum sketch size R
constexpr int kNB = 512;       // nonzeros staged through LDS per row block (one wave)
constexpr int kRowsCap = 128;  // rows per row block
constexpr int kGMax = 2048;    // workgroups of a streaming launch
constexpr int kSegMax = 8;     // column segments of the SpMV (8: one per XCD, run concurrently)

// Storage of the off-diagonal values of C.
enum MatFmt {
    FMT_VAL = 0,   // one value per nonzero
    FMT_PAT = 1,   // every off-diagonal value equals cval: columns only
    FMT_SGN = 2    // every |value| equals cval: column with the sign in bit 31
};

// Scalars of the current iteration, resident in device memory.  Indexing of
// the Lanczos run: basis vector V[j] (j = 0 .. k-1) is stored unnormalised;
// inv[j] is the factor that normalises it.  omega[j] = v_j^T M v_j,
// rho[j] = norm of the vector that becomes V[j+1].
struct DevScalars {
    double omega[kQCap];
    double rho[kQCap];
    double inv[kQCap + 1];
    double coef[kQCap];       // Ritz coefficients u_j * inv[j]
    double h[kQCap];          // reorthogonalisation coefficients
    double comega[kRMax];     // v^T Omega for the normalised Ritz vector
    double xi, vnorm2, inv_vnorm, cv, resid2;
    double p, tau, gamma_eff;
    double d_yb, d_zz, d_gapdot, d_zb2, b2;   // state before the update
    double sum_sq, sum_b;                      // init: sum C_ij^2, sum b
    double c_F, alpha_s;
    int32_t k, done, flags, t_done;
    int32_t err;                               // init validation bits
    int32_t kr;                                // Lanczos steps of the current Ritz vector
    int32_t t_iter;                            // iteration of a replayed graph (IterArgs.dev)
};

// Problem description passed by value to kernels.
template <typename T>
struct Prob {
    int64_t n;
    int R;
    const int32_t* rp;    // off-diagonal CSR, int32[n+1]
    const int32_t* col;
    const T* val;
    double cval;          // the common (absolute) off-diagonal value, FMT_PAT / FMT_SGN
    const double* dC;     // diagonal of C (scaled)
    const double* b;      // scaled b
    const double* lo;     // box constraint set (scaled), or null: K = {b}
    const double* hi;
    int ball;             // 1: K is the ball {||u - b|| <= ball_r} (l2), centred at b
    double ball_r;        // its radius, scaled
    int trace_mode;       // 0: tr X = alpha; 1: tr X <= alpha
    double* z;
    double* y;
    T* s;                 // diagonal shift of D: dC + y + beta (z - b)
    int64_t ld;           // column stride of V, Omega, S: n rounded up to 64
    T* V;                 // Lanczos basis, (qmax+1) columns of stride ld, or 3 rotating columns (vmod = 3)
    int vmod;             // 0: column i at i*ld; 3: column i at (i mod 3)*ld (basis regenerated)
    double* racc;         // Ritz vector accumulator, FP64 (basis regenerated), else null
    T* u;                 // SpMV output
    T* v;                 // Ritz vector (unnormalised)
    const T* Om;          // Omega, n x R column-major (column c at c*ld), or null: generated from Philox
    uint64_t seed, instance;   // Philox key and counter word of Omega (and the start vectors)
    T* S;                 // sketch, n x R column-major (column c at c*ld)
    const int32_t* rb;    // row-block boundaries, int32[nrb+1]
    int nrb;
    const int32_t* qw;    // chunk layouts: column words, 64 quads per chunk
    const T* qv;          // entry-chunk layout: values beside the words
    const int2* qc;       // per chunk: (first row, quads used)
    int64_t nqc;          // chunks
    DevScalars* sc;
    // per-workgroup partial sums, one buffer per producing kernel
    double* p_prep;       // k_prep,        G  x 6
    double* p_spmv;       // k_spmv LANCZOS, Gs x 1
    double* p_upd;        // k_lupdate / k_reorth_apply, G x 1
    double* p_ritz;       // k_ritz,        G  x (RB + 1)
    double* p_obj;        // k_spmv OBJ,    Gs x 2
    double* p_primal;     // k_primal,      G  x 4
    double* p_ball;       // k_ball_norm,   G  x 1
    double* p_ball2;      // k_ball_r2,     G  x 3
    double* p_h;          // k_reorth_dot,  G  x (step + 1)
    int G;                // workgroups of the vector kernels
    int Gs;               // workgroups of the SpMV kernels
    scg_iter_log* logs;
    int T_iters;
};

template <typename T>
__device__ __forceinline__ T* vcol(const Prob<T>& P, int i) {
    return P.V + (size_t)(P.vmod ? i % P.vmod : i) * P.ld;
}

}  // namespace scg

struct scg_ctx {
    scg_params prm;
    int64_t n, nnz_in, nnz_off;
    int64_t ld;     // padded column stride of V, Omega, S
    hipStream_t stream;
    int device;
    int t_next;
    int qmax;
    int G;          // workgroups for vector kernels
    int Gs;         // workgroups for SpMV kernels
    int lanes;      // lanes per row in the SpMV row reduction; 1: the quad-chunk product
    int nseg;       // column segments (1, 2, 4 or 8): segment s gathers only x[s*seglen, (s+1)*seglen)
    bool xseg;      // 8 segments in one launch, segment s on XCD s, partial row sums combined by a second pass
    int64_t seglen;
    int32_t* rp_seg[scg::kSegMax];   // per segment: row pointers into col/val (absolute)
    int2* rbd_seg[scg::kSegMax];     // per segment: row-block descriptors (first row, first nonzero)
    int nrb_seg[scg::kSegMax];
    size_t rb_cap;  // int2 entries available in the row-block area
    int fmt;        // MatFmt of the off-diagonal part
    double cval;    // common (absolute) off-diagonal value, scaled
    int nrb;
    double alpha_orig;
    double c_F;
    double alpha_s;
    // device memory carved from the workspace
    int32_t* rp;
    int32_t* col;
    void* val;
    double* dC;
    double* b;
    double* z;
    double* y;
    void* s;
    void* V;
    void* u;
    void* v;
    void* xpart;    // per-segment raw row sums of the concurrent-segment product (kSegMax x ld), or null
    void* Om;
    void* S;
    int32_t* rb;
    scg::DevScalars* sc;
    double* part;       // partial sums (iteration kernels use fixed slices of it)
    unsigned* counter;  // last-workgroup ticket (initialisation and reconstruction)
    scg_iter_log* logs;
    double* recon;   // reconstruction scratch (n x R FP64 and small matrices)
    double* racc;    // FP64 Ritz accumulator (regenerated basis), else null
    double ball_r;   // radius of the ball constraint set, scaled (constraint_set = 2)
    double* lo;      // box constraint set, scaled (constraint_set = 1), else null
    double* hi;
    size_t recon_bytes;
    // chunk layouts of the off-diagonal entries: padded quads of column words (one
    // off-diagonal magnitude) or unpadded entries with their values (values stored)
    int32_t* qw;     // column words, 256 per chunk (null when not reserved)
    void* qv;        // values of the entry-chunk layout, 256 per chunk (null when not reserved)
    int2* qc;        // per chunk: (first row, quads used)
    int64_t nqc;     // chunks built (0: the matrix does not qualify)
    int64_t qc_cap;  // chunks reserved
    // the sliced entry-chunk layout of the concurrent column segments (spmv_lanes 1, segments 8)
    int32_t* xqw;    // column words, 256 per chunk (null when not reserved)
    void* xqv;       // values beside them
    int2* xqc;       // per chunk: (first row, quads used)
    int64_t xqc_cap; // chunks reserved
    int64_t nxc;     // chunks built (0: not built)
    int64_t xcb[scg::kSegMax + 1];   // chunks of slice s: [xcb[s], xcb[s + 1])
    int4* xlseg;     // long segments: (row, first entry, entries, unused)
    int64_t xlseg_cap;
    int32_t* xlw;    // their column words (at most nnz)
    void* xlv;       // and values
    int64_t xlb[scg::kSegMax + 1];   // long segments of slice s: [xlb[s], xlb[s + 1])
    std::map<int, hipGraphExec_t> graphs;   // one captured iteration per Lanczos step count q (non-null stream)
};

// Arguments of the FP64 Nystrom reconstruction of one sketch (column-major
// S and Omega with column stride ld, storage type by fp32).
struct ReconArgs {
    int64_t n, ld;
    int R, fp32, trace_correct;
    const void* S;
    const void* Om;       // or null: Omega generated from Philox (seed, instance)
    uint64_t seed, instance;
    double tau, alpha;
    double* scratch;      // scg_recon_scratch_doubles(n, R) doubles
    unsigned* counter;    // zeroed ticket word
    hipStream_t stream;
    double* U;            // n x R column-major (stride n)
    double* lambda;       // R
    double* err;          // R or NULL
};
size_t scg_recon_scratch_doubles(int64_t n, int R);
scg_status scg_reconstruct_generic(const ReconArgs& a);
