// HIP kernels (gfx950) of the cooperative CG library that are not the A.D stream:
// layout conversions, low-precision copies of A, refinement steps, and the
// launchers of every kernel (the A.D launchers dispatch to the per-precision
// translation units).
#include "ccg_kernels.h"

#include <algorithm>

#include "ccg_tune_table.h"

namespace ccg {

// ======================================================== layout conversions

// Xr (agent-major n_pad x P, zero padded) <- X (n x p column-major, ldx)
__global__ void k_pack(int n, int n_pad, int p, int P, const double* X, int64_t ldx, double* Xr) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n_pad * P) return;
    const int j = (int)(idx / n_pad);
    const int64_t i = idx - (int64_t)j * n_pad;
    Xr[idx] = (i < n && j < p) ? X[i + j * ldx] : 0.0;
}

__global__ void k_unpack(int n, int n_pad, int p, const double* Xr, double* X, int64_t ldx) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * p) return;
    const int j = (int)(idx / n);
    const int64_t i = idx - (int64_t)j * n;
    X[i + j * ldx] = Xr[(int64_t)j * n_pad + i];
}

__global__ void k_pad_vec(int n, int n_pad, const double* b, double* bp) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_pad) bp[i] = (i < n) ? b[i] : 0.0;
}

// Copy a column-major matrix into one whose leading dimension keeps every column
// 16-byte aligned.
__global__ void k_copy_cols(int n, const double* A, int64_t lda, double* B, int64_t ldb) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * n) return;
    const int64_t c = idx / n, r = idx - c * n;
    B[c * ldb + r] = A[c * lda + r];
}

// ============================================== low-precision copies of A
//
// The FP32 mode streams A32 = A rounded to nearest (ties to even).  The BF16x2 mode
// streams two BF16 planes, hi = A rounded to nearest-even BF16 and lo = (A - hi)
// rounded the same way (A - hi is exact in FP64), so that hi + lo carries 16
// significant bits.  Columns are written with leading dimension ldb (>= n; rows
// n..ldb-1 are zero-filled so 16-byte loads of a column tail read zeros).

// Nearest-even BF16 of a double, rounding once: the double is first cut to FP32
// toward zero with a sticky bit in the last place (round to odd), which keeps the
// information a single rounding needs, then rounded to 8 significant bits.
__device__ __forceinline__ uint16_t bf16_rne(double a) {
    const float f = __double2float_rz(a);
    uint32_t u = __float_as_uint(f);
    if ((double)f != a) u |= 1u;
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__global__ void k_to_f32(int n, const double* A, int64_t lda, float* B, int64_t ldb) {
    const int64_t tot = (int64_t)n * ldb;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < tot;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = idx / ldb, r = idx - c * ldb;
        B[idx] = r < n ? (float)A[c * lda + r] : 0.0f;
    }
}

__global__ void k_to_bf16x2(int n, const double* A, int64_t lda, uint16_t* H, uint16_t* L, int64_t ldb) {
    const int64_t tot = (int64_t)n * ldb;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < tot;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = idx / ldb, r = idx - c * ldb;
        uint16_t h = 0, l = 0;
        if (r < n) {
            const double a = A[c * lda + r];
            h = bf16_rne(a);
            const double hv = (double)__uint_as_float((uint32_t)h << 16);
            l = bf16_rne(a - hv);
        }
        H[idx] = h;
        L[idx] = l;
    }
}

// ================================================= synthetic inputs of the tuner
//
// A symmetric, strictly diagonally dominant n x n matrix (so D^T A D is SPD for any
// full-rank D) and pseudo-random vector blocks, from a counter hash: timing only.
__device__ __forceinline__ double tune_hash(uint64_t x) {
    x *= 0x9E3779B97F4A7C15ull;
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    return (double)(x & 0xffffff) / 16777216.0 - 0.5;
}

__global__ void k_tune_matrix(int n, double* A, int64_t lda) {
    const int64_t tot = (int64_t)n * n;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < tot;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = idx / n, r = idx - c * n;
        const int64_t lo = r < c ? r : c, hi = r < c ? c : r;
        A[c * lda + r] = tune_hash((uint64_t)lo * 1000003ull + (uint64_t)hi) + (r == c ? (double)n : 0.0);
    }
}

__global__ void k_tune_vectors(int64_t cnt, double* d64, float* d32, unsigned seed) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x) {
        const double v = tune_hash((uint64_t)i + ((uint64_t)seed << 40));
        if (d64) d64[i] = v;
        if (d32) d32[i] = (float)v;
    }
}

hipError_t launch_tune_matrix(int n, double* A, int64_t lda, hipStream_t s) {
    const int64_t tot = (int64_t)n * n;
    hipLaunchKernelGGL(k_tune_matrix, dim3((unsigned)std::min<int64_t>((tot + 255) / 256, 8192)), dim3(256), 0, s,
                       n, A, lda);
    return hipGetLastError();
}

hipError_t launch_tune_vectors(int64_t cnt, double* d64, float* d32, unsigned seed, hipStream_t s) {
    hipLaunchKernelGGL(k_tune_vectors, dim3((unsigned)std::min<int64_t>((cnt + 255) / 256, 4096)), dim3(256), 0, s,
                       cnt, d64, d32, seed);
    return hipGetLastError();
}

// ============================== refinement: start an inner solve / apply it
//
// k_inner_init: R = T_j / scale_j (rounded to FP32), D = R, E = 0 for every element
// of the padded block (agents with scale 0 get zero columns).
// k_refine_add: X += E_j * scale_j in FP64.
__global__ void k_inner_init(RefArgs a) {
    const int64_t tot = (int64_t)a.n_pad * a.P;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= tot) return;
    const int j = (int)(idx / a.n_pad);
    const double s = a.scale[j];
    const float r = s > 0.0 ? (float)(a.T[idx] / s) : 0.0f;
    static_cast<float*>(a.R)[idx] = r;
    static_cast<float*>(a.D)[idx] = r;
    static_cast<float*>(a.E)[idx] = 0.0f;
}

__global__ void k_refine_add(RefArgs a) {
    const int64_t tot = (int64_t)a.n_pad * a.P;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= tot) return;
    const int j = (int)(idx / a.n_pad);
    const double s = a.scale[j];
    if (s > 0.0) a.X[idx] = fma((double)static_cast<const float*>(a.E)[idx], s, a.X[idx]);
}

// ================================================== re-inflation of dropped agents
//
// X[:, j] = X[:, best] + d for every agent j in `dropped`, d_i = 2 (z_i >> 11) 2^-53 - 1
// with z_i the (i+1)-th output of SplitMix64 (Steele, Lea, Flood 2014) from the state
// 0x1204 << 48 ^ e << 32 ^ j: the generator's state after i+1 steps is the start
// plus (i+1) golden-ratio increments, so each entry is drawn on its own.  Row i of
// every column is handled by one thread, which reads X[i, best] before any write.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t state0, uint64_t k) {
    uint64_t z = state0 + k * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void k_reinflate(int n, int n_pad, int p, unsigned dropped, int best, int event, double* Xr) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double xb = Xr[(int64_t)best * n_pad + i];
    for (int j = 0; j < p; ++j) {
        if (!((dropped >> j) & 1u)) continue;
        const uint64_t s0 = (0x1204ull << 48) ^ ((uint64_t)event << 32) ^ (uint64_t)j;
        const uint64_t z = splitmix64_at(s0, (uint64_t)i + 1);
        const double d = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
        Xr[(int64_t)j * n_pad + i] = xb + d;
    }
}

hipError_t launch_reinflate(int n, int n_pad, int p, unsigned dropped, int best, int event, double* Xr,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_reinflate, dim3((n + 255) / 256), dim3(256), 0, s, n, n_pad, p, dropped, best, event, Xr);
    return hipGetLastError();
}

// ================================================================== launchers

// A columns per wave and waves per workgroup of the A.D tile for a system: the
// tuning table's choice for (precision, padded agent count, n), else 2 and 4.
static const TuneRow* tune_row(int prec, int P, int n) {
    for (const TuneRow& r : kTuneTable)
        if (r.prec == prec && r.P == P && n <= r.n_max) return &r;
    return nullptr;
}
int ad_cw(int prec, int P, int n) {
    const TuneRow* r = tune_row(prec, P, n);
    return r ? ad_cw_fit(prec, P, r->cw, r->nw) : 2;
}
int ad_nw(int prec, int P, int n) {
    const TuneRow* r = tune_row(prec, P, n);
    return r ? ad_nw_fit(prec, P, r->nw) : 4;
}

// AD rows per A.D tile of a requested shape, as the launchers run it.
int ad_fit_rows(int prec, int P, int cw, int nw) { return ad_cw_fit(prec, P, cw, nw) * ad_nw_fit(prec, P, nw); }
int ad_fit_cw(int prec, int P, int cw, int nw) { return ad_cw_fit(prec, P, cw, nw); }
int ad_fit_nw(int prec, int P, int nw) { return ad_nw_fit(prec, P, nw); }

template <int PREC, int P>
static hipError_t launch_upd_t(const UpdArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((k_upd<PREC, P>), dim3(upd_blocks(a.n_pad, P)), dim3(kWG), 0, s, a);
    return hipGetLastError();
}
template <int PREC, int P>
static hipError_t launch_dir_t(const UpdArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((k_dir<PREC, P>), dim3(upd_blocks(a.n_pad, P)), dim3(kWG), 0, s, a);
    return hipGetLastError();
}
template <int P>
static hipError_t launch_res_t(const ResArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((k_res<P>), dim3(a.n_pad / (kWG / P)), dim3(kWG), 0, s, a);
    return hipGetLastError();
}

#define CCG_DISPATCH_P(P, CALL)                                        \
    switch (P) {                                                       \
        case 1: return CALL(1);                                        \
        case 2: return CALL(2);                                        \
        case 4: return CALL(4);                                        \
        case 8: return CALL(8);                                        \
        case 16: return CALL(16);                                      \
        default: return hipErrorInvalidValue;                          \
    }

// FP64 single systems also run P = 32 (the batched engine takes p <= 16)
#define CCG_DISPATCH_P64(P, CALL)                                      \
    switch (P) {                                                       \
        case 1: return CALL(1);                                        \
        case 2: return CALL(2);                                        \
        case 4: return CALL(4);                                        \
        case 8: return CALL(8);                                        \
        case 16: return CALL(16);                                      \
        case 32: return CALL(32);                                      \
        default: return hipErrorInvalidValue;                          \
    }

static hipError_t launch_ad_any(int prec, int P, int cw, int nw, const AdArgs* one, const AdArgs* sys,
                                const int4* items, int nitems, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    switch (prec) {
        case PREC_F64: return launch_ad_f64(P, cw, nw, one, sys, items, nitems, s, e0, e1);
        case PREC_F32: return launch_ad_f32(P, cw, nw, one, sys, items, nitems, s, e0, e1);
        case PREC_BF16X2: return launch_ad_bf16(P, cw, nw, one, sys, items, nitems, s, e0, e1);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_ad(int prec, int P, const AdArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    return launch_ad_any(prec, P, ad_cw(prec, P, a.n), ad_nw(prec, P, a.n), &a, nullptr, nullptr, 0, s, e0, e1);
}

hipError_t launch_ad_cw(int prec, int P, int cw, int nw, const AdArgs& a, hipStream_t s, hipEvent_t e0,
                        hipEvent_t e1) {
    return launch_ad_any(prec, P, cw, nw, &a, nullptr, nullptr, 0, s, e0, e1);
}

hipError_t launch_small(int prec, int P, const SmallArgs* one, const SmallArgs* sys, const int4* items, int nitems,
                        int steps, hipStream_t s) {
    if (!one && nitems <= 0) return hipSuccess;
    switch (prec) {
        case PREC_F64: return launch_small_f64(P, one, sys, items, nitems, steps, s);
        case PREC_F32: return launch_small_f32(P, one, sys, items, nitems, steps, s);
        case PREC_BF16X2: return launch_small_bf16(P, one, sys, items, nitems, steps, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sym(int P, const SymArgs& sa, const AdArgs& a, int nunits, hipStream_t s, hipEvent_t e0,
                      hipEvent_t e1) {
    return launch_sym_f64(P, sa, a, nunits, s, e0, e1);
}

// The strip list of the symmetric pass for nb blocks: strips of kSymW blocks first,
// then the shorter ones at the ends of the block rows.  One thread.
__global__ void k_sym_units(int nb, int2* units) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int u = 0;
    for (int len = kSymW; len >= 1; --len)
        for (int I = 0; I < nb; ++I)
            for (int J0 = I; J0 < nb; J0 += kSymW)
                if (min(kSymW, nb - J0) == len) units[u++] = int2{I, J0};
}

hipError_t launch_sym_units(int nb, int2* units, hipStream_t s) {
    hipLaunchKernelGGL(k_sym_units, dim3(1), dim3(64), 0, s, nb, units);
    return hipGetLastError();
}

hipError_t launch_upd(int prec, int P, const UpdArgs& a, hipStream_t s) {
    switch (prec) {
#define C64(PP) launch_upd_t<PREC_F64, PP>(a, s)
#define C32(PP) launch_upd_t<PREC_F32, PP>(a, s)
        case PREC_F64: CCG_DISPATCH_P64(P, C64)
        case PREC_F32:
        case PREC_BF16X2: CCG_DISPATCH_P(P, C32)
#undef C64
#undef C32
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_dir(int prec, int P, const UpdArgs& a, hipStream_t s) {
    switch (prec) {
#define C64(PP) launch_dir_t<PREC_F64, PP>(a, s)
#define C32(PP) launch_dir_t<PREC_F32, PP>(a, s)
        case PREC_F64: CCG_DISPATCH_P64(P, C64)
        case PREC_F32:
        case PREC_BF16X2: CCG_DISPATCH_P(P, C32)
#undef C64
#undef C32
        default: return hipErrorInvalidValue;
    }
}

template <int PREC, int P>
static hipError_t launch_upd_batch_t(const UpdArgs* sys, const int4* items, int nitems, hipStream_t s) {
    hipLaunchKernelGGL((k_upd_batch<PREC, P>), dim3(nitems), dim3(kWG), 0, s, sys, items);
    return hipGetLastError();
}
template <int PREC, int P>
static hipError_t launch_dir_batch_t(const UpdArgs* sys, const int4* items, int nitems, hipStream_t s) {
    hipLaunchKernelGGL((k_dir_batch<PREC, P>), dim3(nitems), dim3(kWG), 0, s, sys, items);
    return hipGetLastError();
}
template <int P>
static hipError_t launch_res_batch_t(const ResArgs* sys, const int4* items, int nitems, hipStream_t s) {
    hipLaunchKernelGGL((k_res_batch<P>), dim3(nitems), dim3(kWG), 0, s, sys, items);
    return hipGetLastError();
}

// Batched A.D over (system, tile) items whose systems all use `cw` columns per wave
// and `nw` waves per workgroup.
hipError_t launch_ad_batch(int prec, int P, int cw, int nw, const AdArgs* sys, const int4* items, int nitems,
                           hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    return launch_ad_any(prec, P, cw, nw, nullptr, sys, items, nitems, s, nullptr, nullptr);
}

hipError_t launch_upd_batch(int prec, int P, const UpdArgs* sys, const int4* items, int nitems, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    switch (prec) {
#define C64(PP) launch_upd_batch_t<PREC_F64, PP>(sys, items, nitems, s)
#define C32(PP) launch_upd_batch_t<PREC_F32, PP>(sys, items, nitems, s)
        case PREC_F64: CCG_DISPATCH_P(P, C64)
        case PREC_F32:
        case PREC_BF16X2: CCG_DISPATCH_P(P, C32)
#undef C64
#undef C32
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_dir_batch(int prec, int P, const UpdArgs* sys, const int4* items, int nitems, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    switch (prec) {
#define C64(PP) launch_dir_batch_t<PREC_F64, PP>(sys, items, nitems, s)
#define C32(PP) launch_dir_batch_t<PREC_F32, PP>(sys, items, nitems, s)
        case PREC_F64: CCG_DISPATCH_P(P, C64)
        case PREC_F32:
        case PREC_BF16X2: CCG_DISPATCH_P(P, C32)
#undef C64
#undef C32
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_res_batch(int P, const ResArgs* sys, const int4* items, int nitems, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
#define CR(PP) launch_res_batch_t<PP>(sys, items, nitems, s)
    CCG_DISPATCH_P(P, CR)
#undef CR
}

hipError_t launch_res(int P, const ResArgs& a, hipStream_t s) {
#define CR(PP) launch_res_t<PP>(a, s)
    CCG_DISPATCH_P64(P, CR)
#undef CR
}

hipError_t launch_pack(int n, int n_pad, int p, int P, const double* X, int64_t ldx, double* Xr,
                       hipStream_t s) {
    const int64_t tot = (int64_t)n_pad * P;
    hipLaunchKernelGGL(k_pack, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, n_pad, p, P,
                       X, ldx, Xr);
    return hipGetLastError();
}

hipError_t launch_unpack(int n, int n_pad, int p, const double* Xr, double* X, int64_t ldx,
                         hipStream_t s) {
    const int64_t tot = (int64_t)n * p;
    hipLaunchKernelGGL(k_unpack, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, n_pad, p,
                       Xr, X, ldx);
    return hipGetLastError();
}

hipError_t launch_pad_vec(int n, int n_pad, const double* b, double* bp, hipStream_t s) {
    hipLaunchKernelGGL(k_pad_vec, dim3((n_pad + 255) / 256), dim3(256), 0, s, n, n_pad, b, bp);
    return hipGetLastError();
}

hipError_t launch_copy_cols(int n, const double* A, int64_t lda, double* B, int64_t ldb, hipStream_t s) {
    const int64_t tot = (int64_t)n * n;
    hipLaunchKernelGGL(k_copy_cols, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, A, lda, B,
                       ldb);
    return hipGetLastError();
}

hipError_t launch_convert(int prec, int n, const double* A, int64_t lda, void* hi, void* lo, int64_t ldb,
                          hipStream_t s) {
    const int64_t tot = (int64_t)n * ldb;
    const unsigned grid = (unsigned)std::min<int64_t>((tot + 255) / 256, 8192);
    if (prec == PREC_F32) {
        hipLaunchKernelGGL(k_to_f32, dim3(grid), dim3(256), 0, s, n, A, lda, static_cast<float*>(hi), ldb);
    } else if (prec == PREC_BF16X2) {
        hipLaunchKernelGGL(k_to_bf16x2, dim3(grid), dim3(256), 0, s, n, A, lda, static_cast<uint16_t*>(hi),
                           static_cast<uint16_t*>(lo), ldb);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_inner_init(const RefArgs& a, hipStream_t s) {
    const int64_t tot = (int64_t)a.n_pad * a.P;
    hipLaunchKernelGGL(k_inner_init, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_refine_add(const RefArgs& a, hipStream_t s) {
    const int64_t tot = (int64_t)a.n_pad * a.P;
    hipLaunchKernelGGL(k_refine_add, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

// Number of workgroups of each launch (the host sizes reduction scratch with it).
// (an upper bound over every configuration: at least 4 rows per workgroup)
int ad_workgroups(int n) { return (n + 3) / 4; }
int row_workgroups(int n_pad, int P) { return n_pad / (kWG / P); }

}  // namespace ccg
