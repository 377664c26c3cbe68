// Internal host-side definitions shared by the single-solve driver (ccg_host.cpp)
// and the multi-system engine (ccg_engine.cpp).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/ccg.h"
#include "ccg_device.h"

namespace ccg {
hipError_t launch_ad(int prec, int P, const AdArgs& a, hipStream_t s, hipEvent_t e0 = nullptr,
                     hipEvent_t e1 = nullptr);
hipError_t launch_upd(int prec, int P, const UpdArgs& a, hipStream_t s);
hipError_t launch_dir(int prec, int P, const UpdArgs& a, hipStream_t s);
hipError_t launch_res(int P, const ResArgs& a, hipStream_t s);
hipError_t launch_pack(int n, int n_pad, int p, int P, const double* X, int64_t ldx, double* Xr,
                       hipStream_t s);
hipError_t launch_unpack(int n, int n_pad, int p, const double* Xr, double* X, int64_t ldx,
                         hipStream_t s);
hipError_t launch_pad_vec(int n, int n_pad, const double* b, double* bp, hipStream_t s);
hipError_t launch_copy_cols(int n, const double* A, int64_t lda, double* B, int64_t ldb, hipStream_t s);
hipError_t launch_convert(int prec, int n, const double* A, int64_t lda, void* hi, void* lo, int64_t ldb,
                          hipStream_t s);
hipError_t launch_inner_init(const RefArgs& a, hipStream_t s);
hipError_t launch_reinflate(int n, int n_pad, int p, unsigned dropped, int best, int event, double* Xr,
                            hipStream_t s);
hipError_t launch_refine_add(const RefArgs& a, hipStream_t s);
hipError_t launch_ad_batch(int prec, int P, int cw, int nw, const AdArgs* sys, const int4* items, int nitems,
                           hipStream_t s);
hipError_t launch_ad_cw(int prec, int P, int cw, int nw, const AdArgs& a, hipStream_t s, hipEvent_t e0 = nullptr,
                        hipEvent_t e1 = nullptr);
int ad_cw(int prec, int P, int n);
int ad_nw(int prec, int P, int n);
hipError_t launch_tune_matrix(int n, double* A, int64_t lda, hipStream_t s);
hipError_t launch_tune_vectors(int64_t cnt, double* d64, float* d32, unsigned seed, hipStream_t s);
hipError_t launch_upd_batch(int prec, int P, const UpdArgs* sys, const int4* items, int nitems, hipStream_t s);
hipError_t launch_dir_batch(int prec, int P, const UpdArgs* sys, const int4* items, int nitems, hipStream_t s);
hipError_t launch_res_batch(int P, const ResArgs* sys, const int4* items, int nitems, hipStream_t s);
int ad_fit_rows(int prec, int P, int cw, int nw);
int ad_fit_cw(int prec, int P, int cw, int nw);
int ad_fit_nw(int prec, int P, int nw);
int ad_workgroups(int n);
int row_workgroups(int n_pad, int P);
hipError_t launch_sym(int P, const SymArgs& sa, const AdArgs& a, int nunits, hipStream_t s, hipEvent_t e0 = nullptr,
                      hipEvent_t e1 = nullptr);
hipError_t launch_sym_units(int nb, int2* units, hipStream_t s);
// the small-system tier: one system (one != nullptr) or a batch of (system) items
hipError_t launch_small(int prec, int P, const SmallArgs* one, const SmallArgs* sys, const int4* items, int nitems,
                        int steps, hipStream_t s);
// Systems with n <= kTierMaxN and P <= kTierMaxP run their block steps in the
// small-system tier, in every path (single, batched, served), unless the caller sets
// CCG_NO_TIER.  The bounds are where one workgroup per step was measured faster than
// the multi-workgroup step on MI355X: from n = 128 on, or at P = 8, the one
// workgroup's latency-bound stream of A costs more than the three launches.
constexpr int kTierMaxN = 96;
constexpr int kTierMaxP = 4;
static_assert(kTierMaxN <= kSmallN && kTierMaxP <= kSmallMaxP, "tier bounds within the kernels' shapes");
inline bool small_tier(int P, int n, unsigned flags) {
    return n <= kTierMaxN && P <= kTierMaxP && !(flags & CCG_NO_TIER);
}
// allocation-free solve: the device scratch array (ccg_noalloc.hip)
size_t scratch_bytes();
hipError_t scratch_setup(int device, void** ptr);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);

// The symmetric A.D pass (upper block triangle of A, CCG_SYM_AD) serves FP64 block
// steps of single systems with P <= kSymMaxP and n >= kSymMinN; smaller systems
// stream A whole (their time is set by the step's fixed latency, not by the bytes
// of A).
constexpr int kSymMinN = 1024;
inline bool sym_eligible(int prec, int P, int n) { return prec == PREC_F64 && P <= kSymMaxP && n >= kSymMinN; }
inline int sym_blocks(int n) { return (n + kSymB - 1) / kSymB; }
// strips of kSymW blocks in the upper block triangle of nb blocks
inline int sym_units(int nb) {
    int u = 0;
    for (int I = 0; I < nb; ++I) u += (nb - I + kSymW - 1) / kSymW;
    return u;
}
// bytes of A the symmetric pass reads: every block (I, J), I <= J, whole
inline double sym_bytes_A(int n) {
    double diag = 0.0;
    for (int K = 0; K * kSymB < n; ++K) {
        const double bk = std::min(kSymB, n - K * kSymB);
        diag += bk * bk;
    }
    return 8.0 * 0.5 * ((double)n * n + diag);
}

namespace host {

struct CcgError {
    ccg_status st;
    std::string msg;
};

#define HIP_OK(expr)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            throw CcgError{CCG_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)}; \
    } while (0)

inline int pad_agents(int p) {
    int P = 1;
    while (P < p) P <<= 1;
    return P;
}

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

struct Workspace {
    int n = 0, n_pad = 0, P = 0;
    size_t bytes = 0;
    void* base = nullptr;            // one allocation, carved
    double* Xr = nullptr;            // agent-major n_pad x P (FP64 agents)
    double* bp = nullptr;            // n_pad
    double* R = nullptr;             // agent-major n_pad x P
    double* D = nullptr;
    double* AD = nullptr;
    // low-precision inner solve of the refinement modes (FP32 blocks, agent-major)
    float* E = nullptr;
    float* Rl = nullptr;
    float* Dl = nullptr;
    float* ADl = nullptr;
    RedBuf red_ad{}, red_up{}, red_res{};
    DevState* st = nullptr;
    // symmetric A.D pass (carved on request, for P <= kSymMaxP and n_pad >= kSymMinN)
    double* part = nullptr;          // n_pad/kSymB blocks x as many slots x kSymB x P
    int2* units = nullptr;           // strip list of sym_nb blocks
    int sym_tmax = 0;                // slot stride of part
    int sym_nb = 0;                  // blocks of the strip list in units (0: none built)
};

struct Carver {
    char* p;
    size_t off = 0;
    template <class T> T* take(size_t count) {
        off = (size_t)round_up((int64_t)off, 256);
        T* r = reinterpret_cast<T*>(p ? p + off : nullptr);
        off += count * sizeof(T);
        return r;
    }
};

inline RedBuf carve_red(Carver& cv, int nwg, int ne, int gs = kGroup) {
    const int ngroups = (nwg + gs - 1) / gs;
    RedBuf r;
    r.l1 = cv.take<double>((size_t)nwg * ne);
    r.l2 = cv.take<double>((size_t)ngroups * ne);
    r.cnt = cv.take<unsigned>((size_t)ngroups + 1);
    return r;
}

}  // namespace host
}  // namespace ccg

namespace ccg {
namespace host {
struct Server;
}  // namespace host
}  // namespace ccg

struct ccg_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    size_t budget = 0;
    std::string err;
    ccg::host::Workspace ws;
    ccg::DevState* st_host = nullptr;     // pinned mirror of the device state
    // A.D timing (CCG_PROFILE)
    double prof_ms = 0.0;
    long long prof_launches = 0;
    double prof_bytes = 0.0;              // algorithmic bytes of the timed launches
    std::vector<hipEvent_t> ev_pool;
    // captured block-step graphs, one per round length, all for graph_key
    std::vector<std::pair<int, hipGraphExec_t>> graphs;
    int64_t graph_key[7] = {0, 0, 0, 0, 0, 0, 0};
    // aligned copy of a caller matrix with unaligned columns
    void* acopy = nullptr;
    size_t acopy_bytes = 0;
    // low-precision copy of A (FP32, or the BF16 hi plane followed by the lo plane)
    void* lowA = nullptr;
    size_t lowA_bytes = 0;
    // continuous-batching service (ccg_submit), started on first use
    ccg::host::Server* server = nullptr;
    // device address of this device's scratch array (ccg_solve_noalloc), taken at
    // ccg_create; nullptr if the lookup failed
    void* scratch = nullptr;
};


namespace ccg {
namespace host {

// Stop and join the service thread of a context (no-op without one).
void stop_server(ccg_ctx* c);

// Lay out (or only size, when base == nullptr) the workspace.
// With sym, also the partial sums and strip list of the symmetric A.D pass.
inline size_t carve(Workspace& w, char* base, int n, int n_pad, int P, bool sym = false) {
    Carver cv{base};
    const size_t blk = (size_t)n_pad * P;
    w.Xr = cv.take<double>(blk);
    w.bp = cv.take<double>((size_t)n_pad);
    w.R = cv.take<double>(blk);
    w.D = cv.take<double>(blk);
    w.AD = cv.take<double>(blk);
    w.E = cv.take<float>(blk);
    w.Rl = cv.take<float>(blk);
    w.Dl = cv.take<float>(blk);
    w.ADl = cv.take<float>(blk);
    w.red_ad = carve_red(cv, ad_workgroups(n_pad), P * (P + 1) / 2 + P * P);
    w.red_up = carve_red(cv, upd_blocks(n_pad, P), P * P + P, upd_group(P));
    w.red_res = carve_red(cv, row_workgroups(n_pad, P), P * P + 1);
    w.st = cv.take<DevState>(1);
    if (sym && P <= kSymMaxP && n_pad >= kSymMinN) {
        const int nbp = n_pad / kSymB;
        w.sym_tmax = nbp;
        w.part = cv.take<double>((size_t)nbp * nbp * kSymB * P);
        w.units = cv.take<int2>((size_t)sym_units(nbp));
    }
    return cv.off;
}

inline void check_common(int n, int p, const void* A, int64_t lda, const void* b, const void* X, int64_t ldx) {
    if (n < 1 || p < 1 || p > kMaxP || p > n)
        throw CcgError{CCG_ERR_ARG, "need 1 <= p <= min(n, 32)"};
    if (!A || !b || !X) throw CcgError{CCG_ERR_ARG, "null pointer argument"};
    if (lda < n || ldx < n) throw CcgError{CCG_ERR_ARG, "leading dimension smaller than n"};
}

// Inner tolerance of the next refinement step, from the factor rho by which the last
// outer step lowered the FP64 residual.  When the rounding of the low-precision copy
// limits an outer step to about rho*, solving the correction much more accurately
// than rho* only adds block steps; a quarter of rho keeps the inner solve from
// becoming the limit (the contraction then settles near 4/3 rho*), and the bound
// 0.05 keeps every inner solve doing real work.  Never tighter than inner_tol.
inline double next_inner_tol(double inner_tol, double rho) {
    return std::min(0.05, std::max(inner_tol, 0.25 * rho));
}

inline void set_all_agents(DevState& h, int p) {
    h.m = p;
    h.mask = (p >= 32) ? 0xffffffffu : ((1u << p) - 1u);
    for (int j = 0; j < p; ++j) h.keep[j] = j;
}

inline ccg_opts fill_defaults(const ccg_opts* in) {
    ccg_opts o;
    std::memset(&o, 0, sizeof o);
    if (in) o = *in;
    if (o.inner_tol <= 0.0) o.inner_tol = 1e-4;
    if (o.inner_maxit <= 0) o.inner_maxit = 500;
    if (o.max_refine <= 0) o.max_refine = 60;
    if (o.rank_tau <= 0.0) o.rank_tau = o.prec == CCG_FP64 ? 1e-14 : 1e-12;
    if (o.graph_k <= 0) o.graph_k = 16;
    if (o.max_reinflate <= 0) o.max_reinflate = 3;
    return o;
}

template <class F>
inline ccg_status guarded(ccg_ctx* c, F&& f) {
    if (!c) return CCG_ERR_ARG;
    try {
        HIP_OK(hipSetDevice(c->device));
        c->err.clear();
        return f();
    } catch (const CcgError& e) {
        c->err = e.msg;
        if (e.st == CCG_ERR_DEVICE) {
            // leave the stream usable for the next call where possible
            (void)hipStreamSynchronize(c->stream);
        }
        return e.st;
    } catch (const std::bad_alloc&) {
        c->err = "host allocation failed";
        return CCG_ERR_NOMEM;
    }
}

}  // namespace host
}  // namespace ccg
