// Host side and C interface (include/ccg.h) of the cooperative CG library.
//
// The host side owns one workspace per context, sized for the largest solve so far.
// A solve is: pack X0 into the agent-major block, form R0 = B - A X0 (an A
// stream plus the residual epilogue), then repeat groups of block steps
// (k_ad, k_upd, k_dir) -- captured once into a HIP graph and replayed -- polling
// the device state between groups.  When the recurrence residual passes the test,
// the explicit FP64 residual confirms it or restarts the agents from it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/ccg.h"
#include "ccg_device.h"

#include "ccg_host.h"

using namespace ccg;
using namespace ccg::host;

namespace {

void free_workspace(ccg_ctx* c) {
    for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.second);
    c->graphs.clear();
    if (c->ws.base) (void)hipFree(c->ws.base);
    c->ws = Workspace();
}

// Strip list of the symmetric A.D pass for the workspace's current n (built on the
// device, in stream order, when n changes).
void ensure_sym_units(ccg_ctx* c) {
    Workspace& w = c->ws;
    if (!w.part || w.n < kSymMinN) return;
    const int nb = sym_blocks(w.n);
    if (w.sym_nb == nb) return;
    HIP_OK(launch_sym_units(nb, w.units, c->stream));
    w.sym_nb = nb;
}

// The workspace depends only on (n_pad, P) and on whether it holds the scratch of
// the symmetric A.D pass (sym); the reduction scratch is sized for n_pad rows, which
// covers every n with the same padded size.
void ensure_workspace(ccg_ctx* c, int n, int P, bool sym = false) {
    const int n_pad = (int)round_up(n, kRowAlign);
    Workspace& w = c->ws;
    sym = sym && sym_eligible(PREC_F64, P, n);
    if (w.base && w.n_pad == n_pad && w.P == P && (!sym || w.part)) {
        // rows n..n_pad of AD must read as zero (the A.D kernel stores rows < n only)
        if (w.n != n) {
            HIP_OK(hipMemsetAsync(w.AD, 0, sizeof(double) * (size_t)n_pad * P, c->stream));
            HIP_OK(hipMemsetAsync(w.ADl, 0, sizeof(float) * (size_t)n_pad * P, c->stream));
        }
        w.n = n;
        ensure_sym_units(c);
        return;
    }
    free_workspace(c);
    Workspace nw;
    const size_t bytes = carve(nw, nullptr, n, n_pad, P, sym);
    if (c->budget && bytes + c->acopy_bytes + c->lowA_bytes > c->budget)
        throw CcgError{CCG_ERR_NOMEM, "workspace of " + std::to_string(bytes) + " bytes exceeds the HBM budget"};
    void* base = nullptr;
    if (hipMalloc(&base, bytes) != hipSuccess)
        throw CcgError{CCG_ERR_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed"};
    HIP_OK(hipMemsetAsync(base, 0, bytes, c->stream));
    carve(nw, static_cast<char*>(base), n, n_pad, P, sym);
    nw.base = base;
    nw.bytes = bytes;
    nw.n = n;
    nw.n_pad = n_pad;
    nw.P = P;
    w = nw;
    ensure_sym_units(c);
}

struct Solve {
    ccg_ctx* c;
    int n, p, P, prec;
    const void* A;         // matrix the block steps stream (prec)
    const void* A_lo;      // BF16 lo plane (BF16x2)
    int64_t lda;           // its leading dimension in elements
    const double* A64;     // FP64 matrix of the explicit residual
    int64_t lda64;
    int profile_every;     // time the A.D launches of every n-th round of steps (0: none)
    bool sym_ad = false;   // CCG_SYM_AD: symmetric A.D pass where eligible
    int rounds = 0;        // rounds of block steps run so far
    int ad_cw = 0, ad_nw = 0;   // A.D tile shape (0: the tuned table's)
    unsigned flags = 0;         // the caller's CCG_NO_TIER
};

// The A.D tile shape the block steps of a solve run: the caller's (fitted), else 0
// (the table's choice); and whether the small-system tier may run them.
void set_shape(Solve& s, const ccg_opts& o) {
    s.flags = o.flags & CCG_NO_TIER;
    if (o.ad_cw <= 0 && o.ad_nw <= 0) return;
    const int nw = o.ad_nw > 0 ? o.ad_nw : 4;
    s.ad_nw = ad_fit_nw(s.prec, s.P, nw);
    s.ad_cw = ad_fit_cw(s.prec, s.P, o.ad_cw > 0 ? o.ad_cw : 2, nw);
}

// Block steps of this solve run the symmetric A.D pass.
bool use_sym(const Solve& s) {
    return s.sym_ad && sym_eligible(s.prec, s.P, s.n) && s.c->ws.part && s.c->ws.sym_nb == sym_blocks(s.n);
}

// Block steps of this solve run in the small-system tier (one workgroup per step).
bool use_small(const Solve& s) { return small_tier(s.P, s.n, s.flags); }

// Bytes of A one block step streams, and the algorithmic bytes of its A.D pass
// (A, or its upper triangle, plus the D and R rows) for the kernel timing.
double step_bytes_A(const Solve& s) {
    if (use_sym(s)) return sym_bytes_A(s.n);
    const double sa = s.prec == PREC_F64 ? 8.0 : 4.0;
    return sa * s.n * s.n;
}
double step_alg_bytes(const Solve& s) {
    const double sv = s.prec == PREC_F64 ? 8.0 : 4.0;
    const double vec = 2.0 * sv * s.n * s.p;
    if (use_sym(s)) return 8.0 * 0.5 * (double)s.n * (s.n + 1) + vec;
    const double sa = s.prec == PREC_F64 ? 8.0 : 4.0;
    return sa * s.n * s.n + vec;
}

SymArgs sym_args(const Solve& s) {
    const Workspace& w = s.c->ws;
    SymArgs a;
    a.A = static_cast<const double*>(s.A);
    a.lda = s.lda;
    a.n = s.n;
    a.n_pad = w.n_pad;
    a.nb = sym_blocks(s.n);
    a.tmax = w.sym_tmax;
    a.V = w.D;
    a.part = w.part;
    a.units = w.units;
    a.st = w.st;
    return a;
}

// Timing of the A.D launches requested by the flags: every round (CCG_PROFILE),
// every 4th (CCG_PROFILE_SAMPLED), or none.
int profile_every(const ccg_opts& o) {
    if (o.flags & CCG_PROFILE) return 1;
    if (o.flags & CCG_PROFILE_SAMPLED) return 4;
    return 0;
}

// Vector blocks of the block steps: FP64 for plain cCG, FP32 for the inner solve of
// the refinement modes.
struct Blocks {
    void *X, *R, *D, *AD;
};
Blocks blocks(const Solve& s) {
    const Workspace& w = s.c->ws;
    if (s.prec == PREC_F64) return Blocks{w.Xr, w.R, w.D, w.AD};
    return Blocks{w.E, w.Rl, w.Dl, w.ADl};
}

AdArgs ad_args(const Solve& s, bool product_only) {
    const Workspace& w = s.c->ws;
    AdArgs a;
    a.n = s.n;
    a.n_pad = w.n_pad;
    a.product_only = product_only ? 1 : 0;
    if (product_only) {          // Y = A X in FP64, into the FP64 AD block
        a.A = s.A64;
        a.A_lo = nullptr;
        a.lda = s.lda64;
        a.V = w.Xr;
        a.R = w.R;
        a.AD = w.AD;
    } else {
        const Blocks b = blocks(s);
        a.A = s.A;
        a.A_lo = s.A_lo;
        a.lda = s.lda;
        a.V = b.D;
        a.R = b.R;
        a.AD = b.AD;
    }
    a.red = w.red_ad;
    a.st = w.st;
    return a;
}

void enqueue_residual(const Solve& s, int mode, int set_nb) {
    Workspace& w = s.c->ws;
    // Y = A X in FP64 (the residual is always FP64)
    HIP_OK(launch_ad(PREC_F64, s.P, ad_args(s, true), s.c->stream));
    ResArgs r;
    r.n = s.n;
    r.n_pad = w.n_pad;
    r.p = s.p;
    r.mode = mode;
    r.set_nb = set_nb;
    r.b = w.bp;
    r.Y = w.AD;
    r.R = w.R;
    r.D = w.D;
    r.red = w.red_res;
    r.st = w.st;
    HIP_OK(launch_res(s.P, r, s.c->stream));
}

hipEvent_t pooled_event(ccg_ctx* c, size_t i) {
    while (c->ev_pool.size() <= i) {
        hipEvent_t e;
        HIP_OK(hipEventCreate(&e));
        c->ev_pool.push_back(e);
    }
    return c->ev_pool[i];
}

SmallArgs small_args(const Solve& s) {
    const Workspace& w = s.c->ws;
    const Blocks b = blocks(s);
    SmallArgs a;
    a.A = s.A;
    a.A_lo = s.A_lo;
    a.lda = s.lda;
    a.n = s.n;
    a.X = b.X;
    a.R = b.R;
    a.D = b.D;
    a.st = w.st;
    return a;
}

// One block step: A.D (+ products, rank step, alpha), the X and R update (+ stop
// test and beta), then the direction update; in the small-system tier, one launch.
void enqueue_step(const Solve& s, size_t ev_slot, bool timed) {
    Workspace& w = s.c->ws;
    if (use_small(s)) {
        const SmallArgs sa = small_args(s);
        HIP_OK(launch_small(s.prec, s.P, &sa, nullptr, nullptr, 0, 1, s.c->stream));
        return;
    }
    hipEvent_t e0 = timed ? pooled_event(s.c, 2 * ev_slot) : nullptr;
    hipEvent_t e1 = timed ? pooled_event(s.c, 2 * ev_slot + 1) : nullptr;
    if (use_sym(s)) {
        HIP_OK(launch_sym(s.P, sym_args(s), ad_args(s, false), sym_units(sym_blocks(s.n)), s.c->stream, e0, e1));
    } else {
        if (s.ad_cw)
            HIP_OK(launch_ad_cw(s.prec, s.P, s.ad_cw, s.ad_nw, ad_args(s, false), s.c->stream, e0, e1));
        else
            HIP_OK(launch_ad(s.prec, s.P, ad_args(s, false), s.c->stream, e0, e1));
    }
    const Blocks b = blocks(s);
    UpdArgs u;
    u.n_pad = w.n_pad;
    u.X = b.X;
    u.R = b.R;
    u.D = b.D;
    u.AD = b.AD;
    u.red = w.red_up;
    u.st = w.st;
    HIP_OK(launch_upd(s.prec, s.P, u, s.c->stream));
    HIP_OK(launch_dir(s.prec, s.P, u, s.c->stream));
}

void read_state(ccg_ctx* c) {
    HIP_OK(hipMemcpyAsync(c->st_host, c->ws.st, sizeof(DevState), hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
}

void write_state(ccg_ctx* c) {
    HIP_OK(hipMemcpyAsync(c->ws.st, c->st_host, sizeof(DevState), hipMemcpyHostToDevice, c->stream));
}

void collect_profile(const Solve& s, int steps) {
    ccg_ctx* c = s.c;
    for (int i = 0; i < steps; ++i) {
        float ms = 0.f;
        HIP_OK(hipEventElapsedTime(&ms, c->ev_pool[2 * i], c->ev_pool[2 * i + 1]));
        c->prof_ms += ms;
        c->prof_launches += 1;
        c->prof_bytes += step_alg_bytes(s);
    }
}

// Capture `steps` block steps into a graph.
hipGraphExec_t capture_steps(Solve& s, int steps) {
    ccg_ctx* c = s.c;
    hipGraph_t gr = nullptr;
    HIP_OK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    bool ok = true;
    try {
        for (int i = 0; i < steps; ++i) enqueue_step(s, 0, false);
    } catch (const CcgError&) {
        ok = false;
    }
    const hipError_t e = hipStreamEndCapture(c->stream, &gr);
    if (!ok || e != hipSuccess || !gr) {
        (void)hipGetLastError();
        if (gr) (void)hipGraphDestroy(gr);
        throw CcgError{CCG_ERR_DEVICE, "stream capture of the block step failed"};
    }
    hipGraphExec_t ex = nullptr;
    const hipError_t ei = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    HIP_OK(ei);
    return ex;
}

// Run `steps` block steps, through a captured graph when allowed.  A round whose
// A.D launches are timed runs them directly, each bracketed by its own event pair
// on the stream (the runtime does not time events recorded inside a graph).
// Returns whether this round was timed.
bool run_steps(Solve& s, int steps, bool use_graph) {
    ccg_ctx* c = s.c;
    if (use_small(s)) {
        // the whole round is one launch: one workgroup runs up to `steps` steps
        ++s.rounds;
        const SmallArgs sa = small_args(s);
        HIP_OK(launch_small(s.prec, s.P, &sa, nullptr, nullptr, 0, steps, c->stream));
        return false;
    }
    const bool timed = s.profile_every > 0 && s.rounds % s.profile_every == 0;
    ++s.rounds;
    if (!use_graph || timed) {
        for (int i = 0; i < steps; ++i) enqueue_step(s, (size_t)i, timed);
        return timed;
    }
    // everything a captured step depends on: sizes, precision, workspace, matrix and
    // which A.D pass the steps launch
    const int64_t key[7] = {s.n, s.P, s.prec, (int64_t)(intptr_t)c->ws.base, (int64_t)(intptr_t)s.A,
                            s.lda, use_sym(s) ? 1 : 0};
    if (!std::equal(key, key + 7, c->graph_key)) {
        for (auto& g : c->graphs) HIP_OK(hipGraphExecDestroy(g.second));
        c->graphs.clear();
        std::copy(key, key + 7, c->graph_key);
    }
    hipGraphExec_t ex = nullptr;
    for (auto& g : c->graphs)
        if (g.first == steps) ex = g.second;
    if (!ex) {
        ex = capture_steps(s, steps);
        c->graphs.emplace_back(steps, ex);
    }
    HIP_OK(hipGraphLaunch(ex, c->stream));
    return false;
}

// Block steps of the next round of a solve (FP64, or the inner solve of a
// refinement step, whose target is its inner tolerance).  Each round ends with the host
// reading the device state (about 45 us in which the GPU idles at n = 8192), so
// while the residual is far from the tolerance the rounds grow: from the decay of
// min_j ||R_j|| over the last round (prev -> cur in `done` steps) the steps still
// needed are predicted, and the round takes up to half of them, in powers of two
// from graph_k up to 8 graph_k.  Steps after the stop return at once, so a round
// that overshoots costs a few microseconds per step.  The steps themselves, and so
// the results, do not depend on where the rounds end.
int next_round(int gk, double prev, double cur, int done, double tol) {
    if (!(prev > 0.0) || !(cur > 0.0) || !(tol > 0.0) || done <= 0 || cur >= prev || cur <= tol) return gk;
    const double rate = std::log(cur / prev) / done;      // < 0
    const double left = std::log(tol / cur) / rate;       // predicted steps to go
    int k = gk;
    while (k < 8 * gk && 2.0 * k <= 0.5 * left) k *= 2;
    return k;
}

// The A.D kernel reads columns with 16-byte loads.  A caller matrix whose columns
// are not 16-byte aligned is copied once into a context-owned aligned buffer (lda
// is then updated by the caller from acopy_ld).
const double* aligned_matrix(ccg_ctx* c, int n, const double* A, int64_t& lda) {
    if (reinterpret_cast<uintptr_t>(A) % 16 == 0 && (lda * sizeof(double)) % 16 == 0) return A;
    const int64_t ldb = round_up(n, 2);
    const size_t bytes = sizeof(double) * (size_t)ldb * n;
    if (c->acopy_bytes < bytes) {
        if (c->acopy) (void)hipFree(c->acopy);
        c->acopy = nullptr;
        c->acopy_bytes = 0;
        if (c->budget && bytes + c->ws.bytes > c->budget)
            throw CcgError{CCG_ERR_NOMEM, "aligned copy of A exceeds the HBM budget"};
        if (hipMalloc(&c->acopy, bytes) != hipSuccess)
            throw CcgError{CCG_ERR_NOMEM, "hipMalloc for the aligned copy of A failed"};
        c->acopy_bytes = bytes;
    }
    HIP_OK(launch_copy_cols(n, A, lda, static_cast<double*>(c->acopy), ldb, c->stream));
    lda = ldb;
    return static_cast<const double*>(c->acopy);
}

// Host-pointer staging (CCG_HOST_PTRS): device copies of A, b, X.
struct Staged {
    double *A = nullptr, *b = nullptr, *X = nullptr;
    ~Staged() {
        if (A) (void)hipFree(A);
        if (b) (void)hipFree(b);
        if (X) (void)hipFree(X);
    }
};

void stage_in(ccg_ctx* c, Staged& sg, int n, int p, const double*& A, int64_t& lda, const double*& b,
              double*& X, int64_t& ldx) {
    HIP_OK(hipMalloc(&sg.A, sizeof(double) * (size_t)n * n));
    HIP_OK(hipMalloc(&sg.b, sizeof(double) * (size_t)n));
    HIP_OK(hipMalloc(&sg.X, sizeof(double) * (size_t)n * p));
    HIP_OK(hipMemcpy2DAsync(sg.A, sizeof(double) * n, A, sizeof(double) * lda, sizeof(double) * n, n,
                            hipMemcpyHostToDevice, c->stream));
    HIP_OK(hipMemcpyAsync(sg.b, b, sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
    HIP_OK(hipMemcpy2DAsync(sg.X, sizeof(double) * n, X, sizeof(double) * ldx, sizeof(double) * n, p,
                            hipMemcpyHostToDevice, c->stream));
    A = sg.A;
    lda = n;
    b = sg.b;
    X = sg.X;
    ldx = n;
}

// Plain FP64 cCG on device buffers in the context's workspace c->ws (sized for n
// and p, rows n..n_pad of AD zero); A has 16-byte aligned columns.  Fills info.
ccg_status fp64_steps(ccg_ctx* c, int n, int p, const double* Ause, int64_t lda, const double* b,
                      double* X, int64_t ldx, double tol, int maxit, const ccg_opts& o, ccg_info& info) {
    const int P = pad_agents(p);
    Solve s{c, n, p, P, PREC_F64, Ause, nullptr, lda, Ause, lda, profile_every(o), (o.flags & CCG_SYM_AD) != 0};
    set_shape(s, o);
    Workspace& w = c->ws;
    HIP_OK(launch_pack(n, w.n_pad, p, P, X, ldx, w.Xr, c->stream));
    HIP_OK(launch_pad_vec(n, w.n_pad, b, w.bp, c->stream));
    DevState& h = *c->st_host;
    std::memset(&h, 0, sizeof(DevState));
    h.done = RUNNING;
    h.m = p;
    h.mask = (p >= 32) ? 0xffffffffu : ((1u << p) - 1u);
    for (int j = 0; j < p; ++j) h.keep[j] = j;
    h.maxit = maxit;
    h.tol = tol;
    h.tau = o.rank_tau;
    h.nb = 1.0;
    h.reinflate_left = (o.flags & CCG_REINFLATE) ? o.max_reinflate : 0;
    write_state(c);
    enqueue_residual(s, RES_INIT, 1);
    read_state(c);
    int reinflations = 0;
    const double bytes_iter = (double)n * n * sizeof(double);   // an explicit residual
    const double bytes_step = step_bytes_A(s);
    double bytes = bytes_iter;   // the initial residual
    const bool use_graph = !(o.flags & CCG_NO_GRAPH);
    const int gk = o.graph_k > 0 ? o.graph_k : 16;
    int round_k = gk;
    while (h.done == RUNNING || h.done == RECUR_CONV || h.done == REINFLATE) {
        if (h.done == RUNNING) {
            const int left = maxit - h.iter;
            const int k = left > 0 ? round_k : 1;   // steps past maxit are no-ops
            const int it0 = h.iter;
            const int as0 = h.ad_streams;
            const double res0 = h.minres;
            const bool timed = run_steps(s, k, use_graph);
            read_state(c);
            round_k = next_round(gk, res0, h.minres, h.iter - it0, tol);
            // A.D launches that streamed A (one per step, whose stop test now runs
            // in the update launch, so no launch streams A past the stop)
            const int streamed = h.ad_streams - as0;
            if (timed) collect_profile(s, streamed);
            bytes += bytes_step * streamed;
        }
        if (h.done == RECUR_CONV) {
            enqueue_residual(s, RES_CONFIRM, 0);
            read_state(c);
            bytes += bytes_iter;
        }
        if (h.done == REINFLATE) {
            // the agents outside the kept set restart from the best of those active
            // before the rank step, plus the draw; then the whole block restarts
            const unsigned all = (p >= 32) ? 0xffffffffu : ((1u << p) - 1u);
            const unsigned dropped = all & ~h.mask;
            int best = -1;
            for (int j = 0; j < p; ++j)
                if (((h.prev_mask >> j) & 1u) && (best < 0 || h.norms[j] < h.norms[best])) best = j;
            HIP_OK(launch_reinflate(n, w.n_pad, p, dropped, best, reinflations, w.Xr, c->stream));
            ++reinflations;
            h.done = RUNNING;
            set_all_agents(h, p);
            h.reinflate_left -= 1;
            write_state(c);
            enqueue_residual(s, RES_INIT, 0);
            read_state(c);
            bytes += bytes_iter;
        }
    }
    if (h.done == MAXIT) {
        enqueue_residual(s, RES_FINAL, 0);
        read_state(c);
        bytes += bytes_iter;
    }
    HIP_OK(launch_unpack(n, w.n_pad, p, w.Xr, X, ldx, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    ccg_status st = CCG_OK;
    if (h.done == FAILED) st = (ccg_status)h.status;
    else if (h.done == MAXIT) st = CCG_NOT_CONVERGED;
    info.status = st;
    info.iters = h.iter;
    info.refinements = 0;
    info.restarts = h.restarts;
    info.p_final = h.m;
    info.deflations = h.deflations;
    info.reinflations = reinflations;
    double mn = INFINITY, mx = 0.0;
    int best = -1;
    for (int j = 0; j < p; ++j) {
        const double r = h.norms[j] / h.nb;
        if (r < mn) { mn = r; best = j; }
        if (r > mx) mx = r;
    }
    info.best_agent = best;
    info.rel_res = mn;
    info.rel_res_max = mx;
    info.bytes_A = bytes;
    return st;
}

ccg_status solve_fp64(ccg_ctx* c, int n, int p, const double* A, int64_t lda, const double* b,
                      double* X, int64_t ldx, double tol, int maxit, const ccg_opts& o, ccg_info& info) {
    const double* Ause = aligned_matrix(c, n, A, lda);
    ensure_workspace(c, n, pad_agents(p), (o.flags & CCG_SYM_AD) != 0);
    return fp64_steps(c, n, p, Ause, lda, b, X, ldx, tol, maxit, o, info);
}

// Runs f with the context's workspace replaced by w (restored on every exit).
template <class F>
ccg_status with_workspace(ccg_ctx* c, const Workspace& w, F&& f) {
    struct Swap {
        ccg_ctx* c;
        Workspace saved;
        ~Swap() { c->ws = saved; }
    } sw{c, c->ws};
    c->ws = w;
    return f();
}

// Low-precision copy of A for the FP32 / BF16x2 modes, converted on every solve (the
// caller may change A between calls).  Returns the streamed planes and their
// leading dimension (16-byte aligned columns).
struct LowCopy {
    const void* hi;
    const void* lo;
    int64_t ld;
    double bytes;     // algorithmic bytes of the conversion pass
};

LowCopy low_copy(ccg_ctx* c, int n, const double* A, int64_t lda, int prec) {
    const int64_t ld = round_up(n, prec == PREC_F32 ? 4 : 8);
    const size_t plane = (size_t)ld * n * (prec == PREC_F32 ? sizeof(float) : sizeof(uint16_t));
    const size_t need = prec == PREC_F32 ? plane : 2 * round_up((int64_t)plane, 256);
    if (c->lowA_bytes < need) {
        if (c->lowA) (void)hipFree(c->lowA);
        c->lowA = nullptr;
        c->lowA_bytes = 0;
        if (c->budget && need + c->ws.bytes + c->acopy_bytes > c->budget)
            throw CcgError{CCG_ERR_NOMEM, "low-precision copy of A exceeds the HBM budget"};
        if (hipMalloc(&c->lowA, need) != hipSuccess)
            throw CcgError{CCG_ERR_NOMEM, "hipMalloc for the low-precision copy of A failed"};
        c->lowA_bytes = need;
    }
    char* base = static_cast<char*>(c->lowA);
    void* hi = base;
    void* lo = prec == PREC_F32 ? nullptr : base + round_up((int64_t)plane, 256);
    HIP_OK(launch_convert(prec, n, A, lda, hi, lo, ld, c->stream));
    const double elem = prec == PREC_F32 ? 4.0 : 4.0;   // FP32, or two BF16 planes
    return LowCopy{hi, lo, ld, (double)n * n * (8.0 + elem)};
}

// Mixed precision (FP32 or BF16x2 A): FP64 iterative refinement around a low-
// precision cCG inner solve.  Each outer step forms the explicit FP64 residual
// T = B - A X, scales its columns to unit norm, runs cCG on A E = T in the low-
// precision blocks (FP32 vectors and A.D accumulation; FP64 products, alpha and
// beta) until the best agent's relative residual is below the inner tolerance, and
// adds E * scale to the FP64 agents.  Stops when min_j ||b - A x_j|| / ||b|| <= tol.
// The inner tolerance starts at inner_tol and then follows the contraction of the
// FP64 residual that the last outer step reached (next_inner_tol).  In the last
// steps it is relaxed to 0.1 tol / minres, where less suffices.
ccg_status solve_mixed(ccg_ctx* c, int n, int p, const double* A, int64_t lda, const double* b,
                       double* X, int64_t ldx, double tol, int maxit, const ccg_opts& o, ccg_info& info) {
    const int P = pad_agents(p);
    const int prec = o.prec == CCG_FP32 ? PREC_F32 : PREC_BF16X2;
    const double* A64 = aligned_matrix(c, n, A, lda);
    ensure_workspace(c, n, P);
    const LowCopy lc = low_copy(c, n, A64, lda, prec);
    Solve s{c, n, p, P, prec, lc.hi, lc.lo, lc.ld, A64, lda, profile_every(o)};
    set_shape(s, o);
    Workspace& w = c->ws;
    HIP_OK(launch_pack(n, w.n_pad, p, P, X, ldx, w.Xr, c->stream));
    HIP_OK(launch_pad_vec(n, w.n_pad, b, w.bp, c->stream));
    DevState& h = *c->st_host;
    std::memset(&h, 0, sizeof(DevState));
    h.done = RUNNING;
    set_all_agents(h, p);
    h.maxit = maxit;
    h.tol = tol;
    h.tau = o.rank_tau;
    h.nb = 1.0;
    write_state(c);
    enqueue_residual(s, RES_REFINE, 1);
    read_state(c);
    const double nb = h.nb;     // ||b||; the inner solves use 1 (unit columns)
    const double s_low = 4.0;   // bytes per streamed A element (FP32, or BF16 hi + lo)
    double bytes = lc.bytes + 8.0 * n * n;
    const bool use_graph = !(o.flags & CCG_NO_GRAPH);
    const int gk = o.graph_k > 0 ? o.graph_k : 16;
    int iters = 0, refinements = 0, stall = 0;
    double best = h.minres;
    double in_tol = o.inner_tol;   // inner tolerance (see above)
    double prev = h.minres;        // FP64 residual before the current outer step
    ccg_status st = CCG_OK;
    RefArgs ra{};
    ra.n_pad = w.n_pad;
    ra.P = P;
    ra.T = w.R;
    ra.X = w.Xr;
    ra.E = w.E;
    ra.R = w.Rl;
    ra.D = w.Dl;
    while (h.done == OUTER) {
        if (refinements >= o.max_refine || iters >= maxit) { st = CCG_NOT_CONVERGED; break; }
        // inner solve on A E = T (unit columns)
        unsigned mask = 0u;
        int m = 0;
        for (int j = 0; j < kMaxP; ++j) {
            const double sc = (j < p && std::isfinite(h.norms[j])) ? h.norms[j] : 0.0;
            ra.scale[j] = sc;
            if (sc > 0.0) { mask |= 1u << j; h.keep[m++] = j; }
        }
        HIP_OK(launch_inner_init(ra, c->stream));
        prev = h.minres;
        h.done = RUNNING;
        h.iter = 0;
        h.m = m;
        h.mask = mask;
        // no need to solve the correction more accurately than the outer target:
        // the best agent's residual after this step is about (inner tol) x minres
        h.tol = std::min(0.5, std::max(in_tol, 0.1 * tol / h.minres));
        h.nb = 1.0;
        h.maxit = std::min(o.inner_maxit, maxit - iters);
        write_state(c);
        int round_k = gk;
        while (h.done == RUNNING) {
            const int k = round_k;   // steps past maxit are no-ops
            const int it0 = h.iter;
            const int as0 = h.ad_streams;
            const double res0 = h.minres;
            const bool timed = run_steps(s, k, use_graph);
            read_state(c);
            round_k = next_round(gk, res0, h.minres, h.iter - it0, h.tol);
            const int streamed = h.ad_streams - as0;
            if (timed) collect_profile(s, streamed);
            bytes += s_low * n * n * streamed;
        }
        iters += h.iter;
        if (h.done == FAILED) { st = (ccg_status)h.status; break; }
        HIP_OK(launch_refine_add(ra, c->stream));
        ++refinements;
        // outer FP64 residual
        h.done = RUNNING;
        h.tol = tol;
        h.nb = nb;
        set_all_agents(h, p);
        write_state(c);
        enqueue_residual(s, RES_REFINE, 0);
        read_state(c);
        bytes += 8.0 * n * n;
        if (h.done == FAILED) { st = (ccg_status)h.status; break; }
        if (h.minres >= best) {
            if (++stall >= 3) { st = CCG_ERR_BREAKDOWN; break; }
        } else {
            stall = 0;
        }
        best = std::min(best, h.minres);
        in_tol = next_inner_tol(o.inner_tol, h.minres / prev);
    }
    if (h.done == FAILED && st == CCG_OK) st = (ccg_status)h.status;
    HIP_OK(launch_unpack(n, w.n_pad, p, w.Xr, X, ldx, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    if (st == CCG_ERR_BREAKDOWN) c->err = "refinement made no progress over three outer steps";
    info.status = st;
    info.iters = iters;
    info.refinements = refinements;
    info.restarts = 0;
    info.p_final = p;
    info.deflations = h.deflations;
    double mn = INFINITY, mx = 0.0;
    int bestj = -1;
    for (int j = 0; j < p; ++j) {
        const double r = h.norms[j] / h.nb;
        if (r < mn) { mn = r; bestj = j; }
        if (r > mx) mx = r;
    }
    info.best_agent = bestj;
    info.rel_res = mn;
    info.rel_res_max = mx;
    info.bytes_A = bytes;
    return st;
}

}  // namespace

extern "C" {

ccg_status ccg_create(ccg_ctx** ctx, int device, size_t hbm_budget_bytes, void* hip_stream) {
    if (!ctx) return CCG_ERR_ARG;
    *ctx = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return CCG_ERR_DEVICE;
    if (hipSetDevice(device) != hipSuccess) return CCG_ERR_DEVICE;
    ccg_ctx* c = new ccg_ctx();
    c->device = device;
    c->budget = hbm_budget_bytes;
    if (hip_stream) {
        c->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return CCG_ERR_DEVICE;
        }
        c->own_stream = true;
    }
    if (hipHostMalloc(reinterpret_cast<void**>(&c->st_host), sizeof(DevState), hipHostMallocDefault) != hipSuccess) {
        if (c->own_stream) (void)hipStreamDestroy(c->stream);
        delete c;
        return CCG_ERR_DEVICE;
    }
    std::memset(c->st_host, 0, sizeof(DevState));
    // the device address of this device's scratch array (ccg_solve_noalloc)
    void* sp = nullptr;
    if (scratch_setup(device, &sp) == hipSuccess) {
        c->scratch = sp;
    } else {
        (void)hipGetLastError();
    }
    *ctx = c;
    return CCG_OK;
}

ccg_status ccg_destroy(ccg_ctx* c) {
    if (!c) return CCG_OK;
    (void)hipSetDevice(c->device);
    stop_server(c);
    (void)hipStreamSynchronize(c->stream);
    free_workspace(c);
    if (c->acopy) (void)hipFree(c->acopy);
    if (c->lowA) (void)hipFree(c->lowA);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->st_host) (void)hipHostFree(c->st_host);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return CCG_OK;
}

const char* ccg_last_error(const ccg_ctx* c) { return c ? c->err.c_str() : "null context"; }

// Precision escalation (CCG_ESCALATE): a refinement that breaks down (no progress,
// or a low-precision inner solve whose Gram matrix is not positive or not finite)
// continues from its agents in the next wider precision.
bool escalates(const ccg_opts& o, ccg_status r) {
    return (o.flags & CCG_ESCALATE) && o.prec != CCG_FP64 &&
           (r == CCG_ERR_BREAKDOWN || r == CCG_ERR_NOT_SPD || r == CCG_ERR_NONFINITE);
}

ccg_opts next_precision(const ccg_opts* user, const ccg_opts& cur) {
    ccg_opts u;
    std::memset(&u, 0, sizeof u);
    if (user) u = *user;
    u.prec = cur.prec == CCG_BF16X2 ? CCG_FP32 : CCG_FP64;
    return fill_defaults(&u);
}

void accumulate_stage(ccg_info& acc, const ccg_info& stage) {
    acc.iters += stage.iters;
    acc.refinements += stage.refinements;
    acc.restarts += stage.restarts;
    acc.deflations += stage.deflations;
    acc.reinflations += stage.reinflations;
    acc.bytes_A += stage.bytes_A;
}

ccg_status ccg_solve(ccg_ctx* c, int n, int p, const double* A, int64_t lda, const double* b, double* X,
                     int64_t ldx, double tol, int maxit, const ccg_opts* opts, ccg_info* info) {
    ccg_info local;
    std::memset(&local, 0, sizeof local);
    local.best_agent = -1;
    ccg_status st = guarded(c, [&]() -> ccg_status {
        check_common(n, p, A, lda, b, X, ldx);
        if (!(tol > 0.0)) throw CcgError{CCG_ERR_ARG, "tol must be > 0"};
        if (maxit < 0) throw CcgError{CCG_ERR_ARG, "maxit must be >= 0"};
        const ccg_opts o = fill_defaults(opts);
        if (o.prec != CCG_FP64 && o.prec != CCG_FP32 && o.prec != CCG_BF16X2)
            throw CcgError{CCG_ERR_ARG, "unknown precision mode"};
        if (o.prec != CCG_FP64 && p > kLowMaxP)
            throw CcgError{CCG_ERR_ARG, "p > 16 runs with CCG_FP64 only"};
        if ((o.flags & CCG_REINFLATE) && (o.prec != CCG_FP64 || (o.flags & CCG_ESCALATE)))
            throw CcgError{CCG_ERR_ARG, "CCG_REINFLATE runs with CCG_FP64 only"};
        const auto t0 = std::chrono::steady_clock::now();
        Staged sg;
        double* Xd = X;
        int64_t ldxd = ldx;
        if (o.flags & CCG_HOST_PTRS) stage_in(c, sg, n, p, A, lda, b, Xd, ldxd);
        ccg_status r = CCG_OK;
        ccg_opts oo = o;
        ccg_info acc;
        std::memset(&acc, 0, sizeof acc);
        for (;;) {
            const int left = maxit - acc.iters;
            r = oo.prec == CCG_FP64 ? solve_fp64(c, n, p, A, lda, b, Xd, ldxd, tol, left, oo, local)
                                    : solve_mixed(c, n, p, A, lda, b, Xd, ldxd, tol, left, oo, local);
            accumulate_stage(acc, local);
            if (!escalates(oo, r) || maxit - acc.iters <= 0) break;
            // X holds the agents of the last completed outer step: go on from them in
            // the next wider precision
            oo = next_precision(opts, oo);
        }
        local.prec_final = oo.prec;
        local.iters = acc.iters;
        local.refinements = acc.refinements;
        local.restarts = acc.restarts;
        local.deflations = acc.deflations;
        local.reinflations = acc.reinflations;
        local.bytes_A = acc.bytes_A;
        if (o.flags & CCG_HOST_PTRS) {
            HIP_OK(hipMemcpy2DAsync(X, sizeof(double) * ldx, Xd, sizeof(double) * n, sizeof(double) * n, p,
                                    hipMemcpyDeviceToHost, c->stream));
            HIP_OK(hipStreamSynchronize(c->stream));
        }
        local.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        return r;
    });
    local.status = st;
    if (info) *info = local;
    return st;
}

ccg_status ccg_solve_noalloc(ccg_ctx* c, int n, int p, const double* A, int64_t lda, const double* b,
                             double* X, int64_t ldx, double tol, int maxit, const ccg_opts* opts,
                             ccg_info* info) {
    ccg_info local;
    std::memset(&local, 0, sizeof local);
    local.best_agent = -1;
    ccg_status st = guarded(c, [&]() -> ccg_status {
        check_common(n, p, A, lda, b, X, ldx);
        if (!(tol > 0.0)) throw CcgError{CCG_ERR_ARG, "tol must be > 0"};
        if (maxit < 0) throw CcgError{CCG_ERR_ARG, "maxit must be >= 0"};
        ccg_opts o = fill_defaults(opts);
        if (o.prec != CCG_FP64)
            throw CcgError{CCG_ERR_ARG, "the allocation-free solve runs CCG_FP64 only"};
        if (o.flags & (CCG_HOST_PTRS | CCG_PROFILE | CCG_PROFILE_SAMPLED | CCG_SYM_AD | CCG_ESCALATE |
                       CCG_REINFLATE))
            throw CcgError{CCG_ERR_ARG, "the allocation-free solve takes device pointers and no "
                                        "CCG_HOST_PTRS, CCG_PROFILE*, CCG_SYM_AD or CCG_ESCALATE"};
        if (reinterpret_cast<uintptr_t>(A) % 16 != 0 || (lda * sizeof(double)) % 16 != 0)
            throw CcgError{CCG_ERR_ARG, "the allocation-free solve needs 16-byte aligned columns of A "
                                        "(A aligned, lda even)"};
        if (!c->scratch) throw CcgError{CCG_ERR_DEVICE, "the device scratch array is not available"};
        const int P = pad_agents(p);
        const int n_pad = (int)round_up(n, kRowAlign);
        Workspace w;
        const size_t need = carve(w, nullptr, n, n_pad, P);
        if (need > scratch_bytes())
            throw CcgError{CCG_ERR_NOMEM, "the allocation-free solve needs " + std::to_string(need) +
                                              " bytes of scratch for n = " + std::to_string(n) + ", p = " +
                                              std::to_string(p) + "; the maximum is " +
                                              std::to_string(scratch_bytes())};
        carve(w, static_cast<char*>(c->scratch), n, n_pad, P);
        w.base = nullptr;      // not owned: never freed
        w.bytes = need;
        w.n = n;
        w.n_pad = n_pad;
        w.P = P;
        // the scratch keeps the last call's contents: padded rows, tickets and state
        // start from zero
        HIP_OK(launch_zero(c->scratch, need, c->stream));
        o.flags |= CCG_NO_GRAPH;
        const auto t0 = std::chrono::steady_clock::now();
        const ccg_status r = with_workspace(c, w, [&]() {
            return fp64_steps(c, n, p, A, lda, b, X, ldx, tol, maxit, o, local);
        });
        local.prec_final = CCG_FP64;
        local.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        return r;
    });
    local.status = st;
    if (info) *info = local;
    return st;
}

ccg_status ccg_debug_step(ccg_ctx* c, int n, int p, const double* A, int64_t lda, const double* b,
                          double* X, int64_t ldx, int ksteps, const ccg_opts* opts, double* alphas,
                          double* betas, double* R, double* D) {
    return guarded(c, [&]() -> ccg_status {
        check_common(n, p, A, lda, b, X, ldx);
        if (ksteps < 0) throw CcgError{CCG_ERR_ARG, "ksteps must be >= 0"};
        const ccg_opts o = fill_defaults(opts);
        const int P = pad_agents(p);
        const double* Ause = aligned_matrix(c, n, A, lda);
        Solve s{c, n, p, P, PREC_F64, Ause, nullptr, lda, Ause, lda, 0, (o.flags & CCG_SYM_AD) != 0};
        set_shape(s, o);
        ensure_workspace(c, n, P, s.sym_ad);
        Workspace& w = c->ws;
        HIP_OK(launch_pack(n, w.n_pad, p, P, X, ldx, w.Xr, c->stream));
        HIP_OK(launch_pad_vec(n, w.n_pad, b, w.bp, c->stream));
        DevState& h = *c->st_host;
        std::memset(&h, 0, sizeof(DevState));
        h.done = RUNNING;
        h.m = p;
        h.mask = (p >= 32) ? 0xffffffffu : ((1u << p) - 1u);
        for (int j = 0; j < p; ++j) h.keep[j] = j;
        h.maxit = ksteps + 1;   // never reached: every step runs to the end
        h.tol = -1.0;           // no stop test
        h.tau = o.rank_tau;
        h.nb = 1.0;
        write_state(c);
        enqueue_residual(s, RES_INIT, 1);
        read_state(c);
        for (int k = 0; k < ksteps && h.done == RUNNING; ++k) {
            enqueue_step(s, 0, false);
            read_state(c);
            for (int cc = 0; cc < p; ++cc)
                for (int r = 0; r < p; ++r) {
                    if (alphas) alphas[(size_t)k * p * p + r + cc * p] = h.alpha[r * kMaxP + cc];
                    if (betas) betas[(size_t)k * p * p + r + cc * p] = h.beta[r * kMaxP + cc];
                }
        }
        HIP_OK(launch_unpack(n, w.n_pad, p, w.Xr, X, ldx, c->stream));
        if (R) HIP_OK(launch_unpack(n, w.n_pad, p, w.R, R, n, c->stream));
        if (D) HIP_OK(launch_unpack(n, w.n_pad, p, w.D, D, n, c->stream));
        HIP_OK(hipStreamSynchronize(c->stream));
        if (h.done == FAILED) return (ccg_status)h.status;
        return CCG_OK;
    });
}

ccg_status ccg_convert_matrix(ccg_ctx* c, int n, const double* A, int64_t lda, int prec, void* hi, void* lo) {
    return guarded(c, [&]() -> ccg_status {
        if (n < 1 || !A || !hi || lda < n) throw CcgError{CCG_ERR_ARG, "bad matrix argument"};
        if (prec != CCG_FP32 && prec != CCG_BF16X2) throw CcgError{CCG_ERR_ARG, "prec must be FP32 or BF16X2"};
        if (prec == CCG_BF16X2 && !lo) throw CcgError{CCG_ERR_ARG, "BF16X2 needs the lo plane"};
        HIP_OK(launch_convert(prec == CCG_FP32 ? PREC_F32 : PREC_BF16X2, n, A, lda, hi, lo, n, c->stream));
        HIP_OK(hipStreamSynchronize(c->stream));
        return CCG_OK;
    });
}

ccg_status ccg_tune_ad(ccg_ctx* c, int prec, int p, int n, int cw, int nw, int batched, int reps, double* us) {
    return guarded(c, [&]() -> ccg_status {
        if (n < 1 || p < 1 || p > (prec == CCG_FP64 ? kMaxP : kLowMaxP) || p > n || reps < 1 || !us ||
            (cw != 1 && cw != 2 && cw != 4) ||
            (nw != 4 && nw != 8 && nw != 16) || (batched != 0 && batched != 1))
            throw CcgError{CCG_ERR_ARG, "bad tuning argument"};
        if (prec != CCG_FP64 && prec != CCG_FP32 && prec != CCG_BF16X2) throw CcgError{CCG_ERR_ARG, "bad precision"};
        const int pr = prec == CCG_FP64 ? PREC_F64 : (prec == CCG_FP32 ? PREC_F32 : PREC_BF16X2);
        const int P = pad_agents(p);
        const int64_t lda = round_up(n, 2);
        double* A = nullptr;
        if (hipMalloc(&A, sizeof(double) * (size_t)lda * n) != hipSuccess)
            throw CcgError{CCG_ERR_NOMEM, "tuning matrix allocation failed"};
        struct Free {
            double* p;
            ~Free() { (void)hipFree(p); }
        } fa{A};
        HIP_OK(launch_tune_matrix(n, A, lda, c->stream));
        ensure_workspace(c, n, P);
        Workspace& w = c->ws;
        const int64_t blk = (int64_t)w.n_pad * P;
        HIP_OK(launch_tune_vectors(blk, w.D, w.Dl, 1u, c->stream));
        HIP_OK(launch_tune_vectors(blk, w.R, w.Rl, 2u, c->stream));
        const LowCopy lc = pr == PREC_F64 ? LowCopy{A, nullptr, lda, 0.0} : low_copy(c, n, A, lda, pr);
        Solve s{c, n, p, P, pr, lc.hi, lc.lo, lc.ld, A, lda, 0};
        DevState& h = *c->st_host;
        std::memset(&h, 0, sizeof(DevState));
        h.done = RUNNING;
        set_all_agents(h, p);
        h.maxit = 1 << 30;
        h.tol = 0.0;           // the stop test never passes: every launch runs in full
        h.tau = 1e-14;
        h.nb = 1.0;
        write_state(c);
        hipEvent_t e0 = pooled_event(c, 0), e1 = pooled_event(c, 1);
        const AdArgs a = ad_args(s, false);
        // the batched kernel runs the system's tiles as (system 0, tile) work items
        void* bbuf = nullptr;
        struct FreeB {
            void*& p;
            ~FreeB() { if (p) (void)hipFree(p); }
        } fb{bbuf};
        const int rows = ad_fit_rows(pr, P, cw, nw);
        const int ntiles = (n + rows - 1) / rows;
        AdArgs* d_sys = nullptr;
        int4* d_items = nullptr;
        if (batched) {
            const size_t ioff = round_up((int64_t)sizeof(AdArgs), 256);
            if (hipMalloc(&bbuf, ioff + sizeof(int4) * (size_t)ntiles) != hipSuccess)
                throw CcgError{CCG_ERR_NOMEM, "tuning item list allocation failed"};
            d_sys = static_cast<AdArgs*>(bbuf);
            d_items = reinterpret_cast<int4*>(static_cast<char*>(bbuf) + ioff);
            std::vector<int4> items((size_t)ntiles);
            for (int t = 0; t < ntiles; ++t) items[(size_t)t] = int4{0, t, 0, 0};
            HIP_OK(hipMemcpy(d_sys, &a, sizeof(AdArgs), hipMemcpyHostToDevice));
            HIP_OK(hipMemcpy(d_items, items.data(), sizeof(int4) * (size_t)ntiles, hipMemcpyHostToDevice));
        }
        double tot = 0.0;
        for (int i = 0; i < reps + 2; ++i) {
            if (batched) {
                HIP_OK(hipEventRecord(e0, c->stream));
                HIP_OK(launch_ad_batch(pr, P, cw, nw, d_sys, d_items, ntiles, c->stream));
                HIP_OK(hipEventRecord(e1, c->stream));
            } else {
                HIP_OK(launch_ad_cw(pr, P, cw, nw, a, c->stream, e0, e1));
            }
            HIP_OK(hipStreamSynchronize(c->stream));
            float ms = 0.f;
            HIP_OK(hipEventElapsedTime(&ms, e0, e1));
            if (i >= 2) tot += ms;
        }
        *us = tot * 1e3 / reps;
        return CCG_OK;
    });
}

ccg_status ccg_kernel_time(ccg_ctx* c, double* ms, long long* launches, double* bytes, int reset) {
    if (!c) return CCG_ERR_ARG;
    if (ms) *ms = c->prof_ms;
    if (launches) *launches = c->prof_launches;
    if (bytes) *bytes = c->prof_bytes;
    if (reset) {
        c->prof_ms = 0.0;
        c->prof_launches = 0;
        c->prof_bytes = 0.0;
    }
    return CCG_OK;
}

}  // extern "C"
