// Multi-system engine: many independent cCG solves advanced together by batched
// launches (ccg_solve_batched), and the continuous-batching service built on it
// (ccg_submit / ccg_poll / ccg_wait / ccg_cancel).
//
// Every resident system owns a slot: its device state (one DevState array for all
// slots, so one strided copy reads or writes every state header), its argument
// records for the batched kernels (AdArgs / UpdArgs / ResArgs arrays indexed by
// slot) and its vectors in an arena of device memory.  One host round launches:
//   1. the refinement corrections X += E * scale due this round (per system),
//   2. one batched explicit-residual pass (FP64 A.X, then the residual epilogue)
//      over every system that needs one, per padded agent count,
//   3. the starts of refinement inner solves (per system),
//   4. k block steps over every resident system (k by lane and mode, kRoundSteps):
//      per (precision, padded agent count, tile shape) class, k triples of batched
//      A.D, update and direction launches on a stream of the class, replayed from a graph
//      captured on that stream; the class streams fork from and join back into the
//      engine stream (a step is a no-op for a system that is not running),
// then reads every state header and moves each system through the same phases,
// in the same order, as the single-system driver, so a system's result does not
// depend on the systems it shares launches with.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <exception>
#include <cstddef>
#include <cstdio>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "ccg_host.h"

namespace ccg {
namespace host {
namespace {

constexpr size_t kHeader = offsetof(DevState, alpha);   // state bytes exchanged per round
constexpr int kSlots = 4096;                             // resident systems at most
constexpr size_t kChunk = size_t(1) << 30;               // arena growth step
constexpr size_t kHeadroom = size_t(2) << 30;            // device memory left to others

using Clock = std::chrono::steady_clock;

// First-fit allocator over device memory chunks.  Chunks grow in kChunk steps up
// to the cap (0: what the device reports free, less a headroom) and are returned
// only when the arena is destroyed (hipFree synchronises the device).  The lanes
// of one batched call or of one service share an arena, so it is locked.
class Arena {
  public:
    explicit Arena(size_t cap) : cap_(cap) {}
    ~Arena() {
        for (auto& c : chunks_) (void)hipFree(c.base);
    }
    Arena(const Arena&) = delete;
    Arena& operator=(const Arena&) = delete;

    // nullptr when `bytes` does not fit now
    char* alloc(size_t bytes) {
        std::lock_guard<std::mutex> lk(mu_);
        bytes = (size_t)round_up((int64_t)bytes, 256);
        for (auto& c : chunks_) {
            char* p = take(c, bytes);
            if (p) return p;
        }
        size_t want = std::max(bytes, kChunk);
        if (cap_) {
            if (total_ + bytes > cap_) return nullptr;
            want = std::min(want, cap_ - total_);
        } else {
            size_t fr = 0, tot = 0;
            if (hipMemGetInfo(&fr, &tot) != hipSuccess || fr < bytes + kHeadroom) return nullptr;
            want = std::min(want, fr - kHeadroom);
        }
        void* base = nullptr;
        if (hipMalloc(&base, want) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        chunks_.push_back(Chunk{static_cast<char*>(base), want, {}});
        chunks_.back().free[0] = want;
        total_ += want;
        return take(chunks_.back(), bytes);
    }

    void release(char* p) {
        std::lock_guard<std::mutex> lk(mu_);
        auto u = used_.find(p);
        if (u == used_.end()) return;
        const size_t bytes = u->second;
        used_.erase(u);
        for (auto& c : chunks_) {
            if (p < c.base || p >= c.base + c.size) continue;
            size_t off = (size_t)(p - c.base), size = bytes;
            auto nx = c.free.lower_bound(off);
            if (nx != c.free.end() && off + size == nx->first) {
                size += nx->second;
                nx = c.free.erase(nx);
            }
            if (nx != c.free.begin()) {
                auto pv = std::prev(nx);
                if (pv->first + pv->second == off) {
                    pv->second += size;
                    return;
                }
            }
            c.free[off] = size;
            return;
        }
    }

    // Nothing allocated: a request that does not fit now never will.
    bool empty() const {
        std::lock_guard<std::mutex> lk(mu_);
        return used_.empty();
    }

    // Whether `bytes` could ever fit (the cap, or the device's total memory).
    bool could_fit(size_t bytes) const {
        if (cap_) return bytes <= cap_;
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) return false;
        return bytes + kHeadroom <= tot;
    }

  private:
    struct Chunk {
        char* base;
        size_t size;
        std::map<size_t, size_t> free;   // offset -> size
    };
    char* take(Chunk& c, size_t bytes) {
        for (auto it = c.free.begin(); it != c.free.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, size = it->second;
            c.free.erase(it);
            if (size > bytes) c.free[off + bytes] = size - bytes;
            char* p = c.base + off;
            used_[p] = bytes;
            return p;
        }
        return nullptr;
    }
    mutable std::mutex mu_;
    size_t cap_;
    size_t total_ = 0;
    std::vector<Chunk> chunks_;
    std::unordered_map<char*, size_t> used_;
};

// Systems run in lanes by size: each lane is an engine with its own stream and
// host thread, so the rounds of small systems (a few microseconds per block step)
// do not wait for the block steps of large ones, which take up to milliseconds.
constexpr int kLanes = 2;
constexpr int kLaneSplit = 4096;   // n at or above: the large-system lane
inline int lane_of(int n) { return n >= kLaneSplit ? 1 : 0; }
// Block steps per round: the small-system lane takes long rounds (its steps cost
// microseconds, so the header exchange of a round would weigh on short ones); the
// large-system lane shorter ones, so its phase changes wait less.
constexpr int kRoundSteps[2][kLanes] = {{32, 16},    // batched
                                        {32, 8}};    // served

enum Phase : int {
    PH_INIT_RES,     // waiting for / past the first explicit residual
    PH_STEP,         // FP64 block steps
    PH_CONFIRM,      // FP64 confirmation of the recurrence stop test
    PH_FINAL,        // FP64 report residual after maxit
    PH_INNER,        // low-precision inner solve
    PH_OUTER_RES,    // FP64 residual after a refinement correction
};

struct Sys {
    uint64_t tag = 0;
    int slot = -1;
    // problem
    int n = 0, p = 0, P = 0, prec = PREC_F64;
    // A.D tile shapes (columns per wave, waves per workgroup) of the block step and
    // of the explicit residual
    int cw_step = 2, nw_step = 4, cw_res = 2, nw_res = 4;
    double tol = 0.0;
    int maxit = 0;
    ccg_opts o{};
    double* X_out = nullptr;    // caller's X (device, or host with CCG_HOST_PTRS)
    int64_t ldx = 0;
    bool host = false;
    // device memory
    char* mem = nullptr;
    Workspace w;
    const double* A64 = nullptr;
    int64_t lda64 = 0;
    const void* lowhi = nullptr;
    const void* lowlo = nullptr;
    int64_t ldlow = 0;
    double* Xdev = nullptr;     // device X buffer of a host-pointer system
    // phase machine
    Phase ph = PH_INIT_RES;
    bool res_due = true;        // an explicit residual is launched this round
    int res_mode = RES_INIT;
    int res_set_nb = 1;
    bool refine_due = false;    // X += E * scale this round
    bool inner_start_due = false;
    int iter_before = 0;
    int streams_before = 0;           // A.D launches that streamed A, before the round
    // low-precision outer loop
    double nb = 1.0, best = 0.0;
    int iters = 0, refinements = 0, stall = 0;
    double in_tol = 0.0;        // inner tolerance, following the outer contraction
    double prev_minres = 0.0;   // FP64 residual before the current outer step
    RefArgs ra{};
    // totals of earlier precision stages (CCG_ESCALATE)
    ccg_opts o_user{};
    int iters_done = 0, refinements_done = 0, deflations_done = 0;
    // report
    double bytes = 0.0;
    Clock::time_point t0;
    ccg_status status = CCG_OK;
    bool cancel = false;
};

// The block step's A.D tile shape of a system: the caller's (ccg_opts ad_cw, ad_nw;
// fitted to a shape the launchers run), else the tuned table's.
void step_shape(Sys& sy, const ccg_opts& o) {
    if (o.ad_cw > 0 || o.ad_nw > 0) {
        const int nw = o.ad_nw > 0 ? o.ad_nw : 4;
        sy.nw_step = ad_fit_nw(sy.prec, sy.P, nw);
        sy.cw_step = ad_fit_cw(sy.prec, sy.P, o.ad_cw > 0 ? o.ad_cw : 2, nw);
    } else {
        sy.cw_step = ad_cw(sy.prec, sy.P, sy.n);
        sy.nw_step = ad_nw(sy.prec, sy.P, sy.n);
    }
}

struct Finished {
    uint64_t tag;
    ccg_status status;
    ccg_info info;
};

class Engine {
    // a step class's items: A.D tiles at ad_off, update tiles at up_off in the list
    struct StepRange {
        int prec, P, cw, nw;
        size_t ad_off, ad_n, up_off, up_n, dir_off, dir_n;
    };

  public:
    // class_streams: run the step classes on streams of their own (see rebuild_steps),
    // or all in order on the engine stream.
    Engine(int device, hipStream_t stream, Arena& arena, bool use_graph = true, bool class_streams = true)
        : device_(device), s_(stream), arena_(arena), use_graph_(use_graph), class_streams_on_(class_streams) {
        HIP_OK(hipMalloc(&states_, sizeof(DevState) * kSlots));
        HIP_OK(hipMalloc(&d_ad_, sizeof(AdArgs) * kSlots));
        HIP_OK(hipMalloc(&d_res_ad_, sizeof(AdArgs) * kSlots));
        HIP_OK(hipMalloc(&d_upd_, sizeof(UpdArgs) * kSlots));
        HIP_OK(hipMalloc(&d_small_, sizeof(SmallArgs) * kSlots));
        HIP_OK(hipMalloc(&d_res_, sizeof(ResArgs) * kSlots));
        HIP_OK(hipHostMalloc(reinterpret_cast<void**>(&h_states_), sizeof(DevState) * kSlots,
                             hipHostMallocDefault));
        std::memset(h_states_, 0, sizeof(DevState) * kSlots);
        for (int i = kSlots - 1; i >= 0; --i) free_slots_.push_back(i);
    }
    ~Engine() {
        (void)hipStreamSynchronize(s_);
        (void)hipFree(states_);
        (void)hipFree(d_ad_);
        (void)hipFree(d_res_ad_);
        (void)hipFree(d_upd_);
        (void)hipFree(d_small_);
        (void)hipFree(d_res_);
        for (hipGraphExec_t g : class_graphs_) (void)hipGraphExecDestroy(g);
        for (hipStream_t cs : class_streams_) (void)hipStreamDestroy(cs);
        for (hipEvent_t ev : class_events_) (void)hipEventDestroy(ev);
        if (fork_) (void)hipEventDestroy(fork_);
        if (d_items_) (void)hipFree(d_items_);
        if (h_items_) (void)hipHostFree(h_items_);
        if (d_step_) (void)hipFree(d_step_);
        if (h_step_) (void)hipHostFree(h_step_);
        (void)hipHostFree(h_states_);
    }

    bool idle() const { return live_.empty(); }
    size_t live() const { return live_.size(); }

    // Device bytes a problem needs while resident.
    static size_t footprint(const ccg_problem& pr, const ccg_opts& o) {
        const int P = pad_agents(pr.p);
        const int n_pad = (int)round_up(pr.n, kRowAlign);
        Workspace tmp;
        size_t b = round_up((int64_t)carve(tmp, nullptr, pr.n, n_pad, P), 256);
        const bool host = (o.flags & CCG_HOST_PTRS) != 0;
        const bool aligned = !host && reinterpret_cast<uintptr_t>(pr.A) % 16 == 0 && (pr.lda * 8) % 16 == 0;
        if (!aligned) b += round_up((int64_t)sizeof(double) * round_up(pr.n, 2) * pr.n, 256);
        if (host) b += round_up((int64_t)sizeof(double) * pr.n, 256) + round_up((int64_t)sizeof(double) * pr.n * pr.p, 256);
        if (o.prec == CCG_FP32) b += round_up((int64_t)sizeof(float) * round_up(pr.n, 4) * pr.n, 256);
        if (o.prec == CCG_BF16X2) b += 2 * round_up((int64_t)sizeof(uint16_t) * round_up(pr.n, 8) * pr.n, 256);
        return b;
    }

    bool could_fit(size_t bytes) const { return arena_.could_fit(bytes); }

    // Make a problem resident and enqueue its set-up.  Returns false (nothing done)
    // when there is no slot or no memory for it right now.  Throws CcgError on an
    // invalid problem.
    bool admit(const ccg_problem& pr, uint64_t tag) {
        const ccg_opts o = fill_defaults(&pr.opts);
        check_common(pr.n, pr.p, pr.A, pr.lda, pr.b, pr.X, pr.ldx);
        if (pr.p > kLowMaxP) throw CcgError{CCG_ERR_ARG, "batched and served problems take p <= 16"};
        if (!(pr.tol > 0.0)) throw CcgError{CCG_ERR_ARG, "tol must be > 0"};
        if (pr.maxit < 0) throw CcgError{CCG_ERR_ARG, "maxit must be >= 0"};
        if (o.prec != CCG_FP64 && o.prec != CCG_FP32 && o.prec != CCG_BF16X2)
            throw CcgError{CCG_ERR_ARG, "unknown precision mode"};
        if (o.flags & CCG_REINFLATE)
            throw CcgError{CCG_ERR_ARG, "CCG_REINFLATE is a ccg_solve option (not batched or served)"};
        if (free_slots_.empty()) return false;
        const size_t need = footprint(pr, o);
        char* mem = arena_.alloc(need);
        if (!mem) return false;
        Sys sy;
        sy.tag = tag;
        sy.slot = free_slots_.back();
        free_slots_.pop_back();
        sy.n = pr.n;
        sy.p = pr.p;
        sy.P = pad_agents(pr.p);
        sy.prec = o.prec == CCG_FP64 ? PREC_F64 : (o.prec == CCG_FP32 ? PREC_F32 : PREC_BF16X2);
        step_shape(sy, o);
        if (small_tier(sy.P, pr.n, o.flags)) sy.cw_step = sy.nw_step = 0;   // the tier's class
        sy.cw_res = ad_cw(PREC_F64, sy.P, pr.n);
        sy.nw_res = ad_nw(PREC_F64, sy.P, pr.n);
        sy.tol = pr.tol;
        sy.maxit = pr.maxit;
        sy.o = o;
        sy.o_user = pr.opts;
        sy.X_out = pr.X;
        sy.ldx = pr.ldx;
        sy.host = (o.flags & CCG_HOST_PTRS) != 0;
        sy.mem = mem;
        sy.t0 = Clock::now();
        const int n = sy.n, p = sy.p, P = sy.P;
        const int n_pad = (int)round_up(n, kRowAlign);
        Carver cv{mem};
        const size_t wsb = carve(sy.w, mem, n, n_pad, P);
        sy.w.base = mem;
        sy.w.bytes = wsb;
        sy.w.n = n;
        sy.w.n_pad = n_pad;
        sy.w.P = P;
        cv.off = wsb;
        HIP_OK(hipMemsetAsync(mem, 0, wsb, s_));
        // FP64 matrix (uploaded, or the caller's, copied when its columns are unaligned)
        const double* A = pr.A;
        int64_t lda = pr.lda;
        const double* b = pr.b;
        const double* X0 = pr.X;
        int64_t ldx0 = pr.ldx;
        const bool aligned = !sy.host && reinterpret_cast<uintptr_t>(A) % 16 == 0 && (lda * 8) % 16 == 0;
        if (!aligned) {
            const int64_t ldb = round_up(n, 2);
            double* Ac = cv.take<double>((size_t)ldb * n);
            if (sy.host) {
                HIP_OK(hipMemcpy2DAsync(Ac, sizeof(double) * ldb, A, sizeof(double) * lda, sizeof(double) * n, n,
                                        hipMemcpyHostToDevice, s_));
            } else {
                HIP_OK(launch_copy_cols(n, A, lda, Ac, ldb, s_));
            }
            A = Ac;
            lda = ldb;
        }
        if (sy.host) {
            double* bd = cv.take<double>((size_t)n);
            double* Xd = cv.take<double>((size_t)n * p);
            HIP_OK(hipMemcpyAsync(bd, b, sizeof(double) * n, hipMemcpyHostToDevice, s_));
            HIP_OK(hipMemcpy2DAsync(Xd, sizeof(double) * n, X0, sizeof(double) * ldx0, sizeof(double) * n, p,
                                    hipMemcpyHostToDevice, s_));
            b = bd;
            X0 = Xd;
            ldx0 = n;
            sy.Xdev = Xd;
        }
        sy.A64 = A;
        sy.lda64 = lda;
        if (sy.prec != PREC_F64) {
            const int64_t ld = round_up(n, sy.prec == PREC_F32 ? 4 : 8);
            if (sy.prec == PREC_F32) {
                float* hi = cv.take<float>((size_t)ld * n);
                HIP_OK(launch_convert(PREC_F32, n, A, lda, hi, nullptr, ld, s_));
                sy.lowhi = hi;
            } else {
                uint16_t* hi = cv.take<uint16_t>((size_t)ld * n);
                uint16_t* lo = cv.take<uint16_t>((size_t)ld * n);
                HIP_OK(launch_convert(PREC_BF16X2, n, A, lda, hi, lo, ld, s_));
                sy.lowhi = hi;
                sy.lowlo = lo;
            }
            sy.ldlow = ld;
            sy.bytes += (double)n * n * (8.0 + 4.0);
        }
        HIP_OK(launch_pack(n, n_pad, p, P, X0, ldx0, sy.w.Xr, s_));
        HIP_OK(launch_pad_vec(n, n_pad, b, sy.w.bp, s_));
        // argument records of the batched kernels, and the initial state (written with
        // every header at the start of the next round)
        write_records(sy);
        start_stage(sy);
        sy.ra.n_pad = n_pad;
        sy.ra.P = P;
        sy.ra.T = sy.w.R;
        sy.ra.X = sy.w.Xr;
        sy.ra.E = sy.w.E;
        sy.ra.R = sy.w.Rl;
        sy.ra.D = sy.w.Dl;
        if (sy.slot + 1 > hi_slot_) hi_slot_ = sy.slot + 1;
        live_.push_back(sy);
        items_dirty_ = true;
        return true;
    }

    // Argument records of a system's batched kernels (its current precision).
    void write_records(const Sys& sy) {
        const int n = sy.n, n_pad = sy.w.n_pad;
        DevState* st = states_ + sy.slot;
        AdArgs ad{};
        ad.n = n;
        ad.n_pad = n_pad;
        ad.product_only = 0;
        ad.red = sy.w.red_ad;
        ad.st = st;
        if (sy.prec == PREC_F64) {
            ad.A = sy.A64;
            ad.A_lo = nullptr;
            ad.lda = sy.lda64;
            ad.V = sy.w.D;
            ad.R = sy.w.R;
            ad.AD = sy.w.AD;
        } else {
            ad.A = sy.lowhi;
            ad.A_lo = sy.lowlo;
            ad.lda = sy.ldlow;
            ad.V = sy.w.Dl;
            ad.R = sy.w.Rl;
            ad.AD = sy.w.ADl;
        }
        AdArgs ra = ad;
        ra.product_only = 1;
        ra.A = sy.A64;
        ra.A_lo = nullptr;
        ra.lda = sy.lda64;
        ra.V = sy.w.Xr;
        ra.R = sy.w.R;
        ra.AD = sy.w.AD;
        UpdArgs u{};
        u.n_pad = n_pad;
        if (sy.prec == PREC_F64) {
            u.X = sy.w.Xr; u.R = sy.w.R; u.D = sy.w.D; u.AD = sy.w.AD;
        } else {
            u.X = sy.w.E; u.R = sy.w.Rl; u.D = sy.w.Dl; u.AD = sy.w.ADl;
        }
        u.red = sy.w.red_up;
        u.st = st;
        ResArgs r{};
        r.n = n;
        r.n_pad = n_pad;
        r.p = sy.p;
        r.mode = RES_INIT;
        r.set_nb = 1;
        r.b = sy.w.bp;
        r.Y = sy.w.AD;
        r.R = sy.w.R;
        r.D = sy.w.D;
        r.red = sy.w.red_res;
        r.st = st;
        HIP_OK(hipMemcpyAsync(d_ad_ + sy.slot, &ad, sizeof ad, hipMemcpyHostToDevice, s_));
        HIP_OK(hipMemcpyAsync(d_res_ad_ + sy.slot, &ra, sizeof ra, hipMemcpyHostToDevice, s_));
        HIP_OK(hipMemcpyAsync(d_upd_ + sy.slot, &u, sizeof u, hipMemcpyHostToDevice, s_));
        SmallArgs sm{};
        sm.A = ad.A;
        sm.A_lo = ad.A_lo;
        sm.lda = ad.lda;
        sm.n = n;
        sm.X = u.X;
        sm.R = u.R;
        sm.D = u.D;
        sm.st = st;
        HIP_OK(hipMemcpyAsync(d_small_ + sy.slot, &sm, sizeof sm, hipMemcpyHostToDevice, s_));
        HIP_OK(hipMemcpyAsync(d_res_ + sy.slot, &r, sizeof r, hipMemcpyHostToDevice, s_));
    }

    // Initial state of a (new or escalated) stage: the first explicit residual is due.
    void start_stage(Sys& sy) {
        DevState& h = h_states_[sy.slot];
        std::memset(&h, 0, kHeader);
        h.done = RUNNING;
        set_all_agents(h, sy.p);
        h.maxit = sy.maxit - sy.iters_done;
        h.tol = sy.tol;
        h.tau = sy.o.rank_tau;
        h.nb = 1.0;
        sy.ph = PH_INIT_RES;
        sy.res_due = true;
        sy.res_mode = sy.prec == PREC_F64 ? RES_INIT : RES_REFINE;
        sy.res_set_nb = 1;
        sy.iters = 0;
        sy.refinements = 0;
        sy.stall = 0;
        sy.in_tol = sy.o.inner_tol;
    }

    // CCG_ESCALATE: the refinement broke down; the system goes on from its FP64 agents
    // in the next wider precision, as the single driver does.
    bool escalate(Sys& sy, ccg_status st) {
        if (!(sy.o_user.flags & CCG_ESCALATE) || sy.prec == PREC_F64) return false;
        if (st != CCG_ERR_BREAKDOWN && st != CCG_ERR_NOT_SPD && st != CCG_ERR_NONFINITE) return false;
        const DevState& h = h_states_[sy.slot];
        sy.iters_done += sy.iters;
        sy.refinements_done += sy.refinements;
        sy.deflations_done += h.deflations;
        if (sy.maxit - sy.iters_done <= 0) return false;
        ccg_opts u = sy.o_user;
        u.prec = sy.prec == PREC_BF16X2 ? CCG_FP32 : CCG_FP64;
        sy.o = fill_defaults(&u);
        if (sy.prec == PREC_BF16X2) {
            // the FP32 copy fits where the two BF16 planes were
            const int64_t ld = round_up(sy.n, 4);
            float* hi = reinterpret_cast<float*>(const_cast<void*>(sy.lowhi));
            HIP_OK(launch_convert(PREC_F32, sy.n, sy.A64, sy.lda64, hi, nullptr, ld, s_));
            sy.bytes += (double)sy.n * sy.n * 12.0;
            sy.prec = PREC_F32;
            sy.lowlo = nullptr;
            sy.ldlow = ld;
        } else {
            sy.prec = PREC_F64;
        }
        step_shape(sy, sy.o);
        if (small_tier(sy.P, sy.n, sy.o.flags)) sy.cw_step = sy.nw_step = 0;
        write_records(sy);
        start_stage(sy);
        items_dirty_ = true;
        return true;
    }

    void cancel(uint64_t tag) {
        for (auto& sy : live_)
            if (sy.tag == tag) sy.cancel = true;
    }

    // One host round (see the file comment); k block steps for every resident system.
    // The step work list holds every resident system, whatever its phase: a block
    // step is a no-op for a system whose state is not RUNNING, so the list (and the
    // graph captured from it) only changes when systems are admitted, or when the
    // retired systems' items become a large share of it.
    void round(int k) {
        if (live_.empty()) return;
        // cancelled systems leave before any launch
        for (auto& sy : live_)
            if (sy.cancel) retire(sy, CCG_CANCELLED);
        finish_retired();
        if (live_.empty()) return;
        if (items_dirty_ || dead_items_ * 8 > step_items_total_ || graph_k_ != k) rebuild_steps(k);
        // --- explicit-residual work list
        items_.clear();
        struct Range { int P, cw, nw; size_t ad_off, ad_n, up_off, up_n; };
        std::vector<Range> res_ranges;
        for (int P : {1, 2, 4, 8, 16}) {
            for (int cw : {1, 2, 4}) {
                for (int nw : {4, 8, 16}) {
                    Range rr{P, cw, nw, items_.size(), 0, 0, 0};
                    for (auto& sy : live_) {
                        if (!sy.res_due || sy.P != P || sy.cw_res != cw || sy.nw_res != nw) continue;
                        const int t = (sy.n + cw * nw - 1) / (cw * nw);
                        for (int i = 0; i < t; ++i) items_.push_back(int4{sy.slot, i, 0, 0});
                    }
                    rr.ad_n = items_.size() - rr.ad_off;
                    rr.up_off = items_.size();
                    for (auto& sy : live_) {
                        if (!sy.res_due || sy.P != P || sy.cw_res != cw || sy.nw_res != nw) continue;
                        const int t = sy.w.n_pad / (kWG / P);
                        for (int i = 0; i < t; ++i) items_.push_back(int4{sy.slot, i, sy.res_mode, sy.res_set_nb});
                    }
                    rr.up_n = items_.size() - rr.up_off;
                    if (rr.ad_n) res_ranges.push_back(rr);
                }
            }
        }
        upload_items();
        // --- state headers (host decisions of the previous round)
        for (auto& sy : live_) {
            sy.iter_before = h_states_[sy.slot].iter;
            sy.streams_before = h_states_[sy.slot].ad_streams;
        }
        HIP_OK(hipMemcpy2DAsync(states_, sizeof(DevState), h_states_, sizeof(DevState), kHeader, hi_slot_,
                                hipMemcpyHostToDevice, s_));
        // 1. refinement corrections
        for (auto& sy : live_)
            if (sy.refine_due) HIP_OK(launch_refine_add(sy.ra, s_));
        // 2. explicit residuals
        for (const Range& r : res_ranges) {
            HIP_OK(launch_ad_batch(PREC_F64, r.P, r.cw, r.nw, d_res_ad_, d_items_ + r.ad_off, (int)r.ad_n, s_));
            HIP_OK(launch_res_batch(r.P, d_res_, d_items_ + r.up_off, (int)r.up_n, s_));
        }
        // 3. inner-solve starts
        for (auto& sy : live_)
            if (sy.inner_start_due) HIP_OK(launch_inner_init(sy.ra, s_));
        // 4. block steps: each class's k steps on a stream of its own, forked from
        //    and joined back into the engine stream, or one class after the other on
        //    the engine stream
        if (!step_ranges_.empty() && !class_streams_on_) {
            for (size_t c = 0; c < step_ranges_.size(); ++c) {
                if (use_graph_) {
                    HIP_OK(hipGraphLaunch(class_graphs_[c], s_));
                } else {
                    enqueue_class_round(step_ranges_[c], k, s_);
                }
            }
        } else if (!step_ranges_.empty()) {
            HIP_OK(hipEventRecord(fork_, s_));
            for (size_t c = 0; c < step_ranges_.size(); ++c) {
                hipStream_t cs = class_streams_[c];
                HIP_OK(hipStreamWaitEvent(cs, fork_, 0));
                if (use_graph_) {
                    HIP_OK(hipGraphLaunch(class_graphs_[c], cs));
                } else {
                    enqueue_class_round(step_ranges_[c], k, cs);
                }
                HIP_OK(hipEventRecord(class_events_[c], cs));
                HIP_OK(hipStreamWaitEvent(s_, class_events_[c], 0));
            }
        }
        HIP_OK(hipMemcpy2DAsync(h_states_, sizeof(DevState), states_, sizeof(DevState), kHeader, hi_slot_,
                                hipMemcpyDeviceToHost, s_));
        HIP_OK(hipStreamSynchronize(s_));
        // --- advance every system
        for (auto& sy : live_) advance(sy);
        finish_retired();
    }

    std::vector<Finished> take_finished() {
        std::vector<Finished> f;
        f.swap(finished_);
        return f;
    }

  private:
    void advance(Sys& sy) {
        DevState& h = h_states_[sy.slot];
        const double nn = (double)sy.n * sy.n;
        const double s_step = sy.prec == PREC_F64 ? 8.0 : 4.0;
        // A.D launches that streamed A in this round's block steps
        sy.bytes += s_step * nn * (h.ad_streams - sy.streams_before);
        if (sy.res_due) sy.bytes += 8.0 * nn;
        const bool had_res = sy.res_due;
        sy.res_due = false;
        sy.refine_due = false;
        sy.inner_start_due = false;
        if (sy.prec == PREC_F64) {
            switch (sy.ph) {
                case PH_INIT_RES:
                case PH_CONFIRM:
                case PH_STEP:
                    if (h.done == RUNNING) {
                        sy.ph = PH_STEP;
                    } else if (h.done == RECUR_CONV) {
                        sy.ph = PH_CONFIRM;
                        due_res(sy, RES_CONFIRM, 0);
                    } else if (h.done == MAXIT) {
                        sy.ph = PH_FINAL;
                        due_res(sy, RES_FINAL, 0);
                    } else {
                        retire(sy, h.done == FAILED ? (ccg_status)h.status : CCG_OK);
                    }
                    break;
                case PH_FINAL:
                    retire(sy, h.done == FAILED ? (ccg_status)h.status : CCG_NOT_CONVERGED);
                    break;
                default:
                    retire(sy, CCG_ERR_DEVICE);
            }
            return;
        }
        // refinement modes
        switch (sy.ph) {
            case PH_INIT_RES:
                sy.nb = h.nb;
                sy.best = h.minres;
                decide(sy);
                break;
            case PH_INNER:
                if (h.done == RUNNING) break;
                sy.iters += h.iter;
                if (h.done == FAILED) {
                    retire(sy, (ccg_status)h.status);
                    break;
                }
                sy.refine_due = true;
                ++sy.refinements;
                h.done = RUNNING;
                h.tol = sy.tol;
                h.nb = sy.nb;
                set_all_agents(h, sy.p);
                sy.ph = PH_OUTER_RES;
                due_res(sy, RES_REFINE, 0);
                break;
            case PH_OUTER_RES:
                if (!had_res) break;
                if (h.done == FAILED) {
                    retire(sy, (ccg_status)h.status);
                    break;
                }
                if (h.minres >= sy.best) {
                    if (++sy.stall >= 3) {
                        retire(sy, CCG_ERR_BREAKDOWN);
                        break;
                    }
                } else {
                    sy.stall = 0;
                }
                sy.best = std::min(sy.best, h.minres);
                sy.in_tol = next_inner_tol(sy.o.inner_tol, h.minres / sy.prev_minres);
                decide(sy);
                break;
            default:
                retire(sy, CCG_ERR_DEVICE);
        }
    }

    // Refinement: finished, out of budget, or start the next inner solve.
    void decide(Sys& sy) {
        DevState& h = h_states_[sy.slot];
        if (h.done == FAILED) { retire(sy, (ccg_status)h.status); return; }
        if (h.done != OUTER) { retire(sy, CCG_OK); return; }
        const int budget = sy.maxit - sy.iters_done;   // block steps left for this stage
        if (sy.refinements >= sy.o.max_refine || sy.iters >= budget) {
            retire(sy, CCG_NOT_CONVERGED);
            return;
        }
        unsigned mask = 0u;
        int m = 0;
        for (int j = 0; j < kMaxP; ++j) {
            const double sc = (j < sy.p && std::isfinite(h.norms[j])) ? h.norms[j] : 0.0;
            sy.ra.scale[j] = sc;
            if (sc > 0.0) { mask |= 1u << j; h.keep[m++] = j; }
        }
        h.done = RUNNING;
        h.iter = 0;
        h.m = m;
        h.mask = mask;
        sy.prev_minres = h.minres;
        h.tol = std::min(0.5, std::max(sy.in_tol, 0.1 * sy.tol / h.minres));
        h.nb = 1.0;
        h.maxit = std::min(sy.o.inner_maxit, budget - sy.iters);
        sy.inner_start_due = true;
        sy.ph = PH_INNER;
    }

    void due_res(Sys& sy, int mode, int set_nb) {
        sy.res_due = true;
        sy.res_mode = mode;
        sy.res_set_nb = set_nb;
    }

    // Report a system and copy its agents out (completed in finish_retired).
    void retire(Sys& sy, ccg_status st) {
        if (sy.slot < 0) return;
        if (escalate(sy, st)) return;
        DevState& h = h_states_[sy.slot];
        ccg_info info;
        std::memset(&info, 0, sizeof info);
        info.status = st;
        if (sy.prec == PREC_F64) {
            info.iters = sy.iters_done + h.iter;
            info.refinements = sy.refinements_done;
            info.restarts = h.restarts;
            info.p_final = h.m;
        } else {
            info.iters = sy.iters_done + sy.iters;
            info.refinements = sy.refinements_done + sy.refinements;
            info.restarts = 0;
            info.p_final = sy.p;
        }
        info.deflations = sy.deflations_done + h.deflations;
        info.prec_final = sy.prec == PREC_F64 ? CCG_FP64 : (sy.prec == PREC_F32 ? CCG_FP32 : CCG_BF16X2);
        double mn = INFINITY, mx = 0.0;
        int best = -1;
        for (int j = 0; j < sy.p; ++j) {
            const double r = h.norms[j] / h.nb;
            if (r < mn) { mn = r; best = j; }
            if (r > mx) mx = r;
        }
        info.best_agent = best;
        info.rel_res = mn;
        info.rel_res_max = mx;
        info.bytes_A = sy.bytes;
        double* dst = sy.host ? sy.Xdev : sy.X_out;
        const int64_t ldd = sy.host ? sy.n : sy.ldx;
        HIP_OK(launch_unpack(sy.n, sy.w.n_pad, sy.p, sy.w.Xr, dst, ldd, s_));
        if (sy.host)
            HIP_OK(hipMemcpy2DAsync(sy.X_out, sizeof(double) * sy.ldx, sy.Xdev, sizeof(double) * sy.n,
                                    sizeof(double) * sy.n, sy.p, hipMemcpyDeviceToHost, s_));
        retiring_.push_back(Finished{sy.tag, st, info});
        retiring_mem_.push_back(sy.mem);
        // the slot may still have items in the step work list: its steps must stay
        // no-ops, and the slot is reused only after the list is rebuilt
        h.done = FINISHED;
        pending_slots_.push_back(sy.slot);
        dead_items_ += sy.cw_step ? (size_t)((sy.n + sy.cw_step * sy.nw_step - 1) / (sy.cw_step * sy.nw_step)) : 1;
        sy.slot = -1;
    }

    void finish_retired() {
        if (retiring_.empty()) return;
        HIP_OK(hipStreamSynchronize(s_));
        const auto now = Clock::now();
        for (size_t i = 0; i < retiring_.size(); ++i) {
            for (auto& sy : live_)
                if (sy.tag == retiring_[i].tag && sy.slot < 0)
                    retiring_[i].info.seconds = std::chrono::duration<double>(now - sy.t0).count();
            finished_.push_back(retiring_[i]);
        }
        for (char* m : retiring_mem_) arena_.release(m);
        retiring_.clear();
        retiring_mem_.clear();
        live_.erase(std::remove_if(live_.begin(), live_.end(), [](const Sys& s) { return s.slot < 0; }),
                    live_.end());
        hi_slot_ = 0;
        for (auto& sy : live_) hi_slot_ = std::max(hi_slot_, sy.slot + 1);
        for (int sl : pending_slots_) hi_slot_ = std::max(hi_slot_, sl + 1);
    }

    // Step work list of every resident system, by (precision, P, tile shape) class;
    // uploaded once, and each class's k steps captured into a graph of its own.
    void rebuild_steps(int k) {
        for (int sl : pending_slots_) free_slots_.push_back(sl);
        pending_slots_.clear();
        hi_slot_ = 0;
        for (auto& sy : live_) hi_slot_ = std::max(hi_slot_, sy.slot + 1);
        for (hipGraphExec_t g : class_graphs_) HIP_OK(hipGraphExecDestroy(g));
        class_graphs_.clear();
        std::vector<int4> st;
        step_ranges_.clear();
        step_items_total_ = 0;
        for (int prec : {PREC_F64, PREC_F32, PREC_BF16X2}) {
            for (int P : {1, 2, 4, 8, 16}) {
                // the small-system tier: one work item (workgroup) per system
                StepRange rs{prec, P, 0, 0, st.size(), 0, 0, 0, 0, 0};
                for (auto& sy : live_)
                    if (sy.prec == prec && sy.P == P && sy.cw_step == 0) st.push_back(int4{sy.slot, 0, 0, 0});
                rs.ad_n = st.size() - rs.ad_off;
                rs.up_off = rs.dir_off = st.size();
                if (rs.ad_n) {
                    step_ranges_.push_back(rs);
                    step_items_total_ += rs.ad_n;
                }
                for (int cw : {1, 2, 4}) {
                    for (int nw : {4, 8, 16}) {
                        StepRange r{prec, P, cw, nw, st.size(), 0, 0, 0, 0, 0};
                        for (auto& sy : live_) {
                            if (sy.prec != prec || sy.P != P || sy.cw_step != cw || sy.nw_step != nw) continue;
                            const int t = (sy.n + cw * nw - 1) / (cw * nw);
                            for (int i = 0; i < t; ++i) st.push_back(int4{sy.slot, i, 0, 0});
                        }
                        r.ad_n = st.size() - r.ad_off;
                        r.up_off = st.size();
                        for (auto& sy : live_) {
                            if (sy.prec != prec || sy.P != P || sy.cw_step != cw || sy.nw_step != nw) continue;
                            const int t = upd_blocks(sy.w.n_pad, P);
                            for (int i = 0; i < t; ++i) st.push_back(int4{sy.slot, i, 0, 0});
                        }
                        r.up_n = st.size() - r.up_off;
                        r.dir_off = st.size();
                        for (auto& sy : live_) {
                            if (sy.prec != prec || sy.P != P || sy.cw_step != cw || sy.nw_step != nw) continue;
                            const int t = upd_blocks(sy.w.n_pad, P);
                            for (int i = 0; i < t; ++i) st.push_back(int4{sy.slot, i, 0, 0});
                        }
                        r.dir_n = st.size() - r.dir_off;
                        if (r.ad_n) {
                            step_ranges_.push_back(r);
                            step_items_total_ += r.ad_n;
                        }
                    }
                }
            }
        }
        const size_t n = std::max<size_t>(st.size(), 1);
        if (n > step_cap_) {
            if (d_step_) (void)hipFree(d_step_);
            if (h_step_) (void)hipHostFree(h_step_);
            d_step_ = nullptr;
            h_step_ = nullptr;
            step_cap_ = 0;
            const size_t cap = std::max<size_t>(n * 2, 1 << 16);
            HIP_OK(hipMalloc(&d_step_, sizeof(int4) * cap));
            HIP_OK(hipHostMalloc(reinterpret_cast<void**>(&h_step_), sizeof(int4) * cap, hipHostMallocDefault));
            step_cap_ = cap;
        }
        if (!st.empty()) {
            std::memcpy(h_step_, st.data(), sizeof(int4) * st.size());
            HIP_OK(hipMemcpyAsync(d_step_, h_step_, sizeof(int4) * st.size(), hipMemcpyHostToDevice, s_));
        }
        items_dirty_ = false;
        dead_items_ = 0;
        graph_k_ = k;
        // Classes touch disjoint systems, so each class's k steps form an independent
        // chain on a stream of its own (default priority); the chains run
        // concurrently, overlapping one class's reduction tail with another's
        // stream of A.  Each chain is a linear graph captured on its class stream.
        while (class_streams_on_ && class_streams_.size() < step_ranges_.size()) {
            hipStream_t cs = nullptr;
            HIP_OK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
            class_streams_.push_back(cs);
            hipEvent_t ev = nullptr;
            HIP_OK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
            class_events_.push_back(ev);
        }
        if (!fork_) HIP_OK(hipEventCreateWithFlags(&fork_, hipEventDisableTiming));
        if (!use_graph_) return;
        for (size_t c = 0; c < step_ranges_.size(); ++c) {
            hipStream_t cs = class_streams_on_ ? class_streams_[c] : s_;
            hipGraph_t gr = nullptr;
            HIP_OK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            bool ok = true;
            try {
                enqueue_class_round(step_ranges_[c], k, cs);
            } catch (const CcgError&) {
                ok = false;
            }
            const hipError_t e = hipStreamEndCapture(cs, &gr);
            if (!ok || e != hipSuccess || !gr) {
                (void)hipGetLastError();
                if (gr) (void)hipGraphDestroy(gr);
                throw CcgError{CCG_ERR_DEVICE, "stream capture of the batched block steps failed"};
            }
            hipGraphExec_t ex = nullptr;
            const hipError_t ei = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
            (void)hipGraphDestroy(gr);
            if (ei != hipSuccess || !ex)
                throw CcgError{CCG_ERR_DEVICE, "instantiating the batched block-step graph failed"};
            class_graphs_.push_back(ex);
        }
    }

    // k block steps of one class: one tier launch running k steps per system, or k
    // triples of batched A.D, update and direction launches
    void enqueue_class_round(const StepRange& r, int k, hipStream_t cs) {
        if (r.cw == 0) {
            HIP_OK(launch_small(r.prec, r.P, nullptr, d_small_, d_step_ + r.ad_off, (int)r.ad_n, k, cs));
            return;
        }
        for (int it = 0; it < k; ++it) enqueue_class_step(r, cs);
    }

    void enqueue_class_step(const StepRange& r, hipStream_t cs) {
        HIP_OK(launch_ad_batch(r.prec, r.P, r.cw, r.nw, d_ad_, d_step_ + r.ad_off, (int)r.ad_n, cs));
        HIP_OK(launch_upd_batch(r.prec, r.P, d_upd_, d_step_ + r.up_off, (int)r.up_n, cs));
        HIP_OK(launch_dir_batch(r.prec, r.P, d_upd_, d_step_ + r.dir_off, (int)r.dir_n, cs));
    }

    void upload_items() {
        const size_t n = std::max<size_t>(items_.size(), 1);
        if (n > items_cap_) {
            if (d_items_) (void)hipFree(d_items_);
            if (h_items_) (void)hipHostFree(h_items_);
            d_items_ = nullptr;
            h_items_ = nullptr;
            items_cap_ = 0;
            const size_t cap = std::max<size_t>(n * 2, 1 << 16);
            HIP_OK(hipMalloc(&d_items_, sizeof(int4) * cap));
            HIP_OK(hipHostMalloc(reinterpret_cast<void**>(&h_items_), sizeof(int4) * cap, hipHostMallocDefault));
            items_cap_ = cap;
        }
        if (items_.empty()) return;
        std::memcpy(h_items_, items_.data(), sizeof(int4) * items_.size());
        HIP_OK(hipMemcpyAsync(d_items_, h_items_, sizeof(int4) * items_.size(), hipMemcpyHostToDevice, s_));
    }

    int device_;
    hipStream_t s_;
    Arena& arena_;
    DevState* states_ = nullptr;
    DevState* h_states_ = nullptr;
    AdArgs* d_ad_ = nullptr;
    AdArgs* d_res_ad_ = nullptr;
    UpdArgs* d_upd_ = nullptr;
    SmallArgs* d_small_ = nullptr;
    ResArgs* d_res_ = nullptr;
    int4* d_items_ = nullptr;
    int4* h_items_ = nullptr;
    size_t items_cap_ = 0;
    std::vector<int4> items_;
    std::vector<StepRange> step_ranges_;
    int4* d_step_ = nullptr;
    int4* h_step_ = nullptr;
    size_t step_cap_ = 0;
    bool use_graph_ = true;
    bool class_streams_on_ = true;
    std::vector<hipGraphExec_t> class_graphs_;   // one per step class (use_graph_)
    int graph_k_ = 0;
    std::vector<hipStream_t> class_streams_;
    std::vector<hipEvent_t> class_events_;
    hipEvent_t fork_ = nullptr;
    bool items_dirty_ = true;
    size_t dead_items_ = 0;
    size_t step_items_total_ = 0;
    std::vector<int> pending_slots_;
    std::vector<int> free_slots_;
    int hi_slot_ = 0;
    std::vector<Sys> live_;
    std::vector<Finished> retiring_;
    std::vector<char*> retiring_mem_;
    std::vector<Finished> finished_;
};

// ------------------------------------------------------------------ service

struct Request {
    uint64_t ticket;
    ccg_problem prob;
    Clock::time_point t_submit;
};

struct Result {
    bool done = false;
    ccg_status status = CCG_PENDING;
    ccg_info info{};
    Clock::time_point t_submit;
};

}  // namespace

// One lane of the service: its request queue, pending cancels and thread.
struct ServiceLane {
    std::thread th;
    std::condition_variable wake;      // to the lane's thread
    std::deque<Request> queue;
    std::vector<uint64_t> cancels;
};

struct Server {
    explicit Server(size_t budget) : arena(budget) {}
    std::mutex mu;
    std::condition_variable done_cv;   // to waiters
    ServiceLane lanes[kLanes];
    std::map<uint64_t, Result> results;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::string fatal;                 // a device error that ended the service
    Arena arena;                       // device memory of every lane
};

namespace {

// Service loop of one lane: admit in arrival order while memory allows, advance,
// retire.
void serve(ccg_ctx* c, Server* sv, int lane) {
    ServiceLane& L = sv->lanes[lane];
    (void)hipSetDevice(c->device);
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->fatal = "service stream creation failed";
        sv->done_cv.notify_all();
        for (auto& l : sv->lanes) l.wake.notify_all();
        return;
    }
    try {
        // one stream per lane: a served lane holds few systems, and with fewer streams
        // the small lane's steps wait less behind the large lane's (at 2.6 requests/s:
        // p50 54 -> 48 ms, p99 1.13 -> 1.03 s against streams per class)
        Engine eng(c->device, s, sv->arena, true, false);
        std::map<uint64_t, Clock::time_point> submitted;
        for (;;) {
            std::vector<Request> admit;
            {
                std::unique_lock<std::mutex> lk(sv->mu);
                if (eng.idle())
                    L.wake.wait(lk, [&] {
                        return sv->stop || !sv->fatal.empty() || !L.queue.empty() || !L.cancels.empty();
                    });
                if (sv->stop || !sv->fatal.empty()) break;
                for (uint64_t t : L.cancels) {
                    bool queued = false;
                    for (auto it = L.queue.begin(); it != L.queue.end(); ++it) {
                        if (it->ticket != t) continue;
                        Result& r = sv->results[t];
                        r.done = true;
                        r.status = CCG_CANCELLED;
                        r.info.status = CCG_CANCELLED;
                        L.queue.erase(it);
                        queued = true;
                        break;
                    }
                    if (!queued) eng.cancel(t);
                }
                L.cancels.clear();
                sv->done_cv.notify_all();
                while (!L.queue.empty()) {
                    admit.push_back(L.queue.front());
                    L.queue.pop_front();
                }
            }
            // admission in arrival order; what does not fit goes back to the front
            size_t taken = 0;
            for (; taken < admit.size(); ++taken) {
                const Request& rq = admit[taken];
                const ccg_opts o = fill_defaults(&rq.prob.opts);
                bool ok = false;
                ccg_status err = CCG_OK;
                std::string msg;
                try {
                    if (!eng.could_fit(Engine::footprint(rq.prob, o))) {
                        err = CCG_ERR_NOMEM;
                        msg = "system exceeds the HBM budget";
                    } else {
                        ok = eng.admit(rq.prob, rq.ticket);
                        // nothing resident in any lane and still no room: never fits (one
                        // more try, in case the other lane released its memory meanwhile)
                        if (!ok && eng.idle() && sv->arena.empty()) ok = eng.admit(rq.prob, rq.ticket);
                        if (!ok && eng.idle() && sv->arena.empty()) {
                            err = CCG_ERR_NOMEM;
                            msg = "no device memory for the system";
                        }
                    }
                } catch (const CcgError& e) {
                    err = e.st;
                    msg = e.msg;
                }
                if (err != CCG_OK) {
                    std::lock_guard<std::mutex> lk(sv->mu);
                    Result& r = sv->results[rq.ticket];
                    r.done = true;
                    r.status = err;
                    r.info.status = err;
                    sv->done_cv.notify_all();
                    continue;
                }
                if (!ok) break;
                submitted[rq.ticket] = rq.t_submit;
            }
            if (taken < admit.size()) {
                std::lock_guard<std::mutex> lk(sv->mu);
                for (size_t i = admit.size(); i-- > taken;) L.queue.push_front(admit[i]);
            }
            // the other lane holds the memory this lane waits for
            if (eng.idle() && taken < admit.size()) std::this_thread::sleep_for(std::chrono::microseconds(200));
            eng.round(kRoundSteps[1][lane]);
            auto fin = eng.take_finished();
            if (!fin.empty()) {
                const auto now = Clock::now();
                std::lock_guard<std::mutex> lk(sv->mu);
                for (auto& f : fin) {
                    Result& r = sv->results[f.tag];
                    r.done = true;
                    r.status = f.status;
                    r.info = f.info;
                    auto it = submitted.find(f.tag);
                    if (it != submitted.end()) {
                        r.info.seconds = std::chrono::duration<double>(now - it->second).count();
                        submitted.erase(it);
                    }
                }
                sv->done_cv.notify_all();
            }
        }
    } catch (const CcgError& e) {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->fatal = e.msg;
    } catch (const std::bad_alloc&) {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->fatal = "host allocation failed";
    }
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
    std::lock_guard<std::mutex> lk(sv->mu);
    if (!sv->fatal.empty()) {
        for (auto& kv : sv->results)
            if (!kv.second.done) {
                kv.second.done = true;
                kv.second.status = CCG_ERR_DEVICE;
                kv.second.info.status = CCG_ERR_DEVICE;
            }
        for (auto& l : sv->lanes) l.wake.notify_all();
    }
    sv->done_cv.notify_all();
}

}  // namespace

void stop_server(ccg_ctx* c) {
    Server* sv = c->server;
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    for (auto& l : sv->lanes) {
        l.wake.notify_all();
        if (l.th.joinable()) l.th.join();
    }
    delete sv;
    c->server = nullptr;
}

}  // namespace host
}  // namespace ccg

using namespace ccg;
using namespace ccg::host;

extern "C" {

ccg_status ccg_solve_batched(ccg_ctx* c, int count, const ccg_problem* probs, ccg_info* infos) {
    if (!c) return CCG_ERR_ARG;
    if (count < 0 || (count > 0 && !probs)) return CCG_ERR_ARG;
    if (infos)
        for (int i = 0; i < count; ++i) {
            std::memset(&infos[i], 0, sizeof(ccg_info));
            infos[i].best_agent = -1;
            infos[i].status = CCG_PENDING;
        }
    ccg_status first_err = CCG_OK;
    bool any_nc = false;
    std::mutex rec_mu;
    auto record = [&](int i, ccg_status s, const ccg_info* inf) {
        std::lock_guard<std::mutex> lk(rec_mu);
        if (infos) {
            if (inf) infos[i] = *inf;
            infos[i].status = s;
        }
        if (s < 0 && first_err == CCG_OK) first_err = s;
        if (s == CCG_NOT_CONVERGED) any_nc = true;
    };
    const ccg_status st = guarded(c, [&]() -> ccg_status {
        const bool graphs = !(count > 0 && (probs[0].opts.flags & CCG_NO_GRAPH));
        Arena arena(c->budget);
        std::deque<int> queues[kLanes];
        for (int i = 0; i < count; ++i) queues[lane_of(probs[i].n)].push_back(i);
        std::atomic<bool> abort_lanes{false};
        // one lane: admit in order while memory allows, run rounds until its systems
        // have all retired
        auto run_lane = [&](int lane, hipStream_t s) {
            Engine eng(c->device, s, arena, graphs);
            std::deque<int>& queue = queues[lane];
            while ((!queue.empty() || !eng.idle()) && !abort_lanes.load()) {
                bool wait_memory = false;
                while (!queue.empty()) {
                    const int i = queue.front();
                    const ccg_opts o = fill_defaults(&probs[i].opts);
                    if (!eng.could_fit(Engine::footprint(probs[i], o))) {
                        record(i, CCG_ERR_NOMEM, nullptr);
                        queue.pop_front();
                        continue;
                    }
                    bool ok = false;
                    try {
                        ok = eng.admit(probs[i], (uint64_t)i);
                        // the other lane may have released its memory meanwhile
                        if (!ok && eng.idle() && arena.empty()) ok = eng.admit(probs[i], (uint64_t)i);
                    } catch (const CcgError& e) {
                        if (e.st == CCG_ERR_DEVICE) throw;
                        record(i, e.st, nullptr);
                        queue.pop_front();
                        continue;
                    }
                    if (!ok) {
                        if (eng.idle()) {
                            if (arena.empty()) {   // nothing resident anywhere and still no room
                                record(i, CCG_ERR_NOMEM, nullptr);
                                queue.pop_front();
                                continue;
                            }
                            wait_memory = true;    // the other lane holds the memory
                        }
                        break;
                    }
                    queue.pop_front();
                }
                if (wait_memory) std::this_thread::sleep_for(std::chrono::microseconds(200));
                eng.round(kRoundSteps[0][lane]);
                for (auto& f : eng.take_finished()) record((int)f.tag, f.status, &f.info);
            }
        };
        // the large-system lane runs on a thread and stream of its own
        std::exception_ptr lane_err;
        std::thread big;
        hipStream_t s_big = nullptr;
        if (!queues[1].empty()) {
            HIP_OK(hipStreamCreateWithFlags(&s_big, hipStreamNonBlocking));
            try {
                big = std::thread([&] {
                    try {
                        (void)hipSetDevice(c->device);
                        run_lane(1, s_big);
                    } catch (...) {
                        lane_err = std::current_exception();
                        abort_lanes = true;
                    }
                });
            } catch (const std::system_error&) {
                (void)hipStreamDestroy(s_big);
                throw CcgError{CCG_ERR_DEVICE, "could not start the large-system lane"};
            }
        }
        std::exception_ptr own_err;
        try {
            run_lane(0, c->stream);
        } catch (...) {
            own_err = std::current_exception();
            abort_lanes = true;
        }
        if (big.joinable()) big.join();
        if (s_big) (void)hipStreamDestroy(s_big);
        if (own_err) std::rethrow_exception(own_err);
        if (lane_err) std::rethrow_exception(lane_err);
        return CCG_OK;
    });
    if (st != CCG_OK) return st;
    if (first_err != CCG_OK) return first_err;
    return any_nc ? CCG_NOT_CONVERGED : CCG_OK;
}

ccg_status ccg_submit(ccg_ctx* c, const ccg_problem* prob, uint64_t* ticket) {
    if (!c || !prob || !ticket) return CCG_ERR_ARG;
    int lane = 0;
    try {
        if (!c->server) {
            Server* sv = new Server(c->budget);
            c->server = sv;
            for (int l = 0; l < kLanes; ++l) sv->lanes[l].th = std::thread(serve, c, sv, l);
        }
        Server* sv = c->server;
        std::lock_guard<std::mutex> lk(sv->mu);
        if (!sv->fatal.empty()) {
            c->err = sv->fatal;
            return CCG_ERR_DEVICE;
        }
        const uint64_t t = sv->next_ticket++;
        Result r;
        r.t_submit = Clock::now();
        sv->results[t] = r;
        lane = lane_of(prob->n);
        sv->lanes[lane].queue.push_back(Request{t, *prob, r.t_submit});
        *ticket = t;
    } catch (const std::bad_alloc&) {
        return CCG_ERR_NOMEM;
    } catch (const std::system_error&) {
        c->err = "could not start the service threads";
        stop_server(c);
        return CCG_ERR_DEVICE;
    }
    c->server->lanes[lane].wake.notify_all();
    return CCG_OK;
}

static ccg_status take_result(Server* sv, uint64_t ticket, ccg_info* info, bool wait) {
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->results.find(ticket);
    if (it == sv->results.end()) return CCG_ERR_ARG;
    if (wait) sv->done_cv.wait(lk, [&] { return it->second.done; });
    if (!it->second.done) return CCG_PENDING;
    const ccg_status st = it->second.status;
    if (info) *info = it->second.info;
    sv->results.erase(it);
    return st;
}

ccg_status ccg_poll(ccg_ctx* c, uint64_t ticket, ccg_info* info) {
    if (!c || !c->server) return CCG_ERR_ARG;
    return take_result(c->server, ticket, info, false);
}

ccg_status ccg_wait(ccg_ctx* c, uint64_t ticket, ccg_info* info) {
    if (!c || !c->server) return CCG_ERR_ARG;
    return take_result(c->server, ticket, info, true);
}

ccg_status ccg_cancel(ccg_ctx* c, uint64_t ticket) {
    if (!c || !c->server) return CCG_ERR_ARG;
    Server* sv = c->server;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        auto it = sv->results.find(ticket);
        if (it == sv->results.end()) return CCG_ERR_ARG;
        if (it->second.done) return CCG_OK;
        // the lane that holds the request acts on it; the others find nothing
        for (auto& l : sv->lanes) l.cancels.push_back(ticket);
    }
    for (auto& l : sv->lanes) l.wake.notify_all();
    return CCG_OK;
}

}  // extern "C"
