// Device templates of the block step, shared by the kernel translation units:
// precision traits, the A.D tile (k_ad / k_ad_batch), the update (k_upd), the
// residual epilogue (k_res) and their helpers.  The kernels are instantiated per
// precision in ccg_ad_f64.hip, ccg_ad_f32.hip and ccg_ad_bf16.hip (A.D) and in
// ccg_kernels.hip (the rest), which compile in parallel.
#pragma once

// HIP kernels (gfx950) for the block step of cooperative conjugate gradient.
//
// One block step (Alg. 2 of the paper, sign convention R = B - A X, residual by
// the Table 1 recurrence) is three launches:
//
//   k_ad   : AD = A D, streaming A once.  A is symmetric, so column i of A (which is
//            contiguous in the column-major layout) is row i: each wave streams
//            whole columns with 16-byte non-temporal loads, its lanes splitting the
//            contraction index k, and multiplies them with D rows staged in LDS
//            (double buffered).  Lane sums are folded by a fixed xor butterfly, so
//            every AD row is complete inside one wave: no split-K partials.  Each
//            workgroup adds its rows' share of G = D^T AD and S = D^T R; a two-level
//            fixed-order reduction across workgroups ends in the last workgroup,
//            which runs the rank step of Alg. 3 and alpha = G^{-1} S (FP64).
//   k_upd  : X += D alpha, R_new = R - AD alpha, and the products (AD)^T R_new and
//            diag(R_new^T R_new), summed per group of workgroups.
//   k_dir  : every workgroup adds those shares up in a fixed order and solves
//            beta = -G^{-1} (AD)^T R_new itself, then D = R_new + D beta (masked to
//            active agents); workgroup 0 runs the stop test on the new norms.
//
#include "ccg_device.h"

#include <hip/hip_ext.h>

#include <math.h>

#include <algorithm>
#include <type_traits>

namespace ccg {

// ----------------------------------------------------------------- precision traits

template <int PREC> struct PT;
template <> struct PT<PREC_F64> {
    using TA = double;   // stored A element
    using TV = double;   // vector element (X, R, D, AD)
    using TACC = double; // accumulator of A.D
    static constexpr int E = 2;   // elements per 16-byte load
};
template <> struct PT<PREC_F32> {
    using TA = float;
    using TV = float;
    using TACC = float;
    static constexpr int E = 4;
};
template <> struct PT<PREC_BF16X2> {
    using TA = uint16_t;
    using TV = float;
    using TACC = float;
    static constexpr int E = 8;
};

// Tile configuration of the A.D kernel: CW A columns per wave and NW waves per
// workgroup (so NW*CW AD rows per workgroup, all sharing one staged D chunk), SPC
// wave steps of 64*E contraction elements per staged D chunk, an occupancy hint
// MINW (waves per SIMD) and non-temporal A loads (A is read exactly once per
// launch).  STG rotates each workgroup's starting chunk so that concurrent
// workgroups read different offsets of their columns (the column stride is a large
// power of two).
template <int CW_, int SPC_, int MINW_, bool NT_, bool STG_ = false, int NW_ = 4>
struct AdCfg {
    static constexpr int CW = CW_;
    static constexpr int SPC = SPC_;
    static constexpr int MINW = MINW_;
    static constexpr bool NT = NT_;
    static constexpr bool STG = STG_;
    static constexpr int NW = NW_;
    static constexpr int WG = 64 * NW_;       // threads per workgroup
    static constexpr int ROWS = NW_ * CW_;
};

__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
    return __uint_as_float(((uint32_t)h) << 16);
}

// Load the E elements of one 16-byte chunk of a column, converted to TACC.  hi
// points into the FP64 / FP32 matrix or the BF16 "hi" plane, lo into the BF16 "lo"
// plane at the same offset.  NT selects non-temporal (streaming) loads.
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef unsigned u4v __attribute__((ext_vector_type(4)));

template <bool NT, class T>
__device__ __forceinline__ T ld16(const T* p) {
    if (NT) return __builtin_nontemporal_load(p);
    return *p;
}

template <int PREC, bool NT> struct Loader;

template <bool NT> struct Loader<PREC_F64, NT> {
    __device__ __forceinline__ static void load(const double* hi, const double*, double (&out)[2]) {
        const d2v v = ld16<NT>(reinterpret_cast<const d2v*>(hi));
        out[0] = v.x;
        out[1] = v.y;
    }
    __device__ __forceinline__ static double load1(const double* hi, const double*) { return *hi; }
};
template <bool NT> struct Loader<PREC_F32, NT> {
    __device__ __forceinline__ static void load(const float* hi, const float*, float (&out)[4]) {
        const f4v v = ld16<NT>(reinterpret_cast<const f4v*>(hi));
        out[0] = v.x; out[1] = v.y; out[2] = v.z; out[3] = v.w;
    }
    __device__ __forceinline__ static float load1(const float* hi, const float*) { return *hi; }
};
template <bool NT> struct Loader<PREC_BF16X2, NT> {
    __device__ __forceinline__ static void load(const uint16_t* hi, const uint16_t* lo, float (&out)[8]) {
        const u4v h = ld16<NT>(reinterpret_cast<const u4v*>(hi));
        const u4v l = ld16<NT>(reinterpret_cast<const u4v*>(lo));
        const uint32_t hw[4] = {h.x, h.y, h.z, h.w};
        const uint32_t lw[4] = {l.x, l.y, l.z, l.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            // hi + lo is exact in FP32: both carry 8 significant bits, lo below hi.
            out[2 * q] = __uint_as_float(hw[q] << 16) + __uint_as_float(lw[q] << 16);
            out[2 * q + 1] = __uint_as_float(hw[q] & 0xffff0000u) + __uint_as_float(lw[q] & 0xffff0000u);
        }
    }
    __device__ __forceinline__ static float load1(const uint16_t* hi, const uint16_t* lo) {
        return bf16_to_f32(*hi) + bf16_to_f32(*lo);
    }
};

// ------------------------------------------------------ cross-workgroup reduction
//
// Partial sums pass between workgroups (on MI355X across XCDs, whose L2 caches are
// not coherent with each other) through agent-scope atomic stores and loads, which
// gfx950 issues with the sc1 bit: the stores write through to the device-coherent
// level and the loads read from it, so no L2 writeback or invalidate is needed.  The
// order is: every thread's partial stores, then s_waitcnt vmcnt(0) (each store
// acknowledged by the coherent level), then the ticket fetch-add; the workgroup that
// draws the last ticket waits for the add's return (the ticket value, which decides
// whether it sums at all) before it issues the loads.  The asm statement is a
// compiler barrier for every memory access, and the loads depend on the ticket
// through the workgroup barrier that broadcasts it, so neither the compiler nor the
// memory pipeline can move a load before the add or a store after it.  (An
// acquire-release ticket would add buffer_wbl2 and buffer_inv of the XCD's whole L2
// to every workgroup of every launch, which is what this scheme avoids.)

__device__ __forceinline__ void st_agent(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_agent(const double* p) {
    return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned ticket(unsigned* c) {
    return __hip_atomic_fetch_add(c, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void reset_ticket(unsigned* c) {
    __hip_atomic_store(c, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Wait until every memory operation this thread issued is acknowledged.
__device__ __forceinline__ void stores_done() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Sum, for entry e, the rows m0 .. m0+cnt-1 of src (row stride ne) in row order.
// Loads are issued in unrolled batches of B so that their latencies overlap; the
// batch only groups the loads, the additions stay in row order.
template <int B>
__device__ __forceinline__ double sum_rows(const double* src, int ne, int e, int m0, int cnt) {
    double s = 0.0;
    for (int base = 0; base < cnt; base += B) {
        double v[B];
#pragma unroll
        for (int q = 0; q < B; ++q)
            v[q] = (base + q < cnt) ? ld_agent(&src[(int64_t)(m0 + base + q) * ne + e]) : 0.0;
#pragma unroll
        for (int q = 0; q < B; ++q)
            if (base + q < cnt) s += v[q];
    }
    return s;
}

// out[e] = sum over rows 0..cnt-1 of src (row stride ne), for every e < ne, with the
// rows of each entry split into contiguous slices over spare threads and the slice
// sums added in slice order (a fixed tree).  NTH threads; scratch: NTH doubles of LDS.
template <int B, int NTH>
__device__ __forceinline__ void sum_table(const double* src, int ne, int cnt, double* out, double* scratch) {
    const int tid = threadIdx.x;
    const int tpe = ne >= NTH ? 1 : NTH / ne;          // threads per entry
    const int slice = (cnt + tpe - 1) / tpe;
    for (int e0 = 0; e0 < ne; e0 += NTH / tpe) {
        const int e = e0 + tid / tpe, sub = tid % tpe;
        double s = 0.0;
        if (e < ne && tid / tpe < NTH / tpe) {
            const int m0 = sub * slice;
            s = sum_rows<B>(src, ne, e, m0, max(0, min(slice, cnt - m0)));
        }
        scratch[tid] = s;
        __syncthreads();
        if (sub == 0 && e < ne && tid / tpe < NTH / tpe) {
            double t = scratch[tid];
            for (int q = 1; q < tpe; ++q) t += scratch[tid + q];
            out[e] = t;
        }
        __syncthreads();
    }
}

// The same for ne <= K * NTH with every thread owning the K entries tid + k * NTH:
// the rows are loaded B at a time for all K entries together (K * B loads in flight)
// and added in row order, so each entry gets the bits sum_table gives it.
template <int K, int B, int NTH>
__device__ __forceinline__ void sum_table_k(const double* src, int ne, int cnt, double* out) {
    const int tid = threadIdx.x;
    double s[K];
#pragma unroll
    for (int k = 0; k < K; ++k) s[k] = 0.0;
    for (int base = 0; base < cnt; base += B) {
        double v[K][B];
#pragma unroll
        for (int q = 0; q < B; ++q)
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int e = tid + k * NTH;
                v[k][q] = (base + q < cnt && e < ne) ? ld_agent(&src[(int64_t)(base + q) * ne + e]) : 0.0;
            }
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int q = 0; q < B; ++q)
                if (base + q < cnt) s[k] += v[k][q];
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (tid + k * NTH < ne) out[tid + k * NTH] = s[k];
    __syncthreads();
}

// Sum `ne` values per tile (mine[], LDS) over the nwg tiles of one system, in tile
// order within groups of kGroup and in group order across groups.  Returns true in
// the one workgroup that ends up holding the totals in out[] (LDS).  Tickets are
// reset by their last taker, so the scratch is ready for the next launch.  B: loads
// in flight per thread while summing rows; with B = kGroup a group's rows, and the
// group sums of up to kGroup^2 tiles, take one round trip to memory each where
// every entry has a thread of its own (large ne), at the price of registers that
// the kernels with few agents would pay in occupancy.
template <int B, int NTH>
__device__ __forceinline__ bool grid_reduce(const double* mine, int ne, const RedBuf rb, double* out,
                                            int* s_flag, double* scratch, int bid, int nwg) {
    const int tid = threadIdx.x;
    const int ngroups = (nwg + kGroup - 1) / kGroup;
    const int grp = bid / kGroup;
    const int gsize = min(kGroup, nwg - grp * kGroup);
    for (int e = tid; e < ne; e += NTH) st_agent(&rb.l1[(int64_t)bid * ne + e], mine[e]);
    stores_done();
    __syncthreads();
    if (tid == 0) *s_flag = (ticket(&rb.cnt[grp]) == (unsigned)gsize - 1) ? 1 : 0;
    __syncthreads();
    if (!*s_flag) return false;
    if (tid == 0) reset_ticket(&rb.cnt[grp]);
    if (ngroups == 1) {
        sum_table<B, NTH>(rb.l1, ne, gsize, out, scratch);
        return true;
    }
    // group sum -> level-2 row of this group
    sum_table<B, NTH>(rb.l1 + (int64_t)grp * kGroup * ne, ne, gsize, out, scratch);
    for (int e = tid; e < ne; e += NTH) st_agent(&rb.l2[(int64_t)grp * ne + e], out[e]);
    stores_done();
    __syncthreads();
    if (tid == 0) *s_flag = (ticket(&rb.cnt[ngroups]) == (unsigned)ngroups - 1) ? 1 : 0;
    __syncthreads();
    if (!*s_flag) return false;
    if (tid == 0) reset_ticket(&rb.cnt[ngroups]);
    sum_table<B, NTH>(rb.l2, ne, ngroups, out, scratch);
    return true;
}

// The first level of grid_reduce alone: the last workgroup of each group of GS
// tiles sums its group's rows (tile order) into rb.l2[grp].  Returns true in that
// workgroup.  The group sums are read by a later launch, which adds them up in
// group order.  K > 0 (ne <= K * NTH): the rows go through sum_table_k, B at a time.
template <int B, int NTH, int GS = kGroup, int K = 0>
__device__ __forceinline__ bool group_reduce(const double* mine, int ne, const RedBuf rb, double* out,
                                             int* s_flag, double* scratch, int bid, int nwg) {
    const int tid = threadIdx.x;
    const int grp = bid / GS;
    const int gsize = min(GS, nwg - grp * GS);
    for (int e = tid; e < ne; e += NTH) st_agent(&rb.l1[(int64_t)bid * ne + e], mine[e]);
    stores_done();
    __syncthreads();
    if (tid == 0) *s_flag = (ticket(&rb.cnt[grp]) == (unsigned)gsize - 1) ? 1 : 0;
    __syncthreads();
    if (!*s_flag) return false;
    if (tid == 0) reset_ticket(&rb.cnt[grp]);
    if constexpr (K > 0) sum_table_k<K, B, NTH>(rb.l1 + (int64_t)grp * GS * ne, ne, gsize, out);
    else sum_table<B, NTH>(rb.l1 + (int64_t)grp * GS * ne, ne, gsize, out, scratch);
    for (int e = tid; e < ne; e += NTH) st_agent(&rb.l2[(int64_t)grp * ne + e], out[e]);
    return true;
}

// ------------------------------------------------------------ small p x p algebra
//
// Executed by all threads of one workgroup on LDS arrays (m <= 32), with barriers
// between dependent phases.  Compact m x m matrices are row-major with stride m.

// Greedy pivoted Cholesky of the diagonally scaled G (unit diagonal).  Writes the
// taken compact indices, ascending, to keep[]; returns their count, or -1 when a
// diagonal entry is negative, -2 on a non-finite entry.  Columns with G_ii == 0 are
// never taken.  Same rule as the oracle's rank step.
__device__ __forceinline__ int wg_rank_select(const double* G, int m, double tau, int* keep, double* H, int* sh) {
    const int tid = threadIdx.x;
    const int nth = blockDim.x;
    // sh[0]: status, sh[1]: ncand, sh[2]: ntaken, sh[3]: pivot (or -1 to stop)
    // sh[8..8+m): candidate list, sh[40..40+m): taken list; H: m * m doubles
    if (tid == 0) {
        int st = 0;
        for (int i = 0; i < m && st == 0; ++i) {
            const double g = G[i * m + i];
            if (!isfinite(g)) st = -2;
            else if (g < 0.0) st = -1;
        }
        for (int i = 0; i < m * m && st == 0; ++i)
            if (!isfinite(G[i])) st = -2;
        sh[0] = st;
    }
    __syncthreads();
    if (sh[0] != 0) return sh[0];
    for (int t = tid; t < m * m; t += nth) {
        const int i = t / m, j = t % m;
        const double si = sqrt(G[i * m + i]), sj = sqrt(G[j * m + j]);
        H[t] = (si > 0.0 && sj > 0.0) ? G[t] / (si * sj) : 0.0;
    }
    if (tid == 0) {
        int nc = 0;
        for (int i = 0; i < m; ++i)
            if (G[i * m + i] > 0.0) sh[8 + nc++] = i;
        sh[1] = nc;
        sh[2] = 0;
    }
    __syncthreads();
    for (;;) {
        if (tid == 0) {
            const int nc = sh[1];
            int piv = -1;
            if (nc > 0) {
                int best = 0;
                for (int c = 1; c < nc; ++c)
                    if (H[sh[8 + c] * m + sh[8 + c]] > H[sh[8 + best] * m + sh[8 + best]]) best = c;
                const int cand = sh[8 + best];
                const double d = H[cand * m + cand];
                if (d > tau) {
                    piv = cand;
                    sh[40 + sh[2]] = cand;
                    sh[2] += 1;
                    for (int c = best; c + 1 < nc; ++c) sh[8 + c] = sh[8 + c + 1];
                    sh[1] = nc - 1;
                }
            }
            sh[3] = piv;
        }
        __syncthreads();
        const int piv = sh[3];
        if (piv < 0) break;
        const int nc = sh[1];
        const double r = sqrt(H[piv * m + piv]);
        // entries (ic, ia) of the remaining candidates; the pivot's column, which they
        // read, is not among them, so each thread updates its entries in place
        for (int t = tid; t < nc * nc; t += nth) {
            const int ia = sh[8 + t / nc];
            const int ic = sh[8 + t % nc];
            const double lc = H[ic * m + piv] / r;
            const double la = H[ia * m + piv] / r;
            H[ic * m + ia] = H[ic * m + ia] - lc * la;
        }
        __syncthreads();
    }
    if (tid == 0) {
        const int nt = sh[2];
        for (int a = 0; a < nt; ++a)
            for (int c = a + 1; c < nt; ++c)
                if (sh[40 + c] < sh[40 + a]) { const int t = sh[40 + a]; sh[40 + a] = sh[40 + c]; sh[40 + c] = t; }
        for (int a = 0; a < nt; ++a) keep[a] = sh[40 + a];
    }
    __syncthreads();
    return sh[2];
}

__device__ __forceinline__ void fail_state(DevState* st, int code) {
    st->done = FAILED;
    st->status = code;
}

// ------------------------------------------------ one-wave p x p algebra
//
// The Cholesky factor is formed with lane a holding row a of the matrix in
// registers, the other lanes' values read with v_readlane (uniform, no LDS round
// trip).  The triangular solves then run one right-hand side per lane, entirely in
// that lane's registers, with the factor read from LDS (uniform addresses, so
// every lane gets the same broadcast value).  Inactive agents are identity rows and
// columns, so every loop runs over the compile-time P.

__device__ __forceinline__ double bcast(double v, int src_lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src_lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src_lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// In-place Cholesky of the rows g (lane = row; lanes >= P hold padding): g becomes
// row `lane` of L in its lower part.  Each L entry is formed from the same products,
// in the same order, as the plain left-looking recurrence.  Returns false (uniform)
// on a pivot <= 0 or NaN.
template <int P>
__device__ __forceinline__ bool row_cholesky(double (&g)[P], int lane) {
#pragma unroll
    for (int j = 0; j < P; ++j) {
        const double djj = bcast(g[j], j);
        if (!(djj > 0.0)) return false;
        const double ljj = sqrt(djj);
        if (lane > j) g[j] = g[j] / ljj;
        else if (lane == j) g[j] = ljj;
#pragma unroll
        for (int b = j + 1; b < P; ++b) {
            const double lbj = bcast(g[j], b);
            if (lane > j) g[b] = g[b] - g[j] * lbj;
        }
    }
    return true;
}

// Row `lane` of src (row stride lds) with inactive rows / columns replaced by the
// identity (identity == true) or by zero.
template <int P>
__device__ __forceinline__ void row_load(double (&r)[P], const double* src, int lds, unsigned mask,
                                         bool identity, int lane) {
    const int a = lane < P ? lane : 0;
    const bool ra = (mask >> a) & 1u;
#pragma unroll
    for (int b = 0; b < P; ++b) {
        const bool on = ra && ((mask >> b) & 1u);
        r[b] = on ? src[a * lds + b] : ((identity && a == b) ? 1.0 : 0.0);
    }
}

// The same for a right-hand side kept in LDS (element i at Y[i * P + c], column c
// owned by this lane), with rolled loops: the register-resident form does not fit
// the register budget at P = 16.
template <int P>
__device__ __forceinline__ void col_chol_solve_lds(const double* L, const double* rinv, double* Y, int c) {
#pragma unroll 1
    for (int i = 0; i < P; ++i) {
        double s = Y[i * P + c];
        for (int k = 0; k < i; ++k) s -= L[i * P + k] * Y[k * P + c];
        Y[i * P + c] = s * rinv[i];
    }
#pragma unroll 1
    for (int i = P - 1; i >= 0; --i) {
        double s = Y[i * P + c];
        for (int k = i + 1; k < P; ++k) s -= L[k * P + i] * Y[k * P + c];
        Y[i * P + c] = s * rinv[i];
    }
}

// y <- (L L^T)^{-1} y for one right-hand side held by this lane.  L is row-major
// (stride P) in LDS, rinv[i] = 1 / L[i][i].  Every entry receives its terms in the
// textbook order (forward: k = 0, 1, ..., i - 1; backward: k = i + 1, ..., P - 1) and
// is then scaled by its reciprocal pivot.
// Forward, column-oriented: once y[k] is final, its multiples of column k are taken
// off the entries below, so the P - 1 - k updates of one k are independent and the
// dependent chain is two operations per k instead of one per term.  Backward, row by
// row (a column order would add the terms from P - 1 down).  The factor entries of the
// next column or row are loaded while the current one is used; a scheduling barrier
// per step keeps the compiler from hoisting every step's loads at once.
// LEAN: row by row in both halves without the look-ahead, one row's factor entries
// live at a time, for kernels whose waves have 128 registers (16-wave workgroups),
// where two columns in registers would spill at P = 32.
template <int P, bool LEAN = false>
__device__ __forceinline__ void col_chol_solve(const double* L, const double* rinv, double (&y)[P]) {
    if constexpr (LEAN) {
#pragma unroll
        for (int i = 0; i < P; ++i) {
            double s = y[i];
#pragma unroll
            for (int k = 0; k < i; ++k) s -= L[i * P + k] * y[k];
            y[i] = s * rinv[i];
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int i = P - 1; i >= 0; --i) {
            double s = y[i];
#pragma unroll
            for (int k = i + 1; k < P; ++k) s -= L[k * P + i] * y[k];
            y[i] = s * rinv[i];
            __builtin_amdgcn_sched_barrier(0);
        }
        return;
    }
    double c[P], ri;
#pragma unroll
    for (int i = 1; i < P; ++i) c[i] = L[i * P];
    ri = rinv[0];
#pragma unroll
    for (int k = 0; k < P; ++k) {
        double nx[P], nri = 0.0;
        if (k + 1 < P) {
#pragma unroll
            for (int i = k + 2; i < P; ++i) nx[i] = L[i * P + k + 1];
            nri = rinv[k + 1];
        }
        y[k] = y[k] * ri;
#pragma unroll
        for (int i = k + 1; i < P; ++i) y[i] -= c[i] * y[k];
#pragma unroll
        for (int i = k + 2; i < P; ++i) c[i] = nx[i];
        ri = nri;
        if constexpr (P > 8) __builtin_amdgcn_sched_barrier(0);
    }
    // backward: row i takes column i of L below the diagonal, c[k] = L[k][i] (k > i)
#pragma unroll
    for (int k = 0; k < P; ++k) c[k] = 0.0;
    ri = rinv[P - 1];
#pragma unroll
    for (int i = P - 1; i >= 0; --i) {
        double nx[P], nri = 0.0;
        if (i > 0) {
#pragma unroll
            for (int k = i; k < P; ++k) nx[k] = L[k * P + i - 1];
            nri = rinv[i - 1];
        }
        double s = y[i];
#pragma unroll
        for (int k = i + 1; k < P; ++k) s -= c[k] * y[k];
        y[i] = s * ri;
#pragma unroll
        for (int k = i; k < P; ++k) c[k] = nx[k];
        ri = nri;
        if constexpr (P > 8) __builtin_amdgcn_sched_barrier(0);
    }
}

// Fold M = 2^q values held by every lane of a wave into sums over the 64 lanes:
// each xor round with offset o keeps one half of the live values and adds the
// partner's copy of it, until one value per lane remains, then plain xor adds.
// Returns the index (0..M-1) of the total this lane holds in v[0].
// (the halving is unrolled by recursion over compile-time counts, so every array
// index is a constant and v stays in registers)
template <int M, int O, class T>
struct Fold {
    __device__ static __forceinline__ void run(T* v, int lane, int& idx) {
        if constexpr (O >= 1) {
            if constexpr (M > 1) {
                constexpr int h = M / 2;
                const bool up = (lane & O) != 0;
#pragma unroll
                for (int q = 0; q < h; ++q) {
                    const T send = up ? v[q] : v[q + h];
                    const T keep = up ? v[q + h] : v[q];
                    v[q] = keep + __shfl_xor(send, O);
                }
                if (up) idx += h;
                Fold<h, O / 2, T>::run(v, lane, idx);
            } else {
                v[0] += __shfl_xor(v[0], O);
                Fold<1, O / 2, T>::run(v, lane, idx);
            }
        }
    }
};

template <int M, class T>
__device__ __forceinline__ int wave_fold(T (&v)[M], int lane) {
    int idx = 0;
    Fold<M, 32, T>::run(v, lane, idx);
    return idx;
}

// ============================================================== k_ad: AD = A D

// State of the block step that the last workgroup needs, read at kernel entry so
// that its latency hides under the stream (the previous launches have finished
// writing it).
struct StepState0 {
    unsigned mask;
    double nb, tol, tau;
    int iter, maxit, m;
    int ad_streams;      // (only the A.D launch's last workgroup advances it)
};
__device__ __forceinline__ StepState0 read_state0(const DevState* st) {
    StepState0 s;
    s.mask = st->mask;
    s.nb = st->nb;
    s.tol = st->tol;
    s.tau = st->tau;
    s.iter = st->iter;
    s.maxit = st->maxit;
    s.m = st->m;
    s.ad_streams = st->ad_streams;
    return s;
}

// Thread t < ROWS * P of a workgroup holds element (row i0 + t / P, agent t % P) of
// D and of R (zero for rows >= n), loaded at kernel entry so that the latency of the
// loads hides under the rest of the work.  `early` false: not loaded yet, ad_tail
// loads them itself (the low-precision A.D kernels run at their register limit, and
// two values held through the stream cost them spills).
struct DRval {
    double d, r;
    bool early;
};
template <int PREC, int P, int ROWS>
__device__ __forceinline__ DRval load_dr(const AdArgs& a, int i0) {
    using TV = typename PT<PREC>::TV;
    DRval v{0.0, 0.0, true};
    const int t = threadIdx.x;
    if (t < ROWS * P) {
        const int r = t / P, j = t - (t / P) * P;
        const int i = i0 + r;
        if (i < a.n) {
            v.d = double(static_cast<const TV*>(a.V)[(int64_t)j * a.n_pad + i]);
            v.r = double(static_cast<const TV*>(a.R)[(int64_t)j * a.n_pad + i]);
        }
    }
    return v;
}

// The rank step (Alg. 3) and alpha = G^{-1} S of one block step from the totals in
// gtot (the lower triangle of G = D^T AD, then S = D^T R, FP64), run by all WG
// threads of the workgroup that holds them.  Writes alpha, the Cholesky factor of G
// (kept for beta) and, on a rank drop, the active set to the state.  Returns false
// (uniform) when the step stops: a failure, a re-inflation, or no agent left.  After
// the caller's next barrier, ish[202] holds the active set, the factor of G is in
// sm + P^2 (row-major, stride P) with 1 / L[i][i] at sm + 2 P^2, and alpha also in
// aout[x * P + c] when aout is given (LDS).  LDS: sm 3 P^2 + P doubles, gscr at
// least max(WG, P^2) doubles, ish 256 ints.
template <int P, int WG, bool REG = (P <= 8)>
__device__ __forceinline__ bool step_alpha(const double* gtot, const StepState0& s0, DevState* st, double* sm,
                                           double* gscr, int* ish, double* aout = nullptr) {
    constexpr int OS = P * (P + 1) / 2;
    const double* St = gtot + OS;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const unsigned mask0 = s0.mask;
    const double tau0 = s0.tau;
    const int m0 = s0.m;
    unsigned mask = mask0;
    double* Gs = sm;                          // full symmetric P x P
    double* Lsh = sm + P * P;                 // Cholesky factor, row-major stride P
    double* rinv = sm + 2 * P * P;            // 1 / L[i][i]
    double* lred = gscr;                      // per-lane values reduced by lane 0
    // G is symmetric in exact arithmetic: expand its lower triangle
    for (int t = tid; t < P * P; t += WG) {
        const int x = t / P, y = t - (t / P) * P;
        const int hi = max(x, y), lo = min(x, y);
        Gs[t] = gtot[hi * (hi + 1) / 2 + lo];
    }
    __syncthreads();
    // Fast path: the greedy pivoted factorisation of the diagonally scaled G (Alg. 3)
    // takes its pivots in non-increasing order (each elimination only lowers the
    // remaining diagonal, and the largest is taken), and its last pivot is
    // 1 / (G^-1)_ll of the scaled G for the index l taken last, so every pivot is at
    // least 1 / max_l (scaled G^-1)_ll, which is at least the determinant of the scaled
    // G.  When the determinant exceeds 2 tau (a margin for rounding), or else that bound
    // does, the rank step keeps every agent, and the factor of G in agent order is the
    // one the slow path below would form after running the greedy rule itself.  The
    // determinant is the product of the natural-order pivots; the bound is formed only
    // when the determinant test fails: (scaled G^-1)_ll = G_ll ||L^-1 e_l||^2, lane l
    // solving L y = e_l.
    if (wave == 0) {
        double g[P];
        row_load<P>(g, Gs, P, mask, true, lane);
        const bool ok = row_cholesky<P>(g, lane);
        if (lane < P) {
            double dg = 1.0;
#pragma unroll
            for (int b = 0; b < P; ++b) {
                Lsh[lane * P + b] = b <= lane ? g[b] : 0.0;
                if (b == lane) dg = g[b];
            }
            rinv[lane] = 1.0 / dg;
            lred[lane] = (ok && ((mask >> lane) & 1u)) ? (dg * dg) / Gs[lane * P + lane] : 1.0;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        double det = ok ? 1.0 : 0.0;                 // the same reads and value in every lane
#pragma unroll
        for (int jj = 0; jj < P; ++jj) det *= lred[jj];
        const bool by_det = ok && det > 2.0 * tau0;
        bool keep = by_det;
        if (ok && !by_det) {                         // (uniform)
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            if (lane < P) {
                double y[P];
                double q = 0.0;
#pragma unroll
                for (int k = 0; k < P; ++k) {
                    double t = (k == lane) ? 1.0 : 0.0;
#pragma unroll
                    for (int j = 0; j < k; ++j) t -= Lsh[k * P + j] * y[j];
                    y[k] = t * rinv[k];
                    q = fma(y[k], y[k], q);
                }
                if ((mask >> lane) & 1u) q *= Gs[lane * P + lane];
                lred[lane] = q;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            double mq = 0.0;
#pragma unroll
            for (int jj = 0; jj < P; ++jj) mq = (lred[jj] > mq || lred[jj] != lred[jj]) ? lred[jj] : mq;
            keep = mq * (2.0 * tau0) < 1.0;          // (a NaN is kept, and fails)
        }
        if (lane == 0) ish[200] = keep ? 1 : 0;
    }
    __syncthreads();
    const bool fast = ish[200] != 0;
    if (!fast) {
        int* act = &ish[96];    // active agents (global indices), ascending
        const int m = m0;
        if (tid < m) act[tid] = st->keep[tid];
        __syncthreads();
        double* Gc = sm + 2 * P * P + P;       // compact m x m (below: H)
        double* H = gscr;
        for (int t = tid; t < m * m; t += WG) Gc[t] = Gs[act[t / m] * P + act[t % m]];
        __syncthreads();
        int* kp = &ish[128];
        const int r = wg_rank_select(Gc, m, tau0, kp, H, &ish[0]);
        if (r < 0) {
            if (tid == 0) fail_state(st, r == -2 ? -2 : -3);
            return false;
        }
        if (r > 0 && r < m && st->reinflate_left > 0) {
            // re-inflation instead of the drop: the host restarts the block
            if (tid == 0) {
                unsigned nm = 0u;
                for (int q = 0; q < r; ++q) nm |= 1u << act[kp[q]];
                st->prev_mask = mask;
                st->mask = nm;
                st->done = REINFLATE;
            }
            return false;
        }
        if (r < m) {
            if (tid == 0) {
                unsigned nm = 0u;
                for (int q = 0; q < r; ++q) nm |= 1u << act[kp[q]];
                for (int q = 0; q < r; ++q) st->keep[q] = act[kp[q]];
                st->mask = nm;
                st->m = r;
                st->deflations += 1;
                if (r == 0) st->done = FINISHED;
                ish[201] = (int)nm;
            }
            __syncthreads();
            mask = (unsigned)ish[201];
            if (r == 0) return false;
        }
        if (wave == 0) {
            double g[P];
            row_load<P>(g, Gs, P, mask, true, lane);
            const bool ok = row_cholesky<P>(g, lane);
            if (lane < P) {
                double dg = 1.0;
#pragma unroll
                for (int b = 0; b < P; ++b) {
                    Lsh[lane * P + b] = b <= lane ? g[b] : 0.0;
                    if (b == lane) dg = g[b];
                }
                rinv[lane] = 1.0 / dg;
            }
            if (lane == 0) ish[203] = ok ? 0 : 1;
        }
        __syncthreads();
        if (ish[203]) {
            if (tid == 0) fail_state(st, -3);
            return false;
        }
    }
    if (tid == 0) ish[202] = (int)mask;
    if (wave != 0 || lane >= P) return true;
    // lane c: alpha[:, c] = G^{-1} (D^T R)[:, c] in this lane's registers; the factor
    // is kept for beta, which is solved from the new residual
    const int c = lane;
    const bool ac = (mask >> c) & 1u;
    if constexpr (REG) {
        double y[P];
#pragma unroll
        for (int x = 0; x < P; ++x) y[x] = (ac && ((mask >> x) & 1u)) ? St[x * P + c] : 0.0;
        col_chol_solve<P, (P > 16 && WG > 512)>(Lsh, rinv, y);
#pragma unroll
        for (int x = 0; x < P; ++x) {
            st->alpha[x * kMaxP + c] = y[x];
            st->L[x * kMaxP + c] = Lsh[x * P + c];
            if (aout) aout[x * P + c] = y[x];
        }
    } else {
        double* Yc = sm + 2 * P * P + P;       // column c of alpha at Yc[x * P + c]
#pragma unroll 1
        for (int x = 0; x < P; ++x) Yc[x * P + c] = (ac && ((mask >> x) & 1u)) ? St[x * P + c] : 0.0;
        col_chol_solve_lds<P>(Lsh, rinv, Yc, c);
#pragma unroll 1
        for (int x = 0; x < P; ++x) {
            st->alpha[x * kMaxP + c] = Yc[x * P + c];
            st->L[x * kMaxP + c] = Lsh[x * P + c];
            if (aout) aout[x * P + c] = Yc[x * P + c];
        }
    }
    return true;
}

// LDS of the A.D launch's tail (ad_tail): a kernel declares it __shared__, or lays it
// over staging buffers that are free by the time the tail runs.
template <int P, int ROWS, int WG>
struct TailLds {
    double drw[ROWS * P];                     // D rows of this workgroup
    double rrw[ROWS * P];                     // R rows of this workgroup
    double gmine[P * (P + 1) / 2 + P * P];    // this workgroup's product shares
    double gtot[P * (P + 1) / 2 + P * P];     // grid totals (last workgroup)
    double sm[3 * P * P + P];                 // the p x p algebra (step_alpha)
    double gscr[WG > P * P ? WG : P * P];     // reduction scratch, rank-step matrix
    int ish[256];
};

// The products D^T AD and D^T R over the ROWS AD rows of workgroup `tile` (in adt,
// LDS, row stride P, zero for rows >= n) and the D and R rows (dr, see load_dr),
// their fixed-order reduction over the `ntiles` workgroups, and in the last
// workgroup the rank step (Alg. 3) and alpha, with the Cholesky factor of G kept in
// the state for beta.  WG threads.
// REG: the alpha solve in registers (one right-hand side per lane) at every P; the
// A.D kernels whose streams leave the registers for it (the matrix-core tile) set it.
template <int PREC, int P, int ROWS, int WG, bool REG = (P <= 8)>
__device__ __forceinline__ void ad_tail(const AdArgs& a, const int tile, const int ntiles, const double* adt,
                                        const StepState0& s0, const DRval dr, TailLds<P, ROWS, WG>& L) {
    constexpr int kAdCols = ROWS;
    double* drw = L.drw;
    double* rrw = L.rrw;
    double* gmine = L.gmine;
    double* gtot = L.gtot;
    double* sm = L.sm;
    double* gscr = L.gscr;
    int* ish = L.ish;
    const int tid = threadIdx.x;
    const int i0 = tile * kAdCols;
    const int iter0 = s0.iter, maxit0 = s0.maxit;

    // ---- the workgroup's share of the products over its rows, packed as
    //   G = D^T AD (lower triangle) and S = D^T R (full)
    if (dr.early) {                       // one D and R value per thread (load_dr)
        if (tid < kAdCols * P) {
            const int r = tid / P, j = tid - (tid / P) * P;
            drw[r * P + j] = dr.d;
            rrw[r * P + j] = dr.r;
        }
    } else {
        using TV = typename PT<PREC>::TV;
        for (int t = tid; t < kAdCols * P; t += WG) {
            const int r = t / P, j = t - (t / P) * P;
            const int i = i0 + r;
            const int64_t o = (int64_t)j * a.n_pad + i;
            drw[r * P + j] = i < a.n ? double(static_cast<const TV*>(a.V)[o]) : 0.0;
            rrw[r * P + j] = i < a.n ? double(static_cast<const TV*>(a.R)[o]) : 0.0;
        }
    }
    __syncthreads();
    constexpr int TRI = P * (P + 1) / 2;
    constexpr int OS = TRI;
    constexpr int NE = TRI + P * P;
    for (int e = tid; e < NE; e += WG) {
        const double* Wv;
        int x, y;
        if (e < OS) {                                     // triangle of G
            x = 0;
            while ((x + 1) * (x + 2) / 2 <= e) ++x;
            y = e - x * (x + 1) / 2;
            Wv = adt;
        } else {                                          // S, full
            const int t = e - OS;
            x = t / P;
            y = t - x * P;
            Wv = rrw;
        }
        double s = 0.0;
        for (int r = 0; r < kAdCols; ++r) s = fma(drw[r * P + x], Wv[r * P + y], s);
        gmine[e] = s;
    }
    __syncthreads();
    if (!grid_reduce<(P >= 8 ? kGroup : 16), WG>(gmine, NE, a.red, gtot, &ish[0], gscr, tile, ntiles)) return;

    // ---- last workgroup: rank step (Alg. 3) and alpha
    DevState* st = a.st;
    // (the count read at entry: a load here would hold wave 0, and so the rank step,
    // for a memory round trip)
    if (tid == 0) st->ad_streams = s0.ad_streams + 1;
    if (iter0 >= maxit0) {                    // (the update launch stops the steps first)
        if (tid == 0) st->done = MAXIT;
        return;
    }
    (void)step_alpha<P, WG, REG>(gtot, s0, st, sm, gscr, ish);
}

// One tile (NW * CW rows of AD) of the block step of one system; `tile` of `ntiles`.
template <int PREC, int P, class CFG>
__device__ __forceinline__ void ad_tile(const AdArgs& a, const int tile, const int ntiles) {
    using TA = typename PT<PREC>::TA;
    using TV = typename PT<PREC>::TV;
    using TACC = typename PT<PREC>::TACC;
    constexpr int E = PT<PREC>::E;
    constexpr int KSTEP = 64 * E;
    constexpr int SPC = CFG::SPC;             // wave steps per chunk
    constexpr int KC = SPC * KSTEP;
    constexpr int kCW = CFG::CW;
    constexpr int kAdCols = CFG::ROWS;
    constexpr bool NT = CFG::NT;
    constexpr int NV = kCW * P;               // lane sums per wave
    constexpr int WG = CFG::WG;               // threads of the workgroup
    constexpr int PER = (P * KC + WG - 1) / WG;   // staged D values per thread per chunk
    constexpr bool PART = PER * WG != P * KC;     // the last round of staging is partial
    static_assert(NV <= 64, "lane sums per wave");
    static_assert(PREC != PREC_F64 || kAdCols * P <= WG, "one early D and R value per thread (load_dr)");
    static_assert(512 % KC == 0, "chunks must tile the padded length");

    __shared__ TV dch[2][P * KC];             // D chunk, agent-major: dch[b][j*KC + kk]
    __shared__ double adt[kAdCols * P];       // AD rows of this workgroup
    __shared__ TailLds<P, kAdCols, WG> tl;

    // every A.D launch follows the direction launch of the previous block step (if
    // any): its flag is spent
    if (tile == 0 && threadIdx.x == 0 && a.st->dir_pending) a.st->dir_pending = 0;
    if (!a.product_only && a.st->done != RUNNING) return;
    // state the last workgroup needs, read now so that its latency hides under the
    // stream (the previous launches have finished writing it), and the D and R rows
    // of the products
    const StepState0 s0 = read_state0(a.st);
    const DRval dr = (a.product_only || PREC != PREC_F64) ? DRval{0.0, 0.0, false}
                                                          : load_dr<PREC, P, CFG::ROWS>(a, tile * CFG::ROWS);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int n = a.n;
    const int i0 = tile * kAdCols;                        // first AD row of the workgroup
    const int iw = i0 + wave * kCW;                       // first row of this wave
    const TV* __restrict__ V = static_cast<const TV*>(a.V);
    const int64_t lda = a.lda;
    const TA* colhi[kCW];
    const TA* collo[kCW];
#pragma unroll
    for (int c = 0; c < kCW; ++c) {
        const int i = min(iw + c, n - 1);                 // rows >= n compute a copy, never stored
        colhi[c] = static_cast<const TA*>(a.A) + (int64_t)i * lda;
        collo[c] = (PREC == PREC_BF16X2) ? static_cast<const TA*>(a.A_lo) + (int64_t)i * lda : colhi[c];
    }

    TACC acc[kCW][P];
#pragma unroll
    for (int c = 0; c < kCW; ++c)
#pragma unroll
        for (int j = 0; j < P; ++j) acc[c][j] = TACC(0);

    const int nch = (n + KC - 1) / KC;     // chunks end at <= n_pad: KC divides 512
    // first chunk of this workgroup (rotated when staggering); chunks then wrap
    const int c0 = CFG::STG ? (int)(((unsigned)tile * 13u) % (unsigned)nch) : 0;
    TV pre[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int idx = tid + q * WG;
        const int j = idx / KC, kk = idx - (idx / KC) * KC;
        if (!PART || idx < P * KC) pre[q] = V[(int64_t)j * a.n_pad + c0 * KC + kk];
    }
#pragma unroll
    for (int q = 0; q < PER; ++q)
        if (!PART || tid + q * WG < P * KC) dch[0][tid + q * WG] = pre[q];
    __syncthreads();

    for (int it = 0; it < nch; ++it) {
        const int buf = it & 1;
        int ch = c0 + it;
        if (ch >= nch) ch -= nch;
        const int k0 = ch * KC;
        const bool more = it + 1 < nch;
        if (more) {
            const int nx = (ch + 1 < nch) ? ch + 1 : 0;
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                const int idx = tid + q * WG;
                const int j = idx / KC, kk = idx - (idx / KC) * KC;
                if (!PART || idx < P * KC) pre[q] = V[(int64_t)j * a.n_pad + nx * KC + kk];
            }
        }
        const TV* dc = dch[buf];
        if (k0 + KC <= n) {
#pragma unroll
            for (int s = 0; s < SPC; ++s) {
                const int kk = s * KSTEP + lane * E;
                TACC av[kCW][E];
#pragma unroll
                for (int c = 0; c < kCW; ++c) Loader<PREC, NT>::load(colhi[c] + k0 + kk, collo[c] + k0 + kk, av[c]);
#pragma unroll
                for (int j = 0; j < P; ++j) {
                    TACC d[E];
#pragma unroll
                    for (int e = 0; e < E; ++e) d[e] = TACC(dc[j * KC + kk + e]);
#pragma unroll
                    for (int c = 0; c < kCW; ++c)
#pragma unroll
                        for (int e = 0; e < E; ++e) acc[c][j] = fma(av[c][e], d[e], acc[c][j]);
                }
            }
        } else {
            // last, partial chunk: element loads guarded by k < n
            for (int s = 0; s < SPC; ++s) {
                const int kk = s * KSTEP + lane * E;
                TACC av[kCW][E];
#pragma unroll
                for (int c = 0; c < kCW; ++c)
#pragma unroll
                    for (int e = 0; e < E; ++e)
                        av[c][e] = (k0 + kk + e < n) ? Loader<PREC, NT>::load1(colhi[c] + k0 + kk + e, collo[c] + k0 + kk + e)
                                                     : TACC(0);
#pragma unroll
                for (int j = 0; j < P; ++j) {
                    TACC d[E];
#pragma unroll
                    for (int e = 0; e < E; ++e) d[e] = TACC(dc[j * KC + kk + e]);
#pragma unroll
                    for (int c = 0; c < kCW; ++c)
#pragma unroll
                        for (int e = 0; e < E; ++e) acc[c][j] = fma(av[c][e], d[e], acc[c][j]);
                }
            }
        }
        if (more) {
#pragma unroll
            for (int q = 0; q < PER; ++q)
                if (!PART || tid + q * WG < P * KC) dch[buf ^ 1][tid + q * WG] = pre[q];
        }
        __syncthreads();
    }

    // ---- lane sums -> complete AD rows (fixed butterfly order)
    TACC v[NV];
#pragma unroll
    for (int c = 0; c < kCW; ++c)
#pragma unroll
        for (int j = 0; j < P; ++j) v[c * P + j] = acc[c][j];
    const int idx = wave_fold<NV>(v, lane);
    constexpr int REP = 64 / NV;             // lanes holding the same total
    if (lane % REP == 0) {
        const int c = idx / P, j = idx - (idx / P) * P;
        const int i = iw + c;
        const TV y = TV(v[0]);
        if (i < n) static_cast<TV*>(a.AD)[(int64_t)j * a.n_pad + i] = y;
        adt[(wave * kCW + c) * P + j] = (i < n) ? double(y) : 0.0;   // rows >= n hold copies
    }
    if (a.product_only) return;
    ad_tail<PREC, P, kAdCols, WG>(a, tile, ntiles, adt, s0, dr, tl);
}

template <class CFG>
__host__ __device__ constexpr int ad_tiles(int n) { return (n + CFG::ROWS - 1) / CFG::ROWS; }

template <int PREC, int P, class CFG>
__global__ __launch_bounds__(CFG::WG) __attribute__((amdgpu_waves_per_eu(CFG::MINW))) void k_ad(AdArgs a) {
    ad_tile<PREC, P, CFG>(a, blockIdx.x, gridDim.x);
}

// Many systems in one launch: workgroup w runs tile items[w].y of system items[w].x.
template <int PREC, int P, class CFG>
__global__ __launch_bounds__(CFG::WG) __attribute__((amdgpu_waves_per_eu(CFG::MINW)))
void k_ad_batch(const AdArgs* __restrict__ sys, const int4* __restrict__ items) {
    const int4 it = items[blockIdx.x];
    const AdArgs a = sys[it.x];
    ad_tile<PREC, P, CFG>(a, it.y, ad_tiles<CFG>(a.n));
}

// ------------------------------- A.D on the matrix cores (FP64, P = 16 or 8 agents)
//
// At P = 16 every 8-byte element of A meets 16 multiply-adds, 4 flops per byte: at
// 8 TB/s that is 32 TFLOP/s, which the vector FMA path cannot reach while it also
// reads every D value it multiplies from LDS.  v_mfma_f64_16x16x4_f64 takes a 16 x 4
// slice of A (16 AD rows, 4 contraction indices k) and a 4 x 16 slice of D from one
// register per lane and adds their 16 x 16 product into four accumulator registers:
// lane l holds A(row l % 16, k-slot l / 16), D(k-slot l / 16, agent l % 16) and the
// results (rows l / 16 + 4 v, agent l % 16), v = 0..3 (checked on the device).
//
// The MFMA operand layout spreads a wave's lanes over 16 columns of A; loaded
// straight from memory that makes every load touch 16 columns 64 KB apart, and the
// stream ran at 0.42 of the HBM peak.  So A is staged: a workgroup owns 16 RB
// consecutive columns (AD rows), a contiguous stretch of A, and reads chunks of
// KC = 128 contraction indices of all of them, each wave load one whole kilobyte of
// one column, into LDS (double buffered, the next chunk's loads in flight while the
// current one is multiplied); the D rows of the chunk are staged beside it.  The
// workgroup's NW waves split each chunk's 32 k-steps of 4 between them, each keeping
// its own accumulators; after the stream their partial tiles are added in LDS by a
// fixed binary tree (waves w + h into w for h = NW/2, .., 1), so the result is the
// same on every run, alone or batched.  The tile then goes through the same
// products, reduction and rank step as the vector path (ad_tail).  At P = 8 the
// lanes of agents 8..15 carry zeros: the matrix cores do twice the useful work,
// still far inside their FP64 rate at the HBM stream rate (2 flops per byte of A).

typedef double d4v __attribute__((ext_vector_type(4)));

template <int P, int RB, int NW>
__device__ __forceinline__ void ad_tile_mfma(const AdArgs& a, const int tile, const int ntiles) {
    static_assert(P == 8 || P == 16 || P == 32, "agent blocks of 16 (P = 8: agents 8..15 zero)");
    constexpr int NB = P > 16 ? P / 16 : 1;   // agent blocks of 16
    constexpr int PD = 16 * NB;               // staged agent rows
    constexpr int ROWS = 16 * RB;
    constexpr int WG = 64 * NW;
    constexpr int KC = 128;                   // contraction indices per chunk: one 16-byte
                                              // load per lane of a wave covers a column
    constexpr int LD = KC + 4;                // LDS row stride in doubles (spreads banks)
    constexpr int KS = KC / 4 / NW;           // k-steps of 4 per wave per chunk
    constexpr int CA = ROWS / NW;             // A columns a wave loads per chunk
    constexpr int CD = (P + NW - 1) / NW;     // D agent rows a wave loads per chunk
    constexpr int ASZ = ROWS * LD, DSZ = PD * LD;
    static_assert(KS >= 1 && CA >= 1 && ROWS % NW == 0 && KC == 2 * 64, "tile shape");
    using Tail = TailLds<P, ROWS, WG>;
    static_assert(sizeof(Tail) <= sizeof(double) * 2 * (ASZ + DSZ), "the tail's LDS fits the staging buffers");
    static_assert((NW / 2) * ROWS * P <= 2 * (ASZ + DSZ), "tree partials fit the staging buffers");
    // two chunk buffers of A ([column][k]) and of D ([agent][k]; agents >= P zero),
    // later the tree's partials and the tail's LDS
    __shared__ double stage[2 * (ASZ + DSZ)];
    __shared__ double adt[ROWS * P];          // AD rows of this workgroup
    double* const Ash0 = stage;
    double* const Dsh0 = stage + 2 * ASZ;

    if (tile == 0 && threadIdx.x == 0 && a.st->dir_pending) a.st->dir_pending = 0;
    if (!a.product_only && a.st->done != RUNNING) return;
    const StepState0 s0 = read_state0(a.st);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int r = lane & 15, g = lane >> 4;
    const int n = a.n;
    const int i0 = tile * ROWS;
    const double* __restrict__ A = static_cast<const double*>(a.A);
    const double* __restrict__ V = static_cast<const double*>(a.V);
    if (P < 16) {
        for (int t = tid; t < 2 * (16 - P) * LD; t += WG) {
            const int bf = t / ((16 - P) * LD), o = t - bf * ((16 - P) * LD);
            Dsh0[bf * DSZ + P * LD + o] = 0.0;
        }
    }
    // this wave's share of a chunk: A columns wave + NW q (q < CA), lane l holding
    // k = 2 l, 2 l + 1 of the chunk; D agents wave + NW q (q < CD; a wave whose agent
    // is >= P loads agent P - 1 and does not store it)
    const double* colp[CA];
#pragma unroll
    for (int q = 0; q < CA; ++q) {
        const int i = min(i0 + wave + NW * q, n - 1);   // rows >= n compute a copy, never stored
        colp[q] = A + (int64_t)i * a.lda;
    }
    const double* dcol[CD];
#pragma unroll
    for (int q = 0; q < CD; ++q) dcol[q] = V + (int64_t)min(wave + NW * q, P - 1) * a.n_pad;
    // whole chunks: branch-free loads, so that the loads of the next chunks stay in
    // flight (counted exactly) while the current one is multiplied
    auto load_full = [&](int ch, d2v (&ra)[CA], d2v (&rd)[CD]) {
        const int k = ch * KC + 2 * lane;
#pragma unroll
        for (int q = 0; q < CA; ++q) ra[q] = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(colp[q] + k));
#pragma unroll
        for (int q = 0; q < CD; ++q) rd[q] = *reinterpret_cast<const d2v*>(dcol[q] + k);
    };
    auto store_chunk = [&](int bf, const d2v (&ra)[CA], const d2v (&rd)[CD]) {
#pragma unroll
        for (int q = 0; q < CA; ++q)
            *reinterpret_cast<d2v*>(&Ash0[bf * ASZ + (wave + NW * q) * LD + 2 * lane]) = ra[q];
#pragma unroll
        for (int q = 0; q < CD; ++q) {
            const int j = wave + NW * q;
            if (j < P) *reinterpret_cast<d2v*>(&Dsh0[bf * DSZ + j * LD + 2 * lane]) = rd[q];
        }
    };
    d4v acc[RB][NB];
#pragma unroll
    for (int b = 0; b < RB; ++b)
#pragma unroll
        for (int c = 0; c < NB; ++c) acc[b][c] = d4v{0.0, 0.0, 0.0, 0.0};
    auto mul_chunk = [&](int bf) {
        const double* As = Ash0 + bf * ASZ;
        const double* Ds = Dsh0 + bf * DSZ;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int kk = 4 * (wave * KS + s) + g;
            double dv[NB];
#pragma unroll
            for (int c = 0; c < NB; ++c) dv[c] = Ds[(16 * c + r) * LD + kk];
#pragma unroll
            for (int b = 0; b < RB; ++b) {
                const double av = As[(16 * b + r) * LD + kk];
#pragma unroll
                for (int c = 0; c < NB; ++c) acc[b][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, dv[c], acc[b][c], 0, 0, 0);
            }
        }
    };

    // the whole chunks, two in flight in registers (ring a0/d0, a1/d1) while the one
    // in LDS is multiplied; the loads past the last chunk repeat it (never stored).
    // The scheduling barriers keep each chunk's loads issued ahead of the products of
    // the chunk before it, where the compiler would sink them.  (A third chunk in
    // flight measured no faster.)
    const int nf = n / KC;
    if (nf > 0) {
        d2v a0[CA], d0[CD], a1[CA], d1[CD];
        load_full(0, a0, d0);
        load_full(min(1, nf - 1), a1, d1);
        store_chunk(0, a0, d0);
        __syncthreads();
        for (int c = 0;; c += 2) {
            load_full(min(c + 2, nf - 1), a0, d0);
            __builtin_amdgcn_sched_barrier(0);
            mul_chunk(0);                            // chunk c
            __builtin_amdgcn_sched_barrier(0);
            if (c + 1 >= nf) break;
            store_chunk(1, a1, d1);                  // chunk c + 1
            __syncthreads();
            load_full(min(c + 3, nf - 1), a1, d1);
            __builtin_amdgcn_sched_barrier(0);
            mul_chunk(1);                            // chunk c + 1
            __builtin_amdgcn_sched_barrier(0);
            if (c + 2 >= nf) break;
            store_chunk(0, a0, d0);                  // chunk c + 2
            __syncthreads();
        }
    }
    // the last, partial chunk (n % KC != 0): loads guarded by k < n
    if (n % KC) {
        d2v ra[CA], rd[CD];
        const int k = nf * KC + 2 * lane;
#pragma unroll
        for (int q = 0; q < CA; ++q) {
            ra[q].x = k < n ? colp[q][k] : 0.0;
            ra[q].y = k + 1 < n ? colp[q][k + 1] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < CD; ++q) {
            rd[q].x = k < n ? dcol[q][k] : 0.0;
            rd[q].y = k + 1 < n ? dcol[q][k + 1] : 0.0;
        }
        __syncthreads();                             // every wave is done with both buffers
        store_chunk(0, ra, rd);
        __syncthreads();
        mul_chunk(0);
    }
    __syncthreads();

    // ---- the waves' partial tiles, added by a fixed tree in the (now free) staging
    // buffers; lane (c, g) holds rows g + 4 v of each row block, agent 16 blk + c
    double* part = stage;
    const bool dl = r < P;
#pragma unroll
    for (int h = NW / 2; h >= 1; h >>= 1) {
        if (wave >= h && wave < 2 * h && dl) {
#pragma unroll
            for (int b = 0; b < RB; ++b)
#pragma unroll
                for (int c = 0; c < NB; ++c)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        part[((wave - h) * ROWS + 16 * b + g + 4 * v) * P + 16 * c + r] = acc[b][c][v];
        }
        __syncthreads();
        if (wave < h && dl) {
#pragma unroll
            for (int b = 0; b < RB; ++b)
#pragma unroll
                for (int c = 0; c < NB; ++c)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        acc[b][c][v] += part[(wave * ROWS + 16 * b + g + 4 * v) * P + 16 * c + r];
        }
        __syncthreads();
    }
    if (wave == 0 && dl) {
#pragma unroll
        for (int b = 0; b < RB; ++b)
#pragma unroll
            for (int c = 0; c < NB; ++c)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = 16 * b + g + 4 * v;
                    adt[row * P + 16 * c + r] = (i0 + row < n) ? acc[b][c][v] : 0.0;   // rows >= n hold copies
                }
    }
    __syncthreads();
    // AD rows to memory, each agent's ROWS rows contiguous
    for (int t = tid; t < ROWS * P; t += WG) {
        const int j = t / ROWS, row = t - (t / ROWS) * ROWS;
        if (i0 + row < n) static_cast<double*>(a.AD)[(int64_t)j * a.n_pad + i0 + row] = adt[row * P + j];
    }
    if (a.product_only) return;
    ad_tail<PREC_F64, P, ROWS, WG, true>(a, tile, ntiles, adt, s0, DRval{0.0, 0.0, false},
                                         *reinterpret_cast<Tail*>(stage));
}

// Tile of workgroup b of nb: the workgroups of a launch are handed to the 8 XCDs in
// turn, and this order gives each XCD a contiguous run of tiles (when 8 divides nb).
// Only the placement changes: every tile, and every reduction group of tiles, is the
// same.  Measured on the FP64 matrix-core tile, 3-5 % faster at P = 16 (n = 4096 to
// 32768) and level at P = 32 and at n = 1024-2048; the vector tile at P = 8 ran slower
// with it and keeps the launch order.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    return (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
}

template <int P, int RB, int NW>
__global__ __launch_bounds__(64 * NW) void k_ad_mfma(AdArgs a) {
    ad_tile_mfma<P, RB, NW>(a, xcd_tile(blockIdx.x, gridDim.x), gridDim.x);
}

template <int P, int RB, int NW>
__global__ __launch_bounds__(64 * NW) void k_ad_mfma_batch(const AdArgs* __restrict__ sys,
                                                            const int4* __restrict__ items) {
    const int4 it = items[blockIdx.x];
    const AdArgs a = sys[it.x];
    ad_tile_mfma<P, RB, NW>(a, it.y, (a.n + 16 * RB - 1) / (16 * RB));
}

// ---------------- A.D on the matrix cores with FP32 operands (FP32 and BF16x2 A, P = 8 or 16)
//
// The low-precision modes stream A in 4 bytes per element (FP32, or the BF16 hi and lo
// planes) and keep D in FP32.  At P = 16 that is 8 flops per byte of A, which the vector
// path (FP32 FMAs on D values read from LDS) cannot sustain at the HBM rate.
// v_mfma_f32_16x16x4_f32 multiplies FP32 operands with FP32 accumulation, so A enters
// it as the value the vector path uses (for BF16x2, hi + lo, exact in FP32).  Lane l
// supplies A(row l % 16, k-slot l / 16) and D(k-slot l / 16, agent l % 16), as in the
// FP64 tile, but receives the result rows 4 (l / 16) + v, v = 0..3 (checked on the
// device).  Chunks of KC = 256 contraction indices: one 16-byte load (FP32) or one
// 8-byte load per plane (BF16x2) per lane covers a column; A is converted to FP32 as it
// is stored to LDS.  Double buffering, the waves' split of the k-steps, the fixed tree
// of the waves' partial tiles and the tail are those of the FP64 tile.  At P = 8 the
// lanes of agents 8..15 carry zeros.
typedef unsigned u2v __attribute__((ext_vector_type(2)));

template <int PREC, int P, int RB, int NW>
__device__ __forceinline__ void ad_tile_mma32(const AdArgs& a, const int tile, const int ntiles) {
    static_assert((PREC == PREC_F32 || PREC == PREC_BF16X2) && (P == 8 || P == 16), "FP32 operands, one agent block");
    constexpr bool BF = PREC == PREC_BF16X2;
    constexpr int ROWS = 16 * RB;
    constexpr int WG = 64 * NW;
    constexpr int KC = 256;                   // contraction indices per chunk: 4 per lane
    constexpr int LD = KC + 4;                // LDS row stride in floats (rows 4 banks apart)
    constexpr int KS = KC / 4 / NW;           // k-steps of 4 per wave per chunk
    constexpr int CA = ROWS / NW;             // A columns a wave loads per chunk
    constexpr int CD = (P + NW - 1) / NW;     // D agent rows a wave loads per chunk
    constexpr int ASZ = ROWS * LD, DSZ = 16 * LD;
    static_assert(KS >= 1 && CA >= 1 && ROWS % NW == 0 && KC == 4 * 64, "tile shape");
    using Tail = TailLds<P, ROWS, WG>;
    static_assert(sizeof(Tail) <= sizeof(float) * 2 * (ASZ + DSZ), "the tail's LDS fits the staging buffers");
    static_assert((NW / 2) * ROWS * P <= 2 * (ASZ + DSZ), "tree partials fit the staging buffers");
    // A register slice of one column chunk: 4 FP32 values, or 4 hi and 4 lo BF16 values
    struct ARegF { f4v v; };
    struct ARegB { u2v h, l; };
    using AR = typename std::conditional<BF, ARegB, ARegF>::type;
    __shared__ __align__(16) float stage[2 * (ASZ + DSZ)];
    __shared__ double adt[ROWS * P];          // AD rows of this workgroup
    float* const Ash0 = stage;
    float* const Dsh0 = stage + 2 * ASZ;

    if (tile == 0 && threadIdx.x == 0 && a.st->dir_pending) a.st->dir_pending = 0;
    if (!a.product_only && a.st->done != RUNNING) return;
    const StepState0 s0 = read_state0(a.st);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int r = lane & 15, g = lane >> 4;
    const int n = a.n;
    const int i0 = tile * ROWS;
    using TA = typename PT<PREC>::TA;
    const float* __restrict__ V = static_cast<const float*>(a.V);
    if (P < 16) {
        for (int t = tid; t < 2 * (16 - P) * LD; t += WG) {
            const int bf = t / ((16 - P) * LD), o = t - bf * ((16 - P) * LD);
            Dsh0[bf * DSZ + P * LD + o] = 0.0f;
        }
    }
    // this wave's share of a chunk: A columns wave + NW q (q < CA), lane l holding
    // k = 4 l .. 4 l + 3 of the chunk; D agents wave + NW q (q < CD; a wave whose agent
    // is >= P loads agent P - 1 and does not store it)
    const TA* colp[CA];
    const TA* colq[CA];
#pragma unroll
    for (int q = 0; q < CA; ++q) {
        const int i = min(i0 + wave + NW * q, n - 1);   // rows >= n compute a copy, never stored
        colp[q] = static_cast<const TA*>(a.A) + (int64_t)i * a.lda;
        colq[q] = BF ? static_cast<const TA*>(a.A_lo) + (int64_t)i * a.lda : colp[q];
    }
    const float* dcol[CD];
#pragma unroll
    for (int q = 0; q < CD; ++q) dcol[q] = V + (int64_t)min(wave + NW * q, P - 1) * a.n_pad;
    auto load_full = [&](int ch, AR (&ra)[CA], f4v (&rd)[CD]) {
        const int k = ch * KC + 4 * lane;
#pragma unroll
        for (int q = 0; q < CA; ++q) {
            if constexpr (BF) {
                ra[q].h = __builtin_nontemporal_load(reinterpret_cast<const u2v*>(colp[q] + k));
                ra[q].l = __builtin_nontemporal_load(reinterpret_cast<const u2v*>(colq[q] + k));
            } else {
                ra[q].v = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(colp[q] + k));
            }
        }
#pragma unroll
        for (int q = 0; q < CD; ++q) rd[q] = *reinterpret_cast<const f4v*>(dcol[q] + k);
    };
    // the last, partial chunk: every element guarded by k < n
    auto load_part = [&](int ch, AR (&ra)[CA], f4v (&rd)[CD]) {
        const int k = ch * KC + 4 * lane;
#pragma unroll
        for (int q = 0; q < CA; ++q) {
            if constexpr (BF) {
                unsigned hw[2] = {0u, 0u}, lw[2] = {0u, 0u};
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (k + e < n) {
                        hw[e >> 1] |= (unsigned)colp[q][k + e] << (16 * (e & 1));
                        lw[e >> 1] |= (unsigned)colq[q][k + e] << (16 * (e & 1));
                    }
                ra[q].h = u2v{hw[0], hw[1]};
                ra[q].l = u2v{lw[0], lw[1]};
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) ra[q].v[e] = k + e < n ? colp[q][k + e] : 0.0f;
            }
        }
#pragma unroll
        for (int q = 0; q < CD; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) rd[q][e] = k + e < n ? dcol[q][k + e] : 0.0f;
    };
    auto store_chunk = [&](int bf, const AR (&ra)[CA], const f4v (&rd)[CD]) {
#pragma unroll
        for (int q = 0; q < CA; ++q) {
            f4v v;
            if constexpr (BF) {
                // hi + lo is exact in FP32 (8 significant bits each, lo below hi)
                v.x = __uint_as_float(ra[q].h.x << 16) + __uint_as_float(ra[q].l.x << 16);
                v.y = __uint_as_float(ra[q].h.x & 0xffff0000u) + __uint_as_float(ra[q].l.x & 0xffff0000u);
                v.z = __uint_as_float(ra[q].h.y << 16) + __uint_as_float(ra[q].l.y << 16);
                v.w = __uint_as_float(ra[q].h.y & 0xffff0000u) + __uint_as_float(ra[q].l.y & 0xffff0000u);
            } else {
                v = ra[q].v;
            }
            *reinterpret_cast<f4v*>(&Ash0[bf * ASZ + (wave + NW * q) * LD + 4 * lane]) = v;
        }
#pragma unroll
        for (int q = 0; q < CD; ++q) {
            const int j = wave + NW * q;
            if (j < P) *reinterpret_cast<f4v*>(&Dsh0[bf * DSZ + j * LD + 4 * lane]) = rd[q];
        }
    };
    f4v acc[RB];
#pragma unroll
    for (int b = 0; b < RB; ++b) acc[b] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
    auto mul_chunk = [&](int bf) {
        const float* As = Ash0 + bf * ASZ;
        const float* Ds = Dsh0 + bf * DSZ;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int kk = 4 * (wave * KS + s) + g;
            const float dv = Ds[r * LD + kk];
#pragma unroll
            for (int b = 0; b < RB; ++b)
                acc[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(As[(16 * b + r) * LD + kk], dv, acc[b], 0, 0, 0);
        }
    };

    // the whole chunks, two in flight in registers (ring a0/d0, a1/d1) while the one
    // in LDS is multiplied; the loads past the last chunk repeat it (never stored)
    const int nf = n / KC;
    if (nf > 0) {
        AR a0[CA], a1[CA];
        f4v d0[CD], d1[CD];
        load_full(0, a0, d0);
        load_full(min(1, nf - 1), a1, d1);
        store_chunk(0, a0, d0);
        __syncthreads();
        for (int c = 0;; c += 2) {
            load_full(min(c + 2, nf - 1), a0, d0);
            __builtin_amdgcn_sched_barrier(0);
            mul_chunk(0);                            // chunk c
            __builtin_amdgcn_sched_barrier(0);
            if (c + 1 >= nf) break;
            store_chunk(1, a1, d1);                  // chunk c + 1
            __syncthreads();
            load_full(min(c + 3, nf - 1), a1, d1);
            __builtin_amdgcn_sched_barrier(0);
            mul_chunk(1);                            // chunk c + 1
            __builtin_amdgcn_sched_barrier(0);
            if (c + 2 >= nf) break;
            store_chunk(0, a0, d0);                  // chunk c + 2
            __syncthreads();
        }
    }
    if (n % KC) {
        AR ra[CA];
        f4v rd[CD];
        load_part(nf, ra, rd);
        __syncthreads();                             // every wave is done with both buffers
        store_chunk(0, ra, rd);
        __syncthreads();
        mul_chunk(0);
    }
    __syncthreads();

    // ---- the waves' partial tiles, added by a fixed tree in the (now free) staging
    // buffers; lane (c, g) holds rows 4 g + v of each row block, agent c
    float* part = stage;
    const bool dl = r < P;
#pragma unroll
    for (int h = NW / 2; h >= 1; h >>= 1) {
        if (wave >= h && wave < 2 * h && dl) {
#pragma unroll
            for (int b = 0; b < RB; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) part[((wave - h) * ROWS + 16 * b + 4 * g + v) * P + r] = acc[b][v];
        }
        __syncthreads();
        if (wave < h && dl) {
#pragma unroll
            for (int b = 0; b < RB; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[b][v] += part[(wave * ROWS + 16 * b + 4 * g + v) * P + r];
        }
        __syncthreads();
    }
    if (wave == 0 && dl) {
#pragma unroll
        for (int b = 0; b < RB; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = 16 * b + 4 * g + v;
                adt[row * P + r] = (i0 + row < n) ? double(acc[b][v]) : 0.0;   // rows >= n hold copies
            }
    }
    __syncthreads();
    // AD rows to memory (FP32), each agent's ROWS rows contiguous
    for (int t = tid; t < ROWS * P; t += WG) {
        const int j = t / ROWS, row = t - (t / ROWS) * ROWS;
        if (i0 + row < n) static_cast<float*>(a.AD)[(int64_t)j * a.n_pad + i0 + row] = float(adt[row * P + j]);
    }
    if (a.product_only) return;
    ad_tail<PREC, P, ROWS, WG, true>(a, tile, ntiles, adt, s0, DRval{0.0, 0.0, false},
                                     *reinterpret_cast<Tail*>(stage));
}

// (the XCD-grouped order of xcd_tile for the 32-row shapes only: 1.7 % faster for FP32
// at n = 8192 and 4 % for BF16x2 at n = 32768; with 16 rows it was 7.8 % slower for
// BF16x2 at n = 8192)
template <int PREC, int P, int RB, int NW>
__global__ __launch_bounds__(64 * NW) void k_ad_mma32(AdArgs a) {
    ad_tile_mma32<PREC, P, RB, NW>(a, RB == 2 ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x, gridDim.x);
}

template <int PREC, int P, int RB, int NW>
__global__ __launch_bounds__(64 * NW) void k_ad_mma32_batch(const AdArgs* __restrict__ sys,
                                                             const int4* __restrict__ items) {
    const int4 it = items[blockIdx.x];
    const AdArgs a = sys[it.x];
    ad_tile_mma32<PREC, P, RB, NW>(a, it.y, (a.n + 16 * RB - 1) / (16 * RB));
}

// -------------------------------------------- cross-lane sums of FP64 values (gfx950)
//
// The same reduce-scatter as wave_fold, for doubles, with VALU lane exchanges only:
// offsets 32 and 16 with v_permlane32_swap / v_permlane16_swap (which swap the
// upper half of one register with the lower half of another, so a swap followed by
// one addition leaves each half with its own index summed over the pair), offsets 8,
// 4, 2 and 1 with DPP moves (row rotate by 8, half-row mirror, quad permutes).  Each
// round pairs every lane with one lane of the other half of its group, so after the
// rounds every lane holds the sum over all 64 lanes of the value it ends up with.

__device__ __forceinline__ void dsplit(double v, unsigned& lo, unsigned& hi) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    lo = (unsigned)u;
    hi = (unsigned)(u >> 32);
}
__device__ __forceinline__ double djoin(unsigned lo, unsigned hi) {
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
// x's upper 32 (O = 32) or odd 16-lane rows (O = 16) <-> y's lower / even ones
template <int O>
__device__ __forceinline__ void lane_swap(double& x, double& y) {
    unsigned xl, xh, yl, yh;
    dsplit(x, xl, xh);
    dsplit(y, yl, yh);
    if constexpr (O == 32) {
        const auto l = __builtin_amdgcn_permlane32_swap(xl, yl, false, false);
        const auto h = __builtin_amdgcn_permlane32_swap(xh, yh, false, false);
        x = djoin(l[0], h[0]);
        y = djoin(l[1], h[1]);
    } else {
        static_assert(O == 16, "swap offsets 32 and 16");
        const auto l = __builtin_amdgcn_permlane16_swap(xl, yl, false, false);
        const auto h = __builtin_amdgcn_permlane16_swap(xh, yh, false, false);
        x = djoin(l[0], h[0]);
        y = djoin(l[1], h[1]);
    }
}
// the value of the partner lane at offset O < 16 (8: l ^ 8; 4: the mirror lane in
// the same 8-lane half row, 7 - l % 8; 2 and 1: l ^ 2, l ^ 1)
template <int O>
__device__ __forceinline__ double lane_pair(double v) {
    constexpr int CTRL = O == 8 ? 0x128 : O == 4 ? 0x141 : O == 2 ? 0x4E : 0xB1;
    unsigned lo, hi;
    dsplit(v, lo, hi);
    lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)lo, CTRL, 0xf, 0xf, false);
    hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)hi, CTRL, 0xf, 0xf, false);
    return djoin(lo, hi);
}

template <int M, int O>
struct Fold64 {
    __device__ static __forceinline__ void run(double* v, int lane, int& idx) {
        if constexpr (O >= 1) {
            if constexpr (M > 1) {
                constexpr int h = M / 2;
                if constexpr (O >= 16) {
#pragma unroll
                    for (int q = 0; q < h; ++q) {
                        lane_swap<O>(v[q], v[q + h]);
                        v[q] = v[q] + v[q + h];
                    }
                } else {
                    const bool up = (lane & O) != 0;
#pragma unroll
                    for (int q = 0; q < h; ++q) {
                        const double send = up ? v[q] : v[q + h];
                        const double keep = up ? v[q + h] : v[q];
                        v[q] = keep + lane_pair<O>(send);
                    }
                }
                if (lane & O) idx += h;
                Fold64<h, O / 2>::run(v, lane, idx);
            } else {
                if constexpr (O >= 16) {
                    double x = v[0], y = v[0];
                    lane_swap<O>(x, y);
                    v[0] = x + y;
                } else {
                    v[0] += lane_pair<O>(v[0]);
                }
                Fold64<1, O / 2>::run(v, lane, idx);
            }
        }
    }
};

// Reduce-scatter of M = 2^q doubles per lane over the 64 lanes: returns the index
// (0..M-1) of the total this lane holds in v[0]; 64 / M lanes hold each total.
template <int M>
__device__ __forceinline__ int wave_fold64(double (&v)[M], int lane) {
    int idx = 0;
    Fold64<M, 32>::run(v, lane, idx);
    return idx;
}

// ================================ symmetric A.D: upper block triangle of A only
//
// k_sym streams the blocks A(I, J), I <= J, of 128 x 128, strip by strip (see
// SymArgs).  A workgroup of 4 waves runs one strip of block row I: lane l holds rows
// I*128 + 2l and 2l + 1 (one 16-byte load per column) and the matching D(I) rows in
// registers; wave w takes columns w*32 .. w*32 + 31 of each block, two at a time.
// For column j of block J it adds
//   A(I, J)[:, j] * D[j, :]     to the lane's rows of block I (registers, the whole strip),
//   A(I, J)[:, j]^T D(I)        as a sum over the 128 rows: a fixed xor butterfly over
//                               the lanes, stored as slot I of block J (I < J only).
// The D rows of the wave's 32 columns are staged in a wave-private LDS area, so the
// column stream has no workgroup barrier.  At the end of the strip the four waves'
// block-row sums are added in wave order and stored as slot I + s of block I.
// k_fin adds up each block's slots in slot order and then runs the products, the
// grid reduction and the step algebra of the A.D kernel (ad_tail).

// A(r0 .. r0 + 1, j) of an n x n column-major matrix, zero outside it.  `full`: the
// rows are inside the matrix (uniform over the workgroup).
__device__ __forceinline__ void sym_load(const double* __restrict__ A, int64_t lda, int n, int j, int r0,
                                         bool full, double (&v)[2]) {
    v[0] = 0.0;
    v[1] = 0.0;
    if (j >= n) return;
    const double* col = A + (int64_t)j * lda;
    if (full) {
        const d2v x = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(col + r0));
        v[0] = x.x;
        v[1] = x.y;
    } else {
        if (r0 < n) v[0] = col[r0];
        if (r0 + 1 < n) v[1] = col[r0 + 1];
    }
}

template <int P>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(2))) void k_sym(SymArgs a) {
    constexpr int COLS = kSymB / 4;                 // columns of a block per wave
    constexpr int G = 4;                            // columns per load group
    constexpr int GPB = COLS / G;                   // groups per block and wave
    constexpr int NV = 2 * P;                       // butterfly values per column pair
    constexpr int DPL = (COLS * P + 63) / 64;       // staged D values per lane
    static_assert(P <= kSymMaxP && NV <= 64, "symmetric pass: P <= 8");
    __shared__ double dj[4][COLS * P];              // D rows of each wave's columns
    __shared__ double yred[4][kSymB * P];           // the waves' block-row sums
    if (a.st->done != RUNNING) return;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int2 u = a.units[blockIdx.x];
    const int I = u.x, Js = u.y;
    const int Je = min(Js + kSymW, a.nb);
    const int n = a.n;
    const int64_t lda = a.lda;
    const int64_t np = a.n_pad;
    const int I0 = I * kSymB;
    const int r0 = I0 + 2 * lane;
    const bool full = I0 + kSymB <= n;
    const double* __restrict__ A = a.A;
    const double* __restrict__ V = a.V;

    double di[2][P], yi[2][P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const d2v x = *reinterpret_cast<const d2v*>(V + p * np + r0);
        di[0][p] = x.x;
        di[1][p] = x.y;
        yi[0][p] = 0.0;
        yi[1][p] = 0.0;
    }
    // D rows of this wave's columns of block J, staged value q at dj[wave][c*P + p]
    double dnx[DPL];
    auto dload = [&](int J) {
        const int c0 = J * kSymB + wave * COLS;
#pragma unroll
        for (int m = 0; m < DPL; ++m) {
            const int q = lane + 64 * m;
            const int p = q / COLS, c = q - (q / COLS) * COLS;
            dnx[m] = (q < COLS * P) ? V[p * np + c0 + c] : 0.0;
        }
    };
    // first column of load group g of the strip (4 groups per block and wave)
    auto gcol = [&](int g) { return (Js + g / GPB) * kSymB + wave * COLS + G * (g - (g / GPB) * GPB); };
    auto gload = [&](int g, double (&v)[G][2]) {
        const int j0 = gcol(g);
#pragma unroll
        for (int c = 0; c < G; ++c) sym_load(A, lda, n, j0 + c, r0, full, v[c]);
    };
    auto gwork = [&](int g, double (&v)[G][2]) {
        const int J = Js + g / GPB;
        const int cb = G * (g - (g / GPB) * GPB);           // first column of the group in the wave's 32
        if (cb == 0) {
            // every lane has finished reading the previous block's rows (program
            // order within the wave); stage this block's and fetch the next one's
#pragma unroll
            for (int m = 0; m < DPL; ++m) {
                const int q = lane + 64 * m;
                if (q < COLS * P) {
                    const int p = q / COLS, cc = q - (q / COLS) * COLS;
                    dj[wave][cc * P + p] = dnx[m];
                }
            }
            if (J + 1 < Je) dload(J + 1);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        }
        // rows of block I += A(I, J)[:, group] * D[group, :]
#pragma unroll
        for (int c = 0; c < G; ++c) {
            double dd[P];
#pragma unroll
            for (int p = 0; p < P; ++p) dd[p] = dj[wave][(cb + c) * P + p];
#pragma unroll
            for (int p = 0; p < P; ++p) {
                yi[0][p] = fma(v[c][0], dd[p], yi[0][p]);
                yi[1][p] = fma(v[c][1], dd[p], yi[1][p]);
            }
        }
        // rows of block J += A(I, J)[:, group]^T D(I), a column pair per butterfly
        if (J != I) {
            double* out = a.part + (((int64_t)J * a.tmax + I) * kSymB + wave * COLS + cb) * P;
#pragma unroll
            for (int c = 0; c < G; c += 2) {
                double t[NV];
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int p = 0; p < P; ++p) t[b * P + p] = fma(v[c + b][1], di[1][p], v[c + b][0] * di[0][p]);
                const int idx = wave_fold64<NV>(t, lane);
                if (lane % (64 / NV) == 0) out[c * P + idx] = t[0];
            }
        }
    };
    const int ng = (Je - Js) * GPB;
    double va[G][2], vb[G][2];
    dload(Js);
    gload(0, va);
    for (int g = 0; g < ng; g += 2) {
        if (g + 1 < ng) gload(g + 1, vb);
        gwork(g, va);
        if (g + 1 < ng) {
            if (g + 2 < ng) gload(g + 2, va);
            gwork(g + 1, vb);
        }
    }
    // the strip's sums for block row I: the four waves added in wave order
#pragma unroll
    for (int p = 0; p < P; ++p) {
        yred[wave][(2 * lane) * P + p] = yi[0][p];
        yred[wave][(2 * lane + 1) * P + p] = yi[1][p];
    }
    __syncthreads();
    double* outI = a.part + ((int64_t)I * a.tmax + I + (Js - I) / kSymW) * kSymB * P;
    for (int q = tid; q < kSymB * P; q += kWG) outI[q] = ((yred[0][q] + yred[1][q]) + yred[2][q]) + yred[3][q];
}

// AD rows of the symmetric pass from the partial slots, kFinRows rows per workgroup
// (kSymB % kFinRows == 0, so all rows of a workgroup lie in one block K), then the
// products, the reduction and the step algebra.  Slot t of an output is summed by
// thread phase t mod TPO in slot order; the phases are then added in phase order.
constexpr int kFinRows = 8;

template <int P>
__global__ __launch_bounds__(kWG) void k_fin(SymArgs sa, AdArgs a) {
    constexpr int NO = kFinRows * P;          // outputs of the workgroup
    constexpr int TPO = kWG / NO;             // threads per output
    constexpr int U = 16;                     // loads in flight per thread
    __shared__ double adt[kFinRows * P];
    __shared__ double sub[kWG];
    __shared__ TailLds<P, kFinRows, kWG> tl;
    // (k_sym does not read the state: this launch spends the direction flag)
    if (blockIdx.x == 0 && threadIdx.x == 0 && a.st->dir_pending) a.st->dir_pending = 0;
    if (a.st->done != RUNNING) return;
    const StepState0 s0 = read_state0(a.st);
    const int tid = threadIdx.x;
    const int o = tid % NO, ph = tid / NO;
    const int i0 = blockIdx.x * kFinRows;
    const DRval dr = load_dr<PREC_F64, P, kFinRows>(a, i0);
    const int K = i0 / kSymB;
    const int T = K + (sa.nb - K + kSymW - 1) / kSymW;
    const int64_t stride = (int64_t)kSymB * P;
    const double* src = sa.part + ((int64_t)K * sa.tmax * kSymB + (i0 - K * kSymB)) * P + o;
    double acc = 0.0;
    for (int t0 = ph; t0 < T; t0 += U * TPO) {
        double v[U];
#pragma unroll
        for (int q = 0; q < U; ++q) v[q] = (t0 + q * TPO < T) ? src[(t0 + q * TPO) * stride] : 0.0;
#pragma unroll
        for (int q = 0; q < U; ++q)
            if (t0 + q * TPO < T) acc += v[q];
    }
    sub[tid] = acc;
    __syncthreads();
    if (tid < NO) {
        double y = sub[tid];
        for (int q = 1; q < TPO; ++q) y += sub[tid + q * NO];
        const int r = tid / P, j = tid - (tid / P) * P;
        const int i = i0 + r;
        if (i < a.n) static_cast<double*>(a.AD)[(int64_t)j * a.n_pad + i] = y;
        adt[r * P + j] = (i < a.n) ? y : 0.0;
    }
    // ad_tail's first barrier orders these adt writes before their use
    ad_tail<PREC_F64, P, kFinRows, kWG>(a, blockIdx.x, gridDim.x, adt, s0, dr, tl);
}

// ============ k_upd: X += D alpha, R -= AD alpha, and the products of the new residual
//
// Thread (r, j) of a workgroup owns element (row0 + r, agent j) of a block of
// RB = 256 / P rows.  Each workgroup forms its rows' share of (AD)^T R_new (P x P)
// and of diag(R_new^T R_new) (P values), summed in row order; the last workgroup of
// each group of kGroup blocks adds up its group's shares in block order.  The
// direction launch adds up the group sums.
//
// From P = 16 both launches run on the FP64 matrix cores instead, 64 rows per
// workgroup (upd_tile_mma, dir_tile_mma; the FP32 vectors of the low-precision modes
// are converted on load and rounded on store, the arithmetic staying FP64 as in the
// vector tiles): with one element per thread the update's LDS traffic for the P-term
// row sums, not memory, set its time, and 64-row blocks make 16 (P = 32) or 4
// (P = 16) times fewer group shares of the P^2 + P products for the direction launch
// to add up.

// v_mfma_f64_16x16x4f64 operand layouts, lane l = 16 g + r (r = l % 16, g = l / 16):
// A (16 x 4): A(r, g); B (4 x 16): B(g, r); C (16 x 16): C(g + 4 v, r), v = 0..3.
//
// The update of one wave's 16 rows i0.. (agents in blocks of 16, cb):
//   X_new(i0 + g + 4v, 16 cb + r) = X(...) + sum_k D(i0 + r', k) alpha(k, 16 cb + r)
// as P / 4 products with A = D(i0 + r, 4 kk + g), B = alpha(4 kk + g, 16 cb + r)
// accumulated from zero and then added to X (and AD alpha taken from R), whose C-layout
// elements the lane loads.  The products of the new residual,
//   (AD)^T R_new (x, y) += sum over the 16 rows of AD(i, x) R_new(i, y),
// take the rows as the contraction index in 4 steps s: A = AD(i0 + 4s + g, 16 xb + r)
// (AD loaded a second time, in the C layout) and B = R_new(i0 + 4s + g, 16 yb + r),
// which is the update's output element v = s in place.
template <int PREC, int P>
__device__ __forceinline__ void upd_tile_mma(const UpdArgs& a, const int tile, const int ntiles) {
    static_assert(P % 16 == 0 && kUpdWideRows == 64 && kWG == 256, "4 waves of 16 rows, agent blocks of 16");
    constexpr int NB = P / 16;                  // agent blocks
    constexpr int KK = P / 4;                   // k-steps of the update
    constexpr int NE = P * P + P;               // (AD)^T R_new, then diag(R_new^T R_new)
    __shared__ double part[4][NE];              // the waves' shares
    __shared__ double nsh[4][4][P];             // norm partials [wave][g][agent]
    __shared__ double gsum[NE];
    __shared__ int ish[4];
    DevState* st = a.st;
    if (st->done != RUNNING) return;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int r = lane & 15, g = lane >> 4;
    if (tile == 0 && tid == 0) st->dir_pending = 1;
    const int64_t np = a.n_pad;
    const int64_t i0 = (int64_t)tile * kUpdWideRows + 16 * wave;
    using TV = typename PT<PREC>::TV;        // vectors in FP64, or FP32 (arithmetic in FP64)
    TV* X = static_cast<TV*>(a.X);
    TV* R = static_cast<TV*>(a.R);
    const TV* D = static_cast<const TV*>(a.D);
    const TV* AD = static_cast<const TV*>(a.AD);
    double da[KK], aa[KK], al[KK][NB];
    d4v xc[NB], rc[NB], ac[NB];
#pragma unroll
    for (int kk = 0; kk < KK; ++kk) {
        da[kk] = double(D[(4 * kk + g) * np + i0 + r]);
        aa[kk] = double(AD[(4 * kk + g) * np + i0 + r]);
    }
#pragma unroll
    for (int cb = 0; cb < NB; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t o = (16 * cb + r) * np + i0 + g + 4 * v;
            xc[cb][v] = double(X[o]);
            rc[cb][v] = double(R[o]);
            ac[cb][v] = double(AD[o]);
        }
#pragma unroll
    for (int kk = 0; kk < KK; ++kk)
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) al[kk][cb] = st->alpha[(4 * kk + g) * kMaxP + 16 * cb + r];
    // D alpha and AD alpha summed from zero, then added to X and R with one rounding
    // each: accumulating the partial products onto X itself would round at the scale
    // of X (far larger than its update late in a solve) once per k-step
    d4v sx[NB], sr[NB];
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
        sx[cb] = d4v{0.0, 0.0, 0.0, 0.0};
        sr[cb] = d4v{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < KK; ++kk) {
            sx[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(da[kk], al[kk][cb], sx[cb], 0, 0, 0);
            sr[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(aa[kk], al[kk][cb], sr[cb], 0, 0, 0);
        }
    }
#pragma unroll
    for (int cb = 0; cb < NB; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t o = (16 * cb + r) * np + i0 + g + 4 * v;
            const TV xn = TV(xc[cb][v] + sx[cb][v]);
            const TV rn = TV(rc[cb][v] - sr[cb][v]);
            X[o] = xn;
            R[o] = rn;
            rc[cb][v] = double(rn);              // the products take R_new as stored
        }
    d4v pg[NB][NB];
#pragma unroll
    for (int xb = 0; xb < NB; ++xb)
#pragma unroll
        for (int yb = 0; yb < NB; ++yb) pg[xb][yb] = d4v{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int xb = 0; xb < NB; ++xb)
#pragma unroll
            for (int yb = 0; yb < NB; ++yb)
                pg[xb][yb] = __builtin_amdgcn_mfma_f64_16x16x4f64(ac[xb][s], rc[yb][s], pg[xb][yb], 0, 0, 0);
#pragma unroll
    for (int xb = 0; xb < NB; ++xb)
#pragma unroll
        for (int yb = 0; yb < NB; ++yb)
#pragma unroll
            for (int v = 0; v < 4; ++v) part[wave][(16 * xb + g + 4 * v) * P + 16 * yb + r] = pg[xb][yb][v];
#pragma unroll
    for (int yb = 0; yb < NB; ++yb) {
        double q = 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) q = fma(rc[yb][v], rc[yb][v], q);
        nsh[wave][g][16 * yb + r] = q;
    }
    __syncthreads();
    // the workgroup's share: waves in order (the norms: each wave's rows g + 4v by g)
    double* mine = &part[0][0];
    for (int e = tid; e < NE; e += kWG) {
        double t;
        if (e < P * P) {
            t = part[0][e] + part[1][e] + part[2][e] + part[3][e];
        } else {
            const int y = e - P * P;
            t = 0.0;
#pragma unroll
            for (int w = 0; w < 4; ++w)
#pragma unroll
                for (int gg = 0; gg < 4; ++gg) t += nsh[w][gg][y];
        }
        mine[e] = t;          // (entry e of wave 0's share: read above by this thread only)
    }
    __syncthreads();
    // (a group's 16 rows for the thread's NE / kWG entries: one round of loads)
    (void)group_reduce<upd_group(P), kWG, upd_group(P), (NE + kWG - 1) / kWG>(mine, NE, a.red, gsum, &ish[0], nullptr,
                                                                            tile, ntiles);
}

template <int PREC, int P>
__device__ __forceinline__ void upd_tile(const UpdArgs& a, const int tile, const int ntiles) {
    if constexpr (upd_mma(P)) {
        upd_tile_mma<PREC, P>(a, tile, ntiles);
        return;
    } else {
    using TV = typename PT<PREC>::TV;
    constexpr int RB = kWG / P;
    // Row stride of the row blocks in LDS: P + 1, so that the RB rows read together in
    // the update (one address per row, all lanes of a row alike) fall in distinct banks;
    // with stride P they share one bank and every such read is an RB-way conflict.
    constexpr int PS = P + 1;
    constexpr int NE = P * P + P;       // (AD)^T R_new, then diag(R_new^T R_new)
    __shared__ double al[P * P];
    __shared__ double dt[RB * PS], adt[RB * PS], rt[RB * PS];
    __shared__ double mine[NE], gsum[NE];
    __shared__ double gscr[kWG];
    __shared__ int ish[4];
    DevState* st = a.st;
    if (st->done != RUNNING) return;
    const int tid = threadIdx.x;
    const int r = tid % RB, j = tid / RB;
    const int64_t i = (int64_t)tile * RB + r;
    const int64_t o = (int64_t)j * a.n_pad + i;
    if (tile == 0 && tid == 0) st->dir_pending = 1;
    for (int t = tid; t < P * P; t += kWG) al[t] = st->alpha[(t / P) * kMaxP + (t % P)];
    TV* X = static_cast<TV*>(a.X);
    TV* R = static_cast<TV*>(a.R);
    const double x0 = X[o];
    const double r0 = R[o];
    dt[r * PS + j] = static_cast<const TV*>(a.D)[o];
    adt[r * PS + j] = static_cast<const TV*>(a.AD)[o];
    __syncthreads();
    double sx = 0.0, sr = 0.0;
#pragma unroll
    for (int l = 0; l < P; ++l) {
        sx = fma(dt[r * PS + l], al[l * P + j], sx);
        sr = fma(adt[r * PS + l], al[l * P + j], sr);
    }
    const TV xn = TV(x0 + sx);
    const TV rn = TV(r0 - sr);
    X[o] = xn;
    R[o] = rn;
    rt[r * PS + j] = double(rn);
    __syncthreads();
    for (int e = tid; e < NE; e += kWG) {
        double s = 0.0;
        if (e < P * P) {
            const int x = e / P, y = e - (e / P) * P;
            for (int q = 0; q < RB; ++q) s = fma(adt[q * PS + x], rt[q * PS + y], s);
        } else {
            const int y = e - P * P;
            for (int q = 0; q < RB; ++q) s = fma(rt[q * PS + y], rt[q * PS + y], s);
        }
        mine[e] = s;
    }
    __syncthreads();
    (void)group_reduce<(P >= 8 ? kGroup : 16), kWG>(mine, NE, a.red, gsum, &ish[0], gscr, tile, ntiles);
    }
}

template <int PREC, int P>
__global__ __launch_bounds__(kWG) void k_upd(UpdArgs a) {
    upd_tile<PREC, P>(a, blockIdx.x, gridDim.x);
}

// ====================== k_dir: stop test, beta = -G^{-1} (AD)^T R_new, D = R_new + D beta
//
// Runs when the update launch of this block step ran (dir_pending).  Every
// workgroup adds up the update's group sums in group order, and so holds the
// same totals, bit for bit; from them it solves beta (Alg. 2, with the factor of G
// that the A.D launch kept) and updates the D rows of its block (masked to the
// active agents).  Workgroup 0 also ends the step in the state: the stop test on the
// new residual norms (Alg. 4: smallest agent residual relative to ||b||), beta,
// and the step count.
// The step's report and the stop rule at the top of the next step (Alg. 4: smallest
// agent residual relative to ||b||), by wave 0 of the direction launch's workgroup 0:
// the norms from the totals tot (P x P products, then the P squared norms), beta
// (be: row-major, stride P) to the state, the step count and the stop decision.
// lred: 64 doubles of LDS.
template <int P>
__device__ __forceinline__ void dir_report(DevState* st, const double* tot, const double* be, double* lred,
                                           const unsigned mask, const int lane) {
    double q = INFINITY, bad = 0.0;
    if (lane < P && ((mask >> lane) & 1u)) {
        const double nr = sqrt(tot[P * P + lane]);
        st->norms[lane] = nr;
        if (!isfinite(nr)) bad = 1.0;
        q = nr / st->nb;
    }
    if (lane < P) {
        lred[lane] = q;
        lred[32 + lane] = bad;
#pragma unroll
        for (int x = 0; x < P; ++x) st->beta[x * kMaxP + lane] = be[x * P + lane];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    if (lane == 0) {
        double mn = INFINITY, anybad = 0.0;
#pragma unroll
        for (int jj = 0; jj < P; ++jj) {
            mn = fmin(mn, lred[jj]);
            anybad += lred[32 + jj];
        }
        const int it = st->iter + 1;
        st->minres = mn;
        st->iter = it;
        if (anybad > 0.0) fail_state(st, -2);
        else if (mn <= st->tol) st->done = RECUR_CONV;
        else if (it >= st->maxit) st->done = MAXIT;
    }
}

// Totals of the update's products: its ngrp group sums (rows of NE values in l2) added
// in group order, for the entries tid + h * kWG of this thread, GB groups' loads in
// flight together.
template <int NE, int GB>
__device__ __forceinline__ void sum_groups(const double* l2, const int ngrp, double (&tv)[(NE + kWG - 1) / kWG]) {
    constexpr int NH = (NE + kWG - 1) / kWG;
    const int tid = threadIdx.x;
#pragma unroll
    for (int h = 0; h < NH; ++h) tv[h] = 0.0;
    for (int g0 = 0; g0 < ngrp; g0 += GB) {
        double v[NH][GB];
#pragma unroll
        for (int t = 0; t < GB; ++t)
#pragma unroll
            for (int h = 0; h < NH; ++h) {
                const int e = tid + h * kWG;
                v[h][t] = (g0 + t < ngrp && e < NE) ? l2[(int64_t)(g0 + t) * NE + e] : 0.0;
            }
#pragma unroll
        for (int h = 0; h < NH; ++h)
#pragma unroll
            for (int t = 0; t < GB; ++t)
                if (g0 + t < ngrp) tv[h] += v[h][t];
    }
}

// P = 16 and 32: the direction update on the FP64 matrix cores, 64 rows per workgroup, a
// wave 16 of them: D_new = R_new + D beta as P / 4 products with A = D(i0 + r, 4 kk + g)
// and B = beta(4 kk + g, 16 cb + r) accumulated from zero and added to R_new (layouts as
// in upd_tile_mma).  Every workgroup adds up the group sums and solves beta itself.
template <int PREC, int P>
__device__ __forceinline__ void dir_tile_mma(const UpdArgs& a, const int blk, const int ngrp) {
    static_assert(P % 16 == 0 && kUpdWideRows == 64 && kWG == 256 && (P * P) % kWG == 0, "tile shape");
    constexpr int NB = P / 16, KK = P / 4;
    constexpr int NE = P * P + P;
    constexpr int NH = (NE + kWG - 1) / kWG;
    constexpr int NL = P * P / kWG;
    __shared__ double tot[NE];
    __shared__ double be[P * P];
    __shared__ double Lsh[P * P], rinv[P];
    __shared__ double lred[64];
    DevState* st = a.st;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int r = lane & 15, g = lane >> 4;
    const int64_t np = a.n_pad;
    const int64_t i0 = (int64_t)blk * kUpdWideRows + 16 * wave;
    // (loads only before the flag is tested: nothing is written unless it is set)
    const int pending = st->dir_pending;
    const unsigned mask = st->mask;
    using TV = typename PT<PREC>::TV;        // vectors in FP64, or FP32 (arithmetic in FP64)
    TV* D = static_cast<TV*>(a.D);
    const TV* R = static_cast<const TV*>(a.R);
    double da[KK], lv[NL], tv[NH];
    d4v dc[NB];
#pragma unroll
    for (int kk = 0; kk < KK; ++kk) da[kk] = double(D[(4 * kk + g) * np + i0 + r]);
#pragma unroll
    for (int cb = 0; cb < NB; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) dc[cb][v] = double(R[(16 * cb + r) * np + i0 + g + 4 * v]);
#pragma unroll
    for (int h = 0; h < NL; ++h) {
        const int t = tid + h * kWG;
        lv[h] = st->L[(t / P) * kMaxP + (t % P)];
    }
    sum_groups<NE, 16>(a.red.l2, ngrp, tv);
    if (!pending) return;
#pragma unroll
    for (int h = 0; h < NL; ++h) Lsh[tid + h * kWG] = lv[h];
#pragma unroll
    for (int h = 0; h < NH; ++h)
        if (tid + h * kWG < NE) tot[tid + h * kWG] = tv[h];
    __syncthreads();
    if (tid < P) rinv[tid] = 1.0 / Lsh[tid * P + tid];
    __syncthreads();
    if (wave == 0 && lane < P) {
        // lane c: beta[:, c] = -G^{-1} ((AD)^T R_new)[:, c]
        const int c = lane;
        const bool ac = (mask >> c) & 1u;
        double w[P];
#pragma unroll
        for (int x = 0; x < P; ++x) w[x] = (ac && ((mask >> x) & 1u)) ? -tot[x * P + c] : 0.0;
        col_chol_solve<P>(Lsh, rinv, w);
#pragma unroll
        for (int x = 0; x < P; ++x) be[x * P + c] = w[x];
    }
    __syncthreads();
    // D beta summed from zero, then added to R_new with one rounding
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
        d4v sd = d4v{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < KK; ++kk)
            sd = __builtin_amdgcn_mfma_f64_16x16x4f64(da[kk], be[(4 * kk + g) * P + 16 * cb + r], sd, 0, 0, 0);
        const bool on = (mask >> (16 * cb + r)) & 1u;
#pragma unroll
        for (int v = 0; v < 4; ++v) D[(16 * cb + r) * np + i0 + g + 4 * v] = on ? TV(dc[cb][v] + sd[v]) : TV(0);
    }
    if (blk != 0 || wave != 0) return;
    dir_report<P>(st, tot, be, lred, mask, lane);
}

template <int PREC, int P>
__device__ __forceinline__ void dir_tile(const UpdArgs& a, const int blk, const int ngrp) {
    if constexpr (upd_mma(P)) {
        dir_tile_mma<PREC, P>(a, blk, ngrp);
        return;
    } else {
    using TV = typename PT<PREC>::TV;
    constexpr int RB = kWG / P;
    constexpr int PS = P + 1;           // LDS row stride (see upd_tile)
    constexpr int NE = P * P + P;
    constexpr int NH = (NE + kWG - 1) / kWG;
    __shared__ double tot[NE];
    __shared__ double be[P * P];
    __shared__ double Lsh[P * P], rinv[P];
    __shared__ double lred[64];
    __shared__ double dt[RB * PS];
    DevState* st = a.st;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int r = tid % RB, j = tid / RB;
    const int64_t i = (int64_t)blk * RB + r;
    const int64_t o = (int64_t)j * a.n_pad + i;
    // (loads only before the flag is tested: nothing is written unless it is set)
    const int pending = st->dir_pending;
    const unsigned mask = st->mask;
    TV* D = static_cast<TV*>(a.D);
    const double rv = double(static_cast<const TV*>(a.R)[o]);
    const double dv = double(D[o]);
    const double lv = tid < P * P ? st->L[(tid / P) * kMaxP + (tid % P)] : 0.0;
    // totals of the update's products (kGroup loads in flight per thread)
    double tv[NH];
    sum_groups<NE, kGroup / NH>(a.red.l2, ngrp, tv);
    if (!pending) return;
    dt[r * PS + j] = dv;
    if (tid < P * P) Lsh[tid] = lv;
#pragma unroll
    for (int h = 0; h < NH; ++h)
        if (tid + h * kWG < NE) tot[tid + h * kWG] = tv[h];
    __syncthreads();
    if (tid < P) rinv[tid] = 1.0 / Lsh[tid * P + tid];
    __syncthreads();
    if (wave == 0 && lane < P) {
        // lane c: beta[:, c] = -G^{-1} ((AD)^T R_new)[:, c]
        const int c = lane;
        const bool ac = (mask >> c) & 1u;
        double w[P];
#pragma unroll
        for (int x = 0; x < P; ++x) w[x] = (ac && ((mask >> x) & 1u)) ? -tot[x * P + c] : 0.0;
        col_chol_solve<P>(Lsh, rinv, w);
#pragma unroll
        for (int x = 0; x < P; ++x) be[x * P + c] = w[x];
    }
    __syncthreads();
    double sd = rv;
#pragma unroll
    for (int l = 0; l < P; ++l) sd = fma(dt[r * PS + l], be[l * P + j], sd);
    D[o] = ((mask >> j) & 1u) ? TV(sd) : TV(0);
    if (blk != 0 || wave != 0) return;
    dir_report<P>(st, tot, be, lred, mask, lane);
    }
}

template <int PREC, int P>
__global__ __launch_bounds__(kWG) void k_dir(UpdArgs a) {
    dir_tile<PREC, P>(a, blockIdx.x, (upd_blocks(a.n_pad, P) + upd_group(P) - 1) / upd_group(P));
}

template <int PREC, int P>
__global__ __launch_bounds__(kWG) void k_upd_batch(const UpdArgs* __restrict__ sys, const int4* __restrict__ items) {
    const int4 it = items[blockIdx.x];
    const UpdArgs a = sys[it.x];
    upd_tile<PREC, P>(a, it.y, upd_blocks(a.n_pad, P));
}

template <int PREC, int P>
__global__ __launch_bounds__(kWG) void k_dir_batch(const UpdArgs* __restrict__ sys, const int4* __restrict__ items) {
    const int4 it = items[blockIdx.x];
    const UpdArgs a = sys[it.x];
    dir_tile<PREC, P>(a, it.y, (upd_blocks(a.n_pad, P) + upd_group(P) - 1) / upd_group(P));
}

// ============================================ k_res: T = B - Y, norms, restart

template <int P>
__device__ __forceinline__ void res_tile(const ResArgs& a, const int tile, const int ntiles) {
    constexpr int RB = kWG / P;
    constexpr int NE = P * P + 1;      // T^T T entries, then b^T b
    __shared__ double ts[RB * P];
    __shared__ double bs[RB];
    __shared__ double mine[NE];
    __shared__ double tot[NE];
    __shared__ double gscr[kWG];
    __shared__ int ish[8];
    DevState* st = a.st;
    const int tid = threadIdx.x;
    const int r = tid % RB, j = tid / RB;
    const int64_t i = (int64_t)tile * RB + r;
    const int64_t o = (int64_t)j * a.n_pad + i;
    const unsigned msk = st->mask;
    const double bi = a.b[i];
    if (j == 0) bs[r] = bi;
    const double t = (j < a.p && i < a.n) ? bi - a.Y[o] : 0.0;
    ts[r * P + j] = t;
    if (a.mode != RES_FINAL) a.R[o] = t;
    if (a.mode == RES_INIT || a.mode == RES_CONFIRM) a.D[o] = ((msk >> j) & 1u) ? t : 0.0;
    __syncthreads();
    for (int e = tid; e < NE; e += kWG) {
        double s = 0.0;
        if (e < P * P) {
            const int x = e / P, y = e - (e / P) * P;
            for (int q = 0; q < RB; ++q) s = fma(ts[q * P + x], ts[q * P + y], s);
        } else {
            for (int q = 0; q < RB; ++q) s = fma(bs[q], bs[q], s);
        }
        mine[e] = s;
    }
    __syncthreads();
    if (!grid_reduce<(P >= 8 ? kGroup : 16), kWG>(mine, NE, a.red, tot, &ish[0], gscr, tile, ntiles)) return;
    if (tid == 0) {
        if (a.set_nb) st->nb = sqrt(tot[P * P]);
        double mn = INFINITY;
        bool bad = !isfinite(st->nb);
        for (int jj = 0; jj < a.p; ++jj) {
            const double nr = sqrt(tot[jj * P + jj]);
            st->norms[jj] = nr;
            if (!isfinite(nr)) bad = true;
            if ((msk >> jj) & 1u) mn = fmin(mn, nr / st->nb);
        }
        st->minres = mn;
        if (a.mode != RES_FINAL) {
            if (bad) fail_state(st, -2);
            else if (st->nb == 0.0) fail_state(st, -1);
            else if (mn <= st->tol) st->done = FINISHED;
            else if (a.mode == RES_REFINE) st->done = OUTER;
            else {
                if (a.mode == RES_CONFIRM) st->restarts += 1;
                st->done = (st->iter >= st->maxit) ? MAXIT : RUNNING;
            }
        }
    }
}

template <int P>
__global__ __launch_bounds__(kWG) void k_res(ResArgs a) {
    res_tile<P>(a, blockIdx.x, gridDim.x);
}

// Batched residual: items[w] = (system, tile, mode, set_nb); the mode of each
// system's pass travels with its items.
template <int P>
__global__ __launch_bounds__(kWG) void k_res_batch(const ResArgs* __restrict__ sys, const int4* __restrict__ items) {
    const int4 it = items[blockIdx.x];
    ResArgs a = sys[it.x];
    a.mode = it.z;
    a.set_nb = it.w;
    res_tile<P>(a, it.y, a.n_pad / (kWG / P));
}


// ================================================================ A.D launchers
//
// Tile configuration: CW A columns per wave and NW waves per workgroup (from the
// tuning table, or given); wave steps per staged chunk so that a chunk stages at
// least one value per thread, at most 512 rows; 4 waves per SIMD, non-temporal A
// loads and staggered chunk starts.
template <int PREC, int P, int CW, int NW>
using AdCfgOf = AdCfg<CW,
                      (P * 64 * PT<PREC>::E >= 64 * NW ? 1
                       : (64 * NW / (P * 64 * PT<PREC>::E) > 512 / (64 * PT<PREC>::E)
                              ? 512 / (64 * PT<PREC>::E)
                              : 64 * NW / (P * 64 * PT<PREC>::E))),
                      4, true, true, NW>;

template <int PREC, int P, int CW, int NW>
inline hipError_t launch_ad_t(const AdArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    using C = AdCfgOf<PREC, P, CW, NW>;
    const dim3 grid((a.n + C::ROWS - 1) / C::ROWS);
    // With an event pair the launch records them itself (the kernel's own begin
    // and end), with no separate marker packets around it.
    if (e0) {
        hipExtLaunchKernelGGL((k_ad<PREC, P, C>), grid, dim3(C::WG), 0, s, e0, e1, 0, a);
    } else {
        hipLaunchKernelGGL((k_ad<PREC, P, C>), grid, dim3(C::WG), 0, s, a);
    }
    return hipGetLastError();
}

template <int PREC, int P, int CW, int NW>
inline hipError_t launch_ad_batch_t(const AdArgs* sys, const int4* items, int nitems, hipStream_t s) {
    using C = AdCfgOf<PREC, P, CW, NW>;
    hipLaunchKernelGGL((k_ad_batch<PREC, P, C>), dim3(nitems), dim3(C::WG), 0, s, sys, items);
    return hipGetLastError();
}

// Tile shapes (A columns per wave cw, waves per workgroup nw; a workgroup owns
// cw * nw rows of AD) as the launchers run a request.
//
// Vector tiles: 4 columns per wave only where the accumulators stay small (FP64 up
// to P = 4, FP32 / BF16 up to P = 8), P = 16 at most 2; 8 or 16 waves (one staged D
// chunk shared by more columns, so fewer re-reads of D) only up to P = 8, where a
// thread's registers still fit a quarter of a SIMD's file.
//
// FP64 at P = 16 and P = 8 also has the matrix-core tile (ad_tile_mfma), with 16
// or 32 rows per workgroup (cw * nw) and nw waves splitting the contraction: at
// P = 16 every shape with cw * nw >= 16, (4, 4), (2, 8), (4, 8), (1, 16), (2, 16);
// at P = 8 the shapes with 4 columns per wave, which the vector tile does not run
// there, (4, 4) and (4, 8).  FP32 and BF16x2 at P = 16 have the same shapes on the
// FP32-operand matrix-core tile (ad_tile_mma32).
__host__ __device__ constexpr bool ad_cw4_fits(int prec, int P) {
    return P < 16 && (prec != PREC_F64 || P <= 4);
}
__host__ __device__ constexpr bool ad_has_mfma(int prec, int P) {
    return (prec == PREC_F64 && (P == 32 || P == 16 || P == 8)) ||
           ((prec == PREC_F32 || prec == PREC_BF16X2) && P == 16);
}
__host__ __device__ constexpr int ad_nw_fit(int prec, int P, int nw) {
    return (P >= 16 && !ad_has_mfma(prec, P)) ? 4 : (nw >= 16 ? 16 : (nw >= 8 ? 8 : 4));
}
__host__ __device__ constexpr int ad_cw_fit(int prec, int P, int cw, int nw) {
    if (ad_has_mfma(prec, P) && P == 8) {       // 4 columns per wave: the matrix-core tile
        const int w = ad_nw_fit(prec, P, nw);
        return (cw >= 4 && w <= 8) ? 4 : (cw >= 2 ? 2 : 1);
    }
    if (ad_has_mfma(prec, P)) {
        const int w = ad_nw_fit(prec, P, nw);
        if (w == 4 && P == 32) return 4;                      // matrix cores only
        if (w == 4) return cw >= 4 ? 4 : (cw >= 2 ? 2 : 1);   // 4: matrix cores; 1, 2: vector
        if (w == 8) return cw >= 4 ? 4 : 2;
        return cw >= 2 ? 2 : 1;
    }
    return cw >= 4 ? (ad_cw4_fits(prec, P) ? 4 : 2) : (cw >= 2 ? 2 : 1);
}

// FP64: k_ad_mfma (FP64 operands); FP32 and BF16x2: k_ad_mma32 (FP32 operands)
template <int PREC, int P, int RB, int NW>
inline hipError_t launch_ad_mfma_t(const AdArgs* one, const AdArgs* sys, const int4* items, int nitems,
                                   hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    const dim3 grid = one ? dim3((one->n + 16 * RB - 1) / (16 * RB)) : dim3(nitems);
    if constexpr (PREC == PREC_F64) {
        if (!one) hipLaunchKernelGGL((k_ad_mfma_batch<P, RB, NW>), grid, dim3(64 * NW), 0, s, sys, items);
        else if (e0) hipExtLaunchKernelGGL((k_ad_mfma<P, RB, NW>), grid, dim3(64 * NW), 0, s, e0, e1, 0, *one);
        else hipLaunchKernelGGL((k_ad_mfma<P, RB, NW>), grid, dim3(64 * NW), 0, s, *one);
    } else {
        if (!one) hipLaunchKernelGGL((k_ad_mma32_batch<PREC, P, RB, NW>), grid, dim3(64 * NW), 0, s, sys, items);
        else if (e0) hipExtLaunchKernelGGL((k_ad_mma32<PREC, P, RB, NW>), grid, dim3(64 * NW), 0, s, e0, e1, 0, *one);
        else hipLaunchKernelGGL((k_ad_mma32<PREC, P, RB, NW>), grid, dim3(64 * NW), 0, s, *one);
    }
    return hipGetLastError();
}

// rows: 16 or 32 per workgroup; nw: 4, 8 or 16 waves (fitted shapes only)
template <int PREC, int P>
inline hipError_t launch_ad_mfma(int rows, int nw, const AdArgs* one, const AdArgs* sys, const int4* items,
                                 int nitems, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (rows == 16 && nw == 4) return launch_ad_mfma_t<PREC, P, 1, 4>(one, sys, items, nitems, s, e0, e1);
    if (rows == 16 && nw == 8) return launch_ad_mfma_t<PREC, P, 1, 8>(one, sys, items, nitems, s, e0, e1);
    if (rows == 32 && nw == 8) return launch_ad_mfma_t<PREC, P, 2, 8>(one, sys, items, nitems, s, e0, e1);
    if (rows == 16 && nw == 16) return launch_ad_mfma_t<PREC, P, 1, 16>(one, sys, items, nitems, s, e0, e1);
    if (rows == 32 && nw == 16) return launch_ad_mfma_t<PREC, P, 2, 16>(one, sys, items, nitems, s, e0, e1);
    return hipErrorInvalidValue;
}

template <int PREC, int P, int CW>
inline hipError_t launch_ad_w(int nw, const AdArgs* one, const AdArgs* sys, const int4* items, int nitems,
                              hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if constexpr (P < 16) {
        if (nw >= 16)
            return one ? launch_ad_t<PREC, P, CW, 16>(*one, s, e0, e1)
                       : launch_ad_batch_t<PREC, P, CW, 16>(sys, items, nitems, s);
        if (nw >= 8)
            return one ? launch_ad_t<PREC, P, CW, 8>(*one, s, e0, e1)
                       : launch_ad_batch_t<PREC, P, CW, 8>(sys, items, nitems, s);
    }
    return one ? launch_ad_t<PREC, P, CW, 4>(*one, s, e0, e1) : launch_ad_batch_t<PREC, P, CW, 4>(sys, items, nitems, s);
}

template <int PREC, int P>
inline hipError_t launch_ad_pc(int cw, int nw, const AdArgs* one, const AdArgs* sys, const int4* items,
                               int nitems, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if constexpr (P == 32) {                  // FP64 matrix cores only
        if constexpr (!ad_has_mfma(PREC, P)) {
            return hipErrorInvalidValue;
        } else {
            const int w = ad_nw_fit(PREC, P, nw), c = ad_cw_fit(PREC, P, cw, nw);
            return launch_ad_mfma<PREC, P>(c * w, w, one, sys, items, nitems, s, e0, e1);
        }
    }
    if constexpr (ad_has_mfma(PREC, P)) {
        const int w = ad_nw_fit(PREC, P, nw), c = ad_cw_fit(PREC, P, cw, nw);
        if (P == 16 ? c * w >= 16 : c == 4) return launch_ad_mfma<PREC, P>(c * w, w, one, sys, items, nitems, s, e0, e1);
    }
    constexpr int W4 = ad_cw4_fits(PREC, P) ? 4 : 2;
    if (cw >= 4) return launch_ad_w<PREC, P, W4>(nw, one, sys, items, nitems, s, e0, e1);
    if (cw >= 2) return launch_ad_w<PREC, P, 2>(nw, one, sys, items, nitems, s, e0, e1);
    return launch_ad_w<PREC, P, 1>(nw, one, sys, items, nitems, s, e0, e1);
}

// One system (one != nullptr) or a batch of (system, tile) items.
template <int PREC>
inline hipError_t launch_ad_prec(int P, int cw, int nw, const AdArgs* one, const AdArgs* sys, const int4* items,
                                 int nitems, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    switch (P) {
        case 1: return launch_ad_pc<PREC, 1>(cw, nw, one, sys, items, nitems, s, e0, e1);
        case 2: return launch_ad_pc<PREC, 2>(cw, nw, one, sys, items, nitems, s, e0, e1);
        case 4: return launch_ad_pc<PREC, 4>(cw, nw, one, sys, items, nitems, s, e0, e1);
        case 8: return launch_ad_pc<PREC, 8>(cw, nw, one, sys, items, nitems, s, e0, e1);
        case 16: return launch_ad_pc<PREC, 16>(cw, nw, one, sys, items, nitems, s, e0, e1);
        case 32:
            if constexpr (PREC == PREC_F64) return launch_ad_pc<PREC, 32>(cw, nw, one, sys, items, nitems, s, e0, e1);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

// Entry points of the per-precision translation units.
hipError_t launch_ad_f64(int P, int cw, int nw, const AdArgs* one, const AdArgs* sys, const int4* items,
                         int nitems, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
// Symmetric A.D pass of one FP64 system: k_sym over `nunits` strips, then k_fin.
// With an event pair, e0 is recorded at the start of k_sym and e1 at the end of k_fin.
template <int P>
inline hipError_t launch_sym_t(const SymArgs& sa, const AdArgs& a, int nunits, hipStream_t s, hipEvent_t e0,
                               hipEvent_t e1) {
    const dim3 gs(nunits), gf((a.n + kFinRows - 1) / kFinRows);
    if (e0) {
        hipExtLaunchKernelGGL((k_sym<P>), gs, dim3(kWG), 0, s, e0, nullptr, 0, sa);
    } else {
        hipLaunchKernelGGL((k_sym<P>), gs, dim3(kWG), 0, s, sa);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (e1) {
        hipExtLaunchKernelGGL((k_fin<P>), gf, dim3(kWG), 0, s, nullptr, e1, 0, sa, a);
    } else {
        hipLaunchKernelGGL((k_fin<P>), gf, dim3(kWG), 0, s, sa, a);
    }
    return hipGetLastError();
}
hipError_t launch_sym_f64(int P, const SymArgs& sa, const AdArgs& a, int nunits, hipStream_t s, hipEvent_t e0,
                          hipEvent_t e1);
hipError_t launch_ad_f32(int P, int cw, int nw, const AdArgs* one, const AdArgs* sys, const int4* items,
                         int nitems, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
hipError_t launch_ad_bf16(int P, int cw, int nw, const AdArgs* one, const AdArgs* sys, const int4* items,
                          int nitems, hipStream_t s, hipEvent_t e0, hipEvent_t e1);

}  // namespace ccg

namespace ccg {

// ================= small-system tier: one workgroup runs whole block steps of a system
//
// For n <= kSmallN (= the padded size 512) and P <= kSmallMaxP, a block step of a
// system is latency-bound across workgroups: a grid reduction and three launches
// cost more than streaming A (at most 2 MB in FP64).  Here one workgroup of 512
// threads does the whole step, with D, AD and R staged in LDS, and loops over up to
// `steps` steps per launch; every per-system quantity is summed in a fixed order, so
// a system's result does not depend on the launch it shares or the round lengths.
// Every solve of such a size (single, batched, served) runs this tier.

// out[e] = sum over rows k < nr of f(e, k, .) for e < NE (nr: n rounded up to 64;
// the rows from n on are zero): each entry's rows in RT slices of consecutive rows
// (an FMA chain within a slice), then the slices in order.  part: kSmallWG doubles of
// LDS.
template <int NE, class F>
__device__ __forceinline__ void small_rows_sum(F f, const int nr, double* part, double* out) {
    constexpr int RT = kSmallWG / NE >= 32 ? 32 : (kSmallWG / NE >= 16 ? 16 : (kSmallWG / NE >= 8 ? 8
                       : (kSmallWG / NE >= 4 ? 4 : (kSmallWG / NE >= 2 ? 2 : 1))));
    const int sl = nr / RT;
    const int tid = threadIdx.x;
    for (int t = tid; t < NE * RT; t += kSmallWG) {
        const int e = t / RT, q = t - (t / RT) * RT;
        double s = 0.0;
#pragma unroll 4
        for (int k = q * sl; k < (q + 1) * sl; ++k) s = f(e, k, s);
        part[t] = s;
    }
    __syncthreads();
    for (int e = tid; e < NE; e += kSmallWG) {
        double s = part[e * RT];
        for (int q = 1; q < RT; ++q) s += part[e * RT + q];
        out[e] = s;
    }
    __syncthreads();
}

// A workgroup runs up to `steps` block steps of its system with no memory round trip
// on the step's critical path other than the stream of A: X, D, AD and R stay in LDS
// for the whole launch (written back when it ends), the step
// state lives in LDS (the device state is written for the host as the steps go), and
// each wave loads the A columns of its next pass before it multiplies the current
// ones.  Work runs over the rows below n only (rounded up to 64 for the products).
template <int PREC, int P>
__device__ __forceinline__ void small_steps(const SmallArgs& a, const int steps) {
    using TA = typename PT<PREC>::TA;
    using TV = typename PT<PREC>::TV;
    using TACC = typename PT<PREC>::TACC;
    constexpr int E = PT<PREC>::E;
    constexpr int CW = PREC == PREC_F64 ? 2 : 4;     // A columns per wave pass
    constexpr int N = kSmallN;
    constexpr int NT = kSmallWG;
    constexpr int NWV = NT / 64;
    constexpr int TRI = P * (P + 1) / 2;
    constexpr int NE1 = TRI + P * P;                 // G (lower triangle), S
    constexpr int NE2 = P * P + P;                   // (AD)^T R_new, diag(R_new^T R_new)
    constexpr int NV = CW * P;
    constexpr int PER = P * N / NT;                  // block elements per thread
    constexpr int KI = N / (64 * E);                 // contraction steps of a pass
    static_assert(P <= kSmallMaxP && NV <= 64 && PER * NT == P * N, "tier shape");
    __shared__ TV dsh[P * N], adsh[P * N], rsh[P * N], xsh[P * N];   // agent-major: [j * N + k]
    __shared__ double part[NT];
    __shared__ double g1[NE1], g2[NE2];
    __shared__ double sm[3 * P * P + P];
    __shared__ double gscr[NT];
    __shared__ int ish[256];
    __shared__ double al[P * P], be[P * P];
    __shared__ double lred[64];
    __shared__ StepState0 ss;
    __shared__ int ctl;
    DevState* st = a.st;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int n = a.n;
    TV* X = static_cast<TV*>(a.X);
    TV* R = static_cast<TV*>(a.R);
    TV* D = static_cast<TV*>(a.D);
    const int64_t lda = a.lda;
    const int nr = (n + 63) & ~63;
    const double* Lf = sm + P * P;                // step_alpha's factor of G, stride P
    const double* rinv = sm + 2 * P * P;
    if (tid == 0) {
        ss = read_state0(st);
        ctl = st->done == RUNNING ? 1 : 0;
    }
    // the blocks are agent-major with N rows, so LDS and global share the index
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int idx = tid + q * NT;
        dsh[idx] = D[idx];
        rsh[idx] = R[idx];
        adsh[idx] = TV(0);
        xsh[idx] = X[idx];
    }
    __syncthreads();

    // one pass of a wave: A columns i0 .. i0 + CW - 1 (AD rows; columns >= n are a copy
    // of column n - 1, never stored), the KI contraction steps of the whole column
    auto load_pass = [&](int i0, TACC (&av)[KI][CW][E]) {
#pragma unroll
        for (int c = 0; c < CW; ++c) {
            const int i = min(i0 + c, n - 1);
            const TA* hi = static_cast<const TA*>(a.A) + (int64_t)i * lda;
            const TA* lo = PREC == PREC_BF16X2 ? static_cast<const TA*>(a.A_lo) + (int64_t)i * lda : hi;
#pragma unroll
            for (int it = 0; it < KI; ++it) {
                const int k0 = it * 64 * E + lane * E;
                if (k0 + E <= n) {
                    Loader<PREC, false>::load(hi + k0, lo + k0, av[it][c]);
                } else {
#pragma unroll
                    for (int e = 0; e < E; ++e)
                        av[it][c][e] = (k0 + e < n) ? Loader<PREC, false>::load1(hi + k0 + e, lo + k0 + e) : TACC(0);
                }
            }
        }
    };
    auto mul_pass = [&](int i0, const TACC (&av)[KI][CW][E]) {
        TACC acc[CW][P];
#pragma unroll
        for (int c = 0; c < CW; ++c)
#pragma unroll
            for (int j = 0; j < P; ++j) acc[c][j] = TACC(0);
#pragma unroll
        for (int it = 0; it < KI; ++it) {
            const int k0 = it * 64 * E + lane * E;
#pragma unroll
            for (int j = 0; j < P; ++j) {
                TACC d[E];
#pragma unroll
                for (int e = 0; e < E; ++e) d[e] = TACC(dsh[j * N + k0 + e]);
#pragma unroll
                for (int c = 0; c < CW; ++c)
#pragma unroll
                    for (int e = 0; e < E; ++e) acc[c][j] = fma(av[it][c][e], d[e], acc[c][j]);
            }
            __builtin_amdgcn_sched_barrier(0);   // one contraction step's D values live at a time
        }
        TACC v[NV];
#pragma unroll
        for (int c = 0; c < CW; ++c)
#pragma unroll
            for (int j = 0; j < P; ++j) v[c * P + j] = acc[c][j];
        const int idx = wave_fold<NV>(v, lane);
        constexpr int REP = 64 / NV;
        if (lane % REP == 0) {
            const int c = idx / P, j = idx - (idx / P) * P;
            const int i = i0 + c;
            if (i < n) adsh[j * N + i] = TV(v[0]);
        }
    };

    for (int s = 0; s < steps; ++s) {
        if (!ctl) break;
        const StepState0 s0 = ss;
        // ---- AD = A D: wave w takes A columns (= AD rows, A symmetric) w*CW, w*CW +
        //      NWV*CW, ...; its lanes split the contraction index; one xor fold per pass
        {
            TACC b0[KI][CW][E], b1[KI][CW][E];
            int i0 = wave * CW;
            if (i0 < n) load_pass(i0, b0);
            while (i0 < n) {
                const int i1 = i0 + NWV * CW;
                if (i1 < n) load_pass(i1, b1);
                mul_pass(i0, b0);
                if (i1 >= n) break;
                const int i2 = i1 + NWV * CW;
                if (i2 < n) load_pass(i2, b0);
                mul_pass(i1, b1);
                i0 = i2;
            }
        }
        __syncthreads();
        // ---- G = D^T AD (lower triangle) and S = D^T R, then the rank step and alpha
        small_rows_sum<NE1>(
            [&](int e, int k, double acc) {
                if (e < TRI) {
                    int x = 0;
                    while ((x + 1) * (x + 2) / 2 <= e) ++x;
                    const int y = e - x * (x + 1) / 2;
                    return fma(double(dsh[x * N + k]), double(adsh[y * N + k]), acc);
                }
                const int t = e - TRI, x = t / P, y = t - (t / P) * P;
                return fma(double(dsh[x * N + k]), double(rsh[y * N + k]), acc);
            },
            nr, part, g1);
        if (tid == 0) st->ad_streams += 1;
        if (s0.iter >= s0.maxit) {                    // (the stop rule ends the steps first)
            if (tid == 0) st->done = MAXIT;
            break;
        }
        const bool go = step_alpha<P, NT>(g1, s0, st, sm, gscr, ish, al);
        __syncthreads();
        if (!go) break;
        const unsigned mask = (unsigned)ish[202];
        // ---- X += D alpha, R_new = R - AD alpha (rows < n)
#pragma unroll 1
        for (int q = 0; q < PER; ++q) {
            const int idx = tid + q * NT;
            const int j = idx / N, k = idx - (idx / N) * N;
            if (k < n) {
                double sx = 0.0, sr = 0.0;
#pragma unroll
                for (int l = 0; l < P; ++l) {
                    sx = fma(double(dsh[l * N + k]), al[l * P + j], sx);
                    sr = fma(double(adsh[l * N + k]), al[l * P + j], sr);
                }
                xsh[idx] = TV(double(xsh[idx]) + sx);
                rsh[idx] = TV(double(rsh[idx]) - sr);
            }
        }
        __syncthreads();
        // ---- (AD)^T R_new and the new residual norms; beta and the stop rule
        small_rows_sum<NE2>(
            [&](int e, int k, double acc) {
                if (e < P * P) {
                    const int x = e / P, y = e - (e / P) * P;
                    return fma(double(adsh[x * N + k]), double(rsh[y * N + k]), acc);
                }
                const int y = e - P * P;
                return fma(double(rsh[y * N + k]), double(rsh[y * N + k]), acc);
            },
            nr, part, g2);
        if (wave == 0) {
            if (lane < P) {
                const int c = lane;
                const bool ac = (mask >> c) & 1u;
                double w[P];
#pragma unroll
                for (int x = 0; x < P; ++x) w[x] = (ac && ((mask >> x) & 1u)) ? -g2[x * P + c] : 0.0;
                col_chol_solve<P>(Lf, rinv, w);
#pragma unroll
                for (int x = 0; x < P; ++x) {
                    be[x * P + c] = w[x];
                    st->beta[x * kMaxP + c] = w[x];
                }
            }
            double qv = INFINITY, bad = 0.0;
            if (lane < P && ((mask >> lane) & 1u)) {
                const double nrm = sqrt(g2[P * P + lane]);
                st->norms[lane] = nrm;
                if (!isfinite(nrm)) bad = 1.0;
                qv = nrm / s0.nb;
            }
            if (lane < P) {
                lred[lane] = qv;
                lred[32 + lane] = bad;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            if (lane == 0) {
                double mn = INFINITY, anybad = 0.0;
#pragma unroll
                for (int jj = 0; jj < P; ++jj) {
                    mn = fmin(mn, lred[jj]);
                    anybad += lred[32 + jj];
                }
                const int it = s0.iter + 1;
                st->minres = mn;
                st->iter = it;
                int stop = 1;
                if (anybad > 0.0) fail_state(st, -2);
                else if (mn <= s0.tol) st->done = RECUR_CONV;
                else if (it >= s0.maxit) st->done = MAXIT;
                else stop = 0;
                // the next step's state: one more step, the active set after the rank step
                ss.iter = it;
                ss.mask = mask;
                ss.m = __popc(mask);
                ctl = !stop;
            }
        }
        __syncthreads();
        // ---- D = R_new + D beta (masked to the active agents), built in adsh (AD is
        //      spent; its rows >= n stay zero, as R's and D's do)
#pragma unroll 1
        for (int q = 0; q < PER; ++q) {
            const int idx = tid + q * NT;
            const int j = idx / N, k = idx - (idx / N) * N;
            if (k < n) {
                double sd = double(rsh[idx]);
#pragma unroll
                for (int l = 0; l < P; ++l) sd = fma(double(dsh[l * N + k]), be[l * P + j], sd);
                adsh[idx] = ((mask >> j) & 1u) ? TV(sd) : TV(0);
            }
        }
        __syncthreads();
#pragma unroll 1
        for (int q = 0; q < PER; ++q) {
            const int idx = tid + q * NT;
            const int k = idx - (idx / N) * N;
            if (k < n) {
                dsh[idx] = adsh[idx];
                adsh[idx] = TV(0);
            }
        }
        __syncthreads();
    }
    // ---- the blocks back to memory
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int idx = tid + q * NT;
        X[idx] = xsh[idx];
        R[idx] = rsh[idx];
        D[idx] = dsh[idx];
    }
}

template <int PREC, int P>
__global__ __launch_bounds__(kSmallWG) void k_small(SmallArgs a, int steps) {
    small_steps<PREC, P>(a, steps);
}

// Many systems: workgroup w runs system items[w].x.
template <int PREC, int P>
__global__ __launch_bounds__(kSmallWG) void k_small_batch(const SmallArgs* __restrict__ sys,
                                                          const int4* __restrict__ items, int steps) {
    const SmallArgs a = sys[items[blockIdx.x].x];
    small_steps<PREC, P>(a, steps);
}

hipError_t launch_small_f64(int P, const SmallArgs* one, const SmallArgs* sys, const int4* items, int nitems,
                            int steps, hipStream_t s);
hipError_t launch_small_f32(int P, const SmallArgs* one, const SmallArgs* sys, const int4* items, int nitems,
                            int steps, hipStream_t s);
hipError_t launch_small_bf16(int P, const SmallArgs* one, const SmallArgs* sys, const int4* items, int nitems,
                             int steps, hipStream_t s);

template <int PREC>
inline hipError_t launch_small_prec(int P, const SmallArgs* one, const SmallArgs* sys, const int4* items,
                                    int nitems, int steps, hipStream_t s) {
#define CCG_SMALL(PP)                                                                                       \
    if (one) {                                                                                              \
        hipLaunchKernelGGL((k_small<PREC, PP>), dim3(1), dim3(kSmallWG), 0, s, *one, steps);                \
    } else {                                                                                                \
        hipLaunchKernelGGL((k_small_batch<PREC, PP>), dim3(nitems), dim3(kSmallWG), 0, s, sys, items, steps); \
    }                                                                                                       \
    return hipGetLastError();
    switch (P) {
        case 1: { CCG_SMALL(1) }
        case 2: { CCG_SMALL(2) }
        case 4: { CCG_SMALL(4) }
        case 8: { CCG_SMALL(8) }
        default: return hipErrorInvalidValue;
    }
#undef CCG_SMALL
}

}  // namespace ccg
