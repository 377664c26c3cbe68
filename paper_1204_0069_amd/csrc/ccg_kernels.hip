// HIP kernels (gfx950) for the block step of cooperative conjugate gradient.
//
// One block step (Alg. 2 of the paper, sign convention R = B - A X, residual by
// the Table 1 recurrence) is three launches:
//
//   k_ad   : AD = A D, streamed once over A.  A is column-major, so column k of A
//            times row k of D is an outer-product update of a tile of AD rows;
//            the D row is wave-uniform and arrives by scalar loads.  Partial tiles
//            per column split are summed in a fixed order by the last workgroup of
//            each row tile, which also forms that tile's share of G = D^T A D.  The
//            last tile sums the Gram shares (fixed order), runs the rank test of
//            Alg. 3 and solves G alpha = S (Cholesky, FP64).
//   k_upd  : X += D alpha, R -= AD alpha, and the reductions (AD)^T R, R^T R and
//            D^T R; the last workgroup solves G beta = -(AD)^T R with the cached
//            factor, forms the next S = D_new^T R = R^T R + beta^T (D^T R), the
//            residual norms and the stop test.
//   k_dir  : D = R + D beta (masked to the active agents).
//
// Every reduction is a fixed-order tree over fixed-size tiles, so results depend
// only on (n, p, precision, tile shape), never on timing.
#include "ccg_device.h"

#include <math.h>

namespace ccg {

// ----------------------------------------------------------------- precision traits

template <int PREC> struct PT;
template <> struct PT<PREC_F64> {
    using TA = double;   // stored A element
    using TV = double;   // vector element (X, R, D, AD)
    using TACC = double; // accumulator of A.D
    static constexpr int E = 2;   // elements per 16-byte load
    static constexpr int V = 2;   // 16-byte loads per lane per column
};
template <> struct PT<PREC_F32> {
    using TA = float;
    using TV = float;
    using TACC = float;
    static constexpr int E = 4;
    static constexpr int V = 1;
};
template <> struct PT<PREC_BF16X2> {
    using TA = uint16_t;
    using TV = float;
    using TACC = float;
    static constexpr int E = 8;
    static constexpr int V = 1;
};

template <int PREC> constexpr int tile_rows() { return 64 * PT<PREC>::E * PT<PREC>::V; }

// Columns per unrolled step: keep the uniform D rows of one step within ~64 SGPRs.
template <int PREC, int P> constexpr int unroll() {
    return (sizeof(typename PT<PREC>::TV) * P * 4 <= 256) ? 4 : 2;
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
    return __uint_as_float(((uint32_t)h) << 16);
}

// Load the E elements of one 16-byte chunk of column data, converted to TACC.
// hi points into the FP64 / FP32 matrix or the BF16 "hi" plane, lo into the BF16
// "lo" plane (same offsets).
template <int PREC> struct Loader;

template <> struct Loader<PREC_F64> {
    __device__ __forceinline__ static void load(const double* hi, const double*, double (&out)[2]) {
        const double2 v = *reinterpret_cast<const double2*>(hi);
        out[0] = v.x;
        out[1] = v.y;
    }
    __device__ __forceinline__ static double load1(const double* hi, const double*) { return *hi; }
};
template <> struct Loader<PREC_F32> {
    __device__ __forceinline__ static void load(const float* hi, const float*, float (&out)[4]) {
        const float4 v = *reinterpret_cast<const float4*>(hi);
        out[0] = v.x; out[1] = v.y; out[2] = v.z; out[3] = v.w;
    }
    __device__ __forceinline__ static float load1(const float* hi, const float*) { return *hi; }
};
template <> struct Loader<PREC_BF16X2> {
    __device__ __forceinline__ static void load(const uint16_t* hi, const uint16_t* lo, float (&out)[8]) {
        const uint4 h = *reinterpret_cast<const uint4*>(hi);
        const uint4 l = *reinterpret_cast<const uint4*>(lo);
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

// ----------------------------------------------------------- last-workgroup tickets

// Returns true in every thread of the workgroup that arrives last at *counter
// (expected arrivals: total).  Publishes this workgroup's global writes before the
// ticket and makes every other workgroup's writes visible after it.
__device__ __forceinline__ bool last_arrival(unsigned* counter, unsigned total, int* s_flag) {
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned t = atomicAdd(counter, 1u);
        *s_flag = (t == total - 1) ? 1 : 0;
    }
    __syncthreads();
    const bool last = *s_flag != 0;
    if (last) __threadfence();
    return last;
}

// ------------------------------------------------------------ small p x p algebra
//
// Executed by all threads of one workgroup on LDS arrays (m <= 16), with barriers
// between dependent phases.  Compact m x m matrices are row-major with stride m.

// Greedy pivoted Cholesky of the diagonally scaled G (unit diagonal).  Writes the
// taken compact indices, ascending, to keep[]; returns their count, or -1 when a
// diagonal entry is negative, -2 on a non-finite entry.  Columns with G_ii == 0 are
// never taken.  Same rule as the oracle's rank step.
__device__ int wg_rank_select(const double* G, int m, double tau, int* keep, double* H,
                              int* sh) {
    const int tid = threadIdx.x;
    // sh[0]: status, sh[1]: ncand, sh[2]: ntaken, sh[3]: pivot (or -1 to stop)
    // sh[8..8+m): candidate list, sh[32..32+m): taken list
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
    if (tid < m * m) {
        const int i = tid / m, j = tid % m;
        const double si = sqrt(G[i * m + i]), sj = sqrt(G[j * m + j]);
        H[tid] = (si > 0.0 && sj > 0.0) ? G[tid] / (si * sj) : 0.0;
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
                    sh[32 + sh[2]] = cand;
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
        double upd = 0.0;
        int ia = -1, ic = -1;
        if (tid < nc * nc) {
            ia = sh[8 + tid / nc];
            ic = sh[8 + tid % nc];
            const double lc = H[ic * m + piv] / r;
            const double la = H[ia * m + piv] / r;
            upd = H[ic * m + ia] - lc * la;
        }
        __syncthreads();
        if (ia >= 0) H[ic * m + ia] = upd;
        __syncthreads();
    }
    if (tid == 0) {
        const int nt = sh[2];
        for (int a = 0; a < nt; ++a)
            for (int c = a + 1; c < nt; ++c)
                if (sh[32 + c] < sh[32 + a]) { const int t = sh[32 + a]; sh[32 + a] = sh[32 + c]; sh[32 + c] = t; }
        for (int a = 0; a < nt; ++a) keep[a] = sh[32 + a];
    }
    __syncthreads();
    return sh[2];
}

// Cholesky G = L L^T (m x m compact, natural order).  Returns 0, or -1 when a pivot
// is not positive.
__device__ int wg_cholesky(const double* G, int m, double* L, int* sh) {
    const int tid = threadIdx.x;
    if (tid < m * m) L[tid] = 0.0;
    __syncthreads();
    for (int j = 0; j < m; ++j) {
        if (tid == 0) {
            double d = G[j * m + j];
            for (int k = 0; k < j; ++k) d -= L[j * m + k] * L[j * m + k];
            if (d > 0.0) { L[j * m + j] = sqrt(d); sh[0] = 0; }
            else sh[0] = -1;
        }
        __syncthreads();
        if (sh[0] != 0) return -1;
        const int i = j + 1 + tid;
        if (i < m) {
            double s = G[i * m + j];
            for (int k = 0; k < j; ++k) s -= L[i * m + k] * L[j * m + k];
            L[i * m + j] = s / L[j * m + j];
        }
        __syncthreads();
    }
    return 0;
}

// Z = (L L^T)^{-1} B for q right-hand-side columns (B, Z m x q row-major, stride q).
// One thread per column.
__device__ void wg_chol_solve(const double* L, int m, int q, const double* B, double* Z) {
    const int c = threadIdx.x;
    if (c < q) {
        for (int i = 0; i < m; ++i) {
            double s = B[i * q + c];
            for (int k = 0; k < i; ++k) s -= L[i * m + k] * Z[k * q + c];
            Z[i * q + c] = s / L[i * m + i];
        }
        for (int i = m - 1; i >= 0; --i) {
            double s = Z[i * q + c];
            for (int k = i + 1; k < m; ++k) s -= L[k * m + i] * Z[k * q + c];
            Z[i * q + c] = s / L[i * m + i];
        }
    }
    __syncthreads();
}

__device__ __forceinline__ void fail_state(DevState* st, int code) {
    st->done = FAILED;
    st->status = code;
}

// ============================================================== k_ad: AD = A D
//
// Workgroup (it, ks) covers rows [it*TM, it*TM+TM) and columns [ks*kc, ks*kc+kc);
// its four waves take contiguous quarters of the column range and are summed in
// wave order through LDS.  Lane l owns rows it*TM + v*64*E + l*E + e.

template <int PREC, int P, bool TAIL>
__device__ __forceinline__ void ad_stream(const AdArgs& a, int it, int ks,
                                          typename PT<PREC>::TACC (&acc)[PT<PREC>::V][PT<PREC>::E][P]) {
    using TA = typename PT<PREC>::TA;
    using TV = typename PT<PREC>::TV;
    using TACC = typename PT<PREC>::TACC;
    constexpr int E = PT<PREC>::E;
    constexpr int V = PT<PREC>::V;
    constexpr int TM = tile_rows<PREC>();
    constexpr int U = unroll<PREC, P>();
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int kb0 = ks * a.kc;
    const int ke0 = min(a.n, kb0 + a.kc);
    const int per = (ke0 - kb0 + 3) >> 2;
    const int kb = kb0 + wave * per;
    const int ke = min(ke0, kb + per);
    const int64_t lda = a.lda;
    // wave-uniform column pointers (tile base) and D row pointer
    const TA* chi = static_cast<const TA*>(a.A) + (int64_t)kb * lda + (int64_t)it * TM;
    const TA* clo = (PREC == PREC_BF16X2)
                        ? static_cast<const TA*>(a.A_lo) + (int64_t)kb * lda + (int64_t)it * TM
                        : chi;
    const TV* dp = static_cast<const TV*>(a.V) + (int64_t)kb * P;
    const int loff = lane * E;      // per-lane element offset inside a column tile

#pragma unroll
    for (int v = 0; v < V; ++v)
#pragma unroll
        for (int e = 0; e < E; ++e)
#pragma unroll
            for (int j = 0; j < P; ++j) acc[v][e][j] = TACC(0);

    int k = kb;
    if (!TAIL) {
        for (; k + U <= ke; k += U) {
            TACC av[U][V][E];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int v = 0; v < V; ++v)
                    Loader<PREC>::load(chi + u * lda + loff + v * 64 * E, clo + u * lda + loff + v * 64 * E,
                                       av[u][v]);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                TACC d[P];
#pragma unroll
                for (int j = 0; j < P; ++j) d[j] = TACC(dp[u * P + j]);
#pragma unroll
                for (int v = 0; v < V; ++v)
#pragma unroll
                    for (int e = 0; e < E; ++e)
#pragma unroll
                        for (int j = 0; j < P; ++j) acc[v][e][j] = fma(av[u][v][e], d[j], acc[v][e][j]);
            }
            chi += U * lda;
            clo += U * lda;
            dp += U * P;
        }
    }
    const int row_lane = it * TM + loff;
    for (; k < ke; ++k) {
        TACC av[V][E];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            if (!TAIL) {
                Loader<PREC>::load(chi + loff + v * 64 * E, clo + loff + v * 64 * E, av[v]);
            } else {
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int off = loff + v * 64 * E + e;
                    av[v][e] = (row_lane + v * 64 * E + e < a.n) ? Loader<PREC>::load1(chi + off, clo + off)
                                                                 : TACC(0);
                }
            }
        }
        TACC d[P];
#pragma unroll
        for (int j = 0; j < P; ++j) d[j] = TACC(dp[j]);
#pragma unroll
        for (int v = 0; v < V; ++v)
#pragma unroll
            for (int e = 0; e < E; ++e)
#pragma unroll
                for (int j = 0; j < P; ++j) acc[v][e][j] = fma(av[v][e], d[j], acc[v][e][j]);
        chi += lda;
        clo += lda;
        dp += P;
    }
}

template <int PREC, int P>
__global__ __launch_bounds__(kWG) void k_ad(AdArgs a) {
    using TV = typename PT<PREC>::TV;
    using TACC = typename PT<PREC>::TACC;
    constexpr int E = PT<PREC>::E;
    constexpr int V = PT<PREC>::V;
    constexpr int TM = tile_rows<PREC>();
    __shared__ TACC red[TM * P];           // wave sums; then the reduced AD tile
    __shared__ TV dtile[TM * P];           // D rows of the tile (Gram epilogue)
    __shared__ double gsh[kWG];            // Gram sub-sums / final Gram
    __shared__ double sm[5 * kMaxP * kMaxP];
    __shared__ int ish[128];

    if (!a.product_only && a.st->done != RUNNING) return;
    const int it = blockIdx.x / a.nks;
    const int ks = blockIdx.x - it * a.nks;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;

    TACC acc[V][E][P];
    const bool tail = (it + 1) * TM > a.n;
    if (tail) ad_stream<PREC, P, true>(a, it, ks, acc);
    else ad_stream<PREC, P, false>(a, it, ks, acc);

    // ---- fixed-order sum of the four waves: ((w0 + w1) + w2) + w3
    for (int w = 1; w < 4; ++w) {
        if (wave == w) {
#pragma unroll
            for (int v = 0; v < V; ++v)
#pragma unroll
                for (int e = 0; e < E; ++e)
#pragma unroll
                    for (int j = 0; j < P; ++j) red[(v * 64 * E + lane * E + e) * P + j] = acc[v][e][j];
        }
        __syncthreads();
        if (wave == 0) {
#pragma unroll
            for (int v = 0; v < V; ++v)
#pragma unroll
                for (int e = 0; e < E; ++e)
#pragma unroll
                    for (int j = 0; j < P; ++j) acc[v][e][j] += red[(v * 64 * E + lane * E + e) * P + j];
        }
        __syncthreads();
    }
    // ---- partial tile for this column split
    TACC* part = static_cast<TACC*>(a.part) + ((int64_t)ks * a.n_pad + (int64_t)it * TM) * P;
    if (wave == 0) {
#pragma unroll
        for (int v = 0; v < V; ++v)
#pragma unroll
            for (int e = 0; e < E; ++e)
#pragma unroll
                for (int j = 0; j < P; ++j) part[(v * 64 * E + lane * E + e) * P + j] = acc[v][e][j];
    }
    if (!last_arrival(&a.cnt_tile[it], (unsigned)a.nks, &ish[0])) return;
    if (tid == 0) a.cnt_tile[it] = 0u;

    // ---- last workgroup of the tile: AD tile = sum over splits in split order
    {
        const TACC* p0 = static_cast<const TACC*>(a.part) + (int64_t)it * TM * P;
        TV* ad = static_cast<TV*>(a.AD) + (int64_t)it * TM * P;
        const TV* dv = static_cast<const TV*>(a.V) + (int64_t)it * TM * P;
        for (int idx = tid; idx < TM * P; idx += kWG) {
            TACC s = p0[idx];
            for (int q = 1; q < a.nks; ++q) s += p0[(int64_t)q * a.n_pad * P + idx];
            ad[idx] = TV(s);
            red[idx] = TACC(TV(s));
            dtile[idx] = dv[idx];
        }
    }
    if (a.product_only) return;
    __syncthreads();

    // ---- Gram share of this tile: G_t[x][y] = sum_r D[r][x] * AD[r][y]
    {
        constexpr int NE = P * P;
        constexpr int TPE = (kWG / NE) > 0 ? (kWG / NE) : 1;   // threads per entry
        const int e = tid / TPE, sub = tid - (tid / TPE) * TPE;
        double s = 0.0;
        if (e < NE) {
            const int x = e / P, y = e - (e / P) * P;
            for (int r = sub; r < TM; r += TPE)
                s = fma((double)dtile[r * P + x], (double)red[r * P + y], s);
        }
        gsh[tid] = s;
        __syncthreads();
        if (sub == 0 && e < NE) {
            double t = gsh[tid];
            for (int q = 1; q < TPE; ++q) t += gsh[tid + q];
            a.gpart[(int64_t)it * NE + e] = t;
        }
    }
    if (!last_arrival(&a.st->cnt_all, (unsigned)a.ntiles, &ish[0])) return;

    // ---- last tile: G = sum of shares (tile order), rank step, alpha = G^{-1} S
    DevState* st = a.st;
    if (tid == 0) st->cnt_all = 0u;
    double* Gf = gsh;                       // P x P full Gram
    if (tid < P * P) {
        double t = a.gpart[tid];
        for (int q = 1; q < a.ntiles; ++q) t += a.gpart[(int64_t)q * P * P + tid];
        Gf[tid] = t;
    }
    __syncthreads();
    int* act = &ish[64];    // active agents (global indices), ascending
    int m = st->m;
    if (tid < m) act[tid] = st->keep[tid];
    __syncthreads();
    double* Gc = sm;                         // compact m x m
    double* H = sm + kMaxP * kMaxP;
    double* Lc = sm + 2 * kMaxP * kMaxP;
    double* Sc = sm + 3 * kMaxP * kMaxP;
    double* Zc = sm + 4 * kMaxP * kMaxP;
    if (tid < m * m) {
        const int i = tid / m, j = tid - (tid / m) * m;
        // G is symmetric in exact arithmetic; use the lower triangle of the sum
        const int gi = max(act[i], act[j]), gj = min(act[i], act[j]);
        Gc[tid] = Gf[gi * P + gj];
    }
    __syncthreads();
    int* kp = &ish[96];
    const int r = wg_rank_select(Gc, m, st->tau, kp, H, &ish[0]);
    if (r < 0) {
        if (tid == 0) fail_state(st, r == -2 ? -2 : -3);
        return;
    }
    if (r < m) {
        // deflation: restrict to the kept agents (compact indices kp[0..r))
        double g2 = 0.0;
        int na = 0;
        if (tid < r * r) g2 = Gc[kp[tid / r] * m + kp[tid - (tid / r) * r]];
        if (tid < r) na = act[kp[tid]];
        __syncthreads();
        if (tid < r * r) Gc[tid] = g2;
        if (tid < r) act[tid] = na;
        __syncthreads();
        if (tid == 0) {
            unsigned mask = 0u;
            for (int q = 0; q < r; ++q) mask |= 1u << act[q];
            st->mask = mask;
            st->m = r;
            st->deflations += 1;
            for (int q = 0; q < r; ++q) st->keep[q] = act[q];
        }
        m = r;
        if (m == 0) {
            if (tid == 0) { st->done = FINISHED; }
            return;
        }
    }
    if (wg_cholesky(Gc, m, Lc, &ish[0]) != 0) {
        if (tid == 0) fail_state(st, -3);
        return;
    }
    if (tid < m * m) {
        const int i = tid / m, j = tid - (tid / m) * m;
        Sc[tid] = st->S[act[i] * kMaxP + act[j]];
    }
    __syncthreads();
    wg_chol_solve(Lc, m, m, Sc, Zc);
    // publish alpha (full, zeros off the active block) and the factor
    if (tid < kMaxP * kMaxP) st->alpha[tid] = 0.0;
    __syncthreads();
    if (tid < m * m) {
        const int i = tid / m, j = tid - (tid / m) * m;
        st->alpha[act[i] * kMaxP + act[j]] = Zc[tid];
        st->Lc[tid] = Lc[tid];
    }
}

// ============================================ k_upd: X += D alpha, R -= AD alpha

template <int PREC, int P>
__global__ __launch_bounds__(kWG) void k_upd(UpdArgs a) {
    using TV = typename PT<PREC>::TV;
    constexpr int RB = (P <= 8) ? kWG : kWG / 2;      // rows per workgroup
    __shared__ double al[P * P];
    __shared__ double rs[RB * P], ads[RB * P], ds[RB * P];
    __shared__ double sm[5 * kMaxP * kMaxP];
    __shared__ int ish[128];
    DevState* st = a.st;
    if (st->done != RUNNING) return;
    const int tid = threadIdx.x;
    if (tid < P * P) al[tid] = st->alpha[(tid / P) * kMaxP + (tid % P)];
    __syncthreads();

    TV* X = static_cast<TV*>(a.X);
    TV* R = static_cast<TV*>(a.R);
    const TV* D = static_cast<const TV*>(a.D);
    const TV* AD = static_cast<const TV*>(a.AD);
    const int64_t row0 = (int64_t)blockIdx.x * RB;
    if (tid < RB) {
        const int64_t i = row0 + tid;
        double x[P], rr[P], d[P], ad[P];
#pragma unroll
        for (int j = 0; j < P; ++j) {
            x[j] = X[i * P + j];
            rr[j] = R[i * P + j];
            d[j] = D[i * P + j];
            ad[j] = AD[i * P + j];
        }
#pragma unroll
        for (int j = 0; j < P; ++j) {
            double sx = 0.0, sr = 0.0;
#pragma unroll
            for (int l = 0; l < P; ++l) {
                sx = fma(d[l], al[l * P + j], sx);
                sr = fma(ad[l], al[l * P + j], sr);
            }
            x[j] += sx;
            rr[j] -= sr;
        }
#pragma unroll
        for (int j = 0; j < P; ++j) {
            X[i * P + j] = TV(x[j]);
            R[i * P + j] = TV(rr[j]);
            rs[tid * P + j] = double(TV(rr[j]));
            ads[tid * P + j] = ad[j];
            ds[tid * P + j] = d[j];
        }
    }
    __syncthreads();
    // partial sums over this workgroup's rows: W = AD^T R, Q = R^T R, F = D^T R
    constexpr int NE = 3 * P * P;
    for (int e = tid; e < NE; e += kWG) {
        const int which = e / (P * P);
        const int xy = e - which * P * P;
        const int x = xy / P, y = xy - (xy / P) * P;
        const double* U = which == 0 ? ads : (which == 1 ? rs : ds);
        double s = 0.0;
        for (int r = 0; r < RB; ++r) s = fma(U[r * P + x], rs[r * P + y], s);
        a.upart[(int64_t)blockIdx.x * NE + e] = s;
    }
    if (!last_arrival(&st->cnt_upd, (unsigned)a.nblk, &ish[0])) return;

    // ---- last workgroup: totals in block order, beta, next S, norms, stop test
    if (tid == 0) st->cnt_upd = 0u;
    double* tot = sm;   // 3 x P x P  (fits: 3*256 <= 5*256)
    for (int e = tid; e < NE; e += kWG) {
        double t = a.upart[e];
        for (int q = 1; q < a.nblk; ++q) t += a.upart[(int64_t)q * NE + e];
        tot[e] = t;
    }
    __syncthreads();
    const double* W = tot;
    const double* Q = tot + P * P;
    const double* F = tot + 2 * P * P;
    const int m = st->m;
    int* act = &ish[64];
    if (tid < m) act[tid] = st->keep[tid];
    __syncthreads();
    __shared__ double Lc[kMaxP * kMaxP], Wc[kMaxP * kMaxP], Bc[kMaxP * kMaxP];
    if (tid < m * m) {
        const int i = tid / m, j = tid - (tid / m) * m;
        Lc[tid] = st->Lc[tid];
        Wc[tid] = -W[act[i] * P + act[j]];
    }
    __syncthreads();
    wg_chol_solve(Lc, m, m, Wc, Bc);       // beta = -G^{-1} (AD)^T R
    if (tid < kMaxP * kMaxP) {
        st->beta[tid] = 0.0;
        st->S[tid] = 0.0;
    }
    __syncthreads();
    if (tid < m * m) {
        const int i = tid / m, j = tid - (tid / m) * m;
        st->beta[act[i] * kMaxP + act[j]] = Bc[tid];
        // S_next = R^T R + beta^T (D^T R), restricted to the active agents
        double s = Q[act[i] * P + act[j]];
        for (int l = 0; l < m; ++l) s = fma(Bc[l * m + i], F[act[l] * P + act[j]], s);
        st->S[act[i] * kMaxP + act[j]] = s;
    }
    if (tid == 0) {
        double mn = INFINITY;
        bool bad = false;
        for (int q = 0; q < m; ++q) {
            const int j = act[q];
            const double nr = sqrt(Q[j * P + j]);
            st->norms[j] = nr;
            if (!isfinite(nr)) bad = true;
            mn = fmin(mn, nr / st->nb);
        }
        st->minres = mn;
        st->iter += 1;
        if (bad) fail_state(st, -2);
        else if (mn <= st->tol) st->done = RECUR_CONV;
        else if (st->iter >= st->maxit) st->done = MAXIT;
    }
}

// ====================================================== k_dir: D = R + D beta

template <int PREC, int P>
__global__ __launch_bounds__(kWG) void k_dir(DirArgs a) {
    using TV = typename PT<PREC>::TV;
    __shared__ double be[P * P];
    __shared__ unsigned msk;
    const DevState* st = a.st;
    if (st->done != RUNNING) return;
    const int tid = threadIdx.x;
    if (tid < P * P) be[tid] = st->beta[(tid / P) * kMaxP + (tid % P)];
    if (tid == 0) msk = st->mask;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kWG + tid;
    if (i >= a.n_pad) return;
    const TV* R = static_cast<const TV*>(a.R);
    TV* D = static_cast<TV*>(a.D);
    double d[P];
#pragma unroll
    for (int j = 0; j < P; ++j) d[j] = D[i * P + j];
#pragma unroll
    for (int j = 0; j < P; ++j) {
        double s = R[i * P + j];
#pragma unroll
        for (int l = 0; l < P; ++l) s = fma(d[l], be[l * P + j], s);
        D[i * P + j] = ((msk >> j) & 1u) ? TV(s) : TV(0);
    }
}

// ============================================ k_res: T = B - Y, norms, restart

template <int P>
__global__ __launch_bounds__(kWG) void k_res(ResArgs a) {
    constexpr int RB = (P <= 8) ? kWG : kWG / 2;
    constexpr int NE = P * P + 1;      // T^T T entries, then b^T b
    __shared__ double ts[RB * P];
    __shared__ double bs[RB];
    __shared__ double tot[NE];
    __shared__ int ish[8];
    DevState* st = a.st;
    const int tid = threadIdx.x;
    const int64_t row0 = (int64_t)blockIdx.x * RB;
    const unsigned msk = st->mask;
    if (tid < RB) {
        const int64_t i = row0 + tid;
        const double bi = a.b[i];
        bs[tid] = bi;
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const double t = (j < a.p) ? bi - a.Y[i * P + j] : 0.0;
            ts[tid * P + j] = t;
            if (a.mode != RES_FINAL) {
                a.R[i * P + j] = t;
                a.D[i * P + j] = ((msk >> j) & 1u) ? t : 0.0;
            }
        }
    }
    __syncthreads();
    for (int e = tid; e < NE; e += kWG) {
        double s = 0.0;
        if (e < P * P) {
            const int x = e / P, y = e - (e / P) * P;
            for (int r = 0; r < RB; ++r) s = fma(ts[r * P + x], ts[r * P + y], s);
        } else {
            for (int r = 0; r < RB; ++r) s = fma(bs[r], bs[r], s);
        }
        a.rpart[(int64_t)blockIdx.x * NE + e] = s;
    }
    if (!last_arrival(&st->cnt_res, (unsigned)a.nblk, &ish[0])) return;
    if (tid == 0) st->cnt_res = 0u;
    for (int e = tid; e < NE; e += kWG) {
        double t = a.rpart[e];
        for (int q = 1; q < a.nblk; ++q) t += a.rpart[(int64_t)q * NE + e];
        tot[e] = t;
    }
    __syncthreads();
    if (tid == 0) {
        if (a.set_nb) st->nb = sqrt(tot[P * P]);
        double mn = INFINITY;
        bool bad = !isfinite(st->nb);
        for (int j = 0; j < a.p; ++j) {
            const double nr = sqrt(tot[j * P + j]);
            st->norms[j] = nr;
            if (!isfinite(nr)) bad = true;
            if ((msk >> j) & 1u) mn = fmin(mn, nr / st->nb);
        }
        st->minres = mn;
        if (a.mode != RES_FINAL) {
            if (bad) fail_state(st, -2);
            else if (st->nb == 0.0) fail_state(st, -1);
            else if (mn <= st->tol) st->done = FINISHED;
            else {
                if (a.mode == RES_CONFIRM) st->restarts += 1;
                st->done = (st->iter >= st->maxit) ? MAXIT : RUNNING;
            }
        }
    }
    // next S = D^T R = T^T T on the active agents (D = R = T)
    if (a.mode != RES_FINAL && tid < kMaxP * kMaxP) {
        const int x = tid / kMaxP, y = tid % kMaxP;
        const bool on = x < P && y < P && ((msk >> x) & 1u) && ((msk >> y) & 1u);
        st->S[tid] = on ? tot[x * P + y] : 0.0;
    }
}

// ======================================================== layout conversions

// Xr (n_pad x P row-major, zero padded) <- X (n x p column-major, ldx)
__global__ void k_pack(int n, int n_pad, int p, int P, const double* X, int64_t ldx, double* Xr) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n_pad * P) return;
    const int64_t i = idx / P;
    const int j = (int)(idx - i * P);
    Xr[idx] = (i < n && j < p) ? X[i + j * ldx] : 0.0;
}

__global__ void k_unpack(int n, int p, int P, const double* Xr, double* X, int64_t ldx) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * p) return;
    const int64_t i = idx % n;
    const int j = (int)(idx / n);
    X[i + j * ldx] = Xr[i * P + j];
}

__global__ void k_pad_vec(int n, int n_pad, const double* b, double* bp) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_pad) bp[i] = (i < n) ? b[i] : 0.0;
}

// ================================================================== launchers

template <int PREC, int P>
static hipError_t launch_ad_t(const AdArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((k_ad<PREC, P>), dim3(a.ntiles * a.nks), dim3(kWG), 0, s, a);
    return hipGetLastError();
}
template <int PREC, int P>
static hipError_t launch_upd_t(const UpdArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((k_upd<PREC, P>), dim3(a.nblk), dim3(kWG), 0, s, a);
    return hipGetLastError();
}
template <int PREC, int P>
static hipError_t launch_dir_t(const DirArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((k_dir<PREC, P>), dim3((a.n_pad + kWG - 1) / kWG), dim3(kWG), 0, s, a);
    return hipGetLastError();
}
template <int P>
static hipError_t launch_res_t(const ResArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((k_res<P>), dim3(a.nblk), dim3(kWG), 0, s, a);
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

hipError_t launch_ad(int prec, int P, const AdArgs& a, hipStream_t s) {
    switch (prec) {
#define C64(PP) launch_ad_t<PREC_F64, PP>(a, s)
#define C32(PP) launch_ad_t<PREC_F32, PP>(a, s)
#define CBF(PP) launch_ad_t<PREC_BF16X2, PP>(a, s)
        case PREC_F64: CCG_DISPATCH_P(P, C64)
        case PREC_F32: CCG_DISPATCH_P(P, C32)
        case PREC_BF16X2: CCG_DISPATCH_P(P, CBF)
#undef C64
#undef C32
#undef CBF
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_upd(int prec, int P, const UpdArgs& a, hipStream_t s) {
    switch (prec) {
#define C64(PP) launch_upd_t<PREC_F64, PP>(a, s)
#define C32(PP) launch_upd_t<PREC_F32, PP>(a, s)
        case PREC_F64: CCG_DISPATCH_P(P, C64)
        case PREC_F32:
        case PREC_BF16X2: CCG_DISPATCH_P(P, C32)
#undef C64
#undef C32
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_dir(int prec, int P, const DirArgs& a, hipStream_t s) {
    switch (prec) {
#define C64(PP) launch_dir_t<PREC_F64, PP>(a, s)
#define C32(PP) launch_dir_t<PREC_F32, PP>(a, s)
        case PREC_F64: CCG_DISPATCH_P(P, C64)
        case PREC_F32:
        case PREC_BF16X2: CCG_DISPATCH_P(P, C32)
#undef C64
#undef C32
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_res(int P, const ResArgs& a, hipStream_t s) {
#define CR(PP) launch_res_t<PP>(a, s)
    CCG_DISPATCH_P(P, CR)
#undef CR
}

hipError_t launch_pack(int n, int n_pad, int p, int P, const double* X, int64_t ldx, double* Xr,
                       hipStream_t s) {
    const int64_t tot = (int64_t)n_pad * P;
    hipLaunchKernelGGL(k_pack, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, n_pad, p, P,
                       X, ldx, Xr);
    return hipGetLastError();
}

hipError_t launch_unpack(int n, int p, int P, const double* Xr, double* X, int64_t ldx,
                         hipStream_t s) {
    const int64_t tot = (int64_t)n * p;
    hipLaunchKernelGGL(k_unpack, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, p, P, Xr,
                       X, ldx);
    return hipGetLastError();
}

hipError_t launch_pad_vec(int n, int n_pad, const double* b, double* bp, hipStream_t s) {
    hipLaunchKernelGGL(k_pad_vec, dim3((n_pad + 255) / 256), dim3(256), 0, s, n, n_pad, b, bp);
    return hipGetLastError();
}

int ad_tile_rows(int prec) {
    switch (prec) {
        case PREC_F64: return tile_rows<PREC_F64>();
        case PREC_F32: return tile_rows<PREC_F32>();
        default: return tile_rows<PREC_BF16X2>();
    }
}

}  // namespace ccg
