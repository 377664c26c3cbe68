// Internal device-side definitions shared by the HIP kernels and the host driver.
//
// Vectors X, R, D, AD live on the device as n_pad x P blocks stored agent-major
// (column j = agent j is contiguous: V[j * n_pad + i]), with P the agent count p
// rounded up to 1, 2, 4, 8 or 16 and n_pad = n rounded up to a multiple of 512.
// Rows >= n and columns >= p are kept at zero, so elementwise kernels need no
// guards and sums over padded rows only add exact zeros.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ccg {

constexpr int kMaxP = 32;       // largest padded agent count (FP64 single solves)
constexpr int kLowMaxP = 16;    // ... in the low-precision modes and the batched engine
constexpr int kWG = 256;        // threads per workgroup for every kernel
constexpr int kRowAlign = 512;  // n_pad granularity
constexpr int kGroup = 32;      // workgroups per first-level reduction group

enum Prec : int { PREC_F64 = 0, PREC_F32 = 1, PREC_BF16X2 = 2 };

// Row tiling of the update and direction launches (the same for both): one workgroup
// per block of kWG / P rows (one element per thread), or from P = 16, where both run on
// the FP64 matrix cores, per block of kUpdWideRows rows (4 waves of 16).
constexpr int kUpdWideRows = 64;
static_assert(kRowAlign % kUpdWideRows == 0, "wide update tiles must divide the row padding");
__host__ __device__ constexpr bool upd_mma(int P) { return P >= 16; }
__host__ __device__ inline int upd_blocks(int n_pad, int P) {
    return upd_mma(P) ? n_pad / kUpdWideRows : n_pad / (256 / P);
}
// Workgroups per first-level group of the update's product reduction: at P = 32 the
// 1056 values per workgroup make a group of 16 one round of loads for its summer.
__host__ __device__ constexpr int upd_group(int P) { return P >= 32 ? 16 : kGroup; }

// Device iteration state, one per solve.  Written only by "last workgroup"
// epilogues and by the residual kernel; read by every kernel at entry.
// OUTER: a refinement residual found the solve unfinished; the host starts the
// next inner solve (block steps only run while done == RUNNING).
// REINFLATE: the rank step would drop agents and re-inflation is allowed: the step
// stopped before alpha, mask holds the kept set J and prev_mask the agents active
// before it; the host re-inflates the others and restarts the block.
enum Done : int { RUNNING = 0, RECUR_CONV = 1, FINISHED = 2, MAXIT = 3, FAILED = 4, OUTER = 5, REINFLATE = 6 };

struct DevState {
    int done;          // Done code; kernels are no-ops while done != RUNNING
    int iter;          // completed block steps
    int m;             // active agent count (rank of the last accepted D)
    int status;        // failure code (ccg_status) when done == FAILED
    unsigned mask;     // bit j set <=> agent j active
    int deflations;    // rank-drop events
    int restarts;      // explicit-residual restarts
    int maxit;         // stop after this many block steps
    int dir_pending;   // 1: the update launch of this block step ran, and the direction
                       // launch completes the step (cleared by every A.D launch)
    int ad_streams;    // A.D launches that streamed A in block steps (for byte counts)
    int reinflate_left;  // re-inflation events still allowed (CCG_REINFLATE)
    unsigned prev_mask;  // REINFLATE: the agents active before the rank step
    double nb;         // ||b||_2 (for a refinement inner solve: 1, columns are scaled)
    double tol;        // relative stop tolerance on min_j ||R_j|| / nb
    double tau;        // rank threshold on the scaled pivots
    double minres;     // min over active agents of ||R_j|| / nb (last test)
    int keep[kMaxP];   // active agents, ascending (first m entries)
    double norms[kMaxP];                 // ||R_j|| per agent (last computed)
    double alpha[kMaxP * kMaxP];         // alpha[l*kMaxP + j]: X[:,j] += D[:,l] alpha[l][j]
    double beta[kMaxP * kMaxP];          // beta[l*kMaxP + j]:  D[:,j] = R[:,j] + D[:,l] beta[l][j]
    double L[kMaxP * kMaxP];             // Cholesky factor of G (inactive agents: identity)
};

// Scratch of one fixed-order grid reduction (see grid_reduce in the kernels).
struct RedBuf {
    double* l1;          // nwg x ne partials
    double* l2;          // ngroups x ne group sums
    unsigned* cnt;       // ngroups + 1 tickets, zero between launches
};

// Arguments of the A.D stream kernel.
struct AdArgs {
    const void* A;       // FP64 / FP32 matrix, or the BF16 "hi" plane; column-major, lda
    const void* A_lo;    // BF16 "lo" plane (bf16x2 only)
    int64_t lda;         // leading dimension in elements (lda * element size % 16 == 0)
    int n;               // system size
    int n_pad;           // padded row count of the vector blocks
    int product_only;    // 1: only form Y = A.V (residual); 0: also Gram + alpha
    const void* V;       // operand block D (agent-major, vector type)
    const void* R;       // residual block (agent-major, vector type)
    void* AD;            // result block (agent-major, vector type)
    RedBuf red;          // reduction scratch (ne = P*(P+1)/2 + P*P)
    DevState* st;
};

// Arguments of the symmetric A.D pass (FP64, P <= 8).  AD = A D is formed from the
// blocks A(I, J), I <= J, of a partition of A into kSymB x kSymB blocks: block (I, J)
// adds A(I, J) D(J) to rows I and A(I, J)^T D(I) to rows J, so only the upper block
// triangle of A is read.  Workgroup u runs the strip units[u] = (I, J0) of up to
// kSymW blocks (I, J0 .. J0 + kSymW - 1) and writes its partial sums into part:
// slot I of block J for A(I, J)^T D(I) (I < J), slot I + s of block I for strip s of
// block row I.  Block K has K + ceil((nb - K) / kSymW) <= nb slots.
constexpr int kSymB = 128;      // block size (2 rows per lane of a wave)
constexpr int kSymW = 4;        // blocks per strip
constexpr int kSymMaxP = 8;     // largest padded agent count of the symmetric pass

struct SymArgs {
    const double* A;     // column-major, lda (lda * 8 % 16 == 0); blocks I <= J read
    int64_t lda;
    int n;
    int n_pad;
    int nb;              // ceil(n / kSymB)
    int tmax;            // slot stride of part (>= nb)
    const double* V;     // D block (agent-major, n_pad rows)
    double* part;        // [block][slot][kSymB rows][P] partial sums
    const int2* units;   // (I, J0) per strip, I <= J0
    const DevState* st;
};

// Arguments of the update launch (X += D alpha, R -= AD alpha, and each tile's share
// of (AD)^T R and diag(R^T R) of the new residual) and of the direction launch (the
// totals of those shares, the stop test, beta, and D = R + D beta).
// Arguments of the small-system tier (systems with n <= kSmallN and P <= kSmallMaxP):
// one workgroup runs whole block steps of one system, several per launch.
constexpr int kSmallN = 512;      // the tier's padded size (n_pad == 512)
constexpr int kSmallMaxP = 8;
constexpr int kSmallWG = 512;     // threads of the tier's workgroup
struct SmallArgs {
    const void* A;       // matrix streamed by the block steps (as AdArgs::A)
    const void* A_lo;    // BF16 "lo" plane (bf16x2 only)
    int64_t lda;
    int n;
    void* X;             // agent-major blocks of kSmallN rows (vector type)
    void* R;
    void* D;
    DevState* st;
};

struct UpdArgs {
    int n_pad;
    void* X;             // agent-major blocks (vector type)
    void* R;
    void* D;
    const void* AD;
    RedBuf red;          // products of the update (ne = P*P + P): per block, per group
    DevState* st;
};

// Residual epilogue: T = B - Y, with B = b in every column (FP64).
//   RES_INIT    R = D = T, the start of a solve
//   RES_CONFIRM R = D = T; a failed confirmation restarts the agents from T
//   RES_FINAL   norms only (the report after maxit)
//   RES_REFINE  R = T only: the FP64 residual of an outer refinement step
enum ResMode : int { RES_INIT = 0, RES_CONFIRM = 1, RES_FINAL = 2, RES_REFINE = 3 };

struct ResArgs {
    int n;
    int n_pad;
    int p;               // true agent count (columns >= p ignored)
    int mode;            // ResMode
    int set_nb;          // 1: also set st->nb = ||b||
    const double* b;     // n_pad (zero padded)
    const double* Y;     // agent-major A X
    double* R;           // written in INIT / CONFIRM
    double* D;
    RedBuf red;          // ne = P*P + 1
    DevState* st;
};

// One outer step of the mixed-precision refinement (FP32 / BF16x2 modes).  The
// inner solve works on A E = T with every column of T scaled to unit norm, in the
// low-precision vector blocks; the FP64 agents then take X += E * scale.
struct RefArgs {
    int n_pad;
    int P;
    const double* T;          // FP64 residual block (agent-major)
    double* X;                // FP64 agents (agent-major)
    void* E;                  // inner iterate (FP32)
    void* R;                  // inner residual (FP32)
    void* D;                  // inner direction (FP32)
    double scale[kMaxP];      // ||T_j|| (0: agent j sits out of the inner solve)
};

}  // namespace ccg
