// Internal declarations of libpe (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

namespace pe {

// ---------------------------------------------------------------------------
// GEMM descriptor. Every dense product of the path has the form
//     C[r][s] = epilogue( sum_k A[r][k] * B[s][k] )
// with both operands K-contiguous ("NT"): A rows are state columns (one per
// interval x sample), B rows are operator rows. The K range depends on the
// operator row block: rows s < s_split use [k0a, k1a), rows s >= s_split use
// [k0b, k1b) (the zero blocks of the step operators are skipped).
// ---------------------------------------------------------------------------
struct GemmShape {
    int Mr = 0, Ns = 0;
    const void* A = nullptr;
    long lda = 0;
    const void* B = nullptr;
    long ldb = 0;
    int s_split = 0;
    int k0a = 0, k1a = 0, k0b = 0, k1b = 0;
};

enum EpiMode : int {
    EPI_STORE = 0,   // C = alpha*acc + beta*C0 (+ diag_add on r == s + diag_off)
    EPI_RESID = 1,   // R = f(t) - base - acc               (residual of a step)
    EPI_FSTEP = 2,   // fused fine step: d = ZF(t) - base - acc -> state/history update (ping-pong)
    EPI_COARSE_INIT = 3,   // initial coarse sweep: x_{n+1} = Phi_G x_n + c_n
    EPI_COARSE_DELTA = 4,  // correction of eq. (2.7): x_{n+1}^k = F_n + Phi_G (x_n^k - x_n^{k-1})
    EPI_ADJ_STATE = 6,     // fused adjoint step: [a; nu] <- a - [A; A + Mh] Z^T nu (+ cotangent)
    EPI_FCORR = 7,         // refinement of a fine step: state/history += acc (the correction Z_h[:, u] r)
};

struct Epi {
    int mode = EPI_STORE;
    // EPI_STORE
    double alpha = 1.0, beta = 0.0;
    double diag_add = 0.0;
    int diag_off = 0;
    double* C = nullptr;
    float* C32 = nullptr;  // EPI_STORE: nullable FP32 copy of C (same ldc)
    const double* C0 = nullptr;
    long ldc = 0, ldc0 = 0;
    // EPI_RESID (R64 and R32 nullable): R = f - base - acc (- cres * dres)
    double* R64 = nullptr;
    float* R32 = nullptr;
    long ldr = 0;
    const double* base = nullptr;
    long ldb = 0;
    const double* dres = nullptr;  // nullable: a diagonal term cres * dres[r][s] (ld lddres)
    long lddres = 0;
    double cres = 0.0;
    int src_kind = 0;            // 0: f = 0, 1: low-rank G*H, 2: dense per-interval table
    const double* Gs = nullptr;  // Dp x R
    const double* Hs = nullptr;  // B x R x Tlen
    int R = 0;
    long Tlen = 0;
    int time_mode = 0;           // 0: amplitude per fine step, 1: per interval
    int P = 1;
    int p_step = 0;              // fine step index inside the interval
    int cols_per_b = 1;          // column r -> sample r / cols_per_b, interval r % cols_per_b
    int n_fixed = -1;            // >= 0: every column belongs to this interval (r = sample)
    int rows_per_p = 0;          // > 0: row r is fine step p_step + r / rows_per_p of
                                 // column col_off + r % rows_per_p (rows ordered step-major)
    int col_off = 0;
    int N = 1;
    const double* Fint = nullptr;  // (B*N) x Dp table of per-interval sources
    long ldf = 0;
    // EPI_FSTEP (source fields as for EPI_RESID, with the step operator
    // applied: Gs = Z G, Fint = per-interval Z F; base = Z A x_a)
    const double* din = nullptr;    // state in  [du_prev | u - u_a | w - w_a | dw_prev], ld ldd
    double* dev64 = nullptr;        // state out (FP64), ld ldd
    float* dev32 = nullptr;         // state out (FP32 copy, nullable)
    long ldd = 0;
    int d1p = 0, d2p = 0;
    double* traj = nullptr;         // nullable: full new state xa + deviation at traj + r*ldtraj
    const double* xa = nullptr;     // anchors, ld d1p + d2p
    long ldtraj = 0;
    // EPI_FSTEP with refinement (nullable): the implicit equation's operands
    // [du_new + u - u_a | w - w_a | dw_prev | du_new] (u - u_a of the step's
    // input state; the last block feeds the residual's diagonal term), ld ldd
    double* vr = nullptr;
    // EPI_FCORR uses dev64 / dev32 (state updated in place), ldd, d1p, d2p, traj, ldtraj
    // EPI_COARSE_*  (column r is sample r)
    double* xout = nullptr;         // X^k[b][n+1] = xout + b*ldxo
    long ldxo = 0;
    const double* cs = nullptr;     // INIT: c_n = Z_dt F(t_{n+1}) at cs + b*ldcs (nullable)
    long ldcs = 0;
    const double* fbuf = nullptr;   // DELTA: F(x_n^{k-1}) at fbuf + b*ldfb
    long ldfb = 0;
    const double* xprev = nullptr;  // DELTA: X^{k-1}[b][n+1] at xprev + b*ldxo
    double* dl64 = nullptr;         // DELTA: next change x_{n+1}^k - x_{n+1}^{k-1} (b*ldl)
    float* dl32 = nullptr;
    long ldl = 0;
    const int* active = nullptr;
    // EPI_ADJ_STATE: adjoint state [a | nu], 2*ldr per column; the new nu
    // is also summed into sacc or stored at row r*P + m_step of rho_all
    // (both nullable, ld ldr): the source adjoint is Z^T applied to them
    double* sacc = nullptr;
    double* rho_all = nullptr;
    int m_step = 0;
    const double* s_cur = nullptr;
    double* s_nxt = nullptr;
    float* nu32 = nullptr;          // FP32 copy of nu, ld ldr
    const double* inj = nullptr;    // nullable: cotangent added to both parts, at inj + r*ldinj
    long ldinj = 0;
};

// Tile configuration of one GEMM launch.
struct TileCfg {
    int br = 64, bs = 64, splitk = 1;
    int bk2 = 0;  // 1: twice the base K depth per LDS stage
    int wsk = 0;  // > 0: wave-split-K kernel with this many waves per work-group (64-row tiles)
};

// Workspace for split-K partial planes.
struct GemmWork {
    void* part = nullptr;
    size_t part_bytes = 0;
    // optional hook run on the host between the product kernel and the
    // split-K reduction kernel (used to place timing events)
    void (*between)(void*) = nullptr;
    void* between_arg = nullptr;
};

// One product of a grouped launch (device-resident array of these).
struct GemmItem {
    GemmShape sh;
    Epi epi;
    int tiles_r = 1;  // row tiles of this product for the launch's tile shape
};

// One problem of a grouped coarse step (device-resident array of these):
// x_{n+1} = Phi x_n + c_n (initial sweep, FP64) or the delta-form correction
// x_{n+1}^k = F_n + Phi (x_n^k - x_n^{k-1}) in the path's precision.
struct CoarseItem {
    const double* Phi64 = nullptr;  // Dp x Dp
    const float* Phi32 = nullptr;
    int Dp = 0, B = 0, N = 0;
    long ldX = 0;                   // (N+1) * Dp
    double* Xk = nullptr;           // X^k (B x (N+1) x Dp)
    const double* Xprev = nullptr;  // X^{k-1}
    const double* cs = nullptr;     // B x N x Dp coarse source terms (nullable)
    const double* Fbuf = nullptr;   // B x N x Dp fine values
    double* Dl64[2] = {nullptr, nullptr};  // B x Dp changes (ping-pong)
    float* Dl32[2] = {nullptr, nullptr};
    const int* active = nullptr;    // B flags (nullable: all active)
};

// Launch C = epi(A * B^T) in precision T (float: FP32 MFMA, double: FP64
// MFMA). Returns hipSuccess or an error; throws nothing.
template <typename T>
hipError_t gemm_launch(const GemmShape& sh, const Epi& epi, const TileCfg& cfg, GemmWork& ws,
                       hipStream_t stream);

// Grouped launch of n_wg work-groups over device-resident items (tile shape
// cfg.br x cfg.bs, K depth per cfg.bk2; no split-K).
template <typename T>
hipError_t gemm_grouped_launch(const GemmItem* items, const int* wg_item, const int* wg_tile, int n_wg,
                               const TileCfg& cfg, hipStream_t stream);

// Grouped coarse step n over the first n_wg work-groups of the row table
// (4 operator rows per work-group). delta = 0: initial sweep (FP64),
// delta = 1: correction in precision T, reading changes Dl[c], writing Dl[1-c].
template <typename T>
hipError_t coarse_grouped_launch(const CoarseItem* items, const int* wg_item, const int* wg_row, int n_wg, int n,
                                 int delta, int c, hipStream_t stream);

// Persistent fine sweep (one cooperative launch for all P fused steps of a
// sweep; state columns Mr <= 64). sh: the step > 0 product with A = the even
// steps' FP32 (or FP64) state, A1 the odd steps'; epi: EPI_FSTEP source,
// anchor and layout fields; d64a/d64b, d32a/d32b: the state ping-pong (step 0
// reads a); traj (nullable): per-step states, row (r*P + p). grid: from
// fine_sweep_persistent_grid (the co-resident work-group count; 0 if
// cooperative launches are unavailable).
template <typename T>
int fine_sweep_persistent_grid();
template <typename T>
hipError_t fine_sweep_persistent(const GemmShape& sh, const void* A1, const Epi& epi, double* d64a, double* d64b,
                                 float* d32a, float* d32b, double* traj, int P, int grid, int splitk, void* part,
                                 size_t part_bytes, hipStream_t stream);

// operand offsets, strides and addresses keep 16-byte vector loads aligned
bool gemm_shape_ok(const GemmShape& sh, size_t elem);

// Choose a tile configuration for a product of this shape.
TileCfg choose_tiles(const GemmShape& sh, bool fp32, int n_cu);

// Workspace bytes a launch with cfg needs.
size_t gemm_part_bytes(const GemmShape& sh, const TileCfg& cfg, size_t elem);

}  // namespace pe
