// C ABI of libpe: problem set-up (FP64 factorisations and step operators on
// the GPU), the fine and coarse propagators, and the parareal iteration of
// Algorithm 1 (update (2.7), stopping test (2.8)).
//
// Step of the splitting scheme, eqs. (2.4)-(2.5), written with residuals and
// increments. Per state column keep [du_prev | u | w | dw_prev], where
// du_prev = u_n - u_{n-1}, dw_prev = w_n - w_{n-1} (zero at an interval
// start: every propagator call begins with a fresh history). With
//     r_u = F1 - A11 u - A12 w - (M12/h) dw_prev
//     r_w = F2 - A21 u - A22 w - (M21/h) du_prev
// the step is
//     (M11/h + A11) du = r_u,      M22 dw = h (r_w - A21 du),
// i.e. [du; dw] = Z_h [r_u; r_w] with
//     Z_h = [ K_h^-1            0        ]      K_h = M11/h + A11,
//           [ -Q_h K_h^-1   h M22^-1     ]      Q_h = h M22^-1 A21.
// So one step is two dense products over all columns at once:
//     R = F - A x_a - W_h * dev          (W_h = [[0, A11, A12, M12/h],
//     [du; dw] = Z_h * R                          [M21/h, A21, A22, 0]])
// where x_a is an anchor state (the interval start) and dev the deviation
// from it. K_h^-1 and M22^-1 are formed on the GPU from FP64 Cholesky
// factors. In PE_MIXED the two products run in FP32 on MFMA; the anchor
// residual A x_a, the state accumulation, the coarse propagator and the jump
// norms stay FP64.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/pe.h"
#include "pe_kernels.h"
#include "wg_order.h"

using namespace pe;

namespace {

thread_local std::string g_err;

pe_status fail(pe_status code, const std::string& msg) {
    g_err = msg;
    return code;
}

inline int roundup(int x, int m) { return (x + m - 1) / m * m; }

#define PE_HIP(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(PE_ERR_HIP, std::string(#expr " failed: ") + hipGetErrorString(e_)); \
    } while (0)

#define PE_TRY(expr)                    \
    do {                                \
        pe_status s_ = (expr);          \
        if (s_ < 0) return s_;          \
    } while (0)

}  // namespace

namespace pe {
// error status and message of the calling thread, for the other sources of
// the library
pe_status set_error(pe_status code, const std::string& msg) { return fail(code, msg); }
}  // namespace pe

// captured HIP graphs of repeated launch sequences, keyed by what fixes
// their pointers (first visit eager, second captured, later replayed)
struct GraphCache {
    int use_graphs = 1;
    std::map<std::vector<long>, hipGraphExec_t> graphs;
    std::set<std::vector<long>> seen, bad;
    void clear() {
        for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
        graphs.clear();
        seen.clear();
        bad.clear();
    }
};

// launch timing: HIP event pairs around each launch of a class, recorded on
// the owner's stream, folded into per-class totals when the stream is idle
struct Prof {
    int on = 0;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    std::vector<std::pair<int, size_t>> pending;  // (kind, index of first event)
    double ms[PE_PROF_KINDS] = {0};
    long long n[PE_PROF_KINDS] = {0};
    void reset() {
        pending.clear();
        used = 0;
        for (int k = 0; k < PE_PROF_KINDS; ++k) {
            ms[k] = 0.0;
            n[k] = 0;
        }
    }
    ~Prof() {
        for (hipEvent_t ev : pool) (void)hipEventDestroy(ev);
    }
};

struct pe_problem_s {
    int d1 = 0, d2 = 0, D = 0, d1p = 0, d2p = 0, Dp = 0, N = 0, P = 0;
    double dt = 0, dtf = 0;
    int prec = PE_FP64;
    hipStream_t st = nullptr;
    int own_stream = 0;  // st created by the handle (the caller passed NULL)
    int n_cu = 256;
    int device = 0;  // the device current at creation (the handle's operators live there)

    // operators (padded, row-major)
    double* A64 = nullptr;   // Dp x Dp   full stiffness
    double* M64 = nullptr;   // Dp x Dp   full mass
    // fine step (eqs. (2.4)-(2.5) at dt_fine): increment Z_h R with the
    // residual R = F - A x_a - W_h dev, fused into one product per step:
    // Z_h R = Z_h F - (Z_h A) x_a - (Z_h W_h) dev
    double* Zf64 = nullptr;  // Dp x Dp   Z_h (FP64; whitened coordinates in PE_MIXED)
    double* ZW64 = nullptr;  // Dp x 2Dp  Z_h W_h (PE_FP64)
    float* ZW32 = nullptr;   // Dp x 2Dp  Z_h W_h in FP32, whitened (PE_MIXED)
    double* ZA64 = nullptr;  // Dp x Dp   Z_h A (FP64; whitened in PE_MIXED)
    double* Zc64 = nullptr;  // Dp x Dp   coarse increment operator
    double* PhiG64 = nullptr;  // Dp x Dp   coarse step matrix I - Z_dt A
    float* PhiG32 = nullptr;
    // coarse sweeps as doubling scans (one sample, fresh history): powers
    // Phi_G^(2^l), l < scan_L0 (l = 0 is PhiG), and two (Z + N + 1) x Dp
    // ping-pong buffers whose first Z = 2^(scan_L0 - 1) rows stay zero;
    // scan_L levels for the correction (N terms), scan_L0 for the initial
    // sweep (N + 1 terms)
    int coarse_scan = 1;
    int scan_L = 0, scan_L0 = 0;
    std::vector<double*> pow64, pow64T;  // powers and their transposes
    std::vector<float*> pow32, pow32T;
    // backward (adjoint) scans: (N + 1 + Z) x Dp ping-pong buffers whose
    // rows after N + 1 stay zero
    double* scanA64[2] = {nullptr, nullptr};
    float* scanA32[2] = {nullptr, nullptr};
    double* scan64[2] = {nullptr, nullptr};
    float* scan32[2] = {nullptr, nullptr};
    std::vector<void*> scan_allocs;
    // the coarse sweeps of a batch (PE_MIXED) as the same scan, for B
    // samples: the correction over N terms in bscan_L levels, the initial
    // sweep over N + 1 terms in bscan_L0 levels; FP32 powers Phi_G^(2^l),
    // l = 1..bscan_L0-1 (l = 0 is PhiG32), formed by FP64 squaring, and two
    // B x (Z + N + 1) x Dp ping-pong buffers (FP64 sums, FP32 copies) whose
    // first Z = 2^(bscan_L0 - 1) rows per sample stay zero
    int bscan_L = -1, bscan_L0 = -1, bscan_Z = 0, bscan_B = 0;
    std::vector<float*> bpow32;
    double* bscan64[2] = {nullptr, nullptr};
    float* bscan32[2] = {nullptr, nullptr};
    std::vector<void*> bscan_allocs;
    // PE_MIXED: the fine sweep works in mass-whitened coordinates
    // x~ = Tin x, Tin = blkdiag(L1^T, L2^T) with M11 = L1 L1^T, M22 = L2 L2^T
    // (there M~11 = M~22 = I); x = Tout x~, Tout = Tin^-1; Linv = Tout^T
    double* Aw64 = nullptr;    // Dp x Dp whitened stiffness
    double* Tin64 = nullptr;   // Dp x Dp
    double* Tout64 = nullptr;  // Dp x Dp
    double* Linv64 = nullptr;  // Dp x Dp
    // adjoint (transposed) operators, in the fine sweep's precision and
    // coordinates: [A; A + Mh] Z_h^T (Mh the off-diagonal mass coupling over
    // dt_fine), Phi_G^T; PE_MIXED also keeps Tin^T and the whitened mass
    double* YZ64 = nullptr;    // 2Dp x Dp  [A; A + Mh] Z_h^T: the fused transposed step (PE_FP64)
    float* YZ32 = nullptr;     //            its FP32 copy in whitened coordinates (PE_MIXED)
    double* PhiGT64 = nullptr;
    float* PhiGT32 = nullptr;
    double* TinT64 = nullptr;
    double* Mw64 = nullptr;
    int adj_ops = 0;           // adjoint operators built (on first use)
    double* M12k = nullptr;    // d1p x d2p (ld d2p): M12 in the fine sweep's coordinates
    // PE_MIXED_REFINE (refine = 1; 2: also the sweeps on iterate changes):
    // the implicit V_H1 equation of a fine step in whitened coordinates,
    // Wr = [K~ | A~11 | A~12 | M~12/dt_fine] (d1p x 2Dp, FP64, K~ = I/dt_fine + A~11),
    // applied to [du_new | u - u_a | w - w_a | dw_prev], and the correction
    // operator Zc = Z_h[:, u] (Dp x d1p, FP32)
    int refine = 0;
    double* Wr64 = nullptr;
    float* Zc32 = nullptr;

    // source
    int src_set = 0, B_src = 0, R = 0, Rp = 0, time_mode = 0, src_kind = 0;
    long Tlen = 0;
    double* Gs = nullptr;    // Dp x Rp
    double* Hs = nullptr;    // B x R x Tlen
    double* Fint = nullptr;  // (B*N) x Dp
    double* Gs_w = nullptr;    // whitened copies (PE_MIXED)
    double* Fint_w = nullptr;
    double* CS = nullptr;      // (B*N) x Dp: Z_dt F(t_{n+1}), the coarse step's source term
    double* GT = nullptr;      // Rp x Dp: G^T (source adjoint)
    double* ZGs = nullptr;     // Dp x Rp: Z_h G (whitened in PE_MIXED), the fused step's source
    double* ZGT = nullptr;     // Rp x Dp: its transpose (source adjoint (Z_h G)^T nu)
    double* ZFint = nullptr;   // (B*N) x Dp: Z_h F per interval (dense tables)
    double* GwT = nullptr;     // Rp x Dp: whitened G^T (PE_MIXED)

    // iteration workspace (sized for B_cap samples)
    int B_cap = 0;
    double* Xk[2] = {nullptr, nullptr};  // B x (N+1) x Dp
    double *Fbuf = nullptr, *Xa = nullptr, *Ya = nullptr, *R64 = nullptr;
    double* Dl64[2] = {nullptr, nullptr};  // B x Dp: x_n^k - x_n^{k-1} along the coarse sweep
    float* Dl32[2] = {nullptr, nullptr};
    double* dev64[2] = {nullptr, nullptr};  // fine-step state, ping-pong (N*B x 2Dp)
    float* dev32[2] = {nullptr, nullptr};
    // refinement workspace (PE_MIXED_REFINE): operands of the implicit
    // equation (N*B x 2Dp), the u rows of A x_a (N*B x d1p) and the residual
    // (N*B x d1p, FP32)
    double *Vr = nullptr, *AxU = nullptr;
    float* res32 = nullptr;
    double *E = nullptr, *Yn = nullptr, *Jd = nullptr, *x0p = nullptr, *io = nullptr, *nrm = nullptr;
    int* active_d = nullptr;
    GemmWork gw;

    // adjoint workspace (pe_adjoint / pe_tracking), sized for adj_B samples
    int adj_B = 0, adj_Rp = 0, adj_traj = 0, adj_rho = 0, adj_fdh = 0;
    double *Xb = nullptr, *Qb = nullptr, *Yb = nullptr, *Sacc = nullptr, *Hb = nullptr;
    double *Rho = nullptr, *Ytraj = nullptr, *Inj = nullptr, *Fdh = nullptr, *Fdh_w = nullptr, *rowtmp = nullptr;
    std::vector<void*> adj_allocs;

    // launch timing (pe_profile): HIP event pairs around each launch of a
    // kernel class, on the handle's stream
    Prof prof;

    // tile configuration of the last launch of each profiled class
    int last_cfg[PE_PROF_KINDS][4] = {{0}};

    // persistent fine sweep (one cooperative launch per sweep, opt-in) when
    // the interval columns fit one row tile; co-resident grid per precision
    int persistent = 0;
    int pers_grid[2] = {-1, -1};

    // autotuned tile configurations per product site and shape
    int autotune = 1;
    std::map<std::vector<int>, pe::TileCfg> tuned;
    // PE_FORCE_WSK="bs,waves,splitk": every product whose state columns fit
    // one 64-row tile runs the wave-split-K kernel with this configuration
    pe::TileCfg force_wsk;
    pe::TileCfg force_tiles;  // every product of more than 4 state columns, if force_tiles_on (PE_FORCE_TILES)
    int force_tiles_on = 0;

    // captured HIP graphs of the sweeps, keyed by (kind, B, buffer parity)
    GraphCache gc;

    // waveform-relaxation fine solver (pe_fine_wr, FP64): operators for one
    // alpha and source version, workspace for a chunk of interval columns
    int src_version = 0;
    double wr_alpha = -1.0;
    int wr_src_version = -1, wr_B = -1, wr_NBc = 0, wr_K = 0;
    double *wrO = nullptr, *wrGu = nullptr, *wrZw = nullptr, *wrPhiW = nullptr, *wrM11h = nullptr;
    double *wrGw = nullptr, *wrFintW = nullptr, *wrTw = nullptr;
    double *wrUl = nullptr, *wrWl = nullptr, *wrR = nullptr, *wrRh = nullptr, *wrUh = nullptr;
    double *wrWcat = nullptr, *wrUcat = nullptr, *wrV = nullptr, *wrY = nullptr;
    // grouped launch of the per-frequency solves: items and work-group tables
    // for chunks of wr_tab_nc columns (rebuilt with the operators or workspace)
    GemmItem* wrItems = nullptr;
    int *wrWgI = nullptr, *wrWgT = nullptr;
    int wr_nwg = 0, wr_tab_nc = 0;
    TileCfg wr_cfg;
    std::vector<void*> wr_ops, wr_ws, wr_tab;
    // fine propagator used by pe_solve (pe_set_fine_solver)
    int fine_kind = PE_FINE_STEP;
    double fine_alpha = 0.0;
    int fine_K0 = 0;

    // history carried across intervals (pe_set_history): the states of the
    // iteration are [x | delta] (delta = change over the last fine step), of
    // stride Sx = 2Dp (Sx = Dp with the restarting history); the coarse step
    // on them (2Dp x 2Dp) and its source term (B*N x 2Dp)
    int hist = PE_HIST_RESTART, Sx = 0;
    double* PhiA64 = nullptr;
    float* PhiA32 = nullptr;
    double* CSa = nullptr;
    int csa_version = -1;
    std::vector<void*> hist_ops, hist_src;

    std::vector<void*> op_allocs, ws_allocs;
};

namespace {

pe_status dalloc(pe_problem p, std::vector<void*>& list, void** out, size_t bytes) {
    *out = nullptr;
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(out, bytes);
    if (e != hipSuccess) {
        *out = nullptr;
        (void)hipGetLastError();  // later launches must not report this failure
        return fail(PE_ERR_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " +
                                      hipGetErrorString(e));
    }
    list.push_back(*out);
    return PE_OK;
}

template <typename T>
pe_status dalloc_t(pe_problem p, std::vector<void*>& list, T** out, size_t count) {
    void* v = nullptr;
    PE_TRY(dalloc(p, list, &v, count * sizeof(T)));
    *out = (T*)v;
    return PE_OK;
}

void free_list(std::vector<void*>& list) {
    for (void* v : list) (void)hipFree(v);
    list.clear();
}

// temporary device allocations of one call: released (after the stream has
// drained) when the owner goes out of scope, on every return path
struct TmpList {
    hipStream_t st;
    std::vector<void*> v;
    explicit TmpList(hipStream_t s) : st(s) {}
    ~TmpList() {
        if (!v.empty()) {
            (void)hipStreamSynchronize(st);
            free_list(v);
        }
    }
    TmpList(const TmpList&) = delete;
    TmpList& operator=(const TmpList&) = delete;
};

void graphs_clear(pe_problem p);

// grow the split-K workspace if a launch needs more (synchronises first)
pe_status ensure_gemm_work(pe_problem p, size_t part_bytes) {
    GemmWork& w = p->gw;
    if (part_bytes <= w.part_bytes) return PE_OK;
    PE_HIP(hipStreamSynchronize(p->st));
    graphs_clear(p);
    if (w.part) (void)hipFree(w.part);
    w.part = nullptr;
    w.part_bytes = 0;
    const size_t nb = std::max(part_bytes, (size_t)1 << 20);
    hipError_t e = hipMalloc(&w.part, nb);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(PE_ERR_NOMEM, "split-K workspace allocation failed");
    }
    w.part_bytes = nb;
    return PE_OK;
}

pe_status prof_begin_on(Prof& pf, hipStream_t st, int kind, size_t* slot) {
    *slot = (size_t)-1;
    if (!pf.on || kind < 0) return PE_OK;
    while (pf.pool.size() < pf.used + 2) {
        hipEvent_t ev;
        PE_HIP(hipEventCreate(&ev));
        pf.pool.push_back(ev);
    }
    *slot = pf.used;
    pf.used += 2;
    PE_HIP(hipEventRecord(pf.pool[*slot], st));
    pf.pending.emplace_back(kind, *slot);
    return PE_OK;
}

pe_status prof_end_on(Prof& pf, hipStream_t st, size_t slot) {
    if (slot == (size_t)-1) return PE_OK;
    PE_HIP(hipEventRecord(pf.pool[slot + 1], st));
    return PE_OK;
}

pe_status prof_collect_on(Prof& pf) {
    for (auto& kv : pf.pending) {
        float ms = 0.f;
        PE_HIP(hipEventElapsedTime(&ms, pf.pool[kv.second], pf.pool[kv.second + 1]));
        pf.ms[kv.first] += ms;
        pf.n[kv.first] += 1;
    }
    pf.pending.clear();
    pf.used = 0;
    return PE_OK;
}

pe_status prof_begin(pe_problem p, int kind, size_t* slot) { return prof_begin_on(p->prof, p->st, kind, slot); }

pe_status prof_end(pe_problem p, size_t slot) { return prof_end_on(p->prof, p->st, slot); }

// fold completed event pairs into the per-kind totals (stream must be idle)
pe_status prof_collect(pe_problem p) { return prof_collect_on(p->prof); }

// ---------------------------------------------------------------------------
// HIP graphs: a sweep's launches are recorded once (stream capture) and
// replayed. The first visit of a key runs eagerly (autotuning, workspace
// growth and any other synchronising work happen there); the second visit
// captures. Graphs hold only kernel nodes (no memset nodes). Pointer changes
// (workspace growth, a new source) drop every graph.
// ---------------------------------------------------------------------------
void graphs_clear(pe_problem p) { p->gc.clear(); }

template <typename Fn>
pe_status graph_run_on(GraphCache& gc, hipStream_t st, bool eager, const std::vector<long>& key, Fn&& fn) {
    if (!gc.use_graphs || eager || gc.bad.count(key) || !st) return fn();
    auto it = gc.graphs.find(key);
    if (it != gc.graphs.end()) {
        PE_HIP(hipGraphLaunch(it->second, st));
        return PE_OK;
    }
    if (!gc.seen.count(key)) {
        gc.seen.insert(key);
        return fn();
    }
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        gc.use_graphs = 0;  // this stream cannot be captured: stay eager
        return fn();
    }
    const pe_status s = fn();
    const hipError_t e = hipStreamEndCapture(st, &g);
    hipGraphExec_t ex = nullptr;
    hipError_t ei = hipErrorUnknown;
    if (s == PE_OK && e == hipSuccess && g) ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (s != PE_OK || e != hipSuccess || ei != hipSuccess) {
        // not capturable: keep this sequence eager
        (void)hipGetLastError();
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) {
            hipGraph_t g2 = nullptr;
            (void)hipStreamEndCapture(st, &g2);
            if (g2) (void)hipGraphDestroy(g2);
        }
        gc.bad.insert(key);
        g_err.clear();
        return fn();
    }
    gc.graphs[key] = ex;
    PE_HIP(hipGraphLaunch(ex, st));
    return PE_OK;
}

template <typename Fn>
pe_status graph_run(pe_problem p, const std::vector<long>& key, Fn&& fn) {
    return graph_run_on(p->gc, p->st, p->prof.on != 0, key, fn);
}

// ---------------------------------------------------------------------------
// autotuner: time candidate tile configurations of a product on its real
// operands (output to a scratch buffer, so no side effects) and keep the
// fastest. Choices are looked up first in the read-only database named by
// PE_TUNE_DB and the cache named by PE_TUNE_CACHE (one line per site: key
// fields then br bs bk2 splitk [wsk], wsk > 0 naming the wave-split-K kernel
// with that many waves); new choices are appended to the cache.
// Runs that share these files use identical configurations (identical
// rounding).
// ---------------------------------------------------------------------------
std::vector<int> tune_key(int site, bool fp32, const GemmShape& sh) {
    return {site, fp32 ? 1 : 0, sh.Mr, sh.Ns, sh.s_split, sh.k0a, sh.k1a, sh.k0b, sh.k1b};
}

void tune_file_load(pe_problem p, const char* path) {
    if (!path || !*path) return;
    FILE* f = fopen(path, "r");
    if (!f) return;
    char line[512];
    while (fgets(line, sizeof(line), f)) {
        std::vector<int> v;
        char* tok = strtok(line, " \t\n");
        while (tok) {
            v.push_back(atoi(tok));
            tok = strtok(nullptr, " \t\n");
        }
        if (v.size() != 13 && v.size() != 14) continue;
        TileCfg c;
        c.br = v[9];
        c.bs = v[10];
        c.bk2 = v[11];
        c.splitk = v[12];
        c.wsk = v.size() == 14 ? v[13] : 0;
        v.resize(9);
        p->tuned[v] = c;
    }
    fclose(f);
}

// read-only database shipped with the library (PE_TUNE_DB), then the
// read/append cache (PE_TUNE_CACHE); later entries override earlier ones
void tune_cache_load(pe_problem p) {
    tune_file_load(p, getenv("PE_TUNE_DB"));
    tune_file_load(p, getenv("PE_TUNE_CACHE"));
}

void tune_cache_store(const std::vector<int>& key, const TileCfg& c) {
    const char* path = getenv("PE_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = fopen(path, "a");
    if (!f) return;
    for (int x : key) fprintf(f, "%d ", x);
    fprintf(f, "%d %d %d %d %d\n", c.br, c.bs, c.bk2, c.splitk, c.wsk);
    fclose(f);
}

pe_status ensure_gemm_work(pe_problem p, size_t part_bytes);

template <typename T>
pe_status tune(pe_problem p, const GemmShape& sh, TileCfg* best_out) {
    const bool fp32 = sizeof(T) == 4;
    *best_out = choose_tiles(sh, fp32, p->n_cu);
    double* scratch = nullptr;
    if (hipMalloc((void**)&scratch, sizeof(double) * sh.Mr * sh.Ns) != hipSuccess) {
        (void)hipGetLastError();  // no room to time candidates: keep the default tiles
        return PE_OK;
    }
    hipEvent_t e0, e1;
    PE_HIP(hipEventCreate(&e0));
    PE_HIP(hipEventCreate(&e1));
    Epi epi;
    epi.mode = EPI_STORE;
    epi.C = scratch;
    epi.ldc = sh.Ns;
    const int la = sh.k1a - sh.k0a, lb = sh.k1b - sh.k0b;
    const int kext = std::max(la, lb);
    const int bk0 = fp32 ? 32 : 16;
    const int shapes[6][2] = {{32, 64}, {64, 32}, {64, 64}, {64, 128}, {128, 64}, {128, 128}};
    double best = 1e30;
    for (auto& rs : shapes) {
        for (int bk2 = 0; bk2 < 2; ++bk2) {
            const int bk = bk0 << bk2;
            const int nkt = (kext + bk - 1) / bk;
            const long tiles = (long)((sh.Mr + rs[0] - 1) / rs[0]) * ((sh.Ns + rs[1] - 1) / rs[1]);
            for (int sk = 1; sk <= 32; sk *= 2) {
                if (sk > 1 && (nkt / sk < 2 || tiles * sk > 4L * 2048)) break;
                if (tiles > 2048 && sk > 1) break;
                TileCfg c;
                c.br = rs[0];
                c.bs = rs[1];
                c.bk2 = bk2;
                c.splitk = sk;
                const size_t need = gemm_part_bytes(sh, c, sizeof(T));
                if (need > ((size_t)512 << 20)) continue;
                PE_TRY(ensure_gemm_work(p, need));
                if (gemm_launch<T>(sh, epi, c, p->gw, p->st) != hipSuccess) continue;
                const int reps = 10;
                PE_HIP(hipEventRecord(e0, p->st));
                for (int i = 0; i < reps; ++i) PE_HIP(gemm_launch<T>(sh, epi, c, p->gw, p->st));
                PE_HIP(hipEventRecord(e1, p->st));
                PE_HIP(hipEventSynchronize(e1));
                float ms = 0.f;
                PE_HIP(hipEventElapsedTime(&ms, e0, e1));
                if (getenv("PE_VERBOSE") && atoi(getenv("PE_VERBOSE")) > 1)
                    fprintf(stderr, "[libpe]   candidate %dx%d bk2=%d splitk=%d wsk=%d: %.2f us\n", c.br, c.bs,
                            c.bk2, c.splitk, c.wsk, ms / reps * 1e3);
                if (ms / reps < best) {
                    best = ms / reps;
                    *best_out = c;
                }
            }
        }
    }
    // wave-split-K kernel for products whose state columns fit one 64-row tile
    if (sh.Mr <= 64) {
        const int nst = (kext + 15) / 16;
        const int ws_shapes[4][2] = {{32, 4}, {32, 8}, {16, 4}, {16, 8}};
        for (auto& wc : ws_shapes) {
            const long tiles = (sh.Ns + wc[0] - 1) / wc[0];
            for (int sk = 1; sk <= 32; sk *= 2) {
                if (sk > 1 && (nst / (sk * wc[1]) < 2 || tiles * sk > 4096)) break;
                TileCfg c;
                c.br = 64;
                c.bs = wc[0];
                c.wsk = wc[1];
                c.splitk = sk;
                const size_t need = gemm_part_bytes(sh, c, sizeof(T));
                if (need > ((size_t)512 << 20)) continue;
                PE_TRY(ensure_gemm_work(p, need));
                if (gemm_launch<T>(sh, epi, c, p->gw, p->st) != hipSuccess) continue;
                const int reps = 10;
                PE_HIP(hipEventRecord(e0, p->st));
                for (int i = 0; i < reps; ++i) PE_HIP(gemm_launch<T>(sh, epi, c, p->gw, p->st));
                PE_HIP(hipEventRecord(e1, p->st));
                PE_HIP(hipEventSynchronize(e1));
                float ms = 0.f;
                PE_HIP(hipEventElapsedTime(&ms, e0, e1));
                if (getenv("PE_VERBOSE") && atoi(getenv("PE_VERBOSE")) > 1)
                    fprintf(stderr, "[libpe]   candidate %dx%d bk2=%d splitk=%d wsk=%d: %.2f us\n", c.br, c.bs,
                            c.bk2, c.splitk, c.wsk, ms / reps * 1e3);
                if (ms / reps < best) {
                    best = ms / reps;
                    *best_out = c;
                }
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(scratch);
    if (getenv("PE_VERBOSE"))
        fprintf(stderr, "[libpe] tuned %s Mr=%d Ns=%d K=%d: tile %dx%d bk2=%d splitk=%d wsk=%d (%.2f us)\n",
                fp32 ? "f32" : "f64", sh.Mr, sh.Ns, kext, best_out->br, best_out->bs, best_out->bk2,
                best_out->splitk, best_out->wsk, best * 1e3);
    return PE_OK;
}

constexpr int PROBE_ACC_PER_ROUND = 16;  // independent products per wave per round (k_probe_mfma*)

enum {
    SITE_NONE = -1,
    SITE_FINE_STEP = 7,
    SITE_ANCHOR = 2,
    SITE_NORM = 3,
    SITE_TRAJ = 6,
    SITE_ADJ_STEP = 8,
    SITE_WR_RHS = 9,
    SITE_WR_WSTEP = 10,
    SITE_COARSE_SCAN = 11,
    SITE_REFINE_RES = 12,
    SITE_REFINE_CORR = 13
};

template <typename T>
pe_status gemm(pe_problem p, const GemmShape& sh, const Epi& epi, int force_splitk = 0, int kind = -1,
               int site = SITE_NONE) {
    if (sh.Mr <= 0 || sh.Ns <= 0) return PE_OK;
    TileCfg cfg = choose_tiles(sh, sizeof(T) == 4, p->n_cu);
    if (force_splitk > 0) {
        cfg.splitk = force_splitk;
    } else if (p->force_tiles_on && sh.Mr > 4) {
        cfg = p->force_tiles;
    } else if (p->force_wsk.wsk > 0 && sh.Mr > 4 && sh.Mr <= 64) {
        cfg = p->force_wsk;
    } else if (site != SITE_NONE && p->autotune && sh.Mr > 4) {
        const std::vector<int> key = tune_key(site, sizeof(T) == 4, sh);
        auto it = p->tuned.find(key);
        if (it == p->tuned.end()) {
            TileCfg c;
            PE_TRY(tune<T>(p, sh, &c));
            p->tuned[key] = c;
            tune_cache_store(key, c);
            cfg = c;
        } else {
            cfg = it->second;
        }
    }
    PE_TRY(ensure_gemm_work(p, gemm_part_bytes(sh, cfg, sizeof(T))));
    if (kind >= 0 && kind < PE_PROF_KINDS) {
        const bool gemv = sh.Mr <= 4;
        p->last_cfg[kind][0] = gemv ? 0 : cfg.br;
        p->last_cfg[kind][1] = gemv ? 0 : cfg.bs;
        p->last_cfg[kind][2] = gemv ? 0 : cfg.wsk > 0 ? -cfg.wsk : (sizeof(T) == 4 ? 32 : 16) << cfg.bk2;
        p->last_cfg[kind][3] = gemv ? 0 : cfg.splitk;
    }
    size_t slot;
    PE_TRY(prof_begin(p, kind, &slot));
    // with split-K the reduction kernel is timed as its own class
    struct Hook {
        pe_problem p;
        size_t slot;
        pe_status st;
    } hook{p, slot, PE_OK};
    if (slot != (size_t)-1) {
        p->gw.between = [](void* a) {
            Hook* h = (Hook*)a;
            size_t s2 = (size_t)-1;
            h->st = prof_end(h->p, h->slot);
            if (h->st == PE_OK) h->st = prof_begin(h->p, PE_PROF_SPLITK_REDUCE, &s2);
            h->slot = s2;
        };
        p->gw.between_arg = &hook;
    }
    hipError_t e = gemm_launch<T>(sh, epi, cfg, p->gw, p->st);
    p->gw.between = nullptr;
    p->gw.between_arg = nullptr;
    if (e != hipSuccess)
        return fail(PE_ERR_HIP, std::string("GEMM launch failed: ") + hipGetErrorString(e));
    PE_TRY(hook.st);
    PE_TRY(prof_end(p, hook.slot));
    return PE_OK;
}

GemmShape shape(int Mr, int Ns, const void* A, long lda, const void* B, long ldb, int k0, int k1) {
    GemmShape s;
    s.Mr = Mr;
    s.Ns = Ns;
    s.A = A;
    s.lda = lda;
    s.B = B;
    s.ldb = ldb;
    s.s_split = Ns;
    s.k0a = s.k0b = k0;
    s.k1a = s.k1b = k1;
    return s;
}

Epi store_epi(double* C, long ldc, double alpha = 1.0, const double* C0 = nullptr, long ldc0 = 0,
              double beta = 0.0) {
    Epi e;
    e.mode = EPI_STORE;
    e.C = C;
    e.ldc = ldc;
    e.alpha = alpha;
    e.C0 = C0;
    e.ldc0 = ldc0;
    e.beta = beta;
    return e;
}

// ---------------------------------------------------------------------------
// FP64 Cholesky (blocked, right-looking, 64-wide panels) and the inverse
// K^-1 = L^-T L^-1, all on the GPU. Aemb (nf x nf, nf multiple of 64) is
// overwritten by the factor. On a non-positive pivot returns PE_ERR_NOT_SPD.
// ---------------------------------------------------------------------------
pe_status factor_inverse(pe_problem p, double* Aemb, int nf, double* Kinv, const char* name, int d,
                         double* Zt_out = nullptr) {
    const int nb = 64, nblk = nf / nb;
    TmpList tmpl(p->st);
    std::vector<void*>& tmp = tmpl.v;
    double *Dinv = nullptr, *Zt = nullptr, *T = nullptr;
    int* info = nullptr;
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(p->st);
        free_list(tmp);
    };
    pe_status s;
    if ((s = dalloc_t(p, tmp, &Dinv, (size_t)nblk * nb * nb)) < 0 ||
        (s = dalloc_t(p, tmp, &Zt, (size_t)nf * nf)) < 0 || (s = dalloc_t(p, tmp, &T, (size_t)nf * nb)) < 0 ||
        (s = dalloc_t(p, tmp, &info, 2)) < 0) {
        cleanup();
        return s;
    }
    int h_info[2] = {0, -1};
    PE_HIP(hipMemcpyAsync(info, h_info, sizeof(h_info), hipMemcpyHostToDevice, p->st));
    for (int j = 0; j < nblk; ++j) {
        PE_HIP(chol_diag(Aemb, nf, j, Dinv, info, p->st));
        const int m = nf - (j + 1) * nb;
        if (m <= 0) break;
        double* panel = Aemb + (long)(j + 1) * nb * nf + (long)j * nb;
        // panel <- panel * L_jj^-T (in place: one column tile, no split-K)
        if ((s = gemm<double>(p, shape(m, nb, panel, nf, Dinv + (long)j * nb * nb, nb, 0, nb),
                              store_epi(panel, nf), 1)) < 0) {
            cleanup();
            return s;
        }
        // trailing update  A22 -= L21 L21^T
        double* trail = Aemb + (long)(j + 1) * nb * nf + (long)(j + 1) * nb;
        if ((s = gemm<double>(p, shape(m, m, panel, nf, panel, nf, 0, nb),
                              store_epi(trail, nf, -1.0, trail, nf, 1.0))) < 0) {
            cleanup();
            return s;
        }
    }
    PE_HIP(hipMemcpyAsync(h_info, info, sizeof(h_info), hipMemcpyDeviceToHost, p->st));
    PE_HIP(hipStreamSynchronize(p->st));
    if (h_info[0] != 0) {
        cleanup();
        const int piv = h_info[1];
        return fail(PE_ERR_NOT_SPD, std::string("Cholesky of ") + name + " failed at pivot " +
                                        std::to_string(piv) + (piv >= d ? " (padding)" : ""));
    }
    // forward substitution for Zt = L^-T (row c of Zt = column c of L^-1)
    PE_HIP(hipMemsetAsync(Zt, 0, (size_t)nf * nf * sizeof(double), p->st));
    for (int i = 0; i < nblk; ++i) {
        Epi e = store_epi(T, nb, -1.0);
        e.diag_add = 1.0;
        e.diag_off = i * nb;
        if ((s = gemm<double>(p, shape(nf, nb, Zt, nf, Aemb + (long)i * nb * nf, nf, 0, i * nb), e)) < 0 ||
            (s = gemm<double>(p, shape(nf, nb, T, nb, Dinv + (long)i * nb * nb, nb, 0, nb),
                              store_epi(Zt + (long)i * nb, nf))) < 0) {
            cleanup();
            return s;
        }
    }
    s = PE_OK;
    if (Kinv) s = gemm<double>(p, shape(nf, nf, Zt, nf, Zt, nf, 0, nf), store_epi(Kinv, nf));
    if (s == PE_OK && Zt_out) {
        hipError_t e = hipMemcpyAsync(Zt_out, Zt, sizeof(double) * nf * nf, hipMemcpyDeviceToDevice, p->st);
        if (e != hipSuccess) s = fail(PE_ERR_HIP, "copy of the inverse factor failed");
    }
    cleanup();
    return s;
}

// step operators for step size h: fills Z (Dp x Dp) and, if W != null, W (Dp x 2Dp)
pe_status build_step_ops(pe_problem p, double h, const double* M11, const double* M12,
                         const double* M22inv, const double* A11, const double* A12,
                         const double* A21, const double* A22, double* Z, double* W) {
    const int d1 = p->d1, d2 = p->d2, d1p = p->d1p, d2p = p->d2p, Dp = p->Dp;
    const int nf1 = roundup(d1, 64);
    TmpList tmpl(p->st);
    std::vector<void*>& tmp = tmpl.v;
    double *K = nullptr, *Kinv = nullptr, *Q = nullptr;
    pe_status s;
    if ((s = dalloc_t(p, tmp, &K, (size_t)nf1 * nf1)) < 0 || (s = dalloc_t(p, tmp, &Kinv, (size_t)nf1 * nf1)) < 0 ||
        (s = dalloc_t(p, tmp, &Q, (size_t)std::max(d2p, 1) * std::max(d1p, 1))) < 0) {
        free_list(tmp);
        return s;
    }
    auto done = [&](pe_status r) {
        (void)hipStreamSynchronize(p->st);
        free_list(tmp);
        return r;
    };
    // M11, A11 are d1p x d1p padded copies
    PE_HIP(shifted_embed(K, nf1, A11, M11, d1p, d1, 1.0 / h, p->st));
    char name[64];
    snprintf(name, sizeof(name), "M11/%.3e + A11", h);
    if ((s = factor_inverse(p, K, nf1, Kinv, name, d1)) < 0) return done(s);
    PE_HIP(hipMemsetAsync(Z, 0, (size_t)Dp * Dp * sizeof(double), p->st));
    PE_HIP(place(Z, Dp, 0, 0, Kinv, nf1, d1, d1, 1.0, 0, p->st));
    if (d2 > 0) {
        // Q = h M22^-1 A21  (d2 x d1): C[j][i] = h sum_k M22inv[j][k] A12[i][k]
        PE_HIP(hipMemsetAsync(Q, 0, (size_t)d2p * d1p * sizeof(double), p->st));
        const int nf2 = roundup(d2, 64);
        if ((s = gemm<double>(p, shape(d2, d1, M22inv, nf2, A12, d2p, 0, d2p), store_epi(Q, d1p, h))) < 0)
            return done(s);
        // Z[w rows][u cols] = -Q K^-1
        if ((s = gemm<double>(p, shape(d2, d1, Q, d1p, Kinv, nf1, 0, d1p),
                              store_epi(Z + (long)d1p * Dp, Dp, -1.0))) < 0)
            return done(s);
        PE_HIP(place(Z, Dp, d1p, d1p, M22inv, nf2, d2, d2, h, 0, p->st));
    }
    if (W) {
        const long ldw = 2L * Dp;
        PE_HIP(hipMemsetAsync(W, 0, (size_t)Dp * ldw * sizeof(double), p->st));
        // u rows: [0 | A11 | A12 | M12/h]
        PE_HIP(place(W, ldw, 0, d1p, A11, d1p, d1, d1, 1.0, 0, p->st));
        if (d2 > 0) {
            PE_HIP(place(W, ldw, 0, 2 * d1p, A12, d2p, d1, d2, 1.0, 0, p->st));
            PE_HIP(place(W, ldw, 0, 2 * d1p + d2p, M12, d2p, d1, d2, 1.0 / h, 0, p->st));
            // w rows: [M21/h | A21 | A22 | 0]
            PE_HIP(place(W, ldw, d1p, 0, M12, d2p, d2, d1, 1.0 / h, 1, p->st));
            PE_HIP(place(W, ldw, d1p, d1p, A21, d1p, d2, d1, 1.0, 0, p->st));
            PE_HIP(place(W, ldw, d1p, 2 * d1p, A22, d2p, d2, d2, 1.0, 0, p->st));
        }
    }
    return done(PE_OK);
}

// Second operator of the transposed fine step, Yop = [A; A + Mh] (2Dp x Dp):
// A the full stiffness (Dp x Dp, symmetric) and Mh = [[0, M12/h], [M21/h, 0]]
// the mass coupling of the history terms of eqs. (2.4)-(2.5). M12 is d1 x d2
// with leading dimension ld12.
pe_status build_adj_state_op(pe_problem p, const double* A, const double* M12, long ld12, double h, double* Y) {
    const int d1 = p->d1, d2 = p->d2, d1p = p->d1p, Dp = p->Dp;
    PE_HIP(place(Y, Dp, 0, 0, A, Dp, Dp, Dp, 1.0, 0, p->st));
    PE_HIP(place(Y, Dp, Dp, 0, A, Dp, Dp, Dp, 1.0, 0, p->st));
    if (d2 > 0) {
        PE_HIP(place(Y, Dp, Dp, d1p, M12, ld12, d1, d2, 1.0 / h, 0, p->st, 1));
        PE_HIP(place(Y, Dp, Dp + d1p, 0, M12, ld12, d2, d1, 1.0 / h, 1, p->st, 1));
    }
    return PE_OK;
}

// Mass-whitened blocks for the mixed fine sweep: with L1 L1^T = M11 and
// L2 L2^T = M22 the change of variables u = L1^-T u~, w = L2^-T w~ gives
// M~11 = M~22 = I, M~12 = L1^-1 M12 L2^-T, A~ij = Li^-1 Aij Lj^-T. The
// scheme is the same in these coordinates; its FP32 products are then well
// scaled (the conditioning of M11, M22 no longer amplifies rounding).
pe_status whiten(pe_problem p, std::vector<void*>& tmp, const double* pM11, const double* pM12,
                 const double* pM22, const double* pA11, const double* pA12, const double* pA21,
                 const double* pA22, double** wM12, double** wA11, double** wA12, double** wA21,
                 double** wA22, double** I11, double** I22inv) {
    const int d1 = p->d1, d2 = p->d2, d1p = p->d1p, d2p = p->d2p, Dp = p->Dp;
    const int nf1 = roundup(d1, 64), nf2 = roundup(std::max(d2, 1), 64);
    const int d2q = std::max(d2p, 8);
    double *E1, *Z1, *E2 = nullptr, *Z2 = nullptr, *Li1, *Li2, *X, *M21;
    auto& OL = p->op_allocs;
    PE_TRY(dalloc_t(p, tmp, &E1, (size_t)nf1 * nf1));
    PE_TRY(dalloc_t(p, tmp, &Z1, (size_t)nf1 * nf1));
    PE_TRY(dalloc_t(p, tmp, &Li1, (size_t)d1p * d1p));
    PE_TRY(dalloc_t(p, tmp, &Li2, (size_t)d2q * d2q));
    PE_TRY(dalloc_t(p, tmp, &X, (size_t)std::max(d1p, d2q) * std::max(d1p, d2q)));
    PE_TRY(dalloc_t(p, tmp, &M21, (size_t)d2q * d1p));
    PE_TRY(dalloc_t(p, tmp, wM12, (size_t)d1p * d2q));
    PE_TRY(dalloc_t(p, tmp, wA11, (size_t)d1p * d1p));
    PE_TRY(dalloc_t(p, tmp, wA12, (size_t)d1p * d2q));
    PE_TRY(dalloc_t(p, tmp, wA21, (size_t)d2q * d1p));
    PE_TRY(dalloc_t(p, tmp, wA22, (size_t)d2q * d2q));
    PE_TRY(dalloc_t(p, tmp, I11, (size_t)d1p * d1p));
    PE_TRY(dalloc_t(p, tmp, I22inv, (size_t)nf2 * nf2));
    for (double* z : {*wM12, *wA12}) PE_HIP(hipMemsetAsync(z, 0, sizeof(double) * d1p * d2q, p->st));
    PE_HIP(hipMemsetAsync(*wA21, 0, sizeof(double) * d2q * d1p, p->st));
    PE_HIP(hipMemsetAsync(*wA22, 0, sizeof(double) * d2q * d2q, p->st));
    PE_HIP(hipMemsetAsync(*wA11, 0, sizeof(double) * d1p * d1p, p->st));
    PE_HIP(hipMemsetAsync(Li1, 0, sizeof(double) * d1p * d1p, p->st));
    PE_HIP(hipMemsetAsync(Li2, 0, sizeof(double) * d2q * d2q, p->st));
    PE_HIP(eye(*I11, d1p, d1, p->st));
    PE_HIP(eye(*I22inv, nf2, d2, p->st));
    // factors L (lower part of E) and L^-T (Z)
    PE_HIP(shifted_embed(E1, nf1, pM11, nullptr, d1p, d1, 0.0, p->st));
    PE_TRY(factor_inverse(p, E1, nf1, nullptr, "M11", d1, Z1));
    PE_HIP(tril(E1, nf1, p->st));
    PE_HIP(place(Li1, d1p, 0, 0, Z1, nf1, d1, d1, 1.0, 1, p->st));
    if (d2 > 0) {
        PE_TRY(dalloc_t(p, tmp, &E2, (size_t)nf2 * nf2));
        PE_TRY(dalloc_t(p, tmp, &Z2, (size_t)nf2 * nf2));
        PE_HIP(shifted_embed(E2, nf2, pM22, nullptr, d2p, d2, 0.0, p->st));
        PE_TRY(factor_inverse(p, E2, nf2, nullptr, "M22", d2, Z2));
        PE_HIP(tril(E2, nf2, p->st));
        PE_HIP(place(Li2, d2q, 0, 0, Z2, nf2, d2, d2, 1.0, 1, p->st));
    }
    // transforms (block diagonal, Dp x Dp)
    PE_TRY(dalloc_t(p, OL, &p->Tin64, (size_t)Dp * Dp));
    PE_TRY(dalloc_t(p, OL, &p->Tout64, (size_t)Dp * Dp));
    PE_TRY(dalloc_t(p, OL, &p->Linv64, (size_t)Dp * Dp));
    for (double* m : {p->Tin64, p->Tout64, p->Linv64})
        PE_HIP(hipMemsetAsync(m, 0, sizeof(double) * Dp * Dp, p->st));
    PE_HIP(place(p->Tin64, Dp, 0, 0, E1, nf1, d1, d1, 1.0, 1, p->st));
    PE_HIP(place(p->Tout64, Dp, 0, 0, Z1, nf1, d1, d1, 1.0, 0, p->st));
    PE_HIP(place(p->Linv64, Dp, 0, 0, Z1, nf1, d1, d1, 1.0, 1, p->st));
    if (d2 > 0) {
        PE_HIP(place(p->Tin64, Dp, d1p, d1p, E2, nf2, d2, d2, 1.0, 1, p->st));
        PE_HIP(place(p->Tout64, Dp, d1p, d1p, Z2, nf2, d2, d2, 1.0, 0, p->st));
        PE_HIP(place(p->Linv64, Dp, d1p, d1p, Z2, nf2, d2, d2, 1.0, 1, p->st));
    }
    // A~11 = L1^-1 A11 L1^-T  (two NT products)
    PE_HIP(hipMemsetAsync(X, 0, sizeof(double) * std::max(d1p, d2q) * std::max(d1p, d2q), p->st));
    PE_TRY(gemm<double>(p, shape(d1, d1, Li1, d1p, pA11, d1p, 0, d1p), store_epi(X, d1p)));
    PE_TRY(gemm<double>(p, shape(d1, d1, X, d1p, Li1, d1p, 0, d1p), store_epi(*wA11, d1p)));
    if (d2 > 0) {
        // A~12 = L1^-1 A12 L2^-T (A12 as rows of A21), M~12 likewise
        PE_HIP(hipMemsetAsync(X, 0, sizeof(double) * std::max(d1p, d2q) * std::max(d1p, d2q), p->st));
        PE_TRY(gemm<double>(p, shape(d1, d2, Li1, d1p, pA21, d1p, 0, d1p), store_epi(X, d2p)));
        PE_TRY(gemm<double>(p, shape(d1, d2, X, d2p, Li2, d2q, 0, d2p), store_epi(*wA12, d2p)));
        PE_HIP(hipMemsetAsync(M21, 0, sizeof(double) * d2q * d1p, p->st));
        PE_HIP(place(M21, d1p, 0, 0, pM12, d2p, d2, d1, 1.0, 1, p->st));
        PE_HIP(hipMemsetAsync(X, 0, sizeof(double) * std::max(d1p, d2q) * std::max(d1p, d2q), p->st));
        PE_TRY(gemm<double>(p, shape(d1, d2, Li1, d1p, M21, d1p, 0, d1p), store_epi(X, d2p)));
        PE_TRY(gemm<double>(p, shape(d1, d2, X, d2p, Li2, d2q, 0, d2p), store_epi(*wM12, d2p)));
        PE_HIP(place(*wA21, d1p, 0, 0, *wA12, d2p, d2, d1, 1.0, 1, p->st));
        PE_HIP(hipMemsetAsync(X, 0, sizeof(double) * std::max(d1p, d2q) * std::max(d1p, d2q), p->st));
        PE_TRY(gemm<double>(p, shape(d2, d2, Li2, d2q, pA22, d2p, 0, d2p), store_epi(X, d2p)));
        PE_TRY(gemm<double>(p, shape(d2, d2, X, d2p, Li2, d2q, 0, d2p), store_epi(*wA22, d2p)));
    }
    // whitened full stiffness for the anchor residual
    PE_TRY(dalloc_t(p, OL, &p->Aw64, (size_t)Dp * Dp));
    PE_HIP(hipMemsetAsync(p->Aw64, 0, sizeof(double) * Dp * Dp, p->st));
    PE_HIP(place(p->Aw64, Dp, 0, 0, *wA11, d1p, d1, d1, 1.0, 0, p->st));
    if (d2 > 0) {
        PE_HIP(place(p->Aw64, Dp, 0, d1p, *wA12, d2p, d1, d2, 1.0, 0, p->st));
        PE_HIP(place(p->Aw64, Dp, d1p, 0, *wA21, d1p, d2, d1, 1.0, 0, p->st));
        PE_HIP(place(p->Aw64, Dp, d1p, d1p, *wA22, d2p, d2, d2, 1.0, 0, p->st));
    }
    return PE_OK;
}

pe_status ensure_workspace(pe_problem p, int B) {
    if (B <= p->B_cap) return PE_OK;
    PE_HIP(hipStreamSynchronize(p->st));
    graphs_clear(p);
    free_list(p->ws_allocs);
    const size_t N = p->N, Dp = p->Dp, Sx = p->Sx, Bs = B;
    auto& L = p->ws_allocs;
    PE_TRY(dalloc_t(p, L, &p->Xk[0], Bs * (N + 1) * Sx));
    PE_TRY(dalloc_t(p, L, &p->Xk[1], Bs * (N + 1) * Sx));
    PE_TRY(dalloc_t(p, L, &p->Fbuf, Bs * N * Sx));
    for (int i = 0; i < 2; ++i) {
        PE_TRY(dalloc_t(p, L, &p->Dl64[i], Bs * Sx));
        PE_TRY(dalloc_t(p, L, &p->Dl32[i], Bs * Sx));
    }
    PE_TRY(dalloc_t(p, L, &p->Xa, Bs * N * Dp));
    PE_TRY(dalloc_t(p, L, &p->Ya, Bs * N * Dp));
    PE_TRY(dalloc_t(p, L, &p->R64, Bs * N * Dp));
    PE_TRY(dalloc_t(p, L, &p->dev64[0], Bs * N * 2 * Dp));
    PE_TRY(dalloc_t(p, L, &p->dev64[1], Bs * N * 2 * Dp));
    if (p->prec == PE_MIXED) {
        PE_TRY(dalloc_t(p, L, &p->dev32[0], Bs * N * 2 * Dp));
        PE_TRY(dalloc_t(p, L, &p->dev32[1], Bs * N * 2 * Dp));
    }
    if (p->refine) {
        PE_TRY(dalloc_t(p, L, &p->Vr, Bs * N * 2 * Dp));
        PE_TRY(dalloc_t(p, L, &p->AxU, Bs * N * (size_t)p->d1p));
        PE_TRY(dalloc_t(p, L, &p->res32, Bs * N * (size_t)p->d1p));
    }
    PE_TRY(dalloc_t(p, L, &p->E, Bs * (N + 1) * Sx));
    PE_TRY(dalloc_t(p, L, &p->Yn, Bs * (N + 1) * Dp));
    PE_TRY(dalloc_t(p, L, &p->io, Bs * (N + 1) * Sx));
    PE_TRY(dalloc_t(p, L, &p->Jd, Bs * (N + 1)));
    PE_TRY(dalloc_t(p, L, &p->nrm, Bs * (N + 1)));
    PE_TRY(dalloc_t(p, L, &p->x0p, Bs * Dp));
    PE_TRY(dalloc_t(p, L, &p->active_d, Bs));
    p->B_cap = B;
    return PE_OK;
}

// Dense per-interval source table out[(b, n)][s] = sum_r G[s][r] H[b][r][n]
// (H: B x R x N amplitudes on the handle's G); out_w (nullable) gets the
// whitened copy Linv out.
pe_status interval_table(pe_problem p, int B, const double* H, double* out, double* out_w) {
    const int Dp = p->Dp, N = p->N, R = p->R, Rp = p->Rp;
    double* Ht = nullptr;
    TmpList tmpl(p->st);
    std::vector<void*>& tmp = tmpl.v;
    PE_TRY(dalloc_t(p, tmp, &Ht, (size_t)B * N * Rp));
    pe_status s = PE_OK;
    if (hipMemsetAsync(Ht, 0, sizeof(double) * B * N * Rp, p->st) != hipSuccess)
        s = fail(PE_ERR_HIP, "memset failed");
    for (int b = 0; b < B && s == PE_OK; ++b)
        if (place(Ht + (long)b * N * Rp, Rp, 0, 0, H + (long)b * R * N, N, N, R, 1.0, 1, p->st) != hipSuccess)
            s = fail(PE_ERR_HIP, "source transpose failed");
    if (s == PE_OK) s = gemm<double>(p, shape(B * N, Dp, Ht, Rp, p->Gs, Rp, 0, Rp), store_epi(out, Dp));
    if (s == PE_OK && out_w)
        s = gemm<double>(p, shape(B * N, Dp, out, Dp, p->Linv64, Dp, 0, Dp), store_epi(out_w, Dp));
    (void)hipStreamSynchronize(p->st);
    free_list(tmp);
    return s;
}

// source of the fused fine step with other amplitudes (same G, same time
// layout): kind, amplitudes and, for dense tables, the per-interval Z_h F
// in the sweep's coordinates
struct SrcView {
    int kind = 0;
    const double* Hs = nullptr;
    const double* ZFint = nullptr;
    const double* Fint_w = nullptr;  // the table itself, whitened (refinement residual, PE_MIXED)
};

// source fields of the fused fine step: Z_h G (or the per-interval Z_h F)
void source_fields_step(pe_problem p, Epi& e) {
    e.src_kind = p->src_set ? p->src_kind : 0;
    e.Gs = p->ZGs;
    e.Hs = p->Hs;
    e.R = p->Rp;
    e.Tlen = p->Tlen;
    e.time_mode = p->time_mode;
    e.P = p->P;
    e.N = p->N;
    e.Fint = p->ZFint;
    e.ldf = p->Dp;
}

void source_fields(pe_problem p, Epi& e, bool whitened = false) {
    e.src_kind = p->src_set ? p->src_kind : 0;
    e.Gs = whitened ? p->Gs_w : p->Gs;
    e.Hs = p->Hs;
    e.R = p->Rp;
    e.Tlen = p->Tlen;
    e.time_mode = p->time_mode;
    e.P = p->P;
    e.N = p->N;
    e.Fint = whitened ? p->Fint_w : p->Fint;
    e.ldf = p->Dp;
}

// ---------------------------------------------------------------------------
// propagators
// ---------------------------------------------------------------------------
// F on B*N columns: anchors Xsrc[b][n - n_shift] (row stride ldXb per sample,
// zero for n < n_shift) -> Y (B*N x Dp). Without the source this is the
// homogeneous propagator; with accumulate the result is added to Y.
// sv (nullable) replaces the source amplitudes; traj (nullable) receives the
// state after every fine step, row (b*N + n)*P + p (in the sweep's
// coordinates: whitened in PE_MIXED).
pe_status fine_sweep(pe_problem p, int B, const double* Xsrc, long ldXb, double* Y, bool with_source = true,
                     int n_shift = 0, bool accumulate = false, const SrcView* sv = nullptr,
                     double* traj = nullptr) {
    const int Dp = p->Dp, d1p = p->d1p, d2p = p->d2p, Sx = p->Sx;
    const int rows = B * p->N;
    const bool mixed = p->prec == PE_MIXED;
    const bool hist = p->hist == PE_HIST_CARRY;
    // PE_MIXED_REFINE: the sweeps at the state's scale (with the source),
    // and with refine = 2 also those on iterate changes
    const bool refine = mixed && p->refine && (with_source || p->refine > 1);
    // whitening x~ = Tin x (block diagonal) of rows x Dp: in -> out
    auto whiten_rows = [&](const double* in, double* out, const double* T) -> pe_status {
        GemmShape gt = shape(rows, Dp, in, Dp, T, Dp, 0, d1p);
        gt.s_split = d1p;
        gt.k0b = d1p;
        gt.k1b = Dp;
        return gemm<double>(p, gt, store_epi(out, Dp), 0, PE_PROF_ANCHOR, SITE_ANCHOR);
    };
    if (!mixed) {
        PE_HIP(fine_init(Xsrc, ldXb, -n_shift, p->N, p->Xa, p->dev64[0], nullptr, B, p->N, Dp, p->st, Sx));
    } else {
        // anchors into whitened coordinates: Xa = Tin x
        PE_HIP(fine_init(Xsrc, ldXb, -n_shift, p->N, p->R64, p->dev64[0], p->dev32[0], B, p->N, Dp, p->st, Sx));
        PE_TRY(whiten_rows(p->R64, p->Xa, p->Tin64));
    }
    if (hist) {
        // the carried change over the last fine step starts the step state's
        // history (whitened like the state in PE_MIXED)
        PE_HIP(gather_rows(Xsrc, ldXb, Sx, Dp, -n_shift, p->N, p->R64, B, p->N, Dp, p->st));
        if (mixed) PE_TRY(whiten_rows(p->R64, p->Ya, p->Tin64));
        PE_HIP(hist_put(mixed ? p->Ya : p->R64, p->dev64[0], mixed ? p->dev32[0] : nullptr, rows, Dp, d1p, p->st));
    }
    // anchor term Z_h A x_a (FP64, once per sweep)
    PE_TRY(gemm<double>(p, shape(rows, Dp, p->Xa, Dp, p->ZA64, Dp, 0, Dp), store_epi(p->Ya, Dp), 0,
                        PE_PROF_ANCHOR, SITE_ANCHOR));
    // refinement: the u rows of A x_a (FP64, once per sweep), the anchor
    // part of the implicit equation's residual
    if (refine)
        PE_TRY(gemm<double>(p, shape(rows, d1p, p->Xa, Dp, p->Aw64, Dp, 0, Dp), store_epi(p->AxU, d1p), 0,
                            PE_PROF_ANCHOR, SITE_ANCHOR));
    const long ldS = 2L * Dp;
    // the fused step's epilogue fields (step index and state buffers are per step)
    Epi eb;
    eb.mode = EPI_FSTEP;
    eb.base = p->Ya;
    eb.ldb = Dp;
    source_fields_step(p, eb);
    if (sv) {
        eb.src_kind = sv->kind;
        eb.Hs = sv->Hs;
        eb.Fint = sv->ZFint;
    }
    if (!with_source) eb.src_kind = 0;
    eb.cols_per_b = p->N;
    eb.n_fixed = -1;
    eb.ldd = ldS;
    eb.d1p = d1p;
    eb.d2p = d2p;
    eb.xa = p->Xa;
    eb.ldtraj = (long)p->P * Dp;
    // u-rows of Z_h W_h have no du_prev columns
    GemmShape gs = shape(rows, Dp, mixed ? (const void*)p->dev32[0] : (const void*)p->dev64[0], ldS,
                         mixed ? (const void*)p->ZW32 : (const void*)p->ZW64, ldS, 0, 0);
    gs.s_split = d1p;
    gs.k0a = d1p;
    gs.k1a = 2 * Dp;
    gs.k0b = 0;
    gs.k1b = 2 * Dp;
    bool done = false;
    if (p->persistent && rows <= 64 && !hist && !refine) {
        int& grid = p->pers_grid[mixed ? 1 : 0];
        if (grid < 0) {
            grid = mixed ? fine_sweep_persistent_grid<float>() : fine_sweep_persistent_grid<double>();
            // optional cap on the co-resident grid (fewer work-groups per grid barrier)
            if (const char* gc = getenv("PE_PERSISTENT_GRID")) {
                const int cap = atoi(gc);
                if (cap > 0 && cap < grid) grid = cap;
            }
        }
        if (grid > 0) {
            // split count: about one (tile, split) item per co-resident work-group,
            // at least two K tiles per split
            const int n_tiles = (Dp + 31) / 32;
            const int bk = mixed ? 64 : 32;
            const int ktiles = (2 * Dp + bk - 1) / bk;
            int sk = std::max(1, std::min(16, grid / n_tiles));
            while (sk > 1 && ktiles / sk < 2) --sk;
            const size_t elem = mixed ? sizeof(float) : sizeof(double);
            PE_TRY(ensure_gemm_work(p, (size_t)sk * rows * Dp * elem));
            p->last_cfg[PE_PROF_FINE_SWEEP][0] = 64;
            p->last_cfg[PE_PROF_FINE_SWEEP][1] = 32;
            p->last_cfg[PE_PROF_FINE_SWEEP][2] = bk;
            p->last_cfg[PE_PROF_FINE_SWEEP][3] = sk;
            size_t slot;
            PE_TRY(prof_begin(p, PE_PROF_FINE_SWEEP, &slot));
            const void* A1 = mixed ? (const void*)p->dev32[1] : (const void*)p->dev64[1];
            hipError_t e = mixed ? fine_sweep_persistent<float>(gs, A1, eb, p->dev64[0], p->dev64[1], p->dev32[0],
                                                                p->dev32[1], traj, p->P, grid, sk, p->gw.part,
                                                                p->gw.part_bytes, p->st)
                                 : fine_sweep_persistent<double>(gs, A1, eb, p->dev64[0], p->dev64[1], nullptr,
                                                                 nullptr, traj, p->P, grid, sk, p->gw.part,
                                                                 p->gw.part_bytes, p->st);
            if (e == hipSuccess) {
                PE_TRY(prof_end(p, slot));
                done = true;
            } else {
                (void)hipGetLastError();
                hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
                if (hipStreamIsCapturing(p->st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
                    // not capturable: the caller keeps this sweep eager, so
                    // replays and eager runs take the same path
                    return fail(PE_ERR_HIP, "persistent fine sweep cannot be captured");
                // not launchable on this device: per-step launches from now on
                p->persistent = 0;
                if (slot != (size_t)-1) PE_TRY(prof_end(p, slot));
            }
        }
    }
    for (int step = 0; step < p->P && !done; ++step) {
        const int c = step & 1;
        GemmShape g = gs;
        g.A = mixed ? (const void*)p->dev32[c] : (const void*)p->dev64[c];
        if (step == 0 && !hist) {  // zero deviation: empty K ranges
            g.k0a = g.k1a = g.k0b = g.k1b = 0;
        }
        Epi e = eb;
        e.p_step = step;
        e.din = p->dev64[c];
        e.dev64 = p->dev64[1 - c];
        e.dev32 = mixed ? p->dev32[1 - c] : nullptr;
        e.traj = traj ? traj + (long)step * Dp : nullptr;
        const int kind = step > 0 ? PE_PROF_FINE_STEP : PE_PROF_FINE_FIRST;
        // the first step of a fresh history has no FP32 product (zero
        // deviation): nothing to refine
        const bool ref_step = refine && (step > 0 || hist);
        if (ref_step) e.vr = p->Vr;
        if (mixed)
            PE_TRY(gemm<float>(p, g, e, 0, kind, SITE_FINE_STEP));
        else
            PE_TRY(gemm<double>(p, g, e, 0, kind, SITE_FINE_STEP));
        if (ref_step) {
            // FP64 residual of the implicit V_H1 equation (eq. (2.4)) at the
            // FP32 step's u': r = F~1(t) - (A~ x_a)_u - K~ du - A~11 (u - u_a)
            // - A~12 (w - w_a) - M~12 dw_prev / h, as Wr [du + u - u_a | w - w_a
            // | dw_prev] and the diagonal term du / h
            Epi er;
            er.mode = EPI_RESID;
            er.R32 = p->res32;
            er.ldr = d1p;
            er.base = p->AxU;
            er.ldb = d1p;
            er.dres = p->Vr + d1p + 2 * d2p;
            er.lddres = ldS;
            er.cres = 1.0 / p->dtf;
            source_fields(p, er, true);
            if (sv) {
                er.src_kind = sv->kind;
                er.Hs = sv->Hs;
                er.Fint = sv->Fint_w;
            }
            if (!with_source) er.src_kind = 0;
            er.cols_per_b = p->N;
            er.n_fixed = -1;
            er.p_step = step;
            PE_TRY(gemm<double>(p, shape(rows, d1p, p->Vr, ldS, p->Wr64, ldS, 0, d1p + 2 * d2p), er, 0,
                                PE_PROF_REFINE, SITE_REFINE_RES));
            // FP32 correction of both increments: Z_h[:, u] r
            Epi ec;
            ec.mode = EPI_FCORR;
            ec.dev64 = p->dev64[1 - c];
            ec.dev32 = p->dev32[1 - c];
            ec.ldd = ldS;
            ec.d1p = d1p;
            ec.d2p = d2p;
            ec.traj = e.traj;
            ec.ldtraj = eb.ldtraj;
            PE_TRY(gemm<float>(p, shape(rows, Dp, p->res32, d1p, p->Zc32, d1p, 0, d1p), ec, 0, PE_PROF_REFINE,
                               SITE_REFINE_CORR));
        }
    }
    const double* dfin = p->dev64[p->P & 1];
    if (!mixed) {
        PE_HIP(fine_final(p->Xa, dfin, Y, rows, Dp, d1p, accumulate ? 1 : 0, p->st, Sx));
        // the last step's change: the history handed on
        if (hist) PE_HIP(hist_get(dfin, Y + Dp, Sx, rows, Dp, d1p, accumulate ? 1 : 0, p->st));
    } else {
        // back to the caller's coordinates: Y (+)= Tout (Xa + dev)
        auto unwhiten = [&](double* out) -> pe_status {
            GemmShape gt = shape(rows, Dp, p->R64, Dp, p->Tout64, Dp, 0, d1p);
            gt.s_split = d1p;
            gt.k0b = d1p;
            gt.k1b = Dp;
            return gemm<double>(p, gt, store_epi(out, Sx, 1.0, accumulate ? out : nullptr, Sx, accumulate ? 1.0 : 0.0),
                                0, PE_PROF_ANCHOR, SITE_ANCHOR);
        };
        PE_HIP(fine_final(p->Xa, dfin, p->R64, rows, Dp, d1p, 0, p->st));
        PE_TRY(unwhiten(Y));
        if (hist) {
            PE_HIP(hist_get(dfin, p->R64, Dp, rows, Dp, d1p, 0, p->st));
            PE_TRY(unwhiten(Y + Dp));
        }
    }
    return PE_OK;
}

// Coarse sweep. G is affine, G(x) = Phi_G x + c_n with Phi_G = I - Z_dt A and
// c_n = Z_dt F(t_{n+1}), so the update of eq. (2.7),
//     x_{n+1}^k = G(x_n^k) + F(x_n^{k-1}) - G(x_n^{k-1}),
// is x_{n+1}^k = F(x_n^{k-1}) + Phi_G (x_n^k - x_n^{k-1}): one product per
// coarse step, on the iterate change (FP32 in PE_MIXED: its rounding then
// scales with the change). The initial sweep is x_{n+1}^0 = Phi_G x_n^0 + c_n.
// With carried history the states are [x | delta] (stride Sx = 2Dp), the step
// matrix is [Phi_G; (Phi_G - I)/P] (2Dp x Dp, on x) and c_n = [Z_dt F; Z_dt F / P].
pe_status coarse_sweep_initial(pe_problem p, int B, double* Xk) {
    const int Sx = p->Sx, N = p->N;
    const long ldX = (long)(N + 1) * Sx;
    const bool hist = p->hist == PE_HIST_CARRY;
    const double* cs = hist ? p->CSa : p->CS;
    for (int n = 0; n < N; ++n) {
        Epi e;
        e.mode = EPI_COARSE_INIT;
        e.xout = Xk + (long)(n + 1) * Sx;
        e.ldxo = ldX;
        e.cs = cs ? cs + (long)n * Sx : nullptr;
        e.ldcs = (long)N * Sx;
        PE_TRY(gemm<double>(p, shape(B, Sx, Xk + (long)n * Sx, ldX, hist ? p->PhiA64 : p->PhiG64, p->Dp, 0, p->Dp),
                            e, 0, PE_PROF_COARSE));
    }
    return PE_OK;
}

pe_status coarse_sweep_correct(pe_problem p, int B, double* Xk, const double* Xprev, const int* active) {
    const int Sx = p->Sx, N = p->N;
    const long ldX = (long)(N + 1) * Sx;
    const bool mixed = p->prec == PE_MIXED;
    const bool hist = p->hist == PE_HIST_CARRY;
    int c = 0;
    PE_HIP(zero_fill(mixed ? nullptr : p->Dl64[0], mixed ? p->Dl32[0] : nullptr, (long)B * Sx, p->st));
    for (int n = 0; n < N; ++n) {
        Epi e;
        e.mode = EPI_COARSE_DELTA;
        e.xout = Xk + (long)(n + 1) * Sx;
        e.ldxo = ldX;
        e.xprev = Xprev + (long)(n + 1) * Sx;
        e.fbuf = p->Fbuf + (long)n * Sx;
        e.ldfb = (long)N * Sx;
        e.dl64 = mixed ? nullptr : p->Dl64[1 - c];
        e.dl32 = mixed ? p->Dl32[1 - c] : nullptr;
        e.ldl = Sx;
        e.active = active;
        const int Dp = p->Dp;
        if (mixed)
            PE_TRY(gemm<float>(p, shape(B, Sx, p->Dl32[c], Sx, hist ? p->PhiA32 : p->PhiG32, Dp, 0, Dp), e, 0,
                               PE_PROF_COARSE));
        else
            PE_TRY(gemm<double>(p, shape(B, Sx, p->Dl64[c], Sx, hist ? p->PhiA64 : p->PhiG64, Dp, 0, Dp), e, 0,
                                PE_PROF_COARSE));
        c = 1 - c;
    }
    return PE_OK;
}

// Coarse sweep of one sample as a doubling scan. In change form, with
// d_n = x_n^k - x_n^{k-1} (d_0 = 0), the correction above is the linear
// recurrence
//     d_{n+1} = Phi_G d_n + e_n,    e_n = F(x_n^{k-1}) - x_{n+1}^{k-1},
// so d_n = sum_{j<n} Phi_G^(n-1-j) e_j. Starting from t_n = e_{n-1}, level l
// adds Phi_G^(2^l) t_{n-2^l} to every t_n (rows n <= 2^l read zero rows kept
// in front of the buffer); after ceil(log2 N) levels t_n = d_n, and
// x_n^k = x_n^{k-1} + d_n. One product per level over all N rows replaces N
// dependent coarse steps; the products run in the path's precision on the
// change, as the sequential sweep's do. The powers are formed once per
// problem in FP64 (squarings, with the transposes for the NT products).
pe_status scan_prepare(pe_problem p) {
    if (p->scan_L > 0) return PE_OK;
    const int N = p->N, Dp = p->Dp;
    const bool mixed = p->prec == PE_MIXED;
    int L = 0, L0 = 0;
    while ((1 << L) < N) ++L;
    while ((1 << L0) < N + 1) ++L0;
    const int Z = 1 << (L0 - 1);
    std::vector<void*>& OL = p->scan_allocs;
    TmpList tmpl(p->st);
    std::vector<void*>& tmp = tmpl.v;
    auto done = [&](pe_status r) {
        (void)hipStreamSynchronize(p->st);
        free_list(tmp);
        return r;
    };
    pe_status s;
    p->pow64.assign(L0, nullptr);
    p->pow32.assign(L0, nullptr);
    p->pow64T.assign(L0, nullptr);
    p->pow32T.assign(L0, nullptr);
    p->pow64[0] = p->PhiG64;
    p->pow32[0] = p->PhiG32;
    if ((s = dalloc_t(p, OL, &p->pow64T[0], (size_t)Dp * Dp)) < 0) return done(s);
    PE_HIP(place(p->pow64T[0], Dp, 0, 0, p->PhiG64, Dp, Dp, Dp, 1.0, 1, p->st));
    for (int l = 1; l < L0; ++l) {
        if ((s = dalloc_t(p, OL, &p->pow64[l], (size_t)Dp * Dp)) < 0 ||
            (s = dalloc_t(p, OL, &p->pow64T[l], (size_t)Dp * Dp)) < 0)
            return done(s);
        const double *P = p->pow64[l - 1], *PT = p->pow64T[l - 1];
        // P^2 is the NT product of P with P^T, its transpose that of P^T
        // with P
        if ((s = gemm<double>(p, shape(Dp, Dp, P, Dp, PT, Dp, 0, Dp), store_epi(p->pow64[l], Dp))) < 0 ||
            (s = gemm<double>(p, shape(Dp, Dp, PT, Dp, P, Dp, 0, Dp), store_epi(p->pow64T[l], Dp))) < 0)
            return done(s);
    }
    if (mixed)
        for (int l = 0; l < L; ++l) {
            if (l > 0) {
                if ((s = dalloc_t(p, OL, &p->pow32[l], (size_t)Dp * Dp)) < 0) return done(s);
                PE_HIP(to_f32(p->pow64[l], p->pow32[l], (long)Dp * Dp, p->st));
            }
            if ((s = dalloc_t(p, OL, &p->pow32T[l], (size_t)Dp * Dp)) < 0) return done(s);
            PE_HIP(to_f32(p->pow64T[l], p->pow32T[l], (long)Dp * Dp, p->st));
        }
    const long rows = (long)Z + N + 1;
    for (int c = 0; c < 2; ++c) {
        if ((s = dalloc_t(p, OL, &p->scan64[c], (size_t)rows * Dp)) < 0 ||
            (s = dalloc_t(p, OL, &p->scanA64[c], (size_t)rows * Dp)) < 0)
            return done(s);
        PE_HIP(zero_fill(p->scan64[c], nullptr, rows * Dp, p->st));
        PE_HIP(zero_fill(p->scanA64[c], nullptr, rows * Dp, p->st));
        if (mixed) {
            if ((s = dalloc_t(p, OL, &p->scan32[c], (size_t)rows * Dp)) < 0 ||
                (s = dalloc_t(p, OL, &p->scanA32[c], (size_t)rows * Dp)) < 0)
                return done(s);
            PE_HIP(zero_fill(nullptr, p->scan32[c], rows * Dp, p->st));
            PE_HIP(zero_fill(nullptr, p->scanA32[c], rows * Dp, p->st));
        }
    }
    p->scan_L = L;
    p->scan_L0 = L0;
    return done(PE_OK);
}

// scan operators and buffers of a batch's coarse correction (B samples)
pe_status batch_scan_prepare(pe_problem p, int B) {
    const int N = p->N, Dp = p->Dp;
    int L = 0, L0 = 0;
    while ((1 << L) < N) ++L;       // correction: N terms
    while ((1 << L0) < N + 1) ++L0;  // initial sweep: N + 1 terms (L0 >= 1)
    const int Z = 1 << (L0 - 1);
    if (p->bscan_L == L && p->bscan_L0 == L0 && p->bscan_B == B) return PE_OK;
    PE_HIP(hipStreamSynchronize(p->st));
    free_list(p->bscan_allocs);
    p->bscan_L = p->bscan_L0 = -1;
    std::vector<void*>& OL = p->bscan_allocs;
    p->bpow32.assign(L0, nullptr);
    p->bpow32[0] = p->PhiG32;
    if (L0 > 1) {
        TmpList tmpl(p->st);
        std::vector<void*>& tmp = tmpl.v;
        double *P, *PT, *Q, *QT;
        PE_TRY(dalloc_t(p, tmp, &P, (size_t)Dp * Dp));
        PE_TRY(dalloc_t(p, tmp, &PT, (size_t)Dp * Dp));
        PE_TRY(dalloc_t(p, tmp, &Q, (size_t)Dp * Dp));
        PE_TRY(dalloc_t(p, tmp, &QT, (size_t)Dp * Dp));
        PE_HIP(hipMemcpyAsync(P, p->PhiG64, sizeof(double) * Dp * Dp, hipMemcpyDeviceToDevice, p->st));
        PE_HIP(place(PT, Dp, 0, 0, p->PhiG64, Dp, Dp, Dp, 1.0, 1, p->st));
        for (int l = 1; l < L0; ++l) {
            // P^2 as the NT product of P with P^T (and its transpose, for the next level)
            PE_TRY(gemm<double>(p, shape(Dp, Dp, P, Dp, PT, Dp, 0, Dp), store_epi(Q, Dp)));
            if (l + 1 < L0) PE_TRY(gemm<double>(p, shape(Dp, Dp, PT, Dp, P, Dp, 0, Dp), store_epi(QT, Dp)));
            PE_TRY(dalloc_t(p, OL, &p->bpow32[l], (size_t)Dp * Dp));
            PE_HIP(to_f32(Q, p->bpow32[l], (long)Dp * Dp, p->st));
            std::swap(P, Q);
            std::swap(PT, QT);
        }
        PE_HIP(hipStreamSynchronize(p->st));
    }
    const long rows = (long)B * (Z + N + 1);
    for (int c = 0; c < 2; ++c) {
        PE_TRY(dalloc_t(p, OL, &p->bscan64[c], (size_t)rows * Dp));
        PE_TRY(dalloc_t(p, OL, &p->bscan32[c], (size_t)rows * Dp));
        PE_HIP(zero_fill(p->bscan64[c], p->bscan32[c], rows * Dp, p->st));
    }
    PE_HIP(hipStreamSynchronize(p->st));
    p->bscan_L = L;
    p->bscan_L0 = L0;
    p->bscan_Z = Z;
    p->bscan_B = B;
    return PE_OK;
}

pe_status coarse_sweep_scan(pe_problem p, double* Xk, const double* Xprev, const int* active) {
    const int N = p->N, Dp = p->Dp, L = p->scan_L;
    const int Z = 1 << (p->scan_L0 - 1);
    const bool mixed = p->prec == PE_MIXED;
    const long zoff = (long)Z * Dp;
    PE_HIP(scan_init(p->Fbuf, Xprev, 1, p->scan64[0] + zoff, mixed ? p->scan32[0] + zoff : nullptr, N, Dp, p->st));
    for (int l = 0; l < L; ++l) {
        const int c = l & 1;
        const long shift = (long)(Z - (1 << l)) * Dp;
        Epi e = store_epi(p->scan64[1 - c] + zoff, Dp, 1.0, p->scan64[c] + zoff, Dp, 1.0);
        if (mixed) {
            e.C32 = p->scan32[1 - c] + zoff;
            PE_TRY(gemm<float>(p, shape(N, Dp, p->scan32[c] + shift, Dp, p->pow32[l], Dp, 0, Dp), e, 0,
                               PE_PROF_COARSE, SITE_COARSE_SCAN));
        } else {
            PE_TRY(gemm<double>(p, shape(N, Dp, p->scan64[c] + shift, Dp, p->pow64[l], Dp, 0, Dp), e, 0,
                                PE_PROF_COARSE, SITE_COARSE_SCAN));
        }
    }
    PE_HIP(scan_final(Xprev, p->scan64[L & 1] + zoff, Xk, 1, N, Dp, active, p->st));
    return PE_OK;
}

// Initial sweep x_{n+1} = Phi_G x_n + c_n of one sample as the same scan
// over the N + 1 terms t_0 = x0, t_n = c_{n-1}: after ceil(log2(N + 1))
// levels t_n = x_n (FP64 products on the states, as the sequential initial
// sweep's).
pe_status coarse_sweep_initial_scan(pe_problem p, double* Xk) {
    const int N = p->N, Dp = p->Dp, L0 = p->scan_L0;
    const long zoff = (long)(1 << (L0 - 1)) * Dp;
    PE_HIP(scan_init0(Xk, p->CS, p->scan64[0] + zoff, nullptr, N, Dp, p->st));
    for (int l = 0; l < L0; ++l) {
        const int c = l & 1;
        const long shift = zoff - (long)(1 << l) * Dp;
        Epi e = store_epi(p->scan64[1 - c] + zoff, Dp, 1.0, p->scan64[c] + zoff, Dp, 1.0);
        PE_TRY(gemm<double>(p, shape(N + 1, Dp, p->scan64[c] + shift, Dp, p->pow64[l], Dp, 0, Dp), e, 0,
                            PE_PROF_COARSE, SITE_COARSE_SCAN));
    }
    PE_HIP(scan_final(nullptr, p->scan64[L0 & 1] + zoff + Dp, Xk, 1, N, Dp, nullptr, p->st));
    return PE_OK;
}

// The backward sweeps of the adjoint (one sample) as the same scan with the
// transposed powers, running from n = N down: the correction in change form
// is d_n = Phi_G^T d_{n+1} + e_n (e_n = Fbuf_n - lam_n^{k-1}, d_N = 0), the
// initial sweep lam_n = cs_n + Phi_G^T lam_{n+1} (lam_N = cs_N). Level l adds
// (Phi_G^T)^(2^l) t_{n+2^l}; rows past the data read the zero rows kept
// after it (row N is cleared for the correction's N terms).
pe_status coarse_adj_scan_correct(pe_problem p, double* Lk, const double* Lprev, const int* active) {
    const int N = p->N, Dp = p->Dp, L = p->scan_L;
    const bool mixed = p->prec == PE_MIXED;
    PE_HIP(place(Lk + (long)N * Dp, Dp, 0, 0, Lprev + (long)N * Dp, Dp, 1, Dp, 1.0, 0, p->st));
    for (int c = 0; c < 2; ++c)
        PE_HIP(zero_fill(p->scanA64[c] + (long)N * Dp, mixed ? p->scanA32[c] + (long)N * Dp : nullptr, Dp, p->st));
    PE_HIP(scan_init(p->Fbuf, Lprev, 0, p->scanA64[0], mixed ? p->scanA32[0] : nullptr, N, Dp, p->st));
    for (int l = 0; l < L; ++l) {
        const int c = l & 1;
        const long shift = (long)(1 << l) * Dp;
        Epi e = store_epi(p->scanA64[1 - c], Dp, 1.0, p->scanA64[c], Dp, 1.0);
        if (mixed) {
            e.C32 = p->scanA32[1 - c];
            PE_TRY(gemm<float>(p, shape(N, Dp, p->scanA32[c] + shift, Dp, p->pow32T[l], Dp, 0, Dp), e, 0,
                               PE_PROF_COARSE, SITE_COARSE_SCAN));
        } else {
            PE_TRY(gemm<double>(p, shape(N, Dp, p->scanA64[c] + shift, Dp, p->pow64T[l], Dp, 0, Dp), e, 0,
                                PE_PROF_COARSE, SITE_COARSE_SCAN));
        }
    }
    PE_HIP(scan_final(Lprev, p->scanA64[L & 1], Lk, 0, N, Dp, active, p->st));
    return PE_OK;
}

pe_status coarse_adj_scan_initial(pe_problem p, double* Lk, const double* cs) {
    const int N = p->N, Dp = p->Dp, L0 = p->scan_L0;
    PE_HIP(scan_final(nullptr, cs, p->scanA64[0], 0, N + 1, Dp, nullptr, p->st));
    for (int l = 0; l < L0; ++l) {
        const int c = l & 1;
        const long shift = (long)(1 << l) * Dp;
        Epi e = store_epi(p->scanA64[1 - c], Dp, 1.0, p->scanA64[c], Dp, 1.0);
        PE_TRY(gemm<double>(p, shape(N + 1, Dp, p->scanA64[c] + shift, Dp, p->pow64T[l], Dp, 0, Dp), e, 0,
                            PE_PROF_COARSE, SITE_COARSE_SCAN));
    }
    PE_HIP(scan_final(nullptr, p->scanA64[L0 & 1], Lk, 0, N + 1, Dp, nullptr, p->st));
    return PE_OK;
}

// J_b = max_{j < nr} |Xk[b][n0+j] - Xp[b][n0+j]|_M  (Xp null: plain norms)
// (states of stride Sx: E keeps the whole change, the norm is that of x,
// eq. (2.8))
pe_status jumps_launch(pe_problem p, int B, const double* Xk, const double* Xp, long ldXb, int n0, int nr) {
    const int Dp = p->Dp, Sx = p->Sx;
    PE_HIP(jump_diff(Xk, Xp, ldXb, n0, nr, B, Dp, p->E, p->st, Sx));
    PE_TRY(gemm<double>(p, shape(B * nr, Dp, p->E, Sx, p->M64, Dp, 0, Dp), store_epi(p->Yn, Dp), 0,
                        PE_PROF_NORM, SITE_NORM));
    PE_HIP(jump_reduce(p->E, p->Yn, B, nr, Dp, p->Jd, p->nrm, p->st, Sx));
    return PE_OK;
}

pe_status jumps_read(pe_problem p, int B, double* Jhost) {
    PE_HIP(hipMemcpyAsync(Jhost, p->Jd, sizeof(double) * B, hipMemcpyDeviceToHost, p->st));
    PE_HIP(hipStreamSynchronize(p->st));
    PE_TRY(prof_collect(p));
    return PE_OK;
}

pe_status jumps(pe_problem p, int B, const double* Xk, const double* Xp, long ldXb, int n0, int nr,
                double* Jhost, double* norms_dev) {
    const int Dp = p->Dp, Sx = p->Sx;
    PE_HIP(jump_diff(Xk, Xp, ldXb, n0, nr, B, Dp, p->E, p->st, Sx));
    PE_TRY(gemm<double>(p, shape(B * nr, Dp, p->E, Sx, p->M64, Dp, 0, Dp), store_epi(p->Yn, Dp), 0,
                        PE_PROF_NORM, SITE_NORM));
    PE_HIP(jump_reduce(p->E, p->Yn, B, nr, Dp, p->Jd, norms_dev ? norms_dev : p->nrm, p->st, Sx));
    if (Jhost) {
        PE_HIP(hipMemcpyAsync(Jhost, p->Jd, sizeof(double) * B, hipMemcpyDeviceToHost, p->st));
        PE_HIP(hipStreamSynchronize(p->st));
        PE_TRY(prof_collect(p));
    }
    return PE_OK;
}

// ---------------------------------------------------------------------------
// adjoint
// ---------------------------------------------------------------------------
// The transposed fine step. With the step state s = [du_prev | u | w | dw_prev]
// and the step written as R = F - W s, d = Z R, s' = [du, u + du, w + dw, dw],
// the adjoint of s' maps back through
//     rho = Z^T nu,   a <- a - A rho,   nu <- a - (A + Mh) rho,
// where a is the adjoint of (u, w), nu = a + (adjoint of the history), rho the
// adjoint of the step's source F, and Mh = [[0, M12/h], [M21/h, 0]]. At the
// interval end a = nu = lambda (the history is not an output); at the start
// the fresh history does not depend on the state, so F^T lambda = a there.
// A cotangent of an intermediate state adds to both a and nu.

// Adjoint operators, built at the first adjoint call: Z^T, [A; A + Mh] and
// Phi_G^T in the fine sweep's precision and coordinates; PE_MIXED also
// Tin^T and the whitened mass [[I, M~12], [M~21, I]].
pe_status ensure_adj_ops(pe_problem p) {
    if (p->adj_ops) return PE_OK;
    const int d1 = p->d1, d2 = p->d2, d1p = p->d1p, d2p = p->d2p, Dp = p->Dp;
    auto& OL = p->op_allocs;
    TmpList tmpl(p->st);
    std::vector<void*>& tmp = tmpl.v;
    auto done = [&](pe_status r) {
        (void)hipStreamSynchronize(p->st);
        free_list(tmp);
        return r;
    };
    pe_status s;
    const bool mixed = p->prec == PE_MIXED;
    double *Y64 = nullptr, *YZ = nullptr;
    if ((s = dalloc_t(p, OL, &p->PhiGT64, (size_t)Dp * Dp)) < 0 || (s = dalloc_t(p, tmp, &Y64, (size_t)2 * Dp * Dp)) < 0)
        return done(s);
    PE_HIP(place(p->PhiGT64, Dp, 0, 0, p->PhiG64, Dp, Dp, Dp, 1.0, 1, p->st));
    // [A; A + Mh] Z_h^T (NT product with the rows of Z_h as operator rows)
    if ((s = build_adj_state_op(p, mixed ? p->Aw64 : p->A64, p->M12k, d2p, p->dtf, Y64)) < 0) return done(s);
    if (mixed) {
        if ((s = dalloc_t(p, tmp, &YZ, (size_t)2 * Dp * Dp)) < 0) return done(s);
    } else {
        if ((s = dalloc_t(p, OL, &p->YZ64, (size_t)2 * Dp * Dp)) < 0) return done(s);
        YZ = p->YZ64;
    }
    if ((s = gemm<double>(p, shape(2 * Dp, Dp, Y64, Dp, p->Zf64, Dp, 0, Dp), store_epi(YZ, Dp))) < 0) return done(s);
    if (mixed) {
        double* I = nullptr;
        const int dm = std::max(d1p, d2p);
        if ((s = dalloc_t(p, OL, &p->PhiGT32, (size_t)Dp * Dp)) < 0 ||
            (s = dalloc_t(p, OL, &p->YZ32, (size_t)2 * Dp * Dp)) < 0 ||
            (s = dalloc_t(p, OL, &p->TinT64, (size_t)Dp * Dp)) < 0 ||
            (s = dalloc_t(p, OL, &p->Mw64, (size_t)Dp * Dp)) < 0 || (s = dalloc_t(p, tmp, &I, (size_t)dm * dm)) < 0)
            return done(s);
        PE_HIP(to_f32(p->PhiGT64, p->PhiGT32, (long)Dp * Dp, p->st));
        PE_HIP(to_f32(YZ, p->YZ32, 2L * Dp * Dp, p->st));
        PE_HIP(place(p->TinT64, Dp, 0, 0, p->Tin64, Dp, Dp, Dp, 1.0, 1, p->st));
        PE_HIP(hipMemsetAsync(p->Mw64, 0, sizeof(double) * Dp * Dp, p->st));
        PE_HIP(eye(I, dm, d1, p->st));
        PE_HIP(place(p->Mw64, Dp, 0, 0, I, dm, d1, d1, 1.0, 0, p->st));
        if (d2 > 0) {
            PE_HIP(eye(I, dm, d2, p->st));
            PE_HIP(place(p->Mw64, Dp, d1p, d1p, I, dm, d2, d2, 1.0, 0, p->st));
            PE_HIP(place(p->Mw64, Dp, 0, d1p, p->M12k, d2p, d1, d2, 1.0, 0, p->st));
            PE_HIP(place(p->Mw64, Dp, d1p, 0, p->M12k, d2p, d2, d1, 1.0, 1, p->st));
        }
    }
    p->adj_ops = 1;
    return done(PE_OK);
}

pe_status ensure_adj_workspace(pe_problem p, int B, bool traj, bool rho, bool fdh) {
    const bool grow = B > p->adj_B || std::max(p->Rp, 1) > p->adj_Rp || (traj && !p->adj_traj) ||
                      (rho && !p->adj_rho) || (fdh && !p->adj_fdh);
    if (!grow) return PE_OK;
    B = std::max(B, p->adj_B);
    traj = traj || p->adj_traj;
    rho = rho || p->adj_rho;
    fdh = fdh || p->adj_fdh;
    PE_HIP(hipStreamSynchronize(p->st));
    graphs_clear(p);
    free_list(p->adj_allocs);
    p->Xb = p->Qb = p->Yb = p->Sacc = p->Hb = p->Rho = p->Ytraj = p->Inj = p->Fdh = p->Fdh_w = p->rowtmp =
        nullptr;
    p->adj_B = p->adj_Rp = p->adj_traj = p->adj_rho = p->adj_fdh = 0;
    const size_t N = p->N, P = p->P, Dp = p->Dp, Bs = B, Rp = std::max(p->Rp, 1);
    auto& L = p->adj_allocs;
    PE_TRY(dalloc_t(p, L, &p->Xb, Bs * (N + 1) * Dp));
    PE_TRY(dalloc_t(p, L, &p->Qb, Bs * (N + 1) * Dp));
    PE_TRY(dalloc_t(p, L, &p->Yb, Bs * (N + 1) * Dp));
    PE_TRY(dalloc_t(p, L, &p->Sacc, Bs * N * Dp));
    PE_TRY(dalloc_t(p, L, &p->Hb, Bs * N * (rho ? P : 1) * Rp));
    if (rho) PE_TRY(dalloc_t(p, L, &p->Rho, Bs * N * P * Dp));
    if (traj) {
        PE_TRY(dalloc_t(p, L, &p->Ytraj, Bs * N * P * Dp));
        PE_TRY(dalloc_t(p, L, &p->Inj, Bs * N * P * Dp));
        PE_TRY(dalloc_t(p, L, &p->rowtmp, Bs * N * P));
    }
    if (fdh) {
        PE_TRY(dalloc_t(p, L, &p->Fdh, Bs * N * Dp));
        PE_TRY(dalloc_t(p, L, &p->Fdh_w, Bs * N * Dp));
    }
    p->adj_B = B;
    p->adj_Rp = (int)Rp;
    p->adj_traj = traj;
    p->adj_rho = rho;
    p->adj_fdh = fdh;
    return PE_OK;
}

// Y[b][n] (+)= F_n^T lam[b][n+1] on all B*N intervals, lam rows read from L
// (sample stride ldLb; row n+1 taken when n+1 < nvalid, else zero), plus the
// transposed steps applied to the fine-level cotangents inj (nullable; row
// (b*N + n)*P + p is the cotangent of the state after step p). srcadj: 0 no
// source adjoint, 1 sum rho over the steps into Sacc, 2 every rho into Rho.
pe_status fine_adjoint_sweep(pe_problem p, int B, const double* L, long ldLb, int nvalid, const double* inj,
                             double* Y, bool accumulate, int srcadj) {
    const int Dp = p->Dp, d1p = p->d1p, P = p->P, N = p->N;
    const int rows = B * N;
    const long ldS = 2L * Dp;
    const bool mixed = p->prec == PE_MIXED;
    float* nu32[2] = {mixed ? p->dev32[0] : nullptr, mixed ? p->dev32[1] : nullptr};
    PE_HIP(fine_init(L, ldLb, 1, nvalid, p->Xa, p->dev64[0], nullptr, B, N, Dp, p->st));
    const double* lam0 = p->Xa;
    if (mixed) {
        // lambda~ = Tout^T lambda = Linv lambda (block diagonal)
        GemmShape gt = shape(rows, Dp, p->Xa, Dp, p->Linv64, Dp, 0, d1p);
        gt.s_split = d1p;
        gt.k0b = d1p;
        gt.k1b = Dp;
        PE_TRY(gemm<double>(p, gt, store_epi(p->R64, Dp), 0, PE_PROF_ANCHOR, SITE_ANCHOR));
        lam0 = p->R64;
    }
    // the source adjoint of step p is Z_h^T nu_p: keep the sum of the nu_p
    // over the interval (srcadj 1) or each nu_p (srcadj 2); nu_{P-1} = a
    const long ldinj = (long)P * Dp;
    double* nset = srcadj == 1 ? p->Sacc : (srcadj == 2 ? p->Rho + (long)(P - 1) * Dp : nullptr);
    const long ldset = srcadj == 2 ? (long)P * Dp : Dp;
    PE_HIP(adj_init(lam0, inj ? inj + (long)(P - 1) * Dp : nullptr, ldinj, p->dev64[0], nu32[0], nset, ldset, rows,
                    Dp, p->st));
    double* Sb[2] = {p->dev64[0], p->dev64[1]};
    int c = 0;
    for (int step = P - 1; step >= 0; --step) {
        // [a; nu] <- a - [A; A + Mh] Z_h^T nu  (+ cotangent of the state before this step)
        GemmShape g = shape(rows, 2 * Dp, mixed ? (const void*)nu32[c] : (const void*)(Sb[c] + Dp), mixed ? Dp : ldS,
                            mixed ? (const void*)p->YZ32 : (const void*)p->YZ64, Dp, 0, Dp);
        Epi e;
        e.mode = EPI_ADJ_STATE;
        e.ldr = Dp;
        e.s_cur = Sb[c];
        e.s_nxt = Sb[1 - c];
        e.nu32 = nu32[1 - c];
        e.P = P;
        if (step > 0) {
            if (inj) {
                e.inj = inj + (long)(step - 1) * Dp;
                e.ldinj = ldinj;
            }
            e.sacc = srcadj == 1 ? p->Sacc : nullptr;
            e.rho_all = srcadj == 2 ? p->Rho : nullptr;
            e.m_step = step - 1;
        }
        if (mixed)
            PE_TRY(gemm<float>(p, g, e, 0, PE_PROF_ADJ_STEP, SITE_ADJ_STEP));
        else
            PE_TRY(gemm<double>(p, g, e, 0, PE_PROF_ADJ_STEP, SITE_ADJ_STEP));
        c = 1 - c;
    }
    if (!mixed) {
        PE_HIP(take_a(Sb[c], Y, rows, Dp, accumulate ? 1 : 0, p->st));
    } else {
        // back to the caller's coordinates: Y (+)= Tin^T a~
        GemmShape gt = shape(rows, Dp, Sb[c], ldS, p->TinT64, Dp, 0, d1p);
        gt.s_split = d1p;
        gt.k0b = d1p;
        gt.k1b = Dp;
        PE_TRY(gemm<double>(p, gt, store_epi(Y, Dp, 1.0, accumulate ? Y : nullptr, Dp, accumulate ? 1.0 : 0.0),
                            0, PE_PROF_ANCHOR, SITE_ANCHOR));
    }
    return PE_OK;
}

// Backward coarse sweeps on lambda (B x (N+1) x Dp, row N fixed):
// initial  lam_n = cs_n + Phi_G^T lam_{n+1}, lam_N = cs_N;
// correction  lam_n^k = Fbuf_n + Phi_G^T (lam_{n+1}^k - lam_{n+1}^{k-1}).
pe_status coarse_adj_initial(pe_problem p, int B, double* Lk, const double* cs) {
    const int Dp = p->Dp, N = p->N;
    const long ldX = (long)(N + 1) * Dp;
    PE_HIP(place(Lk + (long)N * Dp, ldX, 0, 0, cs + (long)N * Dp, ldX, B, Dp, 1.0, 0, p->st));
    for (int n = N - 1; n >= 0; --n) {
        Epi e;
        e.mode = EPI_COARSE_INIT;
        e.xout = Lk + (long)n * Dp;
        e.ldxo = ldX;
        e.cs = cs + (long)n * Dp;
        e.ldcs = ldX;
        PE_TRY(gemm<double>(p, shape(B, Dp, Lk + (long)(n + 1) * Dp, ldX, p->PhiGT64, Dp, 0, Dp), e, 0,
                            PE_PROF_COARSE));
    }
    return PE_OK;
}

pe_status coarse_adj_correct(pe_problem p, int B, double* Lk, const double* Lprev, const int* active) {
    const int Dp = p->Dp, N = p->N;
    const long ldX = (long)(N + 1) * Dp;
    const bool mixed = p->prec == PE_MIXED;
    PE_HIP(place(Lk + (long)N * Dp, ldX, 0, 0, Lprev + (long)N * Dp, ldX, B, Dp, 1.0, 0, p->st));
    PE_HIP(zero_fill(mixed ? nullptr : p->Dl64[0], mixed ? p->Dl32[0] : nullptr, (long)B * Dp, p->st));
    int c = 0;
    for (int n = N - 1; n >= 0; --n) {
        Epi e;
        e.mode = EPI_COARSE_DELTA;
        e.xout = Lk + (long)n * Dp;
        e.ldxo = ldX;
        e.xprev = Lprev + (long)n * Dp;
        e.fbuf = p->Fbuf + (long)n * Dp;
        e.ldfb = (long)N * Dp;
        e.dl64 = mixed ? nullptr : p->Dl64[1 - c];
        e.dl32 = mixed ? p->Dl32[1 - c] : nullptr;
        e.ldl = Dp;
        e.active = active;
        if (mixed)
            PE_TRY(gemm<float>(p, shape(B, Dp, p->Dl32[c], Dp, p->PhiGT32, Dp, 0, Dp), e, 0, PE_PROF_COARSE));
        else
            PE_TRY(gemm<double>(p, shape(B, Dp, p->Dl64[c], Dp, p->PhiGT64, Dp, 0, Dp), e, 0, PE_PROF_COARSE));
        c = 1 - c;
    }
    return PE_OK;
}

// Euclidean jumps J_b = max_{j < nr} |Lk[b][n0+j] - Lp[b][n0+j]|_2 (Lp null: norms)
pe_status adj_jumps_launch(pe_problem p, int B, const double* Lk, const double* Lp, int n0, int nr) {
    const int Dp = p->Dp;
    const long ldX = (long)(p->N + 1) * Dp;
    PE_HIP(jump_diff(Lk, Lp, ldX, n0, nr, B, Dp, p->E, p->st));
    PE_HIP(jump_reduce(p->E, p->E, B, nr, Dp, p->Jd, p->nrm, p->st));
    return PE_OK;
}

// Fine levels of the tracked trajectory y (boundary states packed in Yb,
// source amplitudes dH or none) into Ytraj, and Inj = beta dt_fine M y
// (whitened mass in PE_MIXED, where Ytraj holds whitened states).
pe_status tracking_levels(pe_problem p, int B, const double* dH, double beta) {
    const int Dp = p->Dp, N = p->N, P = p->P;
    SrcView sv;
    if (dH && p->src_set && p->src_kind != 0) {
        sv.kind = p->src_kind;
        sv.Hs = dH;
        if (p->src_kind == 2) {
            // per-interval Z_h F of the amplitudes dH, in the sweep's coordinates
            const bool mixed = p->prec == PE_MIXED;
            PE_TRY(interval_table(p, B, dH, p->Fdh, mixed ? p->Fdh_w : nullptr));
            const double* src = mixed ? p->Fdh_w : p->Fdh;
            double* dst = mixed ? p->Fdh : p->Fdh_w;
            PE_TRY(gemm<double>(p, shape(B * N, Dp, src, Dp, p->Zf64, Dp, 0, Dp), store_epi(dst, Dp)));
            sv.ZFint = dst;
            if (mixed) sv.Fint_w = p->Fdh_w;
        }
    }
    PE_TRY(fine_sweep(p, B, p->Yb, (long)(N + 1) * Dp, p->Fbuf, true, 0, false, &sv, p->Ytraj));
    const double* Mx = p->prec == PE_MIXED ? p->Mw64 : p->M64;
    PE_TRY(gemm<double>(p, shape(B * N * P, Dp, p->Ytraj, Dp, Mx, Dp, 0, Dp),
                        store_epi(p->Inj, Dp, beta * p->dtf), 0, -1, SITE_TRAJ));
    return PE_OK;
}

// ---------------------------------------------------------------------------
// batches of different problems
// ---------------------------------------------------------------------------
struct GroupPlan {
    GemmItem* items = nullptr;  // device
    const int* wg_item = nullptr;
    const int* wg_tile = nullptr;
    int n_wg = 0;
};

}  // namespace

struct pe_batch_s {
    int count = 0, prec = PE_FP64, P = 0, N_max = 0;
    std::vector<pe_problem> pr;
    std::vector<int> Bs, J_off;
    int J_total = 0;
    hipStream_t st = nullptr;
    int own_stream = 0;
    // launch plans (built at the first solve; rebuilt when a problem's
    // workspace or sample count changes)
    int planned = 0;
    std::vector<const void*> plan_keys;
    TileCfg cfg;
    std::vector<void*> allocs;
    GroupPlan anc1, anc2, fin[2], nrm_rel, nrm_k;
    std::vector<GroupPlan> resid[2];  // [with source][fine step]
    // PE_MIXED_REFINE: the u rows of A x_a, the FP64 residual products
    // [with source][fine step] and the FP32 corrections [fine step]
    int refine = 0;
    GroupPlan anc3;
    std::vector<GroupPlan> rres[2], rcorr;
    // PE_MIXED: the coarse correction as a doubling scan; level l is one
    // grouped launch over the (problem, sample) items whose problem has
    // more than 2^l intervals
    int scan = 0, scan_L = 0;
    std::vector<GroupPlan> scanp;                    // [level]
    int iscan_L = 0;                                 // the initial sweep as a scan (all problems)
    std::vector<GroupPlan> iscanp;                   // [level]
    std::vector<std::vector<int>> scan_item_g;       // [level][item] -> problem
    std::vector<std::vector<long>> scan_item_tiles;  // [level][item] -> tiles
    std::vector<int*> scan_wi_d, scan_wt_d;          // [level] work-group tables
    CoarseItem* c_init = nullptr;
    CoarseItem* c_corr[2] = {nullptr, nullptr};
    // grouped element-wise steps: one BatchElem per problem, the active
    // problems' indices (act_d[0..n_act-1]) and the largest sample count
    BatchElem* elems_d = nullptr;
    int* act_d = nullptr;
    int n_act = 0, B_max = 0;
    int *c_wg_item = nullptr, *c_wg_row = nullptr;
    std::vector<int> c_nwg;  // coarse step n: work-groups of the problems with N > n
    std::vector<int> order;  // problems by decreasing N
    double* J_all = nullptr;
    GraphCache gc;
    Prof prof;
    // problems still iterating: finished ones leave the launch tables
    std::vector<int> pact, fin_buf;
    std::vector<long> t_fine, t_nk, t_u;  // tiles per problem of the fine, jump and V_H1-row product families
    std::vector<int> tr_fine, tr_nk, tr_u;  // row tiles per problem of the same families
    int *fi_d = nullptr, *ft_d = nullptr, *ki_d = nullptr, *kt_d = nullptr, *ui_d = nullptr, *ut_d = nullptr;
    // XCD-aware work-group order of the grouped products (PE_BATCH_XCD=1:
    // each product on one XCD; 2, the default: the row tiles of each
    // operator column tile on one XCD; 0: plain order)
    int xcd = 0;
    int tables_all = 1;
    long act_hash = 0;
};

namespace {

template <typename T>
pe_status upload(pe_batch bt, const std::vector<T>& v, T** out) {
    *out = nullptr;
    if (v.empty()) return PE_OK;
    void* d = nullptr;
    if (hipMalloc(&d, sizeof(T) * v.size()) != hipSuccess) {
        (void)hipGetLastError();
        return fail(PE_ERR_NOMEM, "device allocation for a batch plan failed");
    }
    bt->allocs.push_back(d);
    PE_HIP(hipMemcpy(d, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
    *out = (T*)d;
    return PE_OK;
}

// device copy of a table with room for any later (padded) version of it
pe_status upload_cap(pe_batch bt, const std::vector<int>& v, size_t cap, int** out) {
    *out = nullptr;
    cap = std::max(cap, v.size());
    if (cap == 0) return PE_OK;
    void* d = nullptr;
    if (hipMalloc(&d, sizeof(int) * cap) != hipSuccess) {
        (void)hipGetLastError();
        return fail(PE_ERR_NOMEM, "device allocation for a batch plan failed");
    }
    bt->allocs.push_back(d);
    if (!v.empty()) PE_HIP(hipMemcpy(d, v.data(), sizeof(int) * v.size(), hipMemcpyHostToDevice));
    *out = (int*)d;
    return PE_OK;
}

// work-group tables of a grouped product family (one product per item);
// dp(item) weighs an item's tiles for the XCD-aware order
template <typename DP>
pe_status group_tables(pe_batch bt, const std::vector<GemmShape>& shapes, const int** wg_item, const int** wg_tile,
                       int* n_wg, DP dp) {
    std::vector<int> wi, wt;
    for (size_t g = 0; g < shapes.size(); ++g) {
        const long tiles = (long)((shapes[g].Mr + bt->cfg.br - 1) / bt->cfg.br) *
                           ((shapes[g].Ns + bt->cfg.bs - 1) / bt->cfg.bs);
        for (long t = 0; t < tiles; ++t) {
            wi.push_back((int)g);
            wt.push_back((int)t);
        }
    }
    std::vector<int> trs(shapes.size());
    for (size_t g = 0; g < shapes.size(); ++g) trs[g] = (shapes[g].Mr + bt->cfg.br - 1) / bt->cfg.br;
    const size_t cap = (bt->xcd == 1 || bt->xcd == 3) ? 8 * wi.size() + 8
                       : bt->xcd == 2                   ? rowtile_cap(wi.size(), trs)
                                                        : wi.size();
    wg_order(bt->xcd, wi, wt, dp, [&](int g) { return trs[g]; });
    int *a = nullptr, *b = nullptr;
    PE_TRY(upload_cap(bt, wi, cap, &a));
    PE_TRY(upload_cap(bt, wt, cap, &b));
    *wg_item = a;
    *wg_tile = b;
    *n_wg = (int)wi.size();
    return PE_OK;
}

pe_status group_plan(pe_batch bt, const std::vector<GemmShape>& sh, const std::vector<Epi>& ep, size_t elem,
                     const int* wg_item, const int* wg_tile, int n_wg, GroupPlan* out) {
    std::vector<GemmItem> items(sh.size());
    for (size_t g = 0; g < sh.size(); ++g) {
        if (!gemm_shape_ok(sh[g], elem)) return fail(PE_ERR_ARG, "batch product operands are not 16-byte aligned");
        items[g].sh = sh[g];
        items[g].epi = ep[g];
        items[g].tiles_r = (sh[g].Mr + bt->cfg.br - 1) / bt->cfg.br;
    }
    PE_TRY(upload(bt, items, &out->items));
    out->wg_item = wg_item;
    out->wg_tile = wg_tile;
    out->n_wg = n_wg;
    return PE_OK;
}

std::vector<const void*> batch_plan_keys(pe_batch bt) {
    std::vector<const void*> k;
    for (int i = 0; i < bt->count; ++i) {
        pe_problem p = bt->pr[i];
        k.push_back(p->Xk[0]);
        k.push_back(p->CS);
        k.push_back(p->Gs);
        k.push_back(p->Fint);
        k.push_back((const void*)(long)bt->Bs[i]);
    }
    return k;
}

pe_status batch_tables(pe_batch bt);

pe_status batch_plan(pe_batch bt) {
    PE_HIP(hipStreamSynchronize(bt->st));
    bt->gc.clear();
    for (void* v : bt->allocs) (void)hipFree(v);
    bt->allocs.clear();
    bt->planned = 0;
    const bool mixed = bt->prec == PE_MIXED;
    const size_t el = mixed ? sizeof(float) : sizeof(double);
    const int G = bt->count;
    std::vector<GemmShape> fine_sh(G), nrel_sh(G), nk_sh(G);
    std::vector<GemmShape> a1(G), a2(G), fsh(G);
    std::vector<Epi> e_a1(G), e_a2(G), e_fin[2], e_nrel(G), e_nk(G);
    e_fin[0].resize(G);
    e_fin[1].resize(G);
    std::vector<std::vector<GemmShape>> r_sh(bt->P, std::vector<GemmShape>(G));
    std::vector<std::vector<Epi>> r_ep[2];
    for (int w = 0; w < 2; ++w) r_ep[w].assign(bt->P, std::vector<Epi>(G));
    // refinement families (PE_MIXED_REFINE)
    std::vector<GemmShape> a3(G), rr_sh(G), rc_sh(G);
    std::vector<Epi> e_a3(G);
    std::vector<std::vector<Epi>> rr_ep[2], rc_ep(bt->P, std::vector<Epi>(G));
    for (int w = 0; w < 2; ++w) rr_ep[w].assign(bt->P, std::vector<Epi>(G));
    for (int g = 0; g < G; ++g) {
        pe_problem p = bt->pr[g];
        const int B = bt->Bs[g], N = p->N, Dp = p->Dp, d1p = p->d1p, d2p = p->d2p, rows = B * N;
        const long ldS = 2L * Dp;
        fine_sh[g] = shape(rows, Dp, nullptr, Dp, nullptr, Dp, 0, Dp);
        // anchors
        a1[g] = shape(rows, Dp, p->R64, Dp, p->Tin64, Dp, 0, d1p);
        a1[g].s_split = d1p;
        a1[g].k0b = d1p;
        a1[g].k1b = Dp;
        e_a1[g] = store_epi(p->Xa, Dp);
        a2[g] = shape(rows, Dp, p->Xa, Dp, p->ZA64, Dp, 0, Dp);
        e_a2[g] = store_epi(p->Ya, Dp);
        // fused fine steps (state ping-pong: step p reads buffer p & 1)
        for (int step = 0; step < bt->P; ++step) {
            const int c = step & 1;
            GemmShape g1 = shape(rows, Dp, mixed ? (const void*)p->dev32[c] : (const void*)p->dev64[c], ldS,
                                 mixed ? (const void*)p->ZW32 : (const void*)p->ZW64, ldS, 0, 0);
            g1.s_split = d1p;
            if (step > 0) {
                g1.k0a = d1p;
                g1.k1a = 2 * Dp;
                g1.k0b = 0;
                g1.k1b = 2 * Dp;
            }
            r_sh[step][g] = g1;
            for (int w = 0; w < 2; ++w) {
                // refined steps: the full sweep's (w = 1), or every sweep's with refine = 2
                const bool ref_step = bt->refine && step > 0 && (w == 1 || bt->refine > 1);
                if (ref_step) {
                    Epi er;
                    er.mode = EPI_RESID;
                    er.R32 = p->res32;
                    er.ldr = d1p;
                    er.base = p->AxU;
                    er.ldb = d1p;
                    er.dres = p->Vr + d1p + 2 * d2p;
                    er.lddres = ldS;
                    er.cres = 1.0 / p->dtf;
                    source_fields(p, er, true);
                    if (!w) er.src_kind = 0;
                    er.cols_per_b = N;
                    er.n_fixed = -1;
                    er.p_step = step;
                    rr_ep[w][step][g] = er;
                }
                Epi e1;
                e1.mode = EPI_FSTEP;
                if (ref_step) e1.vr = p->Vr;
                e1.base = p->Ya;
                e1.ldb = Dp;
                source_fields_step(p, e1);
                if (!w) e1.src_kind = 0;
                e1.cols_per_b = N;
                e1.n_fixed = -1;
                e1.p_step = step;
                e1.din = p->dev64[c];
                e1.dev64 = p->dev64[1 - c];
                e1.dev32 = mixed ? p->dev32[1 - c] : nullptr;
                e1.ldd = ldS;
                e1.d1p = d1p;
                e1.d2p = d2p;
                r_ep[w][step][g] = e1;
            }
            Epi ec;
            ec.mode = EPI_FCORR;
            ec.dev64 = p->dev64[1 - c];
            ec.dev32 = p->dev32[1 - c];
            ec.ldd = ldS;
            ec.d1p = d1p;
            ec.d2p = d2p;
            rc_ep[step][g] = ec;
        }
        if (bt->refine) {
            a3[g] = shape(rows, d1p, p->Xa, Dp, p->Aw64, Dp, 0, Dp);
            e_a3[g] = store_epi(p->AxU, d1p);
            rr_sh[g] = shape(rows, d1p, p->Vr, ldS, p->Wr64, ldS, 0, d1p + 2 * d2p);
            rc_sh[g] = shape(rows, Dp, p->res32, d1p, p->Zc32, d1p, 0, d1p);
        }
        // back to the caller's coordinates (mixed)
        fsh[g] = shape(rows, Dp, p->R64, Dp, p->Tout64, Dp, 0, d1p);
        fsh[g].s_split = d1p;
        fsh[g].k0b = d1p;
        fsh[g].k1b = Dp;
        e_fin[0][g] = store_epi(p->Fbuf, Dp);
        e_fin[1][g] = store_epi(p->Fbuf, Dp, 1.0, p->Fbuf, Dp, 1.0);
        // jump norms
        nrel_sh[g] = shape(B * (N + 1), Dp, p->E, Dp, p->M64, Dp, 0, Dp);
        nk_sh[g] = shape(B * N, Dp, p->E, Dp, p->M64, Dp, 0, Dp);
        e_nrel[g] = store_epi(p->Yn, Dp);
        e_nk[g] = store_epi(p->Yn, Dp);
    }
    const int *fi, *ft, *ri, *rt, *ki, *kt;
    int fn, rn, kn;
    auto dp_of = [&](int g) { return (double)bt->pr[g]->Dp; };
    PE_TRY(group_tables(bt, fine_sh, &fi, &ft, &fn, dp_of));
    PE_TRY(group_tables(bt, nrel_sh, &ri, &rt, &rn, dp_of));
    PE_TRY(group_tables(bt, nk_sh, &ki, &kt, &kn, dp_of));
    if (mixed) {
        PE_TRY(group_plan(bt, a1, e_a1, sizeof(double), fi, ft, fn, &bt->anc1));
        PE_TRY(group_plan(bt, fsh, e_fin[0], sizeof(double), fi, ft, fn, &bt->fin[0]));
        PE_TRY(group_plan(bt, fsh, e_fin[1], sizeof(double), fi, ft, fn, &bt->fin[1]));
    }
    PE_TRY(group_plan(bt, a2, e_a2, sizeof(double), fi, ft, fn, &bt->anc2));
    for (int w = 0; w < 2; ++w) {
        bt->resid[w].assign(bt->P, GroupPlan());
        if (!mixed && !w) continue;  // the FP64 path always sweeps with the source
        for (int step = 0; step < bt->P; ++step)
            PE_TRY(group_plan(bt, r_sh[step], r_ep[w][step], el, fi, ft, fn, &bt->resid[w][step]));
    }
    PE_TRY(group_plan(bt, nrel_sh, e_nrel, sizeof(double), ri, rt, rn, &bt->nrm_rel));
    PE_TRY(group_plan(bt, nk_sh, e_nk, sizeof(double), ki, kt, kn, &bt->nrm_k));
    bt->ui_d = bt->ut_d = nullptr;
    for (int w = 0; w < 2; ++w) bt->rres[w].clear();
    bt->rcorr.clear();
    if (bt->refine) {
        const int *ui, *ut;
        int un;
        PE_TRY(group_tables(bt, a3, &ui, &ut, &un, dp_of));
        PE_TRY(group_plan(bt, a3, e_a3, sizeof(double), ui, ut, un, &bt->anc3));
        for (int w = 0; w < 2; ++w) {
            bt->rres[w].assign(bt->P, GroupPlan());
            if (!w && bt->refine < 2) continue;
            for (int step = 1; step < bt->P; ++step)
                PE_TRY(group_plan(bt, rr_sh, rr_ep[w][step], sizeof(double), ui, ut, un, &bt->rres[w][step]));
        }
        bt->rcorr.assign(bt->P, GroupPlan());
        for (int step = 1; step < bt->P; ++step)
            PE_TRY(group_plan(bt, rc_sh, rc_ep[step], sizeof(float), fi, ft, fn, &bt->rcorr[step]));
        bt->ui_d = (int*)ui;
        bt->ut_d = (int*)ut;
    }
    // coarse sweeps as scans (PE_MIXED; PE_BATCH_SCAN=0 keeps the sequential sweeps)
    bt->scan = 0;
    bt->scan_L = 0;
    bt->iscan_L = 0;
    bt->iscanp.clear();
    bt->scanp.clear();
    bt->scan_item_g.clear();
    bt->scan_item_tiles.clear();
    bt->scan_wi_d.clear();
    bt->scan_wt_d.clear();
    {
        const char* sc = getenv("PE_BATCH_SCAN");
        if (mixed && !(sc && sc[0] == '0')) bt->scan = 1;
    }
    if (bt->scan) {
        for (int g = 0; g < G && bt->scan; ++g) {
            const pe_status s = batch_scan_prepare(bt->pr[g], bt->Bs[g]);
            if (s == PE_ERR_NOMEM) {
                // not enough device memory for the powers: the batch keeps
                // the sequential correction sweep
                for (int h = 0; h <= g; ++h) {
                    pe_problem q = bt->pr[h];
                    (void)hipStreamSynchronize(q->st);
                    free_list(q->bscan_allocs);
                    q->bscan_L = -1;
                }
                g_err.clear();
                bt->scan = 0;
                bt->scan_L = 0;
                break;
            }
            PE_TRY(s);
            bt->scan_L = std::max(bt->scan_L, bt->pr[g]->bscan_L);
        }
    }
    if (bt->scan) {
        bt->scanp.assign(bt->scan_L, GroupPlan());
        bt->scan_item_g.assign(bt->scan_L, {});
        bt->scan_item_tiles.assign(bt->scan_L, {});
        bt->scan_wi_d.assign(bt->scan_L, nullptr);
        bt->scan_wt_d.assign(bt->scan_L, nullptr);
        for (int l = 0; l < bt->scan_L; ++l) {
            const int c = l & 1;
            std::vector<GemmShape> sh;
            std::vector<Epi> ep;
            for (int g = 0; g < G; ++g) {
                pe_problem p = bt->pr[g];
                if (p->bscan_L <= l) continue;
                const int N = p->N, Dp = p->Dp, Z = p->bscan_Z;
                for (int b = 0; b < bt->Bs[g]; ++b) {
                    const long o = ((long)b * (Z + N + 1) + Z) * Dp;
                    const long oa = o - (long)(1 << l) * Dp;
                    sh.push_back(shape(N, Dp, p->bscan32[c] + oa, Dp, p->bpow32[l], Dp, 0, Dp));
                    Epi e = store_epi(p->bscan64[1 - c] + o, Dp, 1.0, p->bscan64[c] + o, Dp, 1.0);
                    e.C32 = p->bscan32[1 - c] + o;
                    ep.push_back(e);
                    bt->scan_item_g[l].push_back(g);
                    bt->scan_item_tiles[l].push_back((long)((N + bt->cfg.br - 1) / bt->cfg.br) *
                                                     ((Dp + bt->cfg.bs - 1) / bt->cfg.bs));
                }
            }
            const int *wi, *wt;
            int wn;
            const std::vector<int>& ig = bt->scan_item_g[l];
            PE_TRY(group_tables(bt, sh, &wi, &wt, &wn, [&](int i) { return (double)bt->pr[ig[i]]->Dp; }));
            PE_TRY(group_plan(bt, sh, ep, sizeof(float), wi, wt, wn, &bt->scanp[l]));
            bt->scan_wi_d[l] = (int*)wi;
            bt->scan_wt_d[l] = (int*)wt;
        }
        // the initial sweep over the N + 1 terms t_0 = x0, t_n = c_{n-1}
        // (tables over every problem: the initial sweep runs before any
        // problem finishes)
        for (int g = 0; g < G; ++g) bt->iscan_L = std::max(bt->iscan_L, bt->pr[g]->bscan_L0);
        bt->iscanp.assign(bt->iscan_L, GroupPlan());
        for (int l = 0; l < bt->iscan_L; ++l) {
            const int c = l & 1;
            std::vector<GemmShape> sh;
            std::vector<Epi> ep;
            std::vector<int> ig;
            for (int g = 0; g < G; ++g) {
                pe_problem p = bt->pr[g];
                if (p->bscan_L0 <= l) continue;
                const int N = p->N, Dp = p->Dp, Z = p->bscan_Z;
                for (int b = 0; b < bt->Bs[g]; ++b) {
                    const long o = ((long)b * (Z + N + 1) + Z) * Dp;
                    const long oa = o - (long)(1 << l) * Dp;
                    sh.push_back(shape(N + 1, Dp, p->bscan32[c] + oa, Dp, p->bpow32[l], Dp, 0, Dp));
                    Epi e = store_epi(p->bscan64[1 - c] + o, Dp, 1.0, p->bscan64[c] + o, Dp, 1.0);
                    e.C32 = p->bscan32[1 - c] + o;
                    ep.push_back(e);
                    ig.push_back(g);
                }
            }
            const int *wi, *wt;
            int wn;
            PE_TRY(group_tables(bt, sh, &wi, &wt, &wn, [&](int i) { return (double)bt->pr[ig[i]]->Dp; }));
            PE_TRY(group_plan(bt, sh, ep, sizeof(float), wi, wt, wn, &bt->iscanp[l]));
        }
    }
    bt->fi_d = (int*)fi;
    bt->ft_d = (int*)ft;
    bt->ki_d = (int*)ki;
    bt->kt_d = (int*)kt;
    bt->t_fine.assign(G, 0);
    bt->t_nk.assign(G, 0);
    bt->t_u.assign(G, 0);
    bt->tr_fine.assign(G, 1);
    bt->tr_nk.assign(G, 1);
    bt->tr_u.assign(G, 1);
    for (int g = 0; g < G; ++g) {
        bt->tr_fine[g] = (fine_sh[g].Mr + bt->cfg.br - 1) / bt->cfg.br;
        bt->tr_nk[g] = (nk_sh[g].Mr + bt->cfg.br - 1) / bt->cfg.br;
        bt->t_fine[g] = (long)bt->tr_fine[g] * ((fine_sh[g].Ns + bt->cfg.bs - 1) / bt->cfg.bs);
        bt->t_nk[g] = (long)bt->tr_nk[g] * ((nk_sh[g].Ns + bt->cfg.bs - 1) / bt->cfg.bs);
        if (bt->refine) {
            bt->tr_u[g] = (a3[g].Mr + bt->cfg.br - 1) / bt->cfg.br;
            bt->t_u[g] = (long)bt->tr_u[g] * ((a3[g].Ns + bt->cfg.bs - 1) / bt->cfg.bs);
        }
    }

    // coarse steps: problems by decreasing N, so the problems still running
    // at step n are a prefix of the row table
    bt->order.resize(G);
    for (int g = 0; g < G; ++g) bt->order[g] = g;
    std::stable_sort(bt->order.begin(), bt->order.end(),
                     [&](int a, int b) { return bt->pr[a]->N > bt->pr[b]->N; });
    std::vector<CoarseItem> ci(G), cc[2];
    cc[0].resize(G);
    cc[1].resize(G);
    std::vector<int> wi, wr, first(G + 1, 0);
    for (int j = 0; j < G; ++j) {
        pe_problem p = bt->pr[bt->order[j]];
        CoarseItem c;
        c.Phi64 = p->PhiG64;
        c.Phi32 = p->PhiG32;
        c.Dp = p->Dp;
        c.B = bt->Bs[bt->order[j]];
        c.N = p->N;
        c.ldX = (long)(p->N + 1) * p->Dp;
        c.Fbuf = p->Fbuf;
        for (int q = 0; q < 2; ++q) {
            c.Dl64[q] = p->Dl64[q];
            c.Dl32[q] = p->Dl32[q];
        }
        CoarseItem a = c;
        a.Xk = p->Xk[0];
        a.cs = p->CS;
        ci[j] = a;
        for (int cur = 0; cur < 2; ++cur) {
            CoarseItem d = c;
            d.Xk = p->Xk[1 - cur];
            d.Xprev = p->Xk[cur];
            d.active = p->active_d;
            cc[cur][j] = d;
        }
        first[j] = (int)wi.size();
        for (int r = 0; r < (p->Dp + 3) / 4; ++r) {
            wi.push_back(j);
            wr.push_back(r);
        }
    }
    first[G] = (int)wi.size();
    PE_TRY(upload(bt, ci, &bt->c_init));
    PE_TRY(upload(bt, cc[0], &bt->c_corr[0]));
    PE_TRY(upload(bt, cc[1], &bt->c_corr[1]));
    PE_TRY(upload(bt, wi, &bt->c_wg_item));
    PE_TRY(upload(bt, wr, &bt->c_wg_row));
    bt->c_nwg.assign(bt->N_max, 0);
    for (int n = 0; n < bt->N_max; ++n) {
        int j = 0;
        while (j < G && bt->pr[bt->order[j]]->N > n) ++j;
        bt->c_nwg[n] = first[j];
    }
    // jump values of every (problem, sample)
    bt->J_off.assign(G, 0);
    bt->J_total = 0;
    for (int g = 0; g < G; ++g) {
        bt->J_off[g] = bt->J_total;
        bt->J_total += bt->Bs[g];
    }
    void* jd = nullptr;
    if (hipMalloc(&jd, sizeof(double) * bt->J_total) != hipSuccess) {
        (void)hipGetLastError();
        return fail(PE_ERR_NOMEM, "device allocation for batch jumps failed");
    }
    bt->allocs.push_back(jd);
    bt->J_all = (double*)jd;
    {
        std::vector<BatchElem> el(G);
        bt->B_max = 0;
        for (int g = 0; g < G; ++g) {
            pe_problem p = bt->pr[g];
            BatchElem& e = el[g];
            e.Xk[0] = p->Xk[0];
            e.Xk[1] = p->Xk[1];
            e.E = p->E;
            e.Yn = p->Yn;
            e.nrm = p->nrm;
            e.J = bt->J_all + bt->J_off[g];
            e.x0p = p->x0p;
            e.Dl64 = p->Dl64[0];
            e.Dl32 = p->Dl32[0];
            e.Xa = p->Xa;
            e.R64 = p->R64;
            e.dev64[0] = p->dev64[0];
            e.dev64[1] = p->dev64[1];
            e.dev32 = p->dev32[0];
            e.Fbuf = p->Fbuf;
            e.CS = p->CS;
            e.active = p->active_d;
            e.B = bt->Bs[g];
            e.N = p->N;
            e.Dp = p->Dp;
            e.d1p = p->d1p;
            if (bt->scan) {
                e.t64[0] = p->bscan64[0];
                e.t64[1] = p->bscan64[1];
                e.t32 = p->bscan32[0];
                e.Z = p->bscan_Z;
                e.L = p->bscan_L;
                e.L0 = p->bscan_L0;
            }
            bt->B_max = std::max(bt->B_max, bt->Bs[g]);
        }
        PE_TRY(upload(bt, el, &bt->elems_d));
        std::vector<int> all(G);
        for (int g = 0; g < G; ++g) all[g] = g;
        PE_TRY(upload(bt, all, &bt->act_d));
        bt->n_act = G;
    }
    bt->plan_keys = batch_plan_keys(bt);
    bt->planned = 1;
    bt->pact.assign(G, 1);
    PE_TRY(batch_tables(bt));
    return PE_OK;
}

// Rebuild the work-group tables of the fine, jump and coarse launches for
// the problems still iterating (bt->pact); the stream must be idle.
pe_status batch_tables(pe_batch bt) {
    const int G = bt->count;
    std::vector<int> fi, ft, ki, kt, wi, wr, ui, ut;
    for (int g = 0; g < G; ++g) {
        if (!bt->pact[g]) continue;
        for (long t = 0; t < bt->t_fine[g]; ++t) {
            fi.push_back(g);
            ft.push_back((int)t);
        }
        for (long t = 0; bt->refine && t < bt->t_u[g]; ++t) {
            ui.push_back(g);
            ut.push_back((int)t);
        }
        for (long t = 0; t < bt->t_nk[g]; ++t) {
            ki.push_back(g);
            kt.push_back((int)t);
        }
    }
    std::vector<int> rows_upto(G + 1, 0);
    for (int j = 0; j < G; ++j) {
        const int g = bt->order[j];
        if (bt->pact[g])
            for (int r = 0; r < (bt->pr[g]->Dp + 3) / 4; ++r) {
                wi.push_back(j);
                wr.push_back(r);
            }
        rows_upto[j + 1] = (int)wi.size();
    }
    for (int n = 0; n < bt->N_max; ++n) {
        int j = 0;
        while (j < G && bt->pr[bt->order[j]]->N > n) ++j;
        bt->c_nwg[n] = rows_upto[j];
    }
    auto put = [&](int* d, const std::vector<int>& v) -> pe_status {
        if (!v.empty()) PE_HIP(hipMemcpy(d, v.data(), sizeof(int) * v.size(), hipMemcpyHostToDevice));
        return PE_OK;
    };
    if (bt->xcd) {
        auto dp_of = [&](int g) { return (double)bt->pr[g]->Dp; };
        wg_order(bt->xcd, fi, ft, dp_of, [&](int g) { return bt->tr_fine[g]; });
        wg_order(bt->xcd, ki, kt, dp_of, [&](int g) { return bt->tr_nk[g]; });
        if (bt->refine) wg_order(bt->xcd, ui, ut, dp_of, [&](int g) { return bt->tr_u[g]; });
    }
    PE_TRY(put(bt->fi_d, fi));
    PE_TRY(put(bt->ft_d, ft));
    PE_TRY(put(bt->ki_d, ki));
    PE_TRY(put(bt->kt_d, kt));
    PE_TRY(put(bt->c_wg_item, wi));
    PE_TRY(put(bt->c_wg_row, wr));
    if (bt->refine) {
        PE_TRY(put(bt->ui_d, ui));
        PE_TRY(put(bt->ut_d, ut));
    }
    {
        std::vector<int> act;
        for (int g = 0; g < G; ++g)
            if (bt->pact[g]) act.push_back(g);
        PE_TRY(put(bt->act_d, act));
        bt->n_act = (int)act.size();
    }
    const int fn = (int)fi.size(), kn = (int)ki.size(), un = (int)ui.size();
    for (GroupPlan* g : {&bt->anc1, &bt->anc2, &bt->fin[0], &bt->fin[1]}) g->n_wg = fn;
    for (int w = 0; w < 2; ++w)
        for (GroupPlan& g : bt->resid[w]) g.n_wg = fn;
    bt->anc3.n_wg = un;
    for (int w = 0; w < 2; ++w)
        for (GroupPlan& g : bt->rres[w]) g.n_wg = un;
    for (GroupPlan& g : bt->rcorr) g.n_wg = fn;
    for (int l = 0; l < bt->scan_L; ++l) {
        std::vector<int> si, st;
        for (size_t i = 0; i < bt->scan_item_g[l].size(); ++i) {
            if (!bt->pact[bt->scan_item_g[l][i]]) continue;
            for (long t = 0; t < bt->scan_item_tiles[l][i]; ++t) {
                si.push_back((int)i);
                st.push_back((int)t);
            }
        }
        if (bt->xcd) {
            const std::vector<int>& ig = bt->scan_item_g[l];
            wg_order(
                bt->xcd, si, st, [&](int i) { return (double)bt->pr[ig[i]]->Dp; },
                [&](int i) { return (bt->pr[ig[i]]->N + bt->cfg.br - 1) / bt->cfg.br; });
        }
        PE_TRY(put(bt->scan_wi_d[l], si));
        PE_TRY(put(bt->scan_wt_d[l], st));
        bt->scanp[l].n_wg = (int)si.size();
    }
    bt->nrm_k.n_wg = kn;
    bt->tables_all = std::count(bt->pact.begin(), bt->pact.end(), 1) == G;
    // graphs are keyed by the active set (the tables' content); repeated
    // solves that pass through the same sets replay them
    unsigned long long h = 1469598103934665603ULL;
    for (int a : bt->pact) h = (h ^ (unsigned long long)(a + 1)) * 1099511628211ULL;
    bt->act_hash = (long)(h >> 1);
    return PE_OK;
}

template <typename T>
pe_status grouped(pe_batch bt, const GroupPlan& g, int kind) {
    TileCfg c = bt->cfg;
    if (sizeof(T) == 8) c.bk2 = 0;
    size_t slot;
    PE_TRY(prof_begin_on(bt->prof, bt->st, kind, &slot));
    const hipError_t e = gemm_grouped_launch<T>(g.items, g.wg_item, g.wg_tile, g.n_wg, c, bt->st);
    if (e != hipSuccess) return fail(PE_ERR_HIP, std::string("grouped product launch failed: ") + hipGetErrorString(e));
    PE_TRY(prof_end_on(bt->prof, bt->st, slot));
    return PE_OK;
}

template <typename T>
pe_status coarse_grouped(pe_batch bt, const CoarseItem* items, int n, int delta, int c) {
    size_t slot;
    PE_TRY(prof_begin_on(bt->prof, bt->st, PE_PROF_COARSE, &slot));
    PE_HIP(coarse_grouped_launch<T>(items, bt->c_wg_item, bt->c_wg_row, bt->c_nwg[n], n, delta, c, bt->st));
    PE_TRY(prof_end_on(bt->prof, bt->st, slot));
    return PE_OK;
}

// F on every interval of every problem (as fine_sweep, one grouped launch per product)
pe_status batch_fine_sweep(pe_batch bt, int cur, bool incremental) {
    const bool mixed = bt->prec == PE_MIXED;
    PE_HIP(grp_fine_init(bt->elems_d, bt->act_d, bt->n_act, cur, incremental ? 1 : 0, mixed ? 1 : 0, bt->st));
    if (mixed) PE_TRY(grouped<double>(bt, bt->anc1, PE_PROF_ANCHOR));
    PE_TRY(grouped<double>(bt, bt->anc2, PE_PROF_ANCHOR));
    const int w = incremental ? 0 : 1;
    const bool refine = bt->refine && (w == 1 || bt->refine > 1);
    if (refine) PE_TRY(grouped<double>(bt, bt->anc3, PE_PROF_ANCHOR));
    for (int step = 0; step < bt->P; ++step) {
        const GroupPlan& r = bt->resid[w][step];
        const int k1 = step > 0 ? PE_PROF_FINE_STEP : PE_PROF_FINE_FIRST;
        if (mixed)
            PE_TRY(grouped<float>(bt, r, k1));
        else
            PE_TRY(grouped<double>(bt, r, k1));
        if (refine && step > 0) {
            PE_TRY(grouped<double>(bt, bt->rres[w][step], PE_PROF_REFINE));
            PE_TRY(grouped<float>(bt, bt->rcorr[step], PE_PROF_REFINE));
        }
    }
    PE_HIP(grp_fine_final(bt->elems_d, bt->act_d, bt->n_act, bt->P, mixed ? 1 : 0, bt->st));
    if (mixed) PE_TRY(grouped<double>(bt, bt->fin[incremental ? 1 : 0], PE_PROF_ANCHOR));
    return PE_OK;
}

// jumps of every problem into J_all: rel (X^0 norms over n = 0..N) or the
// change of iterate xk against 1 - xk over n = 1..N
pe_status batch_jumps(pe_batch bt, int xk, bool rel) {
    PE_HIP(grp_jump_diff(bt->elems_d, bt->act_d, bt->n_act, xk, rel ? 1 : 0, bt->st));
    PE_TRY(grouped<double>(bt, rel ? bt->nrm_rel : bt->nrm_k, PE_PROF_NORM));
    PE_HIP(grp_jump_reduce(bt->elems_d, bt->act_d, bt->n_act, bt->B_max, rel ? 1 : 0, bt->st));
    return PE_OK;
}
pe_status check_handle(pe_problem p) {
    if (!p) return fail(PE_ERR_ARG, "null problem handle");
    return PE_OK;
}

// Coarse step on the history-carrying states [x | delta] (built at the first
// use). G is the one-step coarse propagator with a fresh history, as without
// carried history; it reads x only and hands on its own step's change at the
// fine-step rate:
//   G([x; delta]) = [x + d; d / P],  d = Zc (F - A x),
// i.e. the 2Dp x Dp matrix [Phi_G; (Phi_G - I)/P] on x and the source term
// [Zc F; Zc F / P]. (The parareal limit is fixed by F alone.)
pe_status ensure_hist_ops(pe_problem p) {
    if (p->PhiA64) return PE_OK;
    const int Dp = p->Dp;
    std::vector<void*> L;
    double* phi = nullptr;
    float* phi32 = nullptr;
    pe_status s = dalloc_t(p, L, &phi, (size_t)2 * Dp * Dp);
    if (s == PE_OK && p->prec == PE_MIXED) s = dalloc_t(p, L, &phi32, (size_t)2 * Dp * Dp);
    if (s == PE_OK && hist_phi(p->PhiG64, phi, Dp, p->P, p->st) != hipSuccess) s = fail(PE_ERR_HIP, "hist_phi");
    if (s == PE_OK && phi32 && to_f32(phi, phi32, 2L * Dp * Dp, p->st) != hipSuccess) s = fail(PE_ERR_HIP, "to_f32");
    if (s != PE_OK) {
        (void)hipStreamSynchronize(p->st);
        free_list(L);
        return s;
    }
    p->PhiA64 = phi;
    p->PhiA32 = phi32;
    p->hist_ops = L;
    return PE_OK;
}

// the coarse source term on [x | delta] for the current source
pe_status ensure_hist_src(pe_problem p) {
    if (!p->CS) {
        p->CSa = nullptr;
        return PE_OK;
    }
    if (p->CSa && p->csa_version == p->src_version) return PE_OK;
    PE_HIP(hipStreamSynchronize(p->st));
    free_list(p->hist_src);
    p->CSa = nullptr;
    const long rows = (long)p->B_src * p->N;
    PE_TRY(dalloc_t(p, p->hist_src, &p->CSa, (size_t)rows * 2 * p->Dp));
    PE_HIP(aug_cs(p->CS, p->CSa, rows, p->Dp, p->P, p->st));
    p->csa_version = p->src_version;
    return PE_OK;
}

pe_status hist_unsupported(pe_problem p, const char* what) {
    if (p->hist == PE_HIST_CARRY)
        return fail(PE_ERR_STATE, std::string(what) + " is not available with carried history (pe_set_history)");
    return PE_OK;
}

// ---------------------------------------------------------------------------
// fine propagator by waveform relaxation (Sections 4.1-4.2), FP64, in the
// caller's coordinates. Iteration j on every interval column at once:
//   1. right-hand sides of eq. (4.8) at the levels s = 1..P,
//        R_s = F1_s - (M12/h)(w_{s-1} - w_{s-2}) - A12 w_{s-1}   (w = w^{j-1})
//      plus (M11/h)(u_0 - alpha u_P^{j-1}) at s = 1 (the periodic-like start);
//   2. the all-at-once system (4.12) by the diagonalisation (4.5)-(4.7):
//      scaled transform along time, one solve per frequency, inverse;
//   3. eq. (4.9) sequentially in time with the new u levels:
//        w_s = (I - h M22^-1 A22) w_{s-1} + V_s,
//        V_s = h M22^-1 F2_s - M22^-1 M21 (u_{s-1} - u_{s-2}) - h M22^-1 A21 u_s
//      (V for all s in one product before the sequential part).
// The history at the interval start is reset (w_{-1} = w_0, u_{-1} = u_0) and
// the first iterate continues the start state (w_s^0 = w_0, u_P^0 = u_0).
// Operators (built once per alpha on the GPU):
//   Gu = [M12/h | A12] (d1p x 2d2p), M11h = M11/h, Zw = [M22^-1 M21 | h M22^-1 A21]
//   (d2p x 2d1p), PhiW = I - h M22^-1 A22, the source's w part h M22^-1 G2
//   (or h M22^-1 F2 per interval for dense interval sources), and for each
//   frequency k = 0..K-1 (K = P/2 + 1; the rest are conjugates) the real form
//   O_k = [[Cr, -Ci], [Ci, Cr]] of (d_k M11 + A11)^-1 = Cr + i Ci, d_k = a_k + i b_k
//   the eigenvalues of the alpha-circulant matrix (eq. (4.5)). With the SPD
//   matrices Ar = A11 + a_k M11 (a_k > 0) and S = Ar + b_k^2 M11 Ar^-1 M11:
//   Cr = S^-1, Ci = -b_k S^-1 M11 Ar^-1 (block elimination of the real 2x2
//   form; two Cholesky factorisations, no complex arithmetic, and the
//   condition number is not squared).
// ---------------------------------------------------------------------------
pe_status wr_build_ops(pe_problem p, int B, double alpha) {
    const int d1 = p->d1, d2 = p->d2, d1p = p->d1p, d2p = p->d2p, Dp = p->Dp, P = p->P, N = p->N;
    const double h = p->dtf;
    const int K = P / 2 + 1;
    const bool dense_src = p->src_set && p->src_kind == 2;
    if (p->wr_alpha == alpha && p->wr_src_version == p->src_version && (!dense_src || p->wr_B == B)) return PE_OK;
    PE_HIP(hipStreamSynchronize(p->st));
    graphs_clear(p);
    free_list(p->wr_ops);
    free_list(p->wr_tab);
    p->wr_tab_nc = 0;
    p->wr_alpha = -1.0;
    auto& OL = p->wr_ops;
    const int nf1 = roundup(d1, 64), nf2 = roundup(std::max(d2, 1), 64);
    const long l1 = 2L * d1p, l2 = 2L * std::max(d2p, 1);
    PE_TRY(dalloc_t(p, OL, &p->wrO, (size_t)K * l1 * l1));
    PE_TRY(dalloc_t(p, OL, &p->wrGu, (size_t)d1p * l2));
    PE_TRY(dalloc_t(p, OL, &p->wrM11h, (size_t)d1p * d1p));
    PE_TRY(dalloc_t(p, OL, &p->wrZw, (size_t)std::max(d2p, 1) * l1));
    PE_TRY(dalloc_t(p, OL, &p->wrPhiW, (size_t)std::max(d2p, 1) * std::max(d2p, 1)));
    PE_TRY(dalloc_t(p, OL, &p->wrTw, (size_t)4 * K * P));
    const double* M11 = p->M64;
    const double* A11 = p->A64;
    const double* M12 = p->M64 + d1p;
    const double* A12 = p->A64 + d1p;
    const double* M22 = p->M64 + (long)d1p * Dp + d1p;
    const double* A22 = p->A64 + (long)d1p * Dp + d1p;
    PE_HIP(wr_twiddle(p->wrTw, P, K, alpha, p->st));
    PE_HIP(hipMemsetAsync(p->wrM11h, 0, sizeof(double) * d1p * d1p, p->st));
    PE_HIP(place(p->wrM11h, d1p, 0, 0, M11, Dp, d1, d1, 1.0 / h, 0, p->st));
    PE_HIP(hipMemsetAsync(p->wrGu, 0, sizeof(double) * d1p * l2, p->st));
    PE_HIP(hipMemsetAsync(p->wrZw, 0, sizeof(double) * std::max(d2p, 1) * l1, p->st));
    PE_HIP(hipMemsetAsync(p->wrPhiW, 0, sizeof(double) * std::max(d2p, 1) * std::max(d2p, 1), p->st));
    TmpList tmpl(p->st);
    auto& tmp = tmpl.v;
    if (d2 > 0) {
        PE_HIP(place(p->wrGu, l2, 0, 0, M12, Dp, d1, d2, 1.0 / h, 0, p->st));
        PE_HIP(place(p->wrGu, l2, 0, d2p, A12, Dp, d1, d2, 1.0, 0, p->st));
        double *E2 = nullptr, *M22inv = nullptr;
        PE_TRY(dalloc_t(p, tmp, &E2, (size_t)nf2 * nf2));
        PE_TRY(dalloc_t(p, tmp, &M22inv, (size_t)nf2 * nf2));
        PE_HIP(shifted_embed(E2, nf2, M22, nullptr, Dp, d2, 0.0, p->st));
        PE_TRY(factor_inverse(p, E2, nf2, M22inv, "M22", d2));
        // Zw = [M22^-1 M21 | h M22^-1 A21]: rows of M12 (A12) are the columns of M21 (A21)
        PE_TRY(gemm<double>(p, shape(d2p, d1p, M22inv, nf2, M12, Dp, 0, d2p), store_epi(p->wrZw, l1)));
        PE_TRY(gemm<double>(p, shape(d2p, d1p, M22inv, nf2, A12, Dp, 0, d2p), store_epi(p->wrZw + d1p, l1, h)));
        // PhiW = I - h M22^-1 A22 (A22 symmetric)
        Epi e = store_epi(p->wrPhiW, d2p, -h);
        e.diag_add = 1.0;
        PE_TRY(gemm<double>(p, shape(d2p, d2p, M22inv, nf2, A22, Dp, 0, d2p), e));
        // the source's w part
        if (p->src_set && p->src_kind == 1) {
            PE_TRY(dalloc_t(p, OL, &p->wrGw, (size_t)d2p * p->Rp));
            PE_TRY(gemm<double>(p, shape(d2p, p->Rp, M22inv, nf2, p->GT + d1p, Dp, 0, d2p),
                                store_epi(p->wrGw, p->Rp, h)));
        } else if (dense_src) {
            PE_TRY(dalloc_t(p, OL, &p->wrFintW, (size_t)B * N * d2p));
            PE_TRY(gemm<double>(p, shape(B * N, d2p, p->Fint + d1p, Dp, M22inv, nf2, 0, d2p),
                                store_epi(p->wrFintW, d2p, h)));
        }
    }
    // frequency operators
    double *E = nullptr, *Ari = nullptr, *Si = nullptr, *T1 = nullptr, *T2 = nullptr, *Ci = nullptr;
    PE_TRY(dalloc_t(p, tmp, &E, (size_t)nf1 * nf1));
    PE_TRY(dalloc_t(p, tmp, &Ari, (size_t)nf1 * nf1));
    PE_TRY(dalloc_t(p, tmp, &Si, (size_t)nf1 * nf1));
    PE_TRY(dalloc_t(p, tmp, &T1, (size_t)d1p * d1p));
    PE_TRY(dalloc_t(p, tmp, &T2, (size_t)d1p * d1p));
    PE_TRY(dalloc_t(p, tmp, &Ci, (size_t)d1p * d1p));
    PE_HIP(hipMemsetAsync(p->wrO, 0, sizeof(double) * K * l1 * l1, p->st));
    const double g1 = std::pow(alpha, 1.0 / P);
    for (int k = 0; k < K; ++k) {
        const double th = 2.0 * M_PI * (double)k / (double)P;
        const double a = (1.0 - g1 * std::cos(th)) / h, b = g1 * std::sin(th) / h;
        char name[96];
        snprintf(name, sizeof(name), "A11 + %.6e M11 (frequency %d)", a, k);
        PE_HIP(shifted_embed(E, nf1, A11, M11, Dp, d1, a, p->st));
        PE_TRY(factor_inverse(p, E, nf1, Ari, name, d1));
        double* Ok = p->wrO + (long)k * l1 * l1;
        if (b == 0.0) {
            // real shift (k = 0 and k = P/2): Cr = Ar^-1, Ci = 0
            PE_HIP(place(Ok, l1, 0, 0, Ari, nf1, d1, d1, 1.0, 0, p->st));
            PE_HIP(place(Ok, l1, d1p, d1p, Ari, nf1, d1, d1, 1.0, 0, p->st));
            continue;
        }
        // T1 = M11 Ar^-1, T2 = Ar^-1 M11 = T1^T (Ar^-1, M11 symmetric)
        PE_TRY(gemm<double>(p, shape(d1p, d1p, M11, Dp, Ari, nf1, 0, d1p), store_epi(T1, d1p)));
        PE_TRY(gemm<double>(p, shape(d1p, d1p, Ari, nf1, M11, Dp, 0, d1p), store_epi(T2, d1p)));
        // S = Ar + b^2 M11 Ar^-1 M11, embedded; Cr = S^-1
        PE_HIP(shifted_embed(E, nf1, A11, M11, Dp, d1, a, p->st));
        PE_TRY(gemm<double>(p, shape(d1p, d1p, T1, d1p, M11, Dp, 0, d1p), store_epi(E, nf1, b * b, E, nf1, 1.0)));
        snprintf(name, sizeof(name), "Schur complement of frequency %d", k);
        PE_TRY(factor_inverse(p, E, nf1, Si, name, d1));
        // Ci = -b S^-1 (M11 Ar^-1): row i of the second operand = column i of T1 = row i of T2
        PE_TRY(gemm<double>(p, shape(d1p, d1p, Si, nf1, T2, d1p, 0, d1p), store_epi(Ci, d1p, -b)));
        PE_HIP(place(Ok, l1, 0, 0, Si, nf1, d1, d1, 1.0, 0, p->st));
        PE_HIP(place(Ok, l1, d1p, d1p, Si, nf1, d1, d1, 1.0, 0, p->st));
        PE_HIP(place(Ok, l1, 0, d1p, Ci, d1p, d1, d1, -1.0, 0, p->st));
        PE_HIP(place(Ok, l1, d1p, 0, Ci, d1p, d1, d1, 1.0, 0, p->st));
    }
    PE_HIP(hipStreamSynchronize(p->st));
    p->wr_alpha = alpha;
    p->wr_src_version = p->src_version;
    p->wr_B = B;
    p->wr_K = K;
    return PE_OK;
}

pe_status wr_workspace(pe_problem p, int NBc) {
    if (p->wr_NBc >= NBc) return PE_OK;
    PE_HIP(hipStreamSynchronize(p->st));
    graphs_clear(p);
    free_list(p->wr_ws);
    free_list(p->wr_tab);
    p->wr_tab_nc = 0;
    p->wr_NBc = 0;
    const int P = p->P, K = P / 2 + 1;
    const size_t E1 = (size_t)NBc * p->d1p, E2 = (size_t)NBc * std::max(p->d2p, 1);
    auto& L = p->wr_ws;
    PE_TRY(dalloc_t(p, L, &p->wrUl, (P + 1) * E1));
    PE_TRY(dalloc_t(p, L, &p->wrWl, (P + 1) * E2));
    PE_TRY(dalloc_t(p, L, &p->wrR, P * E1));
    PE_TRY(dalloc_t(p, L, &p->wrRh, K * 2 * E1));
    PE_TRY(dalloc_t(p, L, &p->wrUh, K * 2 * E1));
    PE_TRY(dalloc_t(p, L, &p->wrWcat, P * 2 * E2));
    PE_TRY(dalloc_t(p, L, &p->wrUcat, P * 2 * E1));
    PE_TRY(dalloc_t(p, L, &p->wrV, P * E2));
    PE_TRY(dalloc_t(p, L, &p->wrY, E1));
    p->wr_NBc = NBc;
    return PE_OK;
}

// the K per-frequency solves of a chunk of NBc columns as one grouped launch:
// item k is Uh_k = Rh_k O_k^T (NBc x 2d1p), one work-group per output tile
pe_status wr_tables(pe_problem p, int NBc) {
    if (p->wr_tab_nc == NBc) return PE_OK;
    PE_HIP(hipStreamSynchronize(p->st));
    graphs_clear(p);  // captured iterations point at the old tables
    free_list(p->wr_tab);
    p->wr_tab_nc = 0;
    const int K = p->wr_K;
    const long l1 = 2L * p->d1p;
    TileCfg c;
    c.br = NBc >= 64 ? 64 : 32;
    c.bs = 64;
    c.bk2 = 0;
    c.splitk = 1;
    std::vector<GemmItem> items(K);
    std::vector<int> wi, wt;
    const int tr = (NBc + c.br - 1) / c.br, ts = (int)((l1 + c.bs - 1) / c.bs);
    for (int k = 0; k < K; ++k) {
        items[k].sh = shape(NBc, (int)l1, p->wrRh + (long)k * NBc * l1, l1, p->wrO + (long)k * l1 * l1, l1, 0, (int)l1);
        items[k].epi = store_epi(p->wrUh + (long)k * NBc * l1, l1);
        items[k].tiles_r = tr;
        if (!gemm_shape_ok(items[k].sh, sizeof(double))) return fail(PE_ERR_ARG, "frequency solve shape");
        for (int t = 0; t < tr * ts; ++t) {
            wi.push_back(k);
            wt.push_back(t);
        }
    }
    PE_TRY(dalloc_t(p, p->wr_tab, &p->wrItems, items.size()));
    PE_TRY(dalloc_t(p, p->wr_tab, &p->wrWgI, wi.size()));
    PE_TRY(dalloc_t(p, p->wr_tab, &p->wrWgT, wt.size()));
    PE_HIP(hipMemcpy(p->wrItems, items.data(), sizeof(GemmItem) * items.size(), hipMemcpyHostToDevice));
    PE_HIP(hipMemcpy(p->wrWgI, wi.data(), sizeof(int) * wi.size(), hipMemcpyHostToDevice));
    PE_HIP(hipMemcpy(p->wrWgT, wt.data(), sizeof(int) * wt.size(), hipMemcpyHostToDevice));
    p->wr_nwg = (int)wi.size();
    p->wr_cfg = c;
    p->wr_tab_nc = NBc;
    return PE_OK;
}

// one WR iteration on interval columns c0 .. c0+NBc-1
pe_status wr_iteration(pe_problem p, int c0, int NBc, double alpha) {
    const int d2 = p->d2, d1p = p->d1p, d2p = p->d2p, P = p->P, K = p->wr_K;
    const long E1 = (long)NBc * d1p, E2 = (long)NBc * d2p, l1 = 2L * d1p, l2 = 2L * d2p;
    // 1. right-hand sides of the u-system at s = 1..P (source at each row's level)
    if (d2 > 0) PE_HIP(wr_cat(p->wrWl, p->wrWcat, P, NBc, d2p, 0, p->st));
    {
        Epi e;
        e.mode = EPI_RESID;
        e.R64 = p->wrR;
        e.ldr = d1p;
        source_fields(p, e);
        e.cols_per_b = p->N;
        e.rows_per_p = NBc;
        e.col_off = c0;
        e.p_step = 0;
        PE_TRY(gemm<double>(p, shape(P * NBc, d1p, p->wrWcat, l2, p->wrGu, l2, 0, d2 > 0 ? (int)l2 : 0), e, 0,
                            PE_PROF_WR_RHS, d2 > 0 ? SITE_WR_RHS : SITE_NONE));
    }
    // the periodic-like start at s = 1: + (M11/h)(u_0 - alpha u_P^{j-1})
    PE_HIP(wr_axmy(p->wrY, p->wrUl, p->wrUl + (long)P * E1, alpha, E1, p->st));
    PE_TRY(gemm<double>(p, shape(NBc, d1p, p->wrY, d1p, p->wrM11h, d1p, 0, d1p),
                        store_epi(p->wrR, d1p, 1.0, p->wrR, d1p, 1.0)));
    // 2. all-at-once solve: transform, one solve per frequency, inverse
    PE_HIP(wr_dft(1, p->wrR, p->wrRh, p->wrTw, P, K, NBc, d1p, p->st));
    {
        size_t slot;
        PE_TRY(prof_begin(p, PE_PROF_WR_SOLVE, &slot));
        const hipError_t e = gemm_grouped_launch<double>(p->wrItems, p->wrWgI, p->wrWgT, p->wr_nwg, p->wr_cfg, p->st);
        if (e != hipSuccess) return fail(PE_ERR_HIP, std::string("frequency solves: ") + hipGetErrorString(e));
        PE_TRY(prof_end(p, slot));
    }
    PE_HIP(wr_dft(-1, p->wrUh, p->wrUl, p->wrTw, P, K, NBc, d1p, p->st));
    // 3. eq. (4.9) with the new u levels
    if (d2 > 0) {
        PE_HIP(wr_cat(p->wrUl, p->wrUcat, P, NBc, d1p, 1, p->st));
        Epi e;
        e.mode = EPI_RESID;
        e.R64 = p->wrV;
        e.ldr = d2p;
        source_fields(p, e);
        e.Gs = p->wrGw;
        e.Fint = p->wrFintW;
        e.ldf = d2p;
        e.cols_per_b = p->N;
        e.rows_per_p = NBc;
        e.col_off = c0;
        e.p_step = 0;
        PE_TRY(gemm<double>(p, shape(P * NBc, d2p, p->wrUcat, l1, p->wrZw, l1, 0, (int)l1), e, 0, PE_PROF_WR_RHS,
                            SITE_WR_RHS));
        for (int s = 1; s <= P; ++s)
            PE_TRY(gemm<double>(p, shape(NBc, d2p, p->wrWl + (long)(s - 1) * E2, d2p, p->wrPhiW, d2p, 0, d2p),
                                store_epi(p->wrWl + (long)s * E2, d2p, 1.0, p->wrV + (long)(s - 1) * E2, d2p, 1.0),
                                0, PE_PROF_WR_WSTEP, SITE_WR_WSTEP));
    }
    return PE_OK;
}


// K0 WR iterations on the B*N interval columns: start states X (sample
// stride ldXb; in_dir 1: caller layout rows of D, 2: padded rows of Dp),
// end states to Y (row b*N + n; out_dir -1: caller layout, -2: padded)
pe_status wr_sweep(pe_problem p, int B, const double* X, long ldXb, int in_dir, double* Y, int out_dir,
                   double alpha, int K0) {
    const int N = p->N, NB = B * N;
    PE_TRY(wr_build_ops(p, B, alpha));
    // columns per chunk: the workspace holds about 12 P + 8 levels of a column
    const double col_bytes = 8.0 * ((3.0 * p->P + 1.0 + 2.0 * (p->P / 2 + 1) * 2.0) * p->d1p +
                                    (4.0 * p->P + 1.0) * std::max(p->d2p, 1));
    const int max_cols = std::max(1, (int)std::min<double>(NB, (8.0 * (1 << 30)) / col_bytes));
    const int NBc = std::min(NB, max_cols);
    PE_TRY(wr_workspace(p, NBc));
    for (int c0 = 0; c0 < NB; c0 += NBc) {
        const int nc = std::min(NBc, NB - c0);
        PE_TRY(wr_tables(p, nc));
        PE_HIP(wr_io(in_dir, X, ldXb, nullptr, N, p->d1, p->d2, p->d1p, p->d2p, c0, nc, p->P, p->wrUl, p->wrWl,
                     p->st));
        for (int j = 0; j < K0; ++j)
            PE_TRY(graph_run(p, {20, c0, nc, B}, [&]() -> pe_status { return wr_iteration(p, c0, nc, alpha); }));
        PE_HIP(wr_io(out_dir, nullptr, 0, Y, N, p->d1, p->d2, p->d1p, p->d2p, c0, nc, p->P, p->wrUl, p->wrWl,
                     p->st));
    }
    return PE_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* pe_last_error(void) { return g_err.c_str(); }

int pe_version(void) { return 100; }

pe_status pe_problem_destroy(pe_problem p) {
    if (!p) return PE_OK;
    (void)hipStreamSynchronize(p->st);
    graphs_clear(p);
    free_list(p->ws_allocs);
    free_list(p->adj_allocs);
    free_list(p->op_allocs);
    free_list(p->wr_ops);
    free_list(p->wr_ws);
    free_list(p->wr_tab);
    free_list(p->hist_ops);
    free_list(p->hist_src);
    free_list(p->scan_allocs);
    free_list(p->bscan_allocs);
    if (p->gw.part) (void)hipFree(p->gw.part);
    if (p->own_stream) (void)hipStreamDestroy(p->st);
    delete p;
    return PE_OK;
}

pe_status pe_profile(pe_problem p, int enable) {
    g_err.clear();
    PE_TRY(check_handle(p));
    PE_HIP(hipStreamSynchronize(p->st));
    p->prof.reset();
    p->prof.on = enable ? 1 : 0;
    return PE_OK;
}

pe_status pe_profile_read(pe_problem p, int kind, double* total_ms, long long* launches) {
    g_err.clear();
    PE_TRY(check_handle(p));
    if (kind < 0 || kind >= PE_PROF_KINDS) return fail(PE_ERR_ARG, "unknown profile kind");
    PE_HIP(hipStreamSynchronize(p->st));
    PE_TRY(prof_collect(p));
    if (total_ms) *total_ms = p->prof.ms[kind];
    if (launches) *launches = p->prof.n[kind];
    return PE_OK;
}

pe_status pe_autotune(pe_problem p, int B) {
    g_err.clear();
    PE_TRY(check_handle(p));
    if (B < 1) return fail(PE_ERR_ARG, "need B >= 1");
    if (p->src_set && p->src_kind != 0 && B != p->B_src) return fail(PE_ERR_ARG, "B differs from the source's B");
    PE_TRY(ensure_workspace(p, B));
    const int save = p->autotune;
    p->autotune = 1;
    // one fine sweep and one stopping-test product on zero states visit every tuned site
    PE_HIP(zero_fill(p->Xk[0], nullptr, (long)B * (p->N + 1) * p->Sx, p->st));
    pe_status s = fine_sweep(p, B, p->Xk[0], (long)(p->N + 1) * p->Sx, p->Fbuf);
    if (s == PE_OK) s = jumps(p, B, p->Xk[0], nullptr, (long)(p->N + 1) * p->Sx, 1, p->N, nullptr, nullptr);
    p->autotune = save;
    PE_HIP(hipStreamSynchronize(p->st));
    p->prof.pending.clear();
    p->prof.used = 0;
    return s;
}

pe_status pe_last_tiles(pe_problem p, int kind, int* tiles4) {
    g_err.clear();
    PE_TRY(check_handle(p));
    if (kind < 0 || kind >= PE_PROF_KINDS || !tiles4) return fail(PE_ERR_ARG, "bad arguments");
    for (int i = 0; i < 4; ++i) tiles4[i] = p->last_cfg[kind][i];
    return PE_OK;
}

pe_status pe_problem_info(pe_problem p, int* d1, int* d2, int* N, int* P) {
    PE_TRY(check_handle(p));
    if (d1) *d1 = p->d1;
    if (d2) *d2 = p->d2;
    if (N) *N = p->N;
    if (P) *P = p->P;
    return PE_OK;
}

pe_status pe_problem_create(pe_problem* out, int d1, int d2, const double* M11, const double* M12,
                            const double* M22, const double* A11, const double* A12, const double* A21,
                            const double* A22, double dt_coarse, double dt_fine, int N, int precision,
                            void* hip_stream) {
    g_err.clear();
    if (!out) return fail(PE_ERR_ARG, "out is null");
    *out = nullptr;
    if (d1 < 1 || d2 < 0 || N < 1) return fail(PE_ERR_ARG, "need d1 >= 1, d2 >= 0, N >= 1");
    if (!M11 || !A11 || (d2 > 0 && (!M22 || !A12 || !A22)))
        return fail(PE_ERR_ARG, "required block pointer is null");
    if (!(dt_coarse > 0) || !(dt_fine > 0) || !std::isfinite(dt_coarse) || !std::isfinite(dt_fine))
        return fail(PE_ERR_ARG, "step sizes must be positive and finite");
    const double ratio = dt_coarse / dt_fine;
    const double Pr = std::round(ratio);
    if (Pr < 1 || std::fabs(ratio - Pr) > 1e-12 * Pr || Pr > 1e7)
        return fail(PE_ERR_ARG, "dt_coarse / dt_fine must be a positive integer");
    if (precision != PE_FP64 && precision != PE_MIXED && precision != PE_MIXED_REFINE)
        return fail(PE_ERR_ARG, "unknown precision");
    // PE_MIXED_REFINE is the mixed path with the refinement operators
    int refine = 0;
    if (precision == PE_MIXED_REFINE) {
        precision = PE_MIXED;
        const char* ra = getenv("PE_REFINE_ALL");
        refine = (ra && ra[0] == '1') ? 2 : 1;
    }

    pe_problem p = new pe_problem_s();
    p->d1 = d1;
    p->d2 = d2;
    p->D = d1 + d2;
    p->d1p = roundup(d1, 8);
    p->d2p = roundup(d2, 8);
    p->Dp = p->d1p + p->d2p;
    p->Sx = p->Dp;
    p->N = N;
    p->P = (int)Pr;
    p->dt = dt_coarse;
    p->dtf = dt_fine;
    p->prec = precision;
    p->refine = refine;
    p->st = (hipStream_t)hip_stream;
    if (!p->st) {
        // no stream given: the handle owns one (default priority, non-blocking)
        if (hipStreamCreateWithFlags(&p->st, hipStreamNonBlocking) != hipSuccess) {
            delete p;
            return fail(PE_ERR_HIP, "stream creation failed");
        }
        p->own_stream = 1;
    }
    {
        const char* at = getenv("PE_AUTOTUNE");
        p->autotune = (at && at[0] == '0') ? 0 : 1;
        const char* gr = getenv("PE_GRAPHS");
        p->gc.use_graphs = (gr && gr[0] == '0') ? 0 : 1;
        // persistent fine sweep: opt-in (measured slower than per-step launches
        // replayed from graphs on MI355X: each grid-wide barrier costs tens of µs)
        const char* cs = getenv("PE_COARSE_SCAN");
        p->coarse_scan = (cs && cs[0] == '0') ? 0 : 1;
        const char* pz = getenv("PE_PERSISTENT");
        p->persistent = (pz && pz[0] == '1') ? 1 : 0;
        if (const char* fw = getenv("PE_FORCE_WSK")) {
            int bs = 0, w = 0, sk = 0;
            if (sscanf(fw, "%d,%d,%d", &bs, &w, &sk) == 3 && (bs == 16 || bs == 32) && (w == 4 || w == 8) &&
                sk >= 1 && sk <= 64) {
                p->force_wsk.br = 64;
                p->force_wsk.bs = bs;
                p->force_wsk.wsk = w;
                p->force_wsk.splitk = sk;
            }
        }
        if (const char* ft = getenv("PE_FORCE_TILES")) {
            int br = 0, bs = 0, bk2 = 0, sk = 0;
            const bool shape_ok = sscanf(ft, "%d,%d,%d,%d", &br, &bs, &bk2, &sk) == 4 &&
                                  ((br == 32 && bs == 64) || (br == 64 && bs == 32) || (br == 64 && bs == 64) ||
                                   (br == 64 && bs == 128) || (br == 128 && bs == 64) || (br == 128 && bs == 128));
            if (shape_ok && (bk2 == 0 || bk2 == 1) && sk >= 1 && sk <= 64) {
                p->force_tiles.br = br;
                p->force_tiles.bs = bs;
                p->force_tiles.bk2 = bk2;
                p->force_tiles.splitk = sk;
                p->force_tiles_on = 1;
            }
        }
        tune_cache_load(p);
    }
    int dev = 0;
    (void)hipGetDevice(&dev);
    p->device = dev;
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
        p->n_cu = ncu;

    auto bail = [&](pe_status s) {
        std::string msg = g_err;
        pe_problem_destroy(p);
        g_err = msg;
        return s;
    };
    const int d1p = p->d1p, d2p = p->d2p, Dp = p->Dp;
    auto& OL = p->op_allocs;
    std::vector<void*> tmp;
    auto bail_tmp = [&](pe_status s) {
        (void)hipStreamSynchronize(p->st);
        free_list(tmp);
        return bail(s);
    };
#define CK(expr)                              \
    do {                                      \
        pe_status s__ = (expr);               \
        if (s__ < 0) return bail_tmp(s__);    \
    } while (0)
#define CKH(expr)                                                                              \
    do {                                                                                       \
        hipError_t e__ = (expr);                                                               \
        if (e__ != hipSuccess)                                                                 \
            return bail_tmp(fail(PE_ERR_HIP, std::string(#expr ": ") + hipGetErrorString(e__))); \
    } while (0)

    // symmetry checks (relative 1e-12 of the largest entry)
    {
        unsigned long long* red = nullptr;
        CK(dalloc_t(p, tmp, &red, 2 * 5));
        CKH(hipMemsetAsync(red, 0, sizeof(unsigned long long) * 10, p->st));
        CKH(asym(M11, M11, d1, d1, d1, d1, red + 0, p->st));
        CKH(asym(A11, A11, d1, d1, d1, d1, red + 2, p->st));
        if (d2 > 0) {
            CKH(asym(M22, M22, d2, d2, d2, d2, red + 4, p->st));
            CKH(asym(A22, A22, d2, d2, d2, d2, red + 6, p->st));
            if (A21) CKH(asym(A21, A12, d1, d2, d2, d1, red + 8, p->st));
        }
        unsigned long long h[10];
        CKH(hipMemcpyAsync(h, red, sizeof(h), hipMemcpyDeviceToHost, p->st));
        CKH(hipStreamSynchronize(p->st));
        const char* names[5] = {"M11", "A11", "M22", "A22", "A21 vs A12^T"};
        for (int i = 0; i < 5; ++i) {
            double dmax, amax;
            memcpy(&dmax, &h[2 * i], 8);
            memcpy(&amax, &h[2 * i + 1], 8);
            if (!(dmax <= 1e-12 * amax) && dmax != 0.0)
                return bail_tmp(fail(PE_ERR_ARG, std::string(names[i]) + " is not symmetric (max diff " +
                                                     std::to_string(dmax) + ")"));
        }
    }

    // padded FP64 copies of the blocks
    double *pM11, *pM12, *pM22, *pA11, *pA12, *pA21, *pA22, *M22inv;
    const int nf2 = roundup(std::max(d2, 1), 64);
    CK(dalloc_t(p, tmp, &pM11, (size_t)d1p * d1p));
    CK(dalloc_t(p, tmp, &pA11, (size_t)d1p * d1p));
    CK(dalloc_t(p, tmp, &pM12, (size_t)d1p * std::max(d2p, 8)));
    CK(dalloc_t(p, tmp, &pA12, (size_t)d1p * std::max(d2p, 8)));
    CK(dalloc_t(p, tmp, &pA21, (size_t)std::max(d2p, 8) * d1p));
    CK(dalloc_t(p, tmp, &pM22, (size_t)std::max(d2p, 8) * std::max(d2p, 8)));
    CK(dalloc_t(p, tmp, &pA22, (size_t)std::max(d2p, 8) * std::max(d2p, 8)));
    CK(dalloc_t(p, tmp, &M22inv, (size_t)nf2 * nf2));
    CKH(hipMemsetAsync(pM11, 0, sizeof(double) * d1p * d1p, p->st));
    CKH(hipMemsetAsync(pA11, 0, sizeof(double) * d1p * d1p, p->st));
    CKH(place(pM11, d1p, 0, 0, M11, d1, d1, d1, 1.0, 0, p->st));
    CKH(place(pA11, d1p, 0, 0, A11, d1, d1, d1, 1.0, 0, p->st));
    if (d2 > 0) {
        CKH(hipMemsetAsync(pM12, 0, sizeof(double) * d1p * d2p, p->st));
        CKH(hipMemsetAsync(pA12, 0, sizeof(double) * d1p * d2p, p->st));
        CKH(hipMemsetAsync(pA21, 0, sizeof(double) * d2p * d1p, p->st));
        CKH(hipMemsetAsync(pM22, 0, sizeof(double) * d2p * d2p, p->st));
        CKH(hipMemsetAsync(pA22, 0, sizeof(double) * d2p * d2p, p->st));
        if (M12) CKH(place(pM12, d2p, 0, 0, M12, d2, d1, d2, 1.0, 0, p->st));
        CKH(place(pA12, d2p, 0, 0, A12, d2, d1, d2, 1.0, 0, p->st));
        if (A21)
            CKH(place(pA21, d1p, 0, 0, A21, d1, d2, d1, 1.0, 0, p->st));
        else
            CKH(place(pA21, d1p, 0, 0, A12, d2, d2, d1, 1.0, 1, p->st));
        CKH(place(pM22, d2p, 0, 0, M22, d2, d2, d2, 1.0, 0, p->st));
        CKH(place(pA22, d2p, 0, 0, A22, d2, d2, d2, 1.0, 0, p->st));
        // M22^-1
        double* Mem = nullptr;
        CK(dalloc_t(p, tmp, &Mem, (size_t)nf2 * nf2));
        CKH(shifted_embed(Mem, nf2, pM22, nullptr, d2p, d2, 0.0, p->st));
        CK(factor_inverse(p, Mem, nf2, M22inv, "M22", d2));
    }

    // full stiffness and mass (FP64)
    CK(dalloc_t(p, OL, &p->A64, (size_t)Dp * Dp));
    CK(dalloc_t(p, OL, &p->M64, (size_t)Dp * Dp));
    CKH(hipMemsetAsync(p->A64, 0, sizeof(double) * Dp * Dp, p->st));
    CKH(hipMemsetAsync(p->M64, 0, sizeof(double) * Dp * Dp, p->st));
    CKH(place(p->A64, Dp, 0, 0, pA11, d1p, d1, d1, 1.0, 0, p->st));
    CKH(place(p->M64, Dp, 0, 0, pM11, d1p, d1, d1, 1.0, 0, p->st));
    if (d2 > 0) {
        CKH(place(p->A64, Dp, 0, d1p, pA12, d2p, d1, d2, 1.0, 0, p->st));
        CKH(place(p->A64, Dp, d1p, 0, pA21, d1p, d2, d1, 1.0, 0, p->st));
        CKH(place(p->A64, Dp, d1p, d1p, pA22, d2p, d2, d2, 1.0, 0, p->st));
        CKH(place(p->M64, Dp, 0, d1p, pM12, d2p, d1, d2, 1.0, 0, p->st));
        CKH(place(p->M64, Dp, d1p, 0, pM12, d2p, d2, d1, 1.0, 1, p->st));
        CKH(place(p->M64, Dp, d1p, d1p, pM22, d2p, d2, d2, 1.0, 0, p->st));
    }

    // coarse operator (FP64) and fine operators
    CK(dalloc_t(p, OL, &p->Zc64, (size_t)Dp * Dp));
    CK(build_step_ops(p, dt_coarse, pM11, pM12, M22inv, pA11, pA12, pA21, pA22, p->Zc64, nullptr));
    // coarse step matrix Phi_G = I - Z_dt A  (A symmetric: rows of A serve as columns)
    CK(dalloc_t(p, OL, &p->PhiG64, (size_t)Dp * Dp));
    {
        Epi e = store_epi(p->PhiG64, Dp, -1.0);
        e.diag_add = 1.0;
        CK(gemm<double>(p, shape(Dp, Dp, p->Zc64, Dp, p->A64, Dp, 0, Dp), e));
    }
    if (precision == PE_MIXED) {
        CK(dalloc_t(p, OL, &p->PhiG32, (size_t)Dp * Dp));
        CKH(to_f32(p->PhiG64, p->PhiG32, (long)Dp * Dp, p->st));
    }
    const size_t m12n = (size_t)d1p * std::max(d2p, 8);
    CK(dalloc_t(p, OL, &p->M12k, m12n));
    // fine step operators: Z_h (kept in FP64), the fused Z_h W_h and Z_h A
    CK(dalloc_t(p, OL, &p->Zf64, (size_t)Dp * Dp));
    CK(dalloc_t(p, OL, &p->ZA64, (size_t)Dp * Dp));
    {
        double *W64, *WT, *ZW;
        const double* Aop = p->A64;
        CK(dalloc_t(p, tmp, &W64, (size_t)Dp * 2 * Dp));
        CK(dalloc_t(p, tmp, &WT, (size_t)Dp * 2 * Dp));
        if (precision == PE_FP64) {
            CK(build_step_ops(p, dt_fine, pM11, pM12, M22inv, pA11, pA12, pA21, pA22, p->Zf64, W64));
            CKH(hipMemcpyAsync(p->M12k, pM12, sizeof(double) * m12n, hipMemcpyDeviceToDevice, p->st));
            CK(dalloc_t(p, OL, &p->ZW64, (size_t)Dp * 2 * Dp));
            ZW = p->ZW64;
        } else {
            double *wM12, *wA11, *wA12, *wA21, *wA22, *I11, *I22inv;
            CK(whiten(p, tmp, pM11, pM12, pM22, pA11, pA12, pA21, pA22, &wM12, &wA11, &wA12, &wA21, &wA22,
                      &I11, &I22inv));
            CK(build_step_ops(p, dt_fine, I11, wM12, I22inv, wA11, wA12, wA21, wA22, p->Zf64, W64));
            CKH(hipMemcpyAsync(p->M12k, wM12, sizeof(double) * m12n, hipMemcpyDeviceToDevice, p->st));
            CK(dalloc_t(p, tmp, &ZW, (size_t)Dp * 2 * Dp));
            Aop = p->Aw64;
            if (refine) {
                // Wr = [A~11 | A~12 | M~12/h]: the u rows of W_h = [0 | A~11 |
                // A~12 | M~12/h] past their zero first block. With the
                // operands [du + u - u_a | w - w_a | dw_prev] the product is
                // K~ du + A~11 (u - u_a) + A~12 (w - w_a) + M~12 dw_prev / h
                // (K~ = I/h + A~11) less du / h, which the residual's
                // epilogue subtracts as a diagonal term
                CK(dalloc_t(p, OL, &p->Wr64, (size_t)d1p * 2 * Dp));
                CKH(place(p->Wr64, 2L * Dp, 0, 0, W64 + d1p, 2L * Dp, d1p, d1p + 2 * d2p, 1.0, 0, p->st));
                // Zc = Z_h[:, u]: the solve of a V_H1 residual and its effect
                // on the explicit V_H2 increment
                double* Zc = nullptr;
                CK(dalloc_t(p, tmp, &Zc, (size_t)Dp * d1p));
                CKH(place(Zc, d1p, 0, 0, p->Zf64, Dp, Dp, d1p, 1.0, 0, p->st));
                CK(dalloc_t(p, OL, &p->Zc32, (size_t)Dp * d1p));
                CKH(to_f32(Zc, p->Zc32, (long)Dp * d1p, p->st));
            }
        }
        // Z_h W_h = Z_h (W_h^T)^T: NT product with W_h^T as the operator rows
        CKH(place(WT, Dp, 0, 0, W64, 2L * Dp, 2 * Dp, Dp, 1.0, 1, p->st));
        CK(gemm<double>(p, shape(Dp, 2 * Dp, p->Zf64, Dp, WT, Dp, 0, Dp), store_epi(ZW, 2L * Dp)));
        // Z_h A (A symmetric: its rows serve as the operator rows)
        CK(gemm<double>(p, shape(Dp, Dp, p->Zf64, Dp, Aop, Dp, 0, Dp), store_epi(p->ZA64, Dp)));
        if (precision == PE_MIXED) {
            CK(dalloc_t(p, OL, &p->ZW32, (size_t)Dp * 2 * Dp));
            CKH(to_f32(ZW, p->ZW32, 2L * Dp * Dp, p->st));
        }
    }
    CKH(hipStreamSynchronize(p->st));
    free_list(tmp);
#undef CK
#undef CKH
    *out = p;
    return PE_OK;
}

pe_status pe_source_set(pe_problem p, int B, int R, const double* G, const double* H, int time_mode) {
    g_err.clear();
    PE_TRY(check_handle(p));
    if (B < 1 || R < 0) return fail(PE_ERR_ARG, "need B >= 1 and R >= 0");
    if (time_mode != PE_T_FINE && time_mode != PE_T_INTERVAL) return fail(PE_ERR_ARG, "unknown time_mode");
    if (R > 0 && (!G || !H)) return fail(PE_ERR_ARG, "G and H must be given when R > 0");
    if (time_mode == PE_T_FINE && R > 64) return fail(PE_ERR_ARG, "PE_T_FINE supports R <= 64");
    PE_HIP(hipStreamSynchronize(p->st));
    graphs_clear(p);
    for (void* v : {(void*)p->Gs, (void*)p->Hs, (void*)p->Fint, (void*)p->Gs_w, (void*)p->Fint_w, (void*)p->CS,
                    (void*)p->GT, (void*)p->GwT, (void*)p->ZGs, (void*)p->ZGT, (void*)p->ZFint}) {
        if (!v) continue;
        auto it = std::find(p->op_allocs.begin(), p->op_allocs.end(), v);
        if (it != p->op_allocs.end()) p->op_allocs.erase(it);
        (void)hipFree(v);
    }
    p->Gs = p->Hs = p->Fint = p->Gs_w = p->Fint_w = p->CS = p->GT = p->GwT = p->ZGs = p->ZGT = p->ZFint = nullptr;
    p->src_set = 1;
    p->src_version++;
    p->B_src = B;
    p->R = R;
    p->time_mode = time_mode;
    p->Tlen = (time_mode == PE_T_FINE) ? (long)p->N * p->P : (long)p->N;
    if (R == 0) {
        p->src_kind = 0;
        return PE_OK;
    }
    const int D = p->D, d1 = p->d1, d1p = p->d1p, Dp = p->Dp;
    // per-interval amplitudes with more than a few terms: one dense table
    // Z F per (sample, interval), so the fused step's epilogue reads one value
    // per output instead of 2R (PE_DENSE_SOURCE_R overrides the term count)
    int dense_r = 16;
    if (const char* dr = getenv("PE_DENSE_SOURCE_R")) dense_r = std::max(0, atoi(dr));
    const bool dense = (time_mode == PE_T_INTERVAL && R > dense_r);
    p->Rp = dense ? roundup(R, 2) : R;
    PE_TRY(dalloc_t(p, p->op_allocs, &p->Gs, (size_t)Dp * p->Rp));
    PE_HIP(hipMemsetAsync(p->Gs, 0, sizeof(double) * Dp * p->Rp, p->st));
    PE_HIP(place(p->Gs, p->Rp, 0, 0, G, R, d1, R, 1.0, 0, p->st));
    PE_HIP(place(p->Gs, p->Rp, d1p, 0, G + (long)d1 * R, R, D - d1, R, 1.0, 0, p->st));
    PE_TRY(dalloc_t(p, p->op_allocs, &p->Hs, (size_t)B * R * p->Tlen));
    PE_HIP(hipMemcpyAsync(p->Hs, H, sizeof(double) * B * R * p->Tlen, hipMemcpyDeviceToDevice, p->st));
    if (dense) {
        PE_TRY(dalloc_t(p, p->op_allocs, &p->Fint, (size_t)B * p->N * Dp));
        PE_TRY(interval_table(p, B, p->Hs, p->Fint, nullptr));
        p->src_kind = 2;
    } else {
        p->src_kind = 1;
    }
    // G^T for the source adjoint
    PE_TRY(dalloc_t(p, p->op_allocs, &p->GT, (size_t)p->Rp * Dp));
    PE_HIP(place(p->GT, Dp, 0, 0, p->Gs, p->Rp, p->Rp, Dp, 1.0, 1, p->st));
    {
        // coarse source term c_n = Z_dt F(t_{n+1}) for every (sample, interval)
        double* Fc = nullptr;
        TmpList tmpl(p->st);
        std::vector<void*>& tmp = tmpl.v;
        PE_TRY(dalloc_t(p, tmp, &Fc, (size_t)B * p->N * Dp));
        Epi e;
        e.mode = EPI_RESID;
        e.R64 = Fc;
        e.ldr = Dp;
        source_fields(p, e);
        e.cols_per_b = p->N;
        e.p_step = p->P - 1;
        pe_status s = gemm<double>(p, shape(B * p->N, Dp, Fc, Dp, p->Zc64, Dp, 0, 0), e);
        if (s == PE_OK) s = dalloc_t(p, p->op_allocs, &p->CS, (size_t)B * p->N * Dp);
        if (s == PE_OK) {
            GemmShape g = shape(B * p->N, Dp, Fc, Dp, p->Zc64, Dp, 0, p->d1p);
            g.s_split = p->d1p;
            g.k0b = 0;
            g.k1b = Dp;
            s = gemm<double>(p, g, store_epi(p->CS, Dp));
        }
        (void)hipStreamSynchronize(p->st);
        free_list(tmp);
        if (s < 0) return s;
    }
    if (p->prec == PE_MIXED) {
        // whitened source for the mixed fine sweep: F~ = Tout^T F = Linv F,
        // G~ = Linv G (kept transposed for the source adjoint)
        PE_TRY(dalloc_t(p, p->op_allocs, &p->GwT, (size_t)p->Rp * Dp));
        PE_TRY(gemm<double>(p, shape(p->Rp, Dp, p->GT, Dp, p->Linv64, Dp, 0, Dp), store_epi(p->GwT, Dp)));
        if (p->src_kind == 2) {
            PE_TRY(dalloc_t(p, p->op_allocs, &p->Fint_w, (size_t)B * p->N * Dp));
            PE_TRY(gemm<double>(p, shape(B * p->N, Dp, p->Fint, Dp, p->Linv64, Dp, 0, Dp),
                                store_epi(p->Fint_w, Dp)));
        } else {
            PE_TRY(dalloc_t(p, p->op_allocs, &p->Gs_w, (size_t)Dp * p->Rp));
            PE_HIP(place(p->Gs_w, p->Rp, 0, 0, p->GwT, Dp, Dp, p->Rp, 1.0, 1, p->st));
        }
    }
    // the fused fine step's source: Z_h G, or Z_h F per interval (in the
    // sweep's coordinates)
    const bool mixed = p->prec == PE_MIXED;
    PE_TRY(dalloc_t(p, p->op_allocs, &p->ZGs, (size_t)Dp * p->Rp));
    PE_TRY(gemm<double>(p, shape(Dp, p->Rp, p->Zf64, Dp, mixed ? p->GwT : p->GT, Dp, 0, Dp),
                        store_epi(p->ZGs, p->Rp)));
    PE_TRY(dalloc_t(p, p->op_allocs, &p->ZGT, (size_t)p->Rp * Dp));
    PE_HIP(place(p->ZGT, Dp, 0, 0, p->ZGs, p->Rp, p->Rp, Dp, 1.0, 1, p->st));
    if (p->src_kind == 2) {
        PE_TRY(dalloc_t(p, p->op_allocs, &p->ZFint, (size_t)B * p->N * Dp));
        PE_TRY(gemm<double>(p, shape(B * p->N, Dp, mixed ? p->Fint_w : p->Fint, Dp, p->Zf64, Dp, 0, Dp),
                            store_epi(p->ZFint, Dp)));
    }
    PE_HIP(hipStreamSynchronize(p->st));
    return PE_OK;
}

pe_status pe_fine_propagate(pe_problem p, int B, const double* Xin, double* Y) {
    g_err.clear();
    PE_TRY(check_handle(p));
    if (B < 1 || !Xin || !Y) return fail(PE_ERR_ARG, "bad arguments");
    if (p->src_set && p->src_kind != 0 && B != p->B_src) return fail(PE_ERR_ARG, "B differs from the source's B");
    PE_TRY(ensure_workspace(p, B));
    const long rows = (long)B * p->N;
    const long w = p->Sx / p->Dp;  // states [x | delta] with carried history
    PE_HIP(pack_states(Xin, p->io, rows * w, p->d1, p->d2, p->d1p, p->d2p, p->st));
    PE_TRY(fine_sweep(p, B, p->io, (long)p->N * p->Sx, p->Fbuf));
    PE_HIP(unpack_states(p->Fbuf, Y, rows * w, p->d1, p->d2, p->d1p, p->d2p, p->st));
    PE_HIP(hipStreamSynchronize(p->st));
    PE_TRY(prof_collect(p));
    return PE_OK;
}

pe_status pe_coarse_propagate(pe_problem p, int B, const double* Xin, double* Y) {
    g_err.clear();
    PE_TRY(check_handle(p));
    if (B < 1 || !Xin || !Y) return fail(PE_ERR_ARG, "bad arguments");
    if (p->src_set && p->src_kind != 0 && B != p->B_src) return fail(PE_ERR_ARG, "B differs from the source's B");
    PE_TRY(ensure_workspace(p, B));
    const int Dp = p->Dp;
    const long rows = (long)B * p->N;
    if (p->hist == PE_HIST_CARRY) {
        // one product with the coarse step on [x | delta] for all columns
        const int Sx = p->Sx;
        PE_TRY(ensure_hist_ops(p));
        PE_TRY(ensure_hist_src(p));
        PE_HIP(pack_states(Xin, p->io, rows * 2, p->d1, p->d2, p->d1p, p->d2p, p->st));
        Epi e;
        e.mode = EPI_COARSE_INIT;
        e.xout = p->Fbuf;
        e.ldxo = Sx;
        e.cs = p->CSa;
        e.ldcs = Sx;
        PE_TRY(gemm<double>(p, shape((int)rows, Sx, p->io, Sx, p->PhiA64, Dp, 0, Dp), e));
        PE_HIP(unpack_states(p->Fbuf, Y, rows * 2, p->d1, p->d2, p->d1p, p->d2p, p->st));
        PE_HIP(hipStreamSynchronize(p->st));
        return PE_OK;
    }
    PE_HIP(pack_states(Xin, p->Xa, rows, p->d1, p->d2, p->d1p, p->d2p, p->st));
    Epi e1;
    e1.mode = EPI_RESID;
    e1.R64 = p->R64;
    e1.ldr = Dp;
    source_fields(p, e1);
    e1.cols_per_b = p->N;
    e1.p_step = p->P - 1;
    PE_TRY(gemm<double>(p, shape((int)rows, Dp, p->Xa, Dp, p->A64, Dp, 0, Dp), e1));
    GemmShape g2 = shape((int)rows, Dp, p->R64, Dp, p->Zc64, Dp, 0, p->d1p);
    g2.s_split = p->d1p;
    g2.k0b = 0;
    g2.k1b = Dp;
    PE_TRY(gemm<double>(p, g2, store_epi(p->Ya, Dp, 1.0, p->Xa, Dp, 1.0)));
    PE_HIP(unpack_states(p->Ya, Y, rows, p->d1, p->d2, p->d1p, p->d2p, p->st));
    PE_HIP(hipStreamSynchronize(p->st));
    return PE_OK;
}

// ---------------------------------------------------------------------------
// The coarse propagator without allocations (pe_coarse_propagate_noalloc):
// its workspace - the packed input, the residual, the increment and the
// split-K partial planes - lives in a static device array. Host code never
// uses the array's name as a device address: the address is taken once per
// device with hipGetSymbolAddress and kept.
// ---------------------------------------------------------------------------
constexpr size_t PE_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[PE_SCRATCH_BYTES];

namespace {
constexpr int PE_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[PE_MAX_DEVICES] = {};

// the scratch array's device address on the current device
pe_status scratch_address(int dev, unsigned char** out) {
    if (dev < 0 || dev >= PE_MAX_DEVICES) return fail(PE_ERR_ARG, "device index out of range for the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return fail(PE_ERR_HIP, std::string("hipGetSymbolAddress of the scratch array failed: ") +
                                        hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = (unsigned char*)g_scratch_ptr[dev];
    return PE_OK;
}
}  // namespace

pe_status pe_coarse_propagate_noalloc(pe_problem p, int B, const double* Xin, double* Y) {
    g_err.clear();
    PE_TRY(check_handle(p));
    if (B < 1 || !Xin || !Y) return fail(PE_ERR_ARG, "bad arguments");
    if (p->src_set && p->src_kind != 0 && B != p->B_src) return fail(PE_ERR_ARG, "B differs from the source's B");
    if (p->hist == PE_HIST_CARRY)
        return fail(PE_ERR_STATE, "pe_coarse_propagate_noalloc needs the restarting history (pe_set_history 0)");
    int dev = -1;
    PE_HIP(hipGetDevice(&dev));
    if (dev != p->device) return fail(PE_ERR_ARG, "the handle's device is not the current device");
    const int Dp = p->Dp;
    const long rows = (long)B * p->N;
    const size_t plane = sizeof(double) * (size_t)rows * Dp;
    const size_t fixed = 3 * ((plane + 255) / 256 * 256);
    if (fixed > PE_SCRATCH_BYTES)
        return fail(PE_ERR_ARG, "B*N*D too large for the 64 MiB scratch of pe_coarse_propagate_noalloc (needs " +
                                    std::to_string(fixed) + " bytes)");
    unsigned char* base = nullptr;
    PE_TRY(scratch_address(dev, &base));
    const size_t step = fixed / 3;
    double* xa = (double*)base;
    double* res = (double*)(base + step);
    double* ya = (double*)(base + 2 * step);
    GemmWork ws;
    ws.part = base + fixed;
    ws.part_bytes = PE_SCRATCH_BYTES - fixed;
    // tile choice as pe_coarse_propagate's, split-K only while its planes fit
    auto tiles = [&](const GemmShape& sh) {
        TileCfg c = choose_tiles(sh, false, p->n_cu);
        while (c.splitk > 1 && gemm_part_bytes(sh, c, sizeof(double)) > ws.part_bytes) c.splitk /= 2;
        return c;
    };
    // G(x) = x + Z_dt (F(t_{n+1}) - A x): residual product, then the increment
    PE_HIP(pack_states(Xin, xa, rows, p->d1, p->d2, p->d1p, p->d2p, p->st));
    Epi e1;
    e1.mode = EPI_RESID;
    e1.R64 = res;
    e1.ldr = Dp;
    source_fields(p, e1);
    e1.cols_per_b = p->N;
    e1.p_step = p->P - 1;
    const GemmShape g1 = shape((int)rows, Dp, xa, Dp, p->A64, Dp, 0, Dp);
    PE_HIP(gemm_launch<double>(g1, e1, tiles(g1), ws, p->st));
    GemmShape g2 = shape((int)rows, Dp, res, Dp, p->Zc64, Dp, 0, p->d1p);
    g2.s_split = p->d1p;
    g2.k0b = 0;
    g2.k1b = Dp;
    PE_HIP(gemm_launch<double>(g2, store_epi(ya, Dp, 1.0, xa, Dp, 1.0), tiles(g2), ws, p->st));
    PE_HIP(unpack_states(ya, Y, rows, p->d1, p->d2, p->d1p, p->d2p, p->st));
    PE_HIP(hipStreamSynchronize(p->st));
    return PE_OK;
}

pe_status pe_mass_norms(pe_problem p, int count, const double* X, double* out) {
    g_err.clear();
    PE_TRY(check_handle(p));
    if (count < 1 || !X || !out) return fail(PE_ERR_ARG, "bad arguments");
    const int Dp = p->Dp;
    // workspace rows are B_cap*(N+1); grow if needed
    const int need_B = (count + p->N) / (p->N + 1);
    PE_TRY(ensure_workspace(p, std::max(need_B, 1)));
    PE_HIP(pack_states(X, p->io, count, p->d1, p->d2, p->d1p, p->d2p, p->st));
    PE_HIP(jump_diff(p->io, nullptr, (long)Dp, 0, 1, count, Dp, p->E, p->st));
    PE_TRY(gemm<double>(p, shape(count, Dp, p->E, Dp, p->M64, Dp, 0, Dp), store_epi(p->Yn, Dp)));
    PE_HIP(jump_reduce(p->E, p->Yn, count, 1, Dp, p->Jd, p->nrm, p->st));
    PE_HIP(hipMemcpyAsync(out, p->Jd, sizeof(double) * count, hipMemcpyDeviceToHost, p->st));
    PE_HIP(hipStreamSynchronize(p->st));
    return PE_OK;
}

pe_status pe_solve(pe_problem p, int B, const double* x0, double tol, int norm_mode, int k_max, double* X,
                   int* iters, double* jump_hist) {
    g_err.clear();
    PE_TRY(check_handle(p));
    if (B < 1 || !x0 || !X) return fail(PE_ERR_ARG, "bad arguments");
    if (p->src_set && p->src_kind != 0 && B != p->B_src) return fail(PE_ERR_ARG, "B differs from the source's B");
    if (!(tol >= 0) || k_max < 0 || k_max > p->N) return fail(PE_ERR_ARG, "need tol >= 0 and 0 <= k_max <= N");
    if (norm_mode != PE_NORM_M_ABS && norm_mode != PE_NORM_M_REL) return fail(PE_ERR_ARG, "unknown norm_mode");
    if (p->hist == PE_HIST_CARRY && p->fine_kind == PE_FINE_WR)
        return fail(PE_ERR_STATE, "the waveform-relaxation fine solver restarts the history; use PE_HIST_RESTART");
    PE_TRY(ensure_workspace(p, B));
    const int N = p->N, Dp = p->Dp, Sx = p->Sx;
    const long ldX = (long)(N + 1) * Sx;
    const long w = Sx / Dp;  // 2: states [x | delta] with carried history
    if (p->hist == PE_HIST_CARRY) {
        PE_TRY(ensure_hist_ops(p));
        PE_TRY(ensure_hist_src(p));
    }

    std::vector<int> active(B, 1);
    std::vector<double> thr(B, tol), J(B, 0.0);
    if (iters)
        for (int b = 0; b < B; ++b) iters[b] = 0;
    if (jump_hist)
        for (long i = 0; i < (long)B * k_max; ++i) jump_hist[i] = 0.0;
    PE_HIP(hipMemcpyAsync(p->active_d, active.data(), sizeof(int) * B, hipMemcpyHostToDevice, p->st));

    int cur = 0;
    PE_HIP(pack_states(x0, p->x0p, B, p->d1, p->d2, p->d1p, p->d2p, p->st));
    const long rel = norm_mode == PE_NORM_M_REL ? 1 : 0;
    const bool scan = B == 1 && p->hist != PE_HIST_CARRY && p->coarse_scan && N >= 4;
    if (scan) PE_TRY(scan_prepare(p));
    PE_TRY(graph_run(p, {0, B, rel}, [&]() -> pe_status {
        PE_HIP(set_x0(p->x0p, p->Xk[0], ldX, B, Dp, p->st, Sx));
        if (scan)
            PE_TRY(coarse_sweep_initial_scan(p, p->Xk[0]));
        else
            PE_TRY(coarse_sweep_initial(p, B, p->Xk[0]));
        if (rel) PE_TRY(jumps_launch(p, B, p->Xk[0], nullptr, ldX, 0, N + 1));
        return PE_OK;
    }));
    if (rel) {
        PE_TRY(jumps_read(p, B, thr.data()));
        for (int b = 0; b < B; ++b) thr[b] *= tol;
    }
    int n_active = B;
    for (int k = 1; k <= k_max && n_active > 0; ++k) {
        const int nxt = 1 - cur;
        if (p->fine_kind == PE_FINE_WR) {
            // the paper's fine solver: K0 WR iterations on every interval
            PE_TRY(wr_sweep(p, B, p->Xk[cur], ldX, 2, p->Fbuf, -2, p->fine_alpha, p->fine_K0));
        } else if (p->prec == PE_MIXED && k >= 2) {
            // F is affine: F(x^{k-1}) = F(x^{k-2}) + F_hom(x^{k-1} - x^{k-2}). The
            // change (left in E by the previous jump test, rows n = 1..N) is
            // propagated without source and added to the stored F values, so
            // FP32 rounding scales with the change, not with the state.
            PE_TRY(graph_run(p, {1, B, 2},
                             [&]() { return fine_sweep(p, B, p->E, (long)N * Sx, p->Fbuf, false, 1, true); }));
        } else {
            PE_TRY(graph_run(p, {1, B, cur}, [&]() { return fine_sweep(p, B, p->Xk[cur], ldX, p->Fbuf); }));
        }
        if (n_active < B) PE_HIP(freeze_inactive(p->Xk[cur], p->Xk[nxt], p->active_d, ldX, B, p->st));
        PE_TRY(graph_run(p, {2, B, cur}, [&]() -> pe_status {
            PE_HIP(set_x0(p->x0p, p->Xk[nxt], ldX, B, Dp, p->st, Sx));
            if (scan)
                PE_TRY(coarse_sweep_scan(p, p->Xk[nxt], p->Xk[cur], p->active_d));
            else
                PE_TRY(coarse_sweep_correct(p, B, p->Xk[nxt], p->Xk[cur], p->active_d));
            PE_TRY(jumps_launch(p, B, p->Xk[nxt], p->Xk[cur], ldX, 1, N));
            return PE_OK;
        }));
        PE_TRY(jumps_read(p, B, J.data()));
        cur = nxt;
        for (int b = 0; b < B; ++b) {
            if (!active[b]) continue;
            if (!std::isfinite(J[b])) {
                PE_HIP(unpack_states(p->Xk[cur], X, (long)B * (N + 1) * w, p->d1, p->d2, p->d1p, p->d2p, p->st));
                PE_HIP(hipStreamSynchronize(p->st));
                return fail(PE_ERR_NONFINITE, "non-finite parareal jump for sample " + std::to_string(b) +
                                                  " at iteration " + std::to_string(k));
            }
            if (jump_hist) jump_hist[(long)b * k_max + (k - 1)] = J[b];
            if (iters) iters[b] = k;
            if (J[b] <= thr[b]) {
                active[b] = 0;
                --n_active;
            }
        }
        if (n_active > 0 && n_active < B)
            PE_HIP(hipMemcpyAsync(p->active_d, active.data(), sizeof(int) * B, hipMemcpyHostToDevice, p->st));
    }
    PE_HIP(unpack_states(p->Xk[cur], X, (long)B * (N + 1) * w, p->d1, p->d2, p->d1p, p->d2p, p->st));
    PE_HIP(hipStreamSynchronize(p->st));
    PE_TRY(prof_collect(p));
    return n_active > 0 ? PE_WARN_NOT_CONVERGED : PE_OK;
}


pe_status pe_probe_peaks(void* hip_stream, double* out3) {
    g_err.clear();
    if (!out3) return fail(PE_ERR_ARG, "bad arguments");
    hipStream_t st = (hipStream_t)hip_stream;
    const int blocks = 2048, iters = 2000;
    const long ncopy = (512L << 20) / 16;  // 512 MiB of float4
    void *o = nullptr, *src = nullptr, *dst = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto done = [&](pe_status s) {
        if (st) (void)hipStreamSynchronize(st); else (void)hipDeviceSynchronize();
        for (void* v : {o, src, dst})
            if (v) (void)hipFree(v);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        return s;
    };
    if (hipMalloc(&o, sizeof(double) * blocks * 256) != hipSuccess || hipMalloc(&src, ncopy * 16) != hipSuccess ||
        hipMalloc(&dst, ncopy * 16) != hipSuccess) {
        (void)hipGetLastError();
        return done(fail(PE_ERR_NOMEM, "peak probe buffers"));
    }
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess ||
        hipMemsetAsync(src, 0, ncopy * 16, st) != hipSuccess)
        return done(fail(PE_ERR_HIP, "peak probe set-up"));
    const double mfma_flops = 2.0 * 16 * 16 * 4;  // one 16x16x4 product
    for (int kind = 0; kind < 3; ++kind) {
        double best = 0.0;
        for (int rep = 0; rep < 4; ++rep) {
            if (hipEventRecord(e0, st) != hipSuccess) return done(fail(PE_ERR_HIP, "event"));
            hipError_t e = kind < 2 ? probe_launch(kind, blocks, iters, o, nullptr, 0, st)
                                    : probe_launch(2, 4096, 0, dst, src, ncopy, st);
            if (e != hipSuccess) return done(fail(PE_ERR_HIP, std::string("peak probe: ") + hipGetErrorString(e)));
            if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
                return done(fail(PE_ERR_HIP, "event"));
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (rep == 0 || ms <= 0.f) continue;  // first run warms up
            const double work = kind < 2 ? (double)blocks * 4 * iters * PROBE_ACC_PER_ROUND * mfma_flops
                                         : 2.0 * ncopy * 16;
            best = std::max(best, work / (ms * 1e-3) / 1e12);
        }
        out3[kind] = best;
    }
    return done(PE_OK);
}

pe_status pe_set_history(pe_problem p, int mode) {
    g_err.clear();
    PE_TRY(check_handle(p));
    if (mode != PE_HIST_RESTART && mode != PE_HIST_CARRY) return fail(PE_ERR_ARG, "unknown history mode");
    if (mode == p->hist) return PE_OK;
    if (mode == PE_HIST_CARRY && p->fine_kind == PE_FINE_WR)
        return fail(PE_ERR_STATE, "the waveform-relaxation fine solver restarts the history");
    // the iteration workspace changes its state stride: released and regrown
    PE_HIP(hipStreamSynchronize(p->st));
    graphs_clear(p);
    free_list(p->ws_allocs);
    p->B_cap = 0;
    p->hist = mode;
    p->Sx = mode == PE_HIST_CARRY ? 2 * p->Dp : p->Dp;
    return PE_OK;
}

pe_status pe_set_fine_solver(pe_problem p, int kind, double alpha, int K0) {
    g_err.clear();
    PE_TRY(check_handle(p));
    if (kind == PE_FINE_WR) PE_TRY(hist_unsupported(p, "the waveform-relaxation fine solver"));
    if (kind == PE_FINE_STEP) {
        p->fine_kind = PE_FINE_STEP;
        return PE_OK;
    }
    if (kind != PE_FINE_WR) return fail(PE_ERR_ARG, "unknown fine solver");
    if (p->prec != PE_FP64) return fail(PE_ERR_ARG, "the waveform-relaxation fine solver needs a PE_FP64 handle");
    if (!(alpha > 0.0 && alpha < 1.0)) return fail(PE_ERR_ARG, "need 0 < alpha < 1");
    if (K0 < 1) return fail(PE_ERR_ARG, "need K0 >= 1");
    if (p->P > 128) return fail(PE_ERR_ARG, "waveform relaxation supports P <= 128");
    p->fine_kind = PE_FINE_WR;
    p->fine_alpha = alpha;
    p->fine_K0 = K0;
    return PE_OK;
}

pe_status pe_fine_wr(pe_problem p, int B, const double* Xin, double alpha, int K0, double* Fout) {
    g_err.clear();
    PE_TRY(check_handle(p));
    if (B < 1 || !Xin || !Fout) return fail(PE_ERR_ARG, "bad arguments");
    if (!(alpha > 0.0 && alpha < 1.0)) return fail(PE_ERR_ARG, "need 0 < alpha < 1");
    if (K0 < 0) return fail(PE_ERR_ARG, "need K0 >= 0");
    if (p->P > 128) return fail(PE_ERR_ARG, "waveform relaxation supports P <= 128");
    if (p->src_set && p->src_kind != 0 && B != p->B_src) return fail(PE_ERR_ARG, "B differs from the source's B");
    PE_TRY(hist_unsupported(p, "pe_fine_wr"));
    const int N = p->N, D = p->D;
    const long ldXb = (long)N * D;
    const int NB = B * N;
    if (K0 == 0) {
        PE_HIP(hipMemcpyAsync(Fout, Xin, sizeof(double) * NB * D, hipMemcpyDeviceToDevice, p->st));
        PE_HIP(hipStreamSynchronize(p->st));
        return PE_OK;
    }
    PE_TRY(wr_sweep(p, B, Xin, ldXb, 1, Fout, -1, alpha, K0));
    PE_HIP(hipStreamSynchronize(p->st));
    PE_TRY(prof_collect(p));
    return PE_OK;
}

pe_status pe_tracking(pe_problem p, int B, const double* Ybnd, const double* dH, double beta, double* J) {
    g_err.clear();
    PE_TRY(check_handle(p));
    if (B < 1 || !Ybnd || !J) return fail(PE_ERR_ARG, "bad arguments");
    if (!(beta >= 0)) return fail(PE_ERR_ARG, "need beta >= 0");
    PE_TRY(hist_unsupported(p, "pe_tracking"));
    if (p->src_set && p->src_kind != 0 && B != p->B_src) return fail(PE_ERR_ARG, "B differs from the source's B");
    const bool fdh = dH && p->src_set && p->src_kind == 2;
    PE_TRY(ensure_workspace(p, B));
    PE_TRY(ensure_adj_ops(p));
    PE_TRY(ensure_adj_workspace(p, B, true, false, fdh));
    const long rowsX = (long)B * (p->N + 1);
    PE_HIP(pack_states(Ybnd, p->Yb, rowsX, p->d1, p->d2, p->d1p, p->d2p, p->st));
    PE_TRY(tracking_levels(p, B, dH, beta));
    PE_HIP(sample_dot_sums(p->Ytraj, p->Inj, B, (long)p->N * p->P, p->Dp, 0.5, p->rowtmp, p->Jd, p->st));
    PE_HIP(hipMemcpyAsync(J, p->Jd, sizeof(double) * B, hipMemcpyDeviceToHost, p->st));
    PE_HIP(hipStreamSynchronize(p->st));
    PE_TRY(prof_collect(p));
    return PE_OK;
}

pe_status pe_adjoint(pe_problem p, int B, const double* Xbar, double beta, const double* Ybnd, const double* dH,
                     double tol, int k_max, double* x0bar, double* Hbar, double* Lam, int* iters,
                     double* jump_hist) {
    g_err.clear();
    PE_TRY(check_handle(p));
    if (B < 1 || !x0bar) return fail(PE_ERR_ARG, "bad arguments");
    if (p->src_set && p->src_kind != 0 && B != p->B_src) return fail(PE_ERR_ARG, "B differs from the source's B");
    if (!(tol >= 0) || k_max < 0 || k_max > p->N) return fail(PE_ERR_ARG, "need tol >= 0 and 0 <= k_max <= N");
    if (!(beta >= 0)) return fail(PE_ERR_ARG, "need beta >= 0");
    PE_TRY(hist_unsupported(p, "pe_adjoint"));
    if (beta > 0 && !Ybnd) return fail(PE_ERR_ARG, "beta > 0 needs the tracked trajectory Ybnd");
    const bool track = beta > 0;
    const bool want_h = Hbar && p->src_set && p->R > 0;
    const bool rho_all = want_h && p->time_mode == PE_T_FINE;
    const bool fdh = track && dH && p->src_set && p->src_kind == 2;
    const bool mixed = p->prec == PE_MIXED;
    PE_TRY(ensure_workspace(p, B));
    PE_TRY(ensure_adj_ops(p));
    PE_TRY(ensure_adj_workspace(p, B, track, rho_all, fdh));
    const int N = p->N, Dp = p->Dp;
    const long ldX = (long)(N + 1) * Dp;
    const long rowsX = (long)B * (N + 1);

    if (Xbar)
        PE_HIP(pack_states(Xbar, p->Xb, rowsX, p->d1, p->d2, p->d1p, p->d2p, p->st));
    else
        PE_HIP(zero_fill(p->Xb, nullptr, rowsX * Dp, p->st));
    const double* inj = nullptr;
    if (track) {
        PE_HIP(pack_states(Ybnd, p->Yb, rowsX, p->d1, p->d2, p->d1p, p->d2p, p->st));
        PE_TRY(tracking_levels(p, B, dH, beta));
        inj = p->Inj;
        // coarse stand-in for interval n's tracking term in the initial
        // sweep: beta dt M y_{n+1} at the interval end
        PE_TRY(gemm<double>(p, shape((int)rowsX, Dp, p->Yb, Dp, p->M64, Dp, 0, Dp),
                            store_epi(p->Qb, Dp, beta * p->dt)));
        PE_HIP(zero_row0(p->Qb, ldX, B, Dp, p->st));
    } else {
        PE_HIP(zero_fill(p->Qb, nullptr, rowsX * Dp, p->st));
    }

    std::vector<int> active(B, 1);
    std::vector<double> thr(B, tol), J(B, 0.0);
    if (iters)
        for (int b = 0; b < B; ++b) iters[b] = 0;
    if (jump_hist)
        for (long i = 0; i < (long)B * k_max; ++i) jump_hist[i] = 0.0;
    PE_HIP(hipMemcpyAsync(p->active_d, active.data(), sizeof(int) * B, hipMemcpyHostToDevice, p->st));

    // initial backward coarse sweep on mu = lambda + Q: mu_n = Xbar_n + Q_n + Phi_G^T mu_{n+1}
    int cur = 0;
    PE_HIP(hipMemcpyAsync(p->io, p->Xb, sizeof(double) * rowsX * Dp, hipMemcpyDeviceToDevice, p->st));
    PE_HIP(axpy(p->io, p->Qb, 1.0, rowsX * Dp, p->st));
    const bool scan = B == 1 && p->coarse_scan && N >= 4;
    if (scan) {
        PE_TRY(scan_prepare(p));
        PE_TRY(coarse_adj_scan_initial(p, p->Xk[0], p->io));
    } else {
        PE_TRY(coarse_adj_initial(p, B, p->Xk[0], p->io));
    }
    PE_HIP(axpy(p->Xk[0], p->Qb, -1.0, rowsX * Dp, p->st));
    PE_TRY(adj_jumps_launch(p, B, p->Xk[0], nullptr, 0, N + 1));
    PE_TRY(jumps_read(p, B, thr.data()));
    for (int b = 0; b < B; ++b) thr[b] *= tol;

    int n_active = B;
    for (int k = 1; k <= k_max && n_active > 0; ++k) {
        const int nxt = 1 - cur;
        if (mixed && k >= 2) {
            // the transposed fine map is linear: add its action on the change
            // lam^{k-1} - lam^{k-2} (rows n = 0..N-1 in E) to the stored values
            PE_TRY(graph_run(p, {10, B, 2}, [&]() {
                return fine_adjoint_sweep(p, B, p->E, (long)N * Dp, N, nullptr, p->Fbuf, true, 0);
            }));
        } else {
            PE_TRY(graph_run(p, {10, B, cur, track ? 1 : 0}, [&]() -> pe_status {
                PE_TRY(fine_adjoint_sweep(p, B, p->Xk[cur], ldX, N + 1, inj, p->Fbuf, false, 0));
                PE_HIP(add_rows(p->Fbuf, p->Xb, B, N, Dp, p->st));
                return PE_OK;
            }));
        }
        if (n_active < B) PE_HIP(freeze_inactive(p->Xk[cur], p->Xk[nxt], p->active_d, ldX, B, p->st));
        PE_TRY(graph_run(p, {11, B, cur}, [&]() -> pe_status {
            if (scan)
                PE_TRY(coarse_adj_scan_correct(p, p->Xk[nxt], p->Xk[cur], p->active_d));
            else
                PE_TRY(coarse_adj_correct(p, B, p->Xk[nxt], p->Xk[cur], p->active_d));
            PE_TRY(adj_jumps_launch(p, B, p->Xk[nxt], p->Xk[cur], 0, N));
            return PE_OK;
        }));
        PE_TRY(jumps_read(p, B, J.data()));
        cur = nxt;
        for (int b = 0; b < B; ++b) {
            if (!active[b]) continue;
            if (!std::isfinite(J[b]))
                return fail(PE_ERR_NONFINITE, "non-finite adjoint jump for sample " + std::to_string(b) +
                                                  " at iteration " + std::to_string(k));
            if (jump_hist) jump_hist[(long)b * k_max + (k - 1)] = J[b];
            if (iters) iters[b] = k;
            if (J[b] <= thr[b]) {
                active[b] = 0;
                --n_active;
            }
        }
        if (n_active > 0 && n_active < B)
            PE_HIP(hipMemcpyAsync(p->active_d, active.data(), sizeof(int) * B, hipMemcpyHostToDevice, p->st));
    }
    const double* Lf = p->Xk[cur];
    // gradient with respect to the initial state: lambda_0
    PE_HIP(place(p->x0p, Dp, 0, 0, Lf, ldX, B, Dp, 1.0, 0, p->st));
    PE_HIP(unpack_states(p->x0p, x0bar, B, p->d1, p->d2, p->d1p, p->d2p, p->st));
    if (Lam) PE_HIP(unpack_states(Lf, Lam, rowsX, p->d1, p->d2, p->d1p, p->d2p, p->st));
    if (want_h) {
        // source adjoint: one transposed fine sweep from the final lambda,
        // the nu summed per interval (or kept per step), then (Z_h G)^T nu
        PE_TRY(graph_run(p, {12, B, cur, track ? 1 : 0, rho_all ? 1 : 0}, [&]() {
            return fine_adjoint_sweep(p, B, Lf, ldX, N + 1, inj, p->Fbuf, false, rho_all ? 2 : 1);
        }));
        const int Rp = p->Rp;
        const long tl = p->Tlen;
        const long rows_h = (long)B * tl;
        PE_TRY(gemm<double>(p, shape((int)rows_h, Rp, rho_all ? p->Rho : p->Sacc, Dp, p->ZGT, Dp, 0, Dp),
                            store_epi(p->Hb, Rp)));
        for (int b = 0; b < B; ++b)
            PE_HIP(place(Hbar + (long)b * p->R * tl, tl, 0, 0, p->Hb + (long)b * tl * Rp, Rp, p->R, (int)tl, 1.0, 1,
                         p->st));
    }
    PE_HIP(hipStreamSynchronize(p->st));
    PE_TRY(prof_collect(p));
    return n_active > 0 ? PE_WARN_NOT_CONVERGED : PE_OK;
}

pe_status pe_batch_create(pe_batch* out, int count, const pe_problem* problems, void* hip_stream) {
    g_err.clear();
    if (!out || count < 1 || !problems) return fail(PE_ERR_ARG, "bad arguments");
    *out = nullptr;
    for (int i = 0; i < count; ++i) {
        if (!problems[i]) return fail(PE_ERR_ARG, "null problem handle in the batch");
        PE_TRY(hist_unsupported(problems[i], "a batch"));
    }
    const int prec = problems[0]->prec, P = problems[0]->P;
    for (int i = 1; i < count; ++i) {
        if (problems[i]->prec != prec) return fail(PE_ERR_ARG, "all problems of a batch need the same precision");
        if (problems[i]->P != P) return fail(PE_ERR_ARG, "all problems of a batch need the same step ratio P");
        if (problems[i]->refine != problems[0]->refine)
            return fail(PE_ERR_ARG, "all problems of a batch need the same refinement (PE_MIXED_REFINE or not)");
    }
    pe_batch bt = new pe_batch_s();
    bt->count = count;
    bt->prec = prec;
    bt->refine = problems[0]->refine;
    bt->P = P;
    bt->pr.assign(problems, problems + count);
    for (pe_problem p : bt->pr) bt->N_max = std::max(bt->N_max, p->N);
    const char* gr = getenv("PE_GRAPHS");
    bt->gc.use_graphs = (gr && gr[0] == '0') ? 0 : 1;
    const char* xo = getenv("PE_BATCH_XCD");
    bt->xcd = (xo && xo[0] >= '0' && xo[0] <= '3') ? xo[0] - '0' : 2;
    bt->cfg.br = 64;
    bt->cfg.bs = 64;
    bt->cfg.splitk = 1;
    // 64 x 64 tiles, K depth 32 (FP32) / 16 (FP64): the LDS stages of a
    // work-group take 35 KiB (FP32), four work-groups per CU (measured on the
    // ragged 256-solve batch: 3 % faster than K depth 64, which fits two)
    bt->cfg.bk2 = 0;
    if (const char* t = getenv("PE_BATCH_TILE")) {
        int br = 0, bs = 0, bk2 = 0;
        if (sscanf(t, "%d %d %d", &br, &bs, &bk2) == 3 &&
            ((br == 32 && bs == 64) || (br == 64 && (bs == 64 || bs == 128)) || (br == 128 && bs == 64))) {
            bt->cfg.br = br;
            bt->cfg.bs = bs;
            bt->cfg.bk2 = bk2 ? 1 : 0;
        }
    }
    if (hip_stream) {
        bt->st = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&bt->st, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            delete bt;
            return fail(PE_ERR_HIP, "stream creation failed");
        }
        bt->own_stream = 1;
    }
    *out = bt;
    return PE_OK;
}

pe_status pe_batch_profile(pe_batch bt, int enable) {
    g_err.clear();
    if (!bt) return fail(PE_ERR_ARG, "null batch handle");
    PE_HIP(hipStreamSynchronize(bt->st));
    bt->prof.reset();
    bt->prof.on = enable ? 1 : 0;
    return PE_OK;
}

pe_status pe_batch_profile_read(pe_batch bt, int kind, double* total_ms, long long* launches) {
    g_err.clear();
    if (!bt) return fail(PE_ERR_ARG, "null batch handle");
    if (kind < 0 || kind >= PE_PROF_KINDS) return fail(PE_ERR_ARG, "unknown profile kind");
    PE_HIP(hipStreamSynchronize(bt->st));
    PE_TRY(prof_collect_on(bt->prof));
    if (total_ms) *total_ms = bt->prof.ms[kind];
    if (launches) *launches = bt->prof.n[kind];
    return PE_OK;
}

pe_status pe_batch_destroy(pe_batch bt) {
    if (!bt) return PE_OK;
    (void)hipStreamSynchronize(bt->st);
    bt->gc.clear();
    for (void* v : bt->allocs) (void)hipFree(v);
    if (bt->own_stream) (void)hipStreamDestroy(bt->st);
    delete bt;
    return PE_OK;
}

pe_status pe_batch_solve(pe_batch bt, const double* const* x0, double tol, int norm_mode, int k_max,
                         double* const* X, int* iters) {
    g_err.clear();
    if (!bt || !x0 || !X) return fail(PE_ERR_ARG, "bad arguments");
    if (!(tol >= 0) || k_max < 0) return fail(PE_ERR_ARG, "need tol >= 0 and k_max >= 0");
    if (norm_mode != PE_NORM_M_ABS && norm_mode != PE_NORM_M_REL) return fail(PE_ERR_ARG, "unknown norm_mode");
    const int G = bt->count;
    for (int g = 0; g < G; ++g) {
        if (!x0[g] || !X[g]) return fail(PE_ERR_ARG, "null state pointer for problem " + std::to_string(g));
        PE_TRY(hist_unsupported(bt->pr[g], "a batch"));
    }
    // samples per problem: the B of its source (1 without a source)
    bt->Bs.assign(G, 1);
    for (int g = 0; g < G; ++g) {
        pe_problem p = bt->pr[g];
        if (p->src_set) bt->Bs[g] = p->B_src;
        PE_TRY(ensure_workspace(p, bt->Bs[g]));
        PE_HIP(hipStreamSynchronize(p->st));
    }
    if (!bt->planned || batch_plan_keys(bt) != bt->plan_keys) PE_TRY(batch_plan(bt));
    PE_HIP(hipStreamSynchronize(bt->st));
    bt->pact.assign(G, 1);
    bt->fin_buf.assign(G, 0);
    if (!bt->tables_all) PE_TRY(batch_tables(bt));
    const bool mixed = bt->prec == PE_MIXED;
    const long rel = norm_mode == PE_NORM_M_REL ? 1 : 0;
    std::vector<int> act(bt->J_total, 1), conv(bt->J_total, 0), kcap(G);
    std::vector<double> thr(bt->J_total, tol), J(bt->J_total, 0.0);
    if (iters)
        for (int i = 0; i < bt->J_total; ++i) iters[i] = 0;
    for (int g = 0; g < G; ++g) {
        pe_problem p = bt->pr[g];
        kcap[g] = std::min(k_max, p->N);
        PE_HIP(pack_states(x0[g], p->x0p, bt->Bs[g], p->d1, p->d2, p->d1p, p->d2p, bt->st));
        PE_HIP(hipMemcpyAsync(p->active_d, act.data(), sizeof(int) * bt->Bs[g], hipMemcpyHostToDevice, bt->st));
    }
    int cur = 0;
    PE_TRY(graph_run_on(bt->gc, bt->st, bt->prof.on != 0, {0, rel}, [&]() -> pe_status {
        PE_HIP(grp_set_x0(bt->elems_d, bt->act_d, bt->n_act, 0, 0, bt->st));
        if (bt->scan) {
            // x_{n+1} = Phi_G x_n + c_n summed by the doubling scan over
            // t_0 = x0, t_n = c_{n-1} (FP32 products, FP64 sums)
            PE_HIP(grp_scan_init0(bt->elems_d, bt->act_d, bt->n_act, bt->st));
            for (int l = 0; l < bt->iscan_L; ++l) PE_TRY(grouped<float>(bt, bt->iscanp[l], PE_PROF_COARSE));
            PE_HIP(grp_scan_final0(bt->elems_d, bt->act_d, bt->n_act, bt->st));
        } else {
            for (int n = 0; n < bt->N_max; ++n) PE_TRY(coarse_grouped<double>(bt, bt->c_init, n, 0, 0));
        }
        if (rel) PE_TRY(batch_jumps(bt, 0, true));
        return PE_OK;
    }));
    if (rel) {
        PE_HIP(hipMemcpyAsync(thr.data(), bt->J_all, sizeof(double) * bt->J_total, hipMemcpyDeviceToHost, bt->st));
        PE_HIP(hipStreamSynchronize(bt->st));
        for (double& t : thr) t *= tol;
    }
    // samples of problems with no iteration allowed are done at once
    bool shrink = false;
    for (int g = 0; g < G; ++g)
        if (kcap[g] == 0) {
            for (int b = 0; b < bt->Bs[g]; ++b) act[bt->J_off[g] + b] = 0;
            bt->pact[g] = 0;
            shrink = true;
        }
    auto n_act = [&]() { return (int)std::count(act.begin(), act.end(), 1); };
    if (shrink && n_act() > 0) PE_TRY(batch_tables(bt));
    std::vector<int> pushed(act);
    for (int k = 1; n_act() > 0; ++k) {
        const int nxt = 1 - cur;
        // active flags to the device where they changed
        for (int g = 0; g < G; ++g) {
            if (!bt->pact[g]) continue;
            const int o = bt->J_off[g];
            if (!std::equal(act.begin() + o, act.begin() + o + bt->Bs[g], pushed.begin() + o)) {
                PE_HIP(hipMemcpyAsync(bt->pr[g]->active_d, act.data() + o, sizeof(int) * bt->Bs[g],
                                      hipMemcpyHostToDevice, bt->st));
                std::copy(act.begin() + o, act.begin() + o + bt->Bs[g], pushed.begin() + o);
            }
        }
        const long ah = bt->act_hash;
        if (mixed && k >= 2)
            PE_TRY(graph_run_on(bt->gc, bt->st, bt->prof.on != 0, {1, 2, ah},
                                [&]() { return batch_fine_sweep(bt, cur, true); }));
        else
            PE_TRY(graph_run_on(bt->gc, bt->st, bt->prof.on != 0, {1, cur, ah},
                                [&]() { return batch_fine_sweep(bt, cur, false); }));
        for (int g = 0; g < G; ++g) {
            if (!bt->pact[g]) continue;
            pe_problem p = bt->pr[g];
            const int o = bt->J_off[g];
            if (std::count(act.begin() + o, act.begin() + o + bt->Bs[g], 1) < bt->Bs[g])
                PE_HIP(freeze_inactive(p->Xk[cur], p->Xk[nxt], p->active_d, (long)(p->N + 1) * p->Dp, bt->Bs[g],
                                       bt->st));
        }
        PE_TRY(graph_run_on(bt->gc, bt->st, bt->prof.on != 0, {2, cur, ah}, [&]() -> pe_status {
            PE_HIP(grp_set_x0(bt->elems_d, bt->act_d, bt->n_act, nxt, mixed ? 2 : 1, bt->st));
            if (bt->scan) {
                // change form d_{n+1} = Phi_G d_n + e_n, e_n = F(x_n^{k-1}) - x_{n+1}^{k-1},
                // summed by the doubling scan; then x_n^k = x_n^{k-1} + d_n
                PE_HIP(grp_scan_init(bt->elems_d, bt->act_d, bt->n_act, cur, bt->st));
                for (int l = 0; l < bt->scan_L; ++l) PE_TRY(grouped<float>(bt, bt->scanp[l], PE_PROF_COARSE));
                PE_HIP(grp_scan_final(bt->elems_d, bt->act_d, bt->n_act, cur, nxt, bt->st));
            } else {
                for (int n = 0; n < bt->N_max; ++n) {
                    if (mixed)
                        PE_TRY(coarse_grouped<float>(bt, bt->c_corr[cur], n, 1, n & 1));
                    else
                        PE_TRY(coarse_grouped<double>(bt, bt->c_corr[cur], n, 1, n & 1));
                }
            }
            PE_TRY(batch_jumps(bt, nxt, false));
            return PE_OK;
        }));
        PE_HIP(hipMemcpyAsync(J.data(), bt->J_all, sizeof(double) * bt->J_total, hipMemcpyDeviceToHost, bt->st));
        PE_HIP(hipStreamSynchronize(bt->st));
        PE_TRY(prof_collect_on(bt->prof));
        cur = nxt;
        for (int g = 0; g < G; ++g) {
            for (int b = 0; b < bt->Bs[g]; ++b) {
                const int i = bt->J_off[g] + b;
                if (!act[i]) continue;
                if (!std::isfinite(J[i]))
                    return fail(PE_ERR_NONFINITE, "non-finite parareal jump for problem " + std::to_string(g) +
                                                      " sample " + std::to_string(b) + " at iteration " +
                                                      std::to_string(k));
                if (iters) iters[i] = k;
                if (J[i] <= thr[i]) conv[i] = 1;
                if (conv[i] || k >= kcap[g]) act[i] = 0;
            }
        }
        // problems with no sample left leave the launches; their last
        // iterate stays in buffer fin_buf
        shrink = false;
        for (int g = 0; g < G; ++g) {
            if (!bt->pact[g]) continue;
            const int o = bt->J_off[g];
            if (std::count(act.begin() + o, act.begin() + o + bt->Bs[g], 1) == 0) {
                bt->pact[g] = 0;
                bt->fin_buf[g] = cur;
                shrink = true;
            }
        }
        if (shrink && n_act() > 0) PE_TRY(batch_tables(bt));
    }
    bool all_conv = true;
    for (int g = 0; g < G; ++g) {
        pe_problem p = bt->pr[g];
        const int fb = bt->pact[g] ? cur : bt->fin_buf[g];
        PE_HIP(unpack_states(p->Xk[fb], X[g], (long)bt->Bs[g] * (p->N + 1), p->d1, p->d2, p->d1p, p->d2p, bt->st));
    }
    for (int i = 0; i < bt->J_total; ++i)
        if (!conv[i]) all_conv = false;
    PE_HIP(hipStreamSynchronize(bt->st));
    PE_TRY(prof_collect_on(bt->prof));
    return all_conv ? PE_OK : PE_WARN_NOT_CONVERGED;
}

}  // extern "C"
