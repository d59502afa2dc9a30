// Launchers of the element-wise / reduction kernels of libpe.
#pragma once
#include "pe_internal.h"

namespace pe {
hipError_t pack_states(const double* src, double* dst, long rows, int d1, int d2, int d1p, int d2p,
                       hipStream_t st);
hipError_t unpack_states(const double* src, double* dst, long rows, int d1, int d2, int d1p, int d2p,
                         hipStream_t st);
// states of X have stride sx (0: Dp)
hipError_t fine_init(const double* X, long ldXb, int row_off, int nvalid, double* Xa, double* dev64,
                     float* dev32, int B, int N, int Dp, hipStream_t st, int sx = 0);
hipError_t adj_init(const double* src, const double* add, long ld_add, double* S, float* nu32, double* nu_set,
                    long ld_set, long rows, int Dp, hipStream_t st);
hipError_t axpy(double* y, const double* x, double a, long n, hipStream_t st);
hipError_t zero_row0(double* X, long ldb, int B, int Dp, hipStream_t st);
hipError_t sample_dot_sums(const double* Y, const double* Z, int B, long rows_per_b, int Dp, double scale,
                           double* tmp_rows, double* J, hipStream_t st);
hipError_t take_a(const double* S, double* Y, long rows, int Dp, int accumulate, hipStream_t st);
hipError_t add_rows(double* Y, const double* X, int B, int N, int Dp, hipStream_t st);
hipError_t copy_row(const double* src, double* dst, long ldb, int B, int Dp, hipStream_t st);
hipError_t fine_final(const double* Xa, const double* dev64, double* Y, long rows, int Dp, int d1p,
                      int accumulate, hipStream_t st, long ldy = 0);
hipError_t jump_diff(const double* Xk, const double* Xp, long ldXb, int n0, int nr, int B, int Dp,
                     double* E, hipStream_t st, int sx = 0);
hipError_t jump_reduce(const double* E, const double* Y, int B, int nr, int Dp, double* J, double* norms,
                       hipStream_t st, long lde = 0);
hipError_t freeze_inactive(const double* Xsrc, double* Xdst, const int* active, long ldXb, int B,
                           hipStream_t st);
hipError_t zero_fill(double* a, float* b, long n, hipStream_t st);
// coarse sweep as a scan (one sample): t[n] = F[n] - Xp[n + xrow] (n < N,
// rows of Dp, FP32 copy nullable); X[n + xrow] = Xp[n + xrow] + t[n] (Xp
// nullable: zero) unless the sample is inactive
hipError_t scan_init(const double* F, const double* Xp, int xrow, double* t64, float* t32, int N, int Dp,
                     hipStream_t st);
hipError_t scan_final(const double* Xp, const double* t, double* X, int xrow, int N, int Dp, const int* active,
                      hipStream_t st);
// initial sweep as a scan: t[0] = x0, t[n] = cs[n-1] (n = 1..N; cs nullable:
// zero source). scan_final with Xp = nullptr then copies t[1..N] to X[1..N].
hipError_t scan_init0(const double* x0, const double* cs, double* t, float* t32, int N, int Dp, hipStream_t st);
hipError_t set_x0(const double* x0p, double* X, long ldXb, int B, int Dp, hipStream_t st, int sx = 0);
// carried history
hipError_t gather_rows(const double* X, long ldXb, int sx, int off, int row_off, int nvalid, double* out, int B,
                       int N, int Dp, hipStream_t st);
hipError_t hist_put(const double* H, double* dev64, float* dev32, long rows, int Dp, int d1p, hipStream_t st);
hipError_t hist_get(const double* dev64, double* out, long ldo, long rows, int Dp, int d1p, int accumulate,
                    hipStream_t st);
hipError_t aug_cs(const double* CS, double* CSa, long rows, int Dp, int P, hipStream_t st);
hipError_t hist_phi(const double* Phi, double* out, int Dp, int P, hipStream_t st);
hipError_t place(double* dst, long ldd, int ro, int co, const double* src, long lds, int rows, int cols,
                 double scale, int trans, hipStream_t st, int accumulate = 0);
hipError_t shifted_embed(double* dst, int n, const double* A, const double* Bm, long lds, int d,
                         double cb, hipStream_t st);
hipError_t tril(double* A, int n, hipStream_t st);
hipError_t eye(double* A, int n, int d, hipStream_t st);
hipError_t to_f32(const double* src, float* dst, long n, hipStream_t st);
hipError_t asym(const double* X, const double* Y, long ldx, long ldy, int rows, int cols,
                unsigned long long* out2, hipStream_t st);
hipError_t chol_diag(double* Am, long ld, int j, double* Linv, int* info, hipStream_t st);
// waveform relaxation in time
hipError_t wr_twiddle(double* tw, int P, int K, double alpha, hipStream_t st);
hipError_t wr_dft(int dir, const double* src, double* dst, const double* tw, int P, int K, long NB, int d1p,
                  hipStream_t st);
hipError_t wr_cat(const double* L, double* out, int P, long NB, int d, int mode, hipStream_t st);
hipError_t wr_axmy(double* y, const double* a, const double* b, double alpha, long n, hipStream_t st);
hipError_t wr_io(int dir, const double* X, long ldXb, double* Fout, int N, int d1, int d2, int d1p, int d2p,
                 int c0, int NBc, int P, double* Ul, double* Wl, hipStream_t st);
// Grouped element-wise steps of a batch of different problems: one launch
// covers every active problem (act[0..n_act-1] index the BatchElem array),
// each with the arithmetic and order of the one-problem kernels above.
struct BatchElem {
    double* Xk[2] = {nullptr, nullptr};  // B x (N + 1) x Dp iterates
    double* E = nullptr;                 // jump differences (B x (N + 1) x Dp)
    const double* Yn = nullptr;          // M E
    double* nrm = nullptr;               // B x (N + 1) row norms
    double* J = nullptr;                 // B jumps
    const double* x0p = nullptr;         // B x Dp
    double* Dl64 = nullptr;              // B x Dp change buffer to clear (nullable)
    float* Dl32 = nullptr;
    double* Xa = nullptr;                // fine sweep: anchors (B x N x Dp)
    double* R64 = nullptr;               // mixed: whitened anchors / results
    double* dev64[2] = {nullptr, nullptr};
    float* dev32 = nullptr;
    double* Fbuf = nullptr;              // B x N x Dp fine values
    const double* CS = nullptr;          // B x N x Dp coarse source (nullable)
    double* t64[2] = {nullptr, nullptr}; // scan buffers (B x (Z + N + 1) x Dp)
    float* t32 = nullptr;                // FP32 copy of t64[0]
    const int* active = nullptr;         // B flags
    int B = 0, N = 0, Dp = 0, d1p = 0, Z = 0, L = 0, L0 = 0;
};
// x0 into row 0 of X^xk; zero_mode 1/2 also clears the B x Dp change buffer
// (FP64 / FP32)
hipError_t grp_set_x0(const BatchElem* it, const int* act, int n_act, int xk, int zero_mode, hipStream_t st);
// fine sweep start (incremental: anchors from E with rows shifted by one,
// else from X^cur) and end (mixed: R64, else Fbuf, gets anchors + deviation)
hipError_t grp_fine_init(const BatchElem* it, const int* act, int n_act, int cur, int incremental, int mixed,
                         hipStream_t st);
hipError_t grp_fine_final(const BatchElem* it, const int* act, int n_act, int P, int mixed, hipStream_t st);
// jump differences (rel: the rows n = 0..N of X^xk) and the row norms with the
// per-sample maximum
hipError_t grp_jump_diff(const BatchElem* it, const int* act, int n_act, int xk, int rel, hipStream_t st);
hipError_t grp_jump_reduce(const BatchElem* it, const int* act, int n_act, int Bmax, int rel, hipStream_t st);
// scans of the coarse sweeps: correction (t = F - X^cur rows 1..N, then
// X^nxt = X^cur + t) and initial sweep (t_0 = x0, t_n = c_{n-1}, then X^0
// rows 1..N = t)
hipError_t grp_scan_init(const BatchElem* it, const int* act, int n_act, int cur, hipStream_t st);
hipError_t grp_scan_final(const BatchElem* it, const int* act, int n_act, int cur, int nxt, hipStream_t st);
hipError_t grp_scan_init0(const BatchElem* it, const int* act, int n_act, hipStream_t st);
hipError_t grp_scan_final0(const BatchElem* it, const int* act, int n_act, hipStream_t st);
// peak probes: kind 0 FP32 MFMA, 1 FP64 MFMA (blocks x 256 threads, iters
// rounds of 16 independent 16x16x4 products per wave), 2 copy of n float4
hipError_t probe_launch(int kind, int blocks, int iters, void* out, const void* src, long n, hipStream_t st);
}  // namespace pe
