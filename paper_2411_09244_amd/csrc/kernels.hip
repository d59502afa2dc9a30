// Element-wise and reduction kernels of libpe: state layout conversion, fine
// sweep set-up/finish, parareal jump norms (eq. (2.8)), step-operator
// assembly and the per-block part of the FP64 Cholesky factorisation.
#include "pe_kernels.h"

#include <algorithm>

namespace pe {

static inline dim3 grid1(long n, int bs = 256) {
    long g = (n + bs - 1) / bs;
    if (g > 65535L * 64) g = 65535L * 64;
    return dim3((unsigned)(g < 1 ? 1 : g));
}

// ---------------------------------------------------------------------------
// state layout: user [u (d1) | w (d2)]  <->  internal [u (d1p) | w (d2p)]
// ---------------------------------------------------------------------------
__global__ void k_pack(const double* __restrict__ src, double* __restrict__ dst, long rows, int d1,
                       int d2, int d1p, int d2p) {
    const long Dp = d1p + d2p, D = d1 + d2;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < rows * Dp;
         i += (long)gridDim.x * blockDim.x) {
        const long r = i / Dp;
        const int s = (int)(i - r * Dp);
        double v = 0.0;
        if (s < d1)
            v = src[r * D + s];
        else if (s >= d1p && s < d1p + d2)
            v = src[r * D + d1 + (s - d1p)];
        dst[i] = v;
    }
}

__global__ void k_unpack(const double* __restrict__ src, double* __restrict__ dst, long rows, int d1,
                         int d2, int d1p, int d2p) {
    const long Dp = d1p + d2p, D = d1 + d2;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < rows * D;
         i += (long)gridDim.x * blockDim.x) {
        const long r = i / D;
        const int s = (int)(i - r * D);
        dst[i] = (s < d1) ? src[r * Dp + s] : src[r * Dp + d1p + (s - d1)];
    }
}

hipError_t pack_states(const double* src, double* dst, long rows, int d1, int d2, int d1p, int d2p,
                       hipStream_t st) {
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack, grid1(rows * (d1p + d2p)), dim3(256), 0, st, src, dst, rows, d1, d2,
                       d1p, d2p);
    return hipGetLastError();
}

hipError_t unpack_states(const double* src, double* dst, long rows, int d1, int d2, int d1p, int d2p,
                         hipStream_t st) {
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_unpack, grid1(rows * (long)(d1 + d2)), dim3(256), 0, st, src, dst, rows, d1,
                       d2, d1p, d2p);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// fine sweep: gather anchors X[b][n + row_off] (zero unless
// 0 <= n + row_off < nvalid) into Xa[b*N + n], zero the deviation state;
// afterwards Y (+)= Xa + deviation.
// ---------------------------------------------------------------------------
__global__ void k_fine_init(const double* __restrict__ X, long ldXb, int sx, int row_off, int nvalid,
                            double* __restrict__ Xa, double* __restrict__ dev64, float* __restrict__ dev32,
                            int B, int N, int Dp) {
    const long rows = (long)B * N;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < rows * Dp;
         i += (long)gridDim.x * blockDim.x) {
        const long r = i / Dp;
        const int s = (int)(i - r * Dp);
        const long b = r / N, n = r - b * N;
        const long j = n + row_off;
        Xa[i] = (j >= 0 && j < nvalid) ? X[b * ldXb + j * sx + s] : 0.0;
        dev64[r * 2 * Dp + s] = 0.0;
        dev64[r * 2 * Dp + Dp + s] = 0.0;
        if (dev32) {
            dev32[r * 2 * Dp + s] = 0.0f;
            dev32[r * 2 * Dp + Dp + s] = 0.0f;
        }
    }
}

hipError_t fine_init(const double* X, long ldXb, int row_off, int nvalid, double* Xa, double* dev64,
                     float* dev32, int B, int N, int Dp, hipStream_t st, int sx) {
    hipLaunchKernelGGL(k_fine_init, grid1((long)B * N * Dp), dim3(256), 0, st, X, ldXb, sx > 0 ? sx : Dp,
                       row_off, nvalid, Xa, dev64, dev32, B, N, Dp);
    return hipGetLastError();
}

// Y[r][s] (+)= Xa[r][s] + dev[r][d1p + s]  (u and w deviations sit at d1p + s)
__global__ void k_fine_final(const double* __restrict__ Xa, const double* __restrict__ dev64,
                             double* __restrict__ Y, long ldy, long rows, int Dp, int d1p, int accumulate) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < rows * Dp;
         i += (long)gridDim.x * blockDim.x) {
        const long r = i / Dp;
        const int s = (int)(i - r * Dp);
        const double v = Xa[i] + dev64[r * 2 * Dp + d1p + s];
        double* y = Y + r * ldy + s;
        *y = accumulate ? *y + v : v;
    }
}

hipError_t fine_final(const double* Xa, const double* dev64, double* Y, long rows, int Dp, int d1p,
                      int accumulate, hipStream_t st, long ldy) {
    hipLaunchKernelGGL(k_fine_final, grid1(rows * Dp), dim3(256), 0, st, Xa, dev64, Y, ldy > 0 ? ldy : Dp, rows,
                       Dp, d1p, accumulate);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// jump norms of eq. (2.8): E[b*nr + j] = Xk[b][n0 + j] - Xp[b][n0 + j]
// (Xp may be null: plain norms), then J_b = max_j sqrt(E_j . (M E_j)).
// ---------------------------------------------------------------------------
// (states of stride sx, copied whole: with carried history E holds the
// change of [x | delta], the norm below reads its first Dp entries)
__global__ void k_jump_diff(const double* __restrict__ Xk, const double* __restrict__ Xp, long ldXb,
                            int n0, int nr, int B, int sx, double* __restrict__ E) {
    const long rows = (long)B * nr;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < rows * sx;
         i += (long)gridDim.x * blockDim.x) {
        const long r = i / sx;
        const int s = (int)(i - r * sx);
        const long b = r / nr, j = r - b * nr;
        const long o = b * ldXb + (n0 + j) * sx + s;
        E[i] = Xp ? (Xk[o] - Xp[o]) : Xk[o];
    }
}

hipError_t jump_diff(const double* Xk, const double* Xp, long ldXb, int n0, int nr, int B, int Dp,
                     double* E, hipStream_t st, int sx) {
    if (sx <= 0) sx = Dp;
    hipLaunchKernelGGL(k_jump_diff, grid1((long)B * nr * sx), dim3(256), 0, st, Xk, Xp, ldXb, n0, nr, B,
                       sx, E);
    return hipGetLastError();
}

// one work-group per state row: norms[r] = sqrt(E_r . Y_r) (fixed order)
__global__ __launch_bounds__(256) void k_row_norms(const double* __restrict__ E, long lde,
                                                   const double* __restrict__ Y, int Dp, double* __restrict__ norms) {
    __shared__ double red[4];
    const long r = blockIdx.x;
    double acc = 0.0;
    for (int s = threadIdx.x; s < Dp; s += 256) acc += E[r * lde + s] * Y[r * Dp + s];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double q = (red[0] + red[1]) + (red[2] + red[3]);
        norms[r] = (q == q && q < 1.7e308 && q > -1.7e308) ? sqrt(q > 0.0 ? q : 0.0) : __builtin_nan("");
    }
}

// J[b] = max_j norms[b*nr + j] (NaN if any is NaN)
__global__ void k_sample_max(const double* __restrict__ norms, int B, int nr, double* __restrict__ J) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    double m = 0.0;
    bool bad = false;
    for (int j = 0; j < nr; ++j) {
        const double v = norms[(long)b * nr + j];
        if (!(v == v)) bad = true;
        if (v > m) m = v;
    }
    J[b] = bad ? __builtin_nan("") : m;
}

hipError_t jump_reduce(const double* E, const double* Y, int B, int nr, int Dp, double* J, double* norms,
                       hipStream_t st, long lde) {
    hipLaunchKernelGGL(k_row_norms, dim3((unsigned)((long)B * nr)), dim3(256), 0, st, E, lde > 0 ? lde : Dp, Y, Dp,
                       norms);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sample_max, dim3((B + 63) / 64), dim3(64), 0, st, norms, B, nr, J);
    return hipGetLastError();
}

__global__ void k_zero(double* __restrict__ a, float* __restrict__ b, long n) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        if (a) a[i] = 0.0;
        if (b) b[i] = 0.0f;
    }
}

__global__ void k_scan_init(const double* __restrict__ F, const double* __restrict__ Xp, long xoff,
                            double* __restrict__ t64, float* __restrict__ t32, long n_el) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n_el) return;
    const double v = F[i] - Xp[i + xoff];
    t64[i] = v;
    if (t32) t32[i] = (float)v;
}

hipError_t scan_init(const double* F, const double* Xp, int xrow, double* t64, float* t32, int N, int Dp,
                     hipStream_t st) {
    const long n_el = (long)N * Dp;
    hipLaunchKernelGGL(k_scan_init, dim3((unsigned)((n_el + 255) / 256)), dim3(256), 0, st, F, Xp, (long)xrow * Dp,
                       t64, t32, n_el);
    return hipGetLastError();
}

__global__ void k_scan_final(const double* __restrict__ Xp, const double* __restrict__ t, double* __restrict__ X,
                             long n_el, long xoff, const int* __restrict__ active) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n_el || (active && !active[0])) return;
    X[i + xoff] = (Xp ? Xp[i + xoff] : 0.0) + t[i];
}

__global__ void k_scan_init0(const double* __restrict__ x0, const double* __restrict__ cs, double* __restrict__ t,
                             float* __restrict__ t32, long n_el, int Dp) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n_el) return;
    const double v = i < Dp ? x0[i] : (cs ? cs[i - Dp] : 0.0);
    t[i] = v;
    if (t32) t32[i] = (float)v;
}

hipError_t scan_init0(const double* x0, const double* cs, double* t, float* t32, int N, int Dp, hipStream_t st) {
    const long n_el = (long)(N + 1) * Dp;
    hipLaunchKernelGGL(k_scan_init0, dim3((unsigned)((n_el + 255) / 256)), dim3(256), 0, st, x0, cs, t, t32, n_el,
                       Dp);
    return hipGetLastError();
}

hipError_t scan_final(const double* Xp, const double* t, double* X, int xrow, int N, int Dp, const int* active,
                      hipStream_t st) {
    const long n_el = (long)N * Dp;
    hipLaunchKernelGGL(k_scan_final, dim3((unsigned)((n_el + 255) / 256)), dim3(256), 0, st, Xp, t, X, n_el,
                       (long)xrow * Dp, active);
    return hipGetLastError();
}

hipError_t zero_fill(double* a, float* b, long n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero, grid1(n), dim3(256), 0, st, a, b, n);
    return hipGetLastError();
}

// adjoint sweep state [a | nu] (2Dp per column): a = nu = src (+ add, a
// row of stride ld_add, when given); FP32 copy of nu when nu32 is given; a
// copy of nu at nu_set + r*ld_set when given
__global__ void k_adj_init(const double* __restrict__ src, const double* __restrict__ add, long ld_add,
                           double* __restrict__ S, float* __restrict__ nu32, double* __restrict__ nu_set,
                           long ld_set, long rows, int Dp) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < rows * Dp;
         i += (long)gridDim.x * blockDim.x) {
        const long r = i / Dp;
        const int s = (int)(i - r * Dp);
        double v = src[i];
        if (add) v += add[r * ld_add + s];
        S[r * 2 * Dp + s] = v;
        S[r * 2 * Dp + Dp + s] = v;
        if (nu32) nu32[i] = (float)v;
        if (nu_set) nu_set[r * ld_set + s] = v;
    }
}

hipError_t adj_init(const double* src, const double* add, long ld_add, double* S, float* nu32, double* nu_set,
                    long ld_set, long rows, int Dp, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_init, grid1(rows * Dp), dim3(256), 0, st, src, add, ld_add, S, nu32, nu_set, ld_set,
                       rows, Dp);
    return hipGetLastError();
}

// y += a * x (n elements)
__global__ void k_axpy(double* __restrict__ y, const double* __restrict__ x, double a, long n) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        y[i] += a * x[i];
}

hipError_t axpy(double* y, const double* x, double a, long n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_axpy, grid1(n), dim3(256), 0, st, y, x, a, n);
    return hipGetLastError();
}

// X[b][0][s] = 0 for every sample (rows of Dp, sample stride ldb)
__global__ void k_zero_row0(double* __restrict__ X, long ldb, int B, int Dp) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < (long)B * Dp;
         i += (long)gridDim.x * blockDim.x) {
        const long b = i / Dp;
        X[b * ldb + (i - b * Dp)] = 0.0;
    }
}

hipError_t zero_row0(double* X, long ldb, int B, int Dp, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_row0, grid1((long)B * Dp), dim3(256), 0, st, X, ldb, B, Dp);
    return hipGetLastError();
}

// J[b] = scale * sum over the rows_per_b rows of sample b of dot(Y_row, Z_row):
// one block per row for the dots, then one block per sample sums them in a
// fixed order
__global__ __launch_bounds__(256) void k_row_dots(const double* __restrict__ Y, const double* __restrict__ Z,
                                                  int Dp, double* __restrict__ out) {
    __shared__ double red[4];
    const long r = blockIdx.x;
    double acc = 0.0;
    for (int s = threadIdx.x; s < Dp; s += 256) acc += Y[r * Dp + s] * Z[r * Dp + s];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[r] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void k_sample_sum(const double* __restrict__ v, long rows_per_b, double scale,
                                                    double* __restrict__ J) {
    __shared__ double red[4];
    const long b = blockIdx.x;
    double acc = 0.0;
    for (long j = threadIdx.x; j < rows_per_b; j += 256) acc += v[b * rows_per_b + j];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) J[b] = scale * ((red[0] + red[1]) + (red[2] + red[3]));
}

hipError_t sample_dot_sums(const double* Y, const double* Z, int B, long rows_per_b, int Dp, double scale,
                           double* tmp_rows, double* J, hipStream_t st) {
    const long rows = (long)B * rows_per_b;
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_row_dots, dim3((unsigned)rows), dim3(256), 0, st, Y, Z, Dp, tmp_rows);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sample_sum, dim3((unsigned)B), dim3(256), 0, st, tmp_rows, rows_per_b, scale, J);
    return hipGetLastError();
}

// Y[r][s] (+)= S[r][s]  (the a-part of the adjoint state)
__global__ void k_take_a(const double* __restrict__ S, double* __restrict__ Y, long rows, int Dp, int accumulate) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < rows * Dp;
         i += (long)gridDim.x * blockDim.x) {
        const long r = i / Dp;
        const int s = (int)(i - r * Dp);
        const double v = S[r * 2 * Dp + s];
        Y[i] = accumulate ? Y[i] + v : v;
    }
}

hipError_t take_a(const double* S, double* Y, long rows, int Dp, int accumulate, hipStream_t st) {
    hipLaunchKernelGGL(k_take_a, grid1(rows * Dp), dim3(256), 0, st, S, Y, rows, Dp, accumulate);
    return hipGetLastError();
}

// Y[b][n][s] += X[b][n][s] for n < N (X has N+1 rows per sample, Y has N)
__global__ void k_add_rows(double* __restrict__ Y, const double* __restrict__ X, int B, int N, int Dp) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < (long)B * N * Dp;
         i += (long)gridDim.x * blockDim.x) {
        const long r = i / Dp;
        const int s = (int)(i - r * Dp);
        const long b = r / N, n = r - b * N;
        Y[i] += X[(b * (N + 1) + n) * Dp + s];
    }
}

hipError_t add_rows(double* Y, const double* X, int B, int N, int Dp, hipStream_t st) {
    hipLaunchKernelGGL(k_add_rows, grid1((long)B * N * Dp), dim3(256), 0, st, Y, X, B, N, Dp);
    return hipGetLastError();
}

// X[b][row] = src[b][row] for every sample (rows of length Dp, strides ldb)
__global__ void k_copy_row(const double* __restrict__ src, double* __restrict__ dst, long ldb, int B, int Dp) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < (long)B * Dp;
         i += (long)gridDim.x * blockDim.x) {
        const long b = i / Dp;
        const int s = (int)(i - b * Dp);
        dst[b * ldb + s] = src[b * ldb + s];
    }
}

hipError_t copy_row(const double* src, double* dst, long ldb, int B, int Dp, hipStream_t st) {
    hipLaunchKernelGGL(k_copy_row, grid1((long)B * Dp), dim3(256), 0, st, src, dst, ldb, B, Dp);
    return hipGetLastError();
}

// copy Xsrc[b] -> Xdst[b] for samples that stopped iterating
__global__ void k_freeze(const double* __restrict__ Xsrc, double* __restrict__ Xdst,
                         const int* __restrict__ active, long ldXb, int B) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < (long)B * ldXb;
         i += (long)gridDim.x * blockDim.x) {
        const long b = i / ldXb;
        if (!active[b]) Xdst[i] = Xsrc[i];
    }
}

hipError_t freeze_inactive(const double* Xsrc, double* Xdst, const int* active, long ldXb, int B,
                           hipStream_t st) {
    hipLaunchKernelGGL(k_freeze, grid1((long)B * ldXb), dim3(256), 0, st, Xsrc, Xdst, active, ldXb, B);
    return hipGetLastError();
}

// x0 into row 0 of every sample of X (x_0^k = x_0)
// (states of stride sx >= Dp: the entries past Dp, the carried history, are
// zero at t = 0)
__global__ void k_set_x0(const double* __restrict__ x0p, double* __restrict__ X, long ldXb, int B,
                         int Dp, int sx) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < (long)B * sx;
         i += (long)gridDim.x * blockDim.x) {
        const long b = i / sx;
        const int s = (int)(i - b * sx);
        X[b * ldXb + s] = s < Dp ? x0p[b * Dp + s] : 0.0;
    }
}

hipError_t set_x0(const double* x0p, double* X, long ldXb, int B, int Dp, hipStream_t st, int sx) {
    if (sx <= 0) sx = Dp;
    hipLaunchKernelGGL(k_set_x0, grid1((long)B * sx), dim3(256), 0, st, x0p, X, ldXb, B, Dp, sx);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// grouped element-wise steps of a batch: ch work-groups per active problem
// (64 for 256 or more problems, up to 4096 for one), each striding over
// that problem's elements
// ---------------------------------------------------------------------------
static inline int grp_ch(int n_act) { return std::max(64, std::min(4096, 16384 / std::max(1, n_act))); }

#define GRP_LOOP(n_el) \
    for (long i = (long)(blockIdx.x % ch) * 256 + threadIdx.x; i < (n_el); i += (long)ch * 256)

__global__ void k_grp_set_x0(const BatchElem* __restrict__ it, const int* __restrict__ act, int ch, int xk,
                             int zero_mode) {
    const BatchElem& e = it[act[blockIdx.x / ch]];
    GRP_LOOP((long)e.B * e.Dp) {
        const long b = i / e.Dp;
        const int s = (int)(i - b * e.Dp);
        e.Xk[xk][b * (long)(e.N + 1) * e.Dp + s] = e.x0p[i];
        if (zero_mode == 1) e.Dl64[i] = 0.0;
        if (zero_mode == 2) e.Dl32[i] = 0.0f;
    }
}

__global__ void k_grp_fine_init(const BatchElem* __restrict__ it, const int* __restrict__ act, int ch, int cur, int inc,
                                int mixed) {
    const BatchElem& e = it[act[blockIdx.x / ch]];
    GRP_LOOP((long)e.B * e.N * e.Dp) {
        const int Dp = e.Dp, N = e.N;
        const long r = i / Dp;
        const int s = (int)(i - r * Dp);
        const long b = r / N, n = r - b * N;
        const long j = n + (inc ? -1 : 0);
        const double* X = inc ? e.E : e.Xk[cur];
        const long ldXb = inc ? (long)N * Dp : (long)(N + 1) * Dp;
        double* Xa = mixed ? e.R64 : e.Xa;
        Xa[i] = (j >= 0 && j < N) ? X[b * ldXb + j * Dp + s] : 0.0;
        e.dev64[0][r * 2 * Dp + s] = 0.0;
        e.dev64[0][r * 2 * Dp + Dp + s] = 0.0;
        if (mixed) {
            e.dev32[r * 2 * Dp + s] = 0.0f;
            e.dev32[r * 2 * Dp + Dp + s] = 0.0f;
        }
    }
}

__global__ void k_grp_fine_final(const BatchElem* __restrict__ it, const int* __restrict__ act, int ch, int P,
                                 int mixed) {
    const BatchElem& e = it[act[blockIdx.x / ch]];
    GRP_LOOP((long)e.B * e.N * e.Dp) {
        const int Dp = e.Dp;
        const long r = i / Dp;
        const int s = (int)(i - r * Dp);
        const double v = e.Xa[i] + e.dev64[P & 1][r * 2 * Dp + e.d1p + s];
        (mixed ? e.R64 : e.Fbuf)[r * Dp + s] = v;
    }
}

__global__ void k_grp_jump_diff(const BatchElem* __restrict__ it, const int* __restrict__ act, int ch, int xk,
                                int rel) {
    const BatchElem& e = it[act[blockIdx.x / ch]];
    const int nr0 = rel ? e.N + 1 : e.N;
    GRP_LOOP((long)e.B * nr0 * e.Dp) {
        const int Dp = e.Dp, nr = rel ? e.N + 1 : e.N, n0 = rel ? 0 : 1;
        const long r = i / Dp;
        const int s = (int)(i - r * Dp);
        const long b = r / nr, j = r - b * nr;
        const long o = b * (long)(e.N + 1) * Dp + (n0 + j) * Dp + s;
        e.E[i] = rel ? e.Xk[xk][o] : (e.Xk[xk][o] - e.Xk[1 - xk][o]);
    }
}

// one work-group per (problem, sample): the sample's row norms (each row
// reduced exactly as k_row_norms does) and their maximum (as k_sample_max)
__global__ __launch_bounds__(256) void k_grp_jump_reduce(const BatchElem* __restrict__ it, const int* __restrict__ act,
                                                         int Bmax, int rel) {
    const BatchElem& e = it[act[blockIdx.x / Bmax]];
    const int b = blockIdx.x % Bmax;
    if (b >= e.B) return;
    __shared__ double red[4];
    const int Dp = e.Dp, nr = rel ? e.N + 1 : e.N;
    double m = 0.0;
    bool bad = false;
    for (int j = 0; j < nr; ++j) {
        const long r = (long)b * nr + j;
        double acc = 0.0;
        for (int s = threadIdx.x; s < Dp; s += 256) acc += e.E[r * Dp + s] * e.Yn[r * Dp + s];
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            const double q = (red[0] + red[1]) + (red[2] + red[3]);
            const double v = (q == q && q < 1.7e308 && q > -1.7e308) ? sqrt(q > 0.0 ? q : 0.0) : __builtin_nan("");
            e.nrm[r] = v;
            if (!(v == v)) bad = true;
            if (v > m) m = v;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) e.J[b] = bad ? __builtin_nan("") : m;
}

__global__ void k_grp_scan_init(const BatchElem* __restrict__ it, const int* __restrict__ act, int ch, int cur) {
    const BatchElem& e = it[act[blockIdx.x / ch]];
    GRP_LOOP((long)e.B * e.N * e.Dp) {
        const long per = (long)e.N * e.Dp;
        const long b = i / per, j = i - b * per;
        const long o = (b * (long)(e.Z + e.N + 1) + e.Z) * e.Dp + j;
        const double v = e.Fbuf[i] - e.Xk[cur][b * (long)(e.N + 1) * e.Dp + e.Dp + j];
        e.t64[0][o] = v;
        e.t32[o] = (float)v;
    }
}

__global__ void k_grp_scan_final(const BatchElem* __restrict__ it, const int* __restrict__ act, int ch, int cur,
                                 int nxt) {
    const BatchElem& e = it[act[blockIdx.x / ch]];
    GRP_LOOP((long)e.B * e.N * e.Dp) {
        const long per = (long)e.N * e.Dp;
        const long b = i / per, j = i - b * per;
        if (!e.active[b]) continue;
        const long o = (b * (long)(e.Z + e.N + 1) + e.Z) * e.Dp + j;
        const long x = b * (long)(e.N + 1) * e.Dp + e.Dp + j;
        e.Xk[nxt][x] = e.Xk[cur][x] + e.t64[e.L & 1][o];
    }
}

__global__ void k_grp_scan_init0(const BatchElem* __restrict__ it, const int* __restrict__ act, int ch) {
    const BatchElem& e = it[act[blockIdx.x / ch]];
    GRP_LOOP((long)e.B * (e.N + 1) * e.Dp) {
        const long per = (long)(e.N + 1) * e.Dp;
        const long b = i / per, j = i - b * per;
        const long o = (b * (long)(e.Z + e.N + 1) + e.Z) * e.Dp + j;
        const double v = j < e.Dp ? e.Xk[0][b * per + j] : (e.CS ? e.CS[b * (long)e.N * e.Dp + j - e.Dp] : 0.0);
        e.t64[0][o] = v;
        e.t32[o] = (float)v;
    }
}

__global__ void k_grp_scan_final0(const BatchElem* __restrict__ it, const int* __restrict__ act, int ch) {
    const BatchElem& e = it[act[blockIdx.x / ch]];
    GRP_LOOP((long)e.B * e.N * e.Dp) {
        const long per = (long)e.N * e.Dp;
        const long b = i / per, j = i - b * per;
        const long o = (b * (long)(e.Z + e.N + 1) + e.Z) * e.Dp + e.Dp + j;
        e.Xk[0][b * (long)(e.N + 1) * e.Dp + e.Dp + j] = 0.0 + e.t64[e.L0 & 1][o];
    }
}
#undef GRP_LOOP

static inline dim3 grp_grid(int n_act) { return dim3((unsigned)(n_act * grp_ch(n_act))); }

hipError_t grp_set_x0(const BatchElem* it, const int* act, int n_act, int xk, int zero_mode, hipStream_t st) {
    if (n_act <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_grp_set_x0, grp_grid(n_act), dim3(256), 0, st, it, act, grp_ch(n_act), xk, zero_mode);
    return hipGetLastError();
}
hipError_t grp_fine_init(const BatchElem* it, const int* act, int n_act, int cur, int incremental, int mixed,
                         hipStream_t st) {
    if (n_act <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_grp_fine_init, grp_grid(n_act), dim3(256), 0, st, it, act, grp_ch(n_act), cur, incremental,
                       mixed);
    return hipGetLastError();
}
hipError_t grp_fine_final(const BatchElem* it, const int* act, int n_act, int P, int mixed, hipStream_t st) {
    if (n_act <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_grp_fine_final, grp_grid(n_act), dim3(256), 0, st, it, act, grp_ch(n_act), P, mixed);
    return hipGetLastError();
}
hipError_t grp_jump_diff(const BatchElem* it, const int* act, int n_act, int xk, int rel, hipStream_t st) {
    if (n_act <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_grp_jump_diff, grp_grid(n_act), dim3(256), 0, st, it, act, grp_ch(n_act), xk, rel);
    return hipGetLastError();
}
hipError_t grp_jump_reduce(const BatchElem* it, const int* act, int n_act, int Bmax, int rel, hipStream_t st) {
    if (n_act <= 0 || Bmax <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_grp_jump_reduce, dim3((unsigned)(n_act * Bmax)), dim3(256), 0, st, it, act, Bmax, rel);
    return hipGetLastError();
}
hipError_t grp_scan_init(const BatchElem* it, const int* act, int n_act, int cur, hipStream_t st) {
    if (n_act <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_grp_scan_init, grp_grid(n_act), dim3(256), 0, st, it, act, grp_ch(n_act), cur);
    return hipGetLastError();
}
hipError_t grp_scan_final(const BatchElem* it, const int* act, int n_act, int cur, int nxt, hipStream_t st) {
    if (n_act <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_grp_scan_final, grp_grid(n_act), dim3(256), 0, st, it, act, grp_ch(n_act), cur, nxt);
    return hipGetLastError();
}
hipError_t grp_scan_init0(const BatchElem* it, const int* act, int n_act, hipStream_t st) {
    if (n_act <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_grp_scan_init0, grp_grid(n_act), dim3(256), 0, st, it, act, grp_ch(n_act));
    return hipGetLastError();
}
hipError_t grp_scan_final0(const BatchElem* it, const int* act, int n_act, hipStream_t st) {
    if (n_act <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_grp_scan_final0, grp_grid(n_act), dim3(256), 0, st, it, act, grp_ch(n_act));
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// operator assembly
// ---------------------------------------------------------------------------
// generic placement: dst[(ro + i) * ldd + co + j] = scale * (trans ? src[j*lds + i] : src[i*lds + j])
__global__ void k_place(double* __restrict__ dst, long ldd, int ro, int co, const double* __restrict__ src,
                        long lds, int rows, int cols, double scale, int trans, int accumulate) {
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < (long)rows * cols;
         t += (long)gridDim.x * blockDim.x) {
        const int i = (int)(t / cols), j = (int)(t - (long)i * cols);
        const double v = trans ? src[(long)j * lds + i] : src[(long)i * lds + j];
        double* d = dst + (long)(ro + i) * ldd + co + j;
        *d = accumulate ? *d + scale * v : scale * v;
    }
}

hipError_t place(double* dst, long ldd, int ro, int co, const double* src, long lds, int rows, int cols,
                 double scale, int trans, hipStream_t st, int accumulate) {
    if (rows <= 0 || cols <= 0 || !src) return hipSuccess;
    hipLaunchKernelGGL(k_place, grid1((long)rows * cols), dim3(256), 0, st, dst, ldd, ro, co, src, lds,
                       rows, cols, scale, trans, accumulate);
    return hipGetLastError();
}

// dst = A + c*B on a rows x cols block (row-major, lds), written into a
// square padded buffer of size n with identity on the padding diagonal
__global__ void k_shifted_embed(double* __restrict__ dst, int n, const double* __restrict__ A,
                                const double* __restrict__ Bm, long lds, int d, double cb) {
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < (long)n * n;
         t += (long)gridDim.x * blockDim.x) {
        const int i = (int)(t / n), j = (int)(t - (long)i * n);
        double v;
        if (i < d && j < d)
            v = A[(long)i * lds + j] + (Bm ? cb * Bm[(long)i * lds + j] : 0.0);
        else
            v = (i == j) ? 1.0 : 0.0;
        dst[t] = v;
    }
}

hipError_t shifted_embed(double* dst, int n, const double* A, const double* Bm, long lds, int d,
                         double cb, hipStream_t st) {
    hipLaunchKernelGGL(k_shifted_embed, grid1((long)n * n), dim3(256), 0, st, dst, n, A, Bm, lds, d, cb);
    return hipGetLastError();
}

__global__ void k_to_f32(const double* __restrict__ src, float* __restrict__ dst, long n) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        dst[i] = (float)src[i];
}

// zero the strict upper triangle of an n x n row-major matrix
__global__ void k_tril(double* __restrict__ A, int n) {
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < (long)n * n;
         t += (long)gridDim.x * blockDim.x) {
        const int i = (int)(t / n), j = (int)(t - (long)i * n);
        if (j > i) A[t] = 0.0;
    }
}

hipError_t tril(double* A, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_tril, grid1((long)n * n), dim3(256), 0, st, A, n);
    return hipGetLastError();
}

// identity on the leading d x d block of an n x n matrix, zero elsewhere
__global__ void k_eye(double* __restrict__ A, int n, int d) {
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < (long)n * n;
         t += (long)gridDim.x * blockDim.x) {
        const int i = (int)(t / n), j = (int)(t - (long)i * n);
        A[t] = (i == j && i < d) ? 1.0 : 0.0;
    }
}

hipError_t eye(double* A, int n, int d, hipStream_t st) {
    hipLaunchKernelGGL(k_eye, grid1((long)n * n), dim3(256), 0, st, A, n, d);
    return hipGetLastError();
}

hipError_t to_f32(const double* src, float* dst, long n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_to_f32, grid1(n), dim3(256), 0, st, src, dst, n);
    return hipGetLastError();
}

// max |X[i][j] - Y[j][i]| and max |X[i][j]| (Y = X for a symmetry test);
// non-negative doubles order like their bit patterns
__global__ void k_asym(const double* __restrict__ X, const double* __restrict__ Y, long ldx, long ldy,
                       int rows, int cols, unsigned long long* __restrict__ out) {
    double dmax = 0.0, amax = 0.0;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < (long)rows * cols;
         t += (long)gridDim.x * blockDim.x) {
        const int i = (int)(t / cols), j = (int)(t - (long)i * cols);
        const double x = X[(long)i * ldx + j];
        const double y = Y[(long)j * ldy + i];
        const double d = fabs(x - y);
        if (!(d <= dmax)) dmax = (d == d) ? d : 1.0e308;
        const double a = fabs(x);
        if (!(a <= amax)) amax = (a == a) ? a : 1.0e308;
    }
    atomicMax(&out[0], (unsigned long long)__double_as_longlong(dmax));
    atomicMax(&out[1], (unsigned long long)__double_as_longlong(amax));
}

hipError_t asym(const double* X, const double* Y, long ldx, long ldy, int rows, int cols,
                unsigned long long* out2, hipStream_t st) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_asym, dim3(256), dim3(256), 0, st, X, Y, ldx, ldy, rows, cols, out2);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Cholesky of the 64 x 64 diagonal block (j, j) of a padded SPD matrix, in
// LDS, plus the inverse of the factor block. A non-positive pivot records
// (block, pivot) in info (first failure wins) and poisons the block.
// ---------------------------------------------------------------------------
constexpr int NB = 64;

__global__ __launch_bounds__(256) void k_chol_diag(double* __restrict__ Am, long ld, int j,
                                                   double* __restrict__ Linv, int* __restrict__ info) {
    __shared__ double L[NB][NB + 1];
    __shared__ double X[NB][NB + 1];
    const int tid = threadIdx.x;
    const long o = (long)j * NB;
    for (int t = tid; t < NB * NB; t += 256) {
        const int r = t / NB, c = t % NB;
        L[r][c] = Am[(o + r) * ld + o + c];
    }
    __syncthreads();
    for (int k = 0; k < NB; ++k) {
        if (tid == 0) {
            const double d = L[k][k];
            if (!(d > 0.0)) {
                if (info[0] == 0) {
                    info[0] = 1;
                    info[1] = j * NB + k;
                }
                L[k][k] = __builtin_nan("");
            } else {
                L[k][k] = sqrt(d);
            }
        }
        __syncthreads();
        for (int i = k + 1 + tid; i < NB; i += 256) L[i][k] /= L[k][k];
        __syncthreads();
        for (int t = tid; t < NB * NB; t += 256) {
            const int i = t / NB, c = t % NB;
            if (i > k && c > k && c <= i) L[i][c] -= L[i][k] * L[c][k];
        }
        __syncthreads();
    }
    // inverse of the lower-triangular factor, one column per thread
    if (tid < NB) {
        const int c = tid;
        for (int i = 0; i < NB; ++i) X[i][c] = 0.0;
        for (int i = c; i < NB; ++i) {
            double v = (i == c) ? 1.0 : 0.0;
            for (int m = c; m < i; ++m) v -= L[i][m] * X[m][c];
            X[i][c] = v / L[i][i];
        }
    }
    __syncthreads();
    for (int t = tid; t < NB * NB; t += 256) {
        const int r = t / NB, c = t % NB;
        Am[(o + r) * ld + o + c] = (c <= r) ? L[r][c] : 0.0;
        Linv[(long)j * NB * NB + r * NB + c] = (c <= r) ? X[r][c] : 0.0;
    }
}

hipError_t chol_diag(double* Am, long ld, int j, double* Linv, int* info, hipStream_t st) {
    hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(256), 0, st, Am, ld, j, Linv, info);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// waveform relaxation in time (Sections 4.1-4.2): the transforms of the
// alpha-circulant diagonalisation and the staging of the level differences.
// Level-major layouts: level l of a (levels x NB x d) array is the NB x d
// block at l * NB * d; E = NB * d elements per level.
// ---------------------------------------------------------------------------
// Tables for P levels and K = P/2 + 1 frequencies (real data, so the
// frequencies P-K+1 .. P-1 are the conjugates of 1 .. K-2 for even P):
//   fwd[k][q]       =  alpha^(q/P) cos(2 pi k q/P)   real part of frequency k
//   fwd[K + k][q]   = -alpha^(q/P) sin(2 pi k q/P)   imaginary part
//   inv[k][q]       =  w_k alpha^(-q/P) cos(2 pi k q/P) / P
//   inv[K + k][q]   = -w_k alpha^(-q/P) sin(2 pi k q/P) / P
// w_k = 1 for k = 0 and for k = P/2 (P even), 2 otherwise; level q + 1 of the
// interval is time index q. fwd occupies [0, 2KP), inv [2KP, 4KP).
__global__ void k_wr_twiddle(double* __restrict__ tw, int P, int K, double log_alpha) {
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < 4L * K * P; t += (long)gridDim.x * blockDim.x) {
        const int which = (int)(t / ((long)K * P));
        const int k = (int)((t / P) % K), q = (int)(t % P);
        double sn, cs;
        sincospi(2.0 * (double)(((long)k * q) % P) / (double)P, &sn, &cs);
        const double g = exp(log_alpha * (double)q / (double)P);
        const double wk = (k == 0 || 2 * k == P) ? 1.0 : 2.0;
        double v;
        switch (which) {
            case 0: v = g * cs; break;
            case 1: v = -g * sn; break;
            case 2: v = wk * cs / (g * (double)P); break;
            default: v = -wk * sn / (g * (double)P); break;
        }
        tw[t] = v;
    }
}

hipError_t wr_twiddle(double* tw, int P, int K, double alpha, hipStream_t st) {
    hipLaunchKernelGGL(k_wr_twiddle, grid1(4L * K * P), dim3(256), 0, st, tw, P, K, log(alpha));
    return hipGetLastError();
}

// forward transform along time: R (P levels x NB x d1p) -> Rh (K x NB x
// [re (d1p) | im (d1p)]). A work-group takes WR_TE consecutive elements,
// stages their P levels in LDS and produces all 2K outputs of them.
constexpr int WR_TE = 32;
__global__ __launch_bounds__(256) void k_wr_dft_fwd(const double* __restrict__ R, double* __restrict__ Rh,
                                                    const double* __restrict__ tw, int P, int K, long E,
                                                    int d1p) {
    extern __shared__ double sh[];
    const long e0 = blockIdx.x * (long)WR_TE;
    for (int t = threadIdx.x; t < P * WR_TE; t += blockDim.x) {
        const int q = t / WR_TE, j = t % WR_TE;
        const long e = e0 + j;
        sh[t] = e < E ? R[(long)q * E + e] : 0.0;
    }
    __syncthreads();
    const long NB = E / d1p;
    for (int t = threadIdx.x; t < 2 * K * WR_TE; t += blockDim.x) {
        const int j = t % WR_TE, kk = t / WR_TE;
        const long e = e0 + j;
        if (e >= E) continue;
        const double* w = tw + (long)kk * P;
        double acc = 0.0;
        for (int q = 0; q < P; ++q) acc = fma(w[q], sh[q * WR_TE + j], acc);
        const int part = kk / K, k = kk % K;
        const long c = e / d1p;
        const int i = (int)(e - c * d1p);
        Rh[((long)k * NB + c) * 2 * d1p + (long)part * d1p + i] = acc;
    }
}

// inverse transform: Uh (K x NB x [re | im]) -> levels 1..P of U (level
// q + 1 = sum over the 2K table rows of inv[kk][q] times part kk of Uh)
__global__ __launch_bounds__(256) void k_wr_dft_inv(const double* __restrict__ Uh, double* __restrict__ U,
                                                    const double* __restrict__ tinv, int P, int K, long E,
                                                    int d1p) {
    extern __shared__ double sh[];
    const long e0 = blockIdx.x * (long)WR_TE;
    const long NB = E / d1p;
    for (int t = threadIdx.x; t < 2 * K * WR_TE; t += blockDim.x) {
        const int kk = t / WR_TE, j = t % WR_TE;
        const long e = e0 + j;
        double v = 0.0;
        if (e < E) {
            const int part = kk / K, k = kk % K;
            const long c = e / d1p;
            const int i = (int)(e - c * d1p);
            v = Uh[((long)k * NB + c) * 2 * d1p + (long)part * d1p + i];
        }
        sh[t] = v;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < P * WR_TE; t += blockDim.x) {
        const int q = t / WR_TE, j = t % WR_TE;
        const long e = e0 + j;
        if (e >= E) continue;
        double acc = 0.0;
        for (int kk = 0; kk < 2 * K; ++kk) acc = fma(tinv[(long)kk * P + q], sh[kk * WR_TE + j], acc);
        U[(long)(q + 1) * E + e] = acc;
    }
}

hipError_t wr_dft(int dir, const double* src, double* dst, const double* tw, int P, int K, long NB, int d1p,
                  hipStream_t st) {
    const long E = NB * d1p;
    const dim3 g((unsigned)((E + WR_TE - 1) / WR_TE));
    if (dir > 0) {
        const size_t lds = sizeof(double) * (size_t)P * WR_TE;
        hipLaunchKernelGGL(k_wr_dft_fwd, g, dim3(256), lds, st, src, dst, tw, P, K, E, d1p);
    } else {
        const size_t lds = sizeof(double) * (size_t)2 * K * WR_TE;
        hipLaunchKernelGGL(k_wr_dft_inv, g, dim3(256), lds, st, src, dst, tw + 2L * K * P, P, K, E, d1p);
    }
    return hipGetLastError();
}

// staging for the two products of an iteration, s = 1..P (level s-1 of the
// output): mode 0 (w): [w_{s-1} - w_{s-2} | w_{s-1}], w_{-1} = w_0;
// mode 1 (u): [u_{s-1} - u_{s-2} | u_s], u_{-1} = u_0
__global__ void k_wr_cat(const double* __restrict__ L, double* __restrict__ out, int P, long NB, int d, int mode) {
    const long E = NB * d;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < (long)P * E; t += (long)gridDim.x * blockDim.x) {
        const int s1 = (int)(t / E);
        const long rem = t - (long)s1 * E;
        const double a = L[(long)s1 * E + rem];
        const double b = s1 >= 1 ? L[(long)(s1 - 1) * E + rem] : a;
        const double second = mode ? L[(long)(s1 + 1) * E + rem] : a;
        const long c = rem / d;
        const int i = (int)(rem - c * d);
        double* o = out + ((long)s1 * NB + c) * 2 * d;
        o[i] = a - b;
        o[d + i] = second;
    }
}

hipError_t wr_cat(const double* L, double* out, int P, long NB, int d, int mode, hipStream_t st) {
    hipLaunchKernelGGL(k_wr_cat, grid1((long)P * NB * d), dim3(256), 0, st, L, out, P, NB, d, mode);
    return hipGetLastError();
}

// y = a - alpha b
__global__ void k_wr_axmy(double* __restrict__ y, const double* __restrict__ a, const double* __restrict__ b,
                          double alpha, long n) {
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x)
        y[t] = a[t] - alpha * b[t];
}

hipError_t wr_axmy(double* y, const double* a, const double* b, double alpha, long n, hipStream_t st) {
    hipLaunchKernelGGL(k_wr_axmy, grid1(n), dim3(256), 0, st, y, a, b, alpha, n);
    return hipGetLastError();
}

// Start of a WR run on columns c0 .. c0+NBc-1 (column c = b N + n, start
// state row n of sample b in X, sample stride ldXb): level 0 of U and W, the
// initial waveform w_s = w_0 (s = 1..P) and u_P = u_0. dir < 0 writes the end
// states (level P) to Fout (row c0 + c) instead. |dir| = 1: rows in the
// caller's layout [u (d1) | w (d2)]; |dir| = 2: padded rows [u (d1p) | w (d2p)].
__global__ void k_wr_io(int dir, const double* __restrict__ X, long ldXb, double* __restrict__ Fout, int N,
                        int d1, int d2, int d1p, int d2p, int c0, int NBc, int P, double* __restrict__ Ul,
                        double* __restrict__ Wl) {
    const bool padded = dir == 2 || dir == -2;
    const int D = d1 + d2, Dp = d1p + d2p;
    const int ld = padded ? Dp : D, wo = padded ? d1p : d1;  // row length, offset of the w part
    const int du = padded ? d1p : d1, dw = padded ? d2p : d2;  // stored lengths
    const long E1 = (long)NBc * d1p, E2 = (long)NBc * d2p;
    if (dir > 0) {
        for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < (long)NBc * Dp;
             t += (long)gridDim.x * blockDim.x) {
            const int c = (int)(t / Dp), s = (int)(t % Dp);
            const int cg = c0 + c, b = cg / N, n = cg % N;
            const double* x = X + (long)b * ldXb + (long)n * ld;
            if (s < d1p) {
                const double v = s < du ? x[s] : 0.0;
                Ul[(long)c * d1p + s] = v;
                Ul[(long)P * E1 + (long)c * d1p + s] = v;
            } else {
                const int j = s - d1p;
                const double v = j < dw ? x[wo + j] : 0.0;
                for (int l = 0; l <= P; ++l) Wl[(long)l * E2 + (long)c * d2p + j] = v;
            }
        }
    } else {
        for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < (long)NBc * ld;
             t += (long)gridDim.x * blockDim.x) {
            const int c = (int)(t / ld), s = (int)(t % ld);
            const double v = s < wo ? (s < d1p ? Ul[(long)P * E1 + (long)c * d1p + s] : 0.0)
                                    : Wl[(long)P * E2 + (long)c * d2p + (s - wo)];
            Fout[(long)(c0 + c) * ld + s] = v;
        }
    }
}

hipError_t wr_io(int dir, const double* X, long ldXb, double* Fout, int N, int d1, int d2, int d1p, int d2p,
                 int c0, int NBc, int P, double* Ul, double* Wl, hipStream_t st) {
    const bool padded = dir == 2 || dir == -2;
    const long n = (long)NBc * (dir > 0 || padded ? d1p + d2p : d1 + d2);
    hipLaunchKernelGGL(k_wr_io, grid1(n), dim3(256), 0, st, dir, X, ldXb, Fout, N, d1, d2, d1p, d2p, c0, NBc, P,
                       Ul, Wl);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// carried history (states [x | delta] of 2Dp, delta = the change over the last
// fine step): gather, placement into the fine-step state and back, the
// coarse step's augmented source and operator
// ---------------------------------------------------------------------------
// out[b*N + n][s] = X[b][n + row_off][off + s] (zero unless 0 <= n + row_off < nvalid)
__global__ void k_gather_rows(const double* __restrict__ X, long ldXb, int sx, int off, int row_off, int nvalid,
                              double* __restrict__ out, int B, int N, int Dp) {
    const long rows = (long)B * N;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < rows * Dp;
         i += (long)gridDim.x * blockDim.x) {
        const long r = i / Dp;
        const int s = (int)(i - r * Dp);
        const long b = r / N, n = r - b * N;
        const long j = n + row_off;
        out[i] = (j >= 0 && j < nvalid) ? X[b * ldXb + j * sx + off + s] : 0.0;
    }
}

hipError_t gather_rows(const double* X, long ldXb, int sx, int off, int row_off, int nvalid, double* out, int B,
                       int N, int Dp, hipStream_t st) {
    hipLaunchKernelGGL(k_gather_rows, grid1((long)B * N * Dp), dim3(256), 0, st, X, ldXb, sx, off, row_off, nvalid,
                       out, B, N, Dp);
    return hipGetLastError();
}

// history rows H (rows x Dp, [du | dw]) into the fine-step state
// [du_prev | u - u_a | w - w_a | dw_prev] (2Dp per row), both precisions
__global__ void k_hist_put(const double* __restrict__ H, double* __restrict__ dev64, float* __restrict__ dev32,
                           long rows, int Dp, int d1p) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < rows * Dp;
         i += (long)gridDim.x * blockDim.x) {
        const long r = i / Dp;
        const int s = (int)(i - r * Dp);
        const long o = r * 2 * Dp + (s < d1p ? s : Dp + s);
        const double v = H[i];
        dev64[o] = v;
        if (dev32) dev32[o] = (float)v;
    }
}

hipError_t hist_put(const double* H, double* dev64, float* dev32, long rows, int Dp, int d1p, hipStream_t st) {
    hipLaunchKernelGGL(k_hist_put, grid1(rows * Dp), dim3(256), 0, st, H, dev64, dev32, rows, Dp, d1p);
    return hipGetLastError();
}

// out[r][s] (+)= history of the fine-step state (the last step's change)
__global__ void k_hist_get(const double* __restrict__ dev64, double* __restrict__ out, long ldo, long rows,
                           int Dp, int d1p, int accumulate) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < rows * Dp;
         i += (long)gridDim.x * blockDim.x) {
        const long r = i / Dp;
        const int s = (int)(i - r * Dp);
        const double v = dev64[r * 2 * Dp + (s < d1p ? s : Dp + s)];
        double* y = out + r * ldo + s;
        *y = accumulate ? *y + v : v;
    }
}

hipError_t hist_get(const double* dev64, double* out, long ldo, long rows, int Dp, int d1p, int accumulate,
                    hipStream_t st) {
    hipLaunchKernelGGL(k_hist_get, grid1(rows * Dp), dim3(256), 0, st, dev64, out, ldo, rows, Dp, d1p, accumulate);
    return hipGetLastError();
}

// CSa[r] = [CS[r]; CS[r] / P]: the coarse step's source term on [x | delta]
__global__ void k_aug_cs(const double* __restrict__ CS, double* __restrict__ CSa, long rows, int Dp, double invP) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < rows * 2 * Dp;
         i += (long)gridDim.x * blockDim.x) {
        const long r = i / (2 * Dp);
        const int s = (int)(i - r * 2 * Dp);
        CSa[i] = s < Dp ? CS[r * Dp + s] : invP * CS[r * Dp + s - Dp];
    }
}

hipError_t aug_cs(const double* CS, double* CSa, long rows, int Dp, int P, hipStream_t st) {
    hipLaunchKernelGGL(k_aug_cs, grid1(rows * 2 * Dp), dim3(256), 0, st, CS, CSa, rows, Dp, 1.0 / P);
    return hipGetLastError();
}

// the coarse step on [x | delta] (2Dp x Dp: it reads x only):
//   [Phi_G; (Phi_G - I)/P]
__global__ void k_hist_phi(const double* __restrict__ Phi, double* __restrict__ out, int Dp, double invP) {
    const long n = (long)Dp * Dp;
    for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < 2 * n; t += (long)gridDim.x * blockDim.x) {
        const long u = t < n ? t : t - n;
        const int i = (int)(u / Dp), j = (int)(u - (long)i * Dp);
        out[t] = t < n ? Phi[u] : invP * (Phi[u] - (i == j ? 1.0 : 0.0));
    }
}

hipError_t hist_phi(const double* Phi, double* out, int Dp, int P, hipStream_t st) {
    hipLaunchKernelGGL(k_hist_phi, grid1(2L * Dp * Dp), dim3(256), 0, st, Phi, out, Dp, 1.0 / P);
    return hipGetLastError();
}

}  // namespace pe
