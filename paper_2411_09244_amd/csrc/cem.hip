// Set-up pipeline on the GPU: the CEM-GMsFEM basis functions of Section 3.1
// (eq. (3.2)) on every oversampled patch, and the Galerkin blocks of eq. (3.8)
// with the source factors.
//
// Basis. For coarse element i with oversampled patch K_i^+ (K_i plus `layers`
// coarse layers, clipped to the domain) the basis functions phi_j^(i),
// j < J, minimise the energy a(phi, phi) over H^1_0(K_i^+) subject to
// s(phi, psi_l^(k)) = delta_{(k,l),(i,j)} for every auxiliary function of
// every element k of the patch. With A the kappa-weighted Q1 stiffness on
// the patch's interior nodes and C the constraint matrix (row (k, l) =
// (S_k psi_l^(k))^T on the patch nodes), the saddle-point system
//     [A C^T; C 0] [phi; mu] = [0; e_(i,j)]
// gives phi = A^-1 C^T S^-1 e_(i,j) with S = C A^-1 C^T. Numbering the
// patch's interior nodes row by row makes A banded with half-bandwidth
// nx + 1 (nx nodes per row), so per patch:
//   1. banded Cholesky A = L L^T (one work-group; the active (bw+1)^2
//      window lives in LDS, stiffness entries are formed from kappa as rows
//      enter the window);
//   2. Y = L^-1 C^T by a forward sweep over the rows, one thread per
//      constraint column;
//   3. S = Y^T Y;
//   4. Cholesky of S in LDS, z = S^-1 e_(i,j) for the J functions of
//      element i, w = Y z, and phi = L^-T w by a backward sweep.
// Projection. Every basis function is scattered into a dense row of
// Psi^T (one row per function, fine-grid interior nodes as columns); the
// fine mass and stiffness are applied by their 9-point stencils, the Gram
// matrices Psi^T M Psi and Psi^T K Psi and the source factors Psi^T b come
// from the FP64 MFMA product kernel, and a last kernel normalises every
// function to unit L2 norm, symmetrises the diagonal blocks and writes the
// blocks of the V_H1 / V_H2 split (the J1 lowest eigen-indices of every
// element span V_H1, the next J2 span V_H2).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/pe.h"
#include "pe_internal.h"

namespace pe {

pe_status set_error(pe_status code, const std::string& msg);

namespace {

constexpr int CEM_WN = 64;     // largest band window (half-bandwidth + 1)
constexpr int CEM_NAUX = 128;  // largest number of constraints per patch
constexpr int CEM_LDS_S = CEM_NAUX * CEM_NAUX;  // doubles of the step-4 LDS area

struct CemGeom {
    int n, n_c, m, layers, J;  // J: constraint slots per element in the constraint data
    // per-element function counts (nullable: J for every element) and the
    // first function of every element in the element-major order (n_c^2 + 1)
    const int* cnt = nullptr;
    const int* foff = nullptr;
    long lb_stride;  // doubles of band storage per patch
    long y_stride;   // doubles of Y per patch (rows x CEM_NAUX)
    long ldp;        // row length of Psi^T (fine interior nodes, padded)
    int n_dof1;      // interior nodes per side, n - 1
};

struct Patch {
    int ex0, ey0, nex, ney;  // first coarse element and element counts
    int gx0, gy0;            // global node of patch node 0
    int nx, ny, nf;          // interior nodes per row, rows, total
    int bw, wn;              // half-bandwidth nx + 1, window bw + 1
    int naux;                // constraints: sum of the patch elements' counts
    int ai;                  // position of the patch's own element
    int aoff, jown;          // its first constraint and its count
};

__device__ inline int elem_count(const CemGeom& g, int k) { return g.cnt ? g.cnt[k] : g.J; }

__device__ inline Patch patch_of(const CemGeom& g, int i) {
    Patch p;
    const int ey = i / g.n_c, ex = i % g.n_c;
    const int ey0 = max(ey - g.layers, 0), ey1 = min(ey + g.layers, g.n_c - 1);
    const int ex0 = max(ex - g.layers, 0), ex1 = min(ex + g.layers, g.n_c - 1);
    p.ex0 = ex0;
    p.ey0 = ey0;
    p.nex = ex1 - ex0 + 1;
    p.ney = ey1 - ey0 + 1;
    p.gx0 = ex0 * g.m + 1;
    p.gy0 = ey0 * g.m + 1;
    p.nx = p.nex * g.m - 1;
    p.ny = p.ney * g.m - 1;
    p.nf = p.nx * p.ny;
    p.bw = p.nx + 1;
    p.wn = p.bw + 1;
    p.ai = (ey - ey0) * p.nex + (ex - ex0);
    p.naux = 0;
    p.aoff = 0;
    for (int a = 0; a < p.nex * p.ney; ++a) {
        if (a == p.ai) p.aoff = p.naux;
        p.naux += elem_count(g, (ey0 + a / p.nex) * g.n_c + ex0 + a % p.nex);
    }
    p.jown = elem_count(g, i);
    return p;
}

// constraint q of a patch -> (patch element a, slot l)
__device__ inline void constraint_slot(const CemGeom& g, const Patch& p, int q, int* a, int* l) {
    int rem = q, k = 0;
    for (; k < p.nex * p.ney - 1; ++k) {
        const int c = elem_count(g, (p.ey0 + k / p.nex) * g.n_c + p.ex0 + k % p.nex);
        if (rem < c) break;
        rem -= c;
    }
    *a = k;
    *l = rem;
}

// Q1 stiffness between interior fine nodes (gy, gx) and (hy, hx): the
// element matrix kappa/6 [[4,-1,-2,-1],...] summed over the cells that
// contain both nodes (node (y, x) is a corner of cells (y-1|y, x-1|x)).
__device__ inline double q1_stiff(const double* __restrict__ kappa, int n, int gy, int gx, int hy, int hx) {
    const int dy = hy - gy, dx = hx - gx;
    if (dy < -1 || dy > 1 || dx < -1 || dx > 1) return 0.0;
    auto k = [&](int cy, int cx) { return kappa[(long)cy * n + cx]; };
    if (dy == 0 && dx == 0) return (4.0 / 6.0) * (k(gy - 1, gx - 1) + k(gy - 1, gx) + k(gy, gx - 1) + k(gy, gx));
    if (dy == 0) {
        const int cx = min(gx, hx);
        return (-1.0 / 6.0) * (k(gy - 1, cx) + k(gy, cx));
    }
    if (dx == 0) {
        const int cy = min(gy, hy);
        return (-1.0 / 6.0) * (k(cy, gx - 1) + k(cy, gx));
    }
    return (-2.0 / 6.0) * k(min(gy, hy), min(gx, hx));
}

// stiffness between patch nodes r and c
__device__ inline double patch_stiff(const double* __restrict__ kappa, const CemGeom& g, const Patch& p, int r,
                                     int c) {
    const int ry = r / p.nx, rx = r - ry * p.nx;
    const int cy = c / p.nx, cx = c - cy * p.nx;
    return q1_stiff(kappa, g.n, p.gy0 + ry, p.gx0 + rx, p.gy0 + cy, p.gx0 + cx);
}

// constraint (patch element a, slot l) at patch node r: the constraint
// data of element k (S_k psi_l^(k) for CEM, the region integrals for NLMC)
// at the node if it belongs to element k, else 0
__device__ inline double constraint(const double* __restrict__ spsi, const CemGeom& g, const Patch& p, int a,
                                    int l, int r) {
    const int ky = p.ey0 + a / p.nex, kx = p.ex0 + a % p.nex;
    const int ry = r / p.nx, rx = r - ry * p.nx;
    const int ly = p.gy0 + ry - ky * g.m, lx = p.gx0 + rx - kx * g.m;
    if (ly < 0 || ly > g.m || lx < 0 || lx > g.m) return 0.0;
    const int k = ky * g.n_c + kx;
    return spsi[((long)k * (g.m + 1) * (g.m + 1) + ly * (g.m + 1) + lx) * g.J + l];
}

// 1. banded Cholesky of the patch stiffness. Lb row r holds L[r][r - d] at
// d = 0..bw. info[i] = 0, or the 1-based row of a non-positive pivot.
__global__ __launch_bounds__(256) void k_cem_band_chol(const CemGeom g, const double* __restrict__ kappa,
                                                       double* __restrict__ Lb, int* __restrict__ info) {
    __shared__ double win[CEM_WN * CEM_WN];
    __shared__ double col[CEM_WN];
    const int i = blockIdx.x, tid = threadIdx.x;
    const Patch p = patch_of(g, i);
    const int nf = p.nf, bw = p.bw, wn = p.wn;
    double* L = Lb + (long)i * g.lb_stride;
    // rows 0..bw of the window: entries (r, c), max(0, r - bw) <= c <= r
    for (int idx = tid; idx < wn * wn; idx += 256) {
        const int r = idx / wn, d = idx - r * wn;
        if (r < nf && d <= r) win[(r % wn) * wn + (r - d) % wn] = patch_stiff(kappa, g, p, r, r - d);
    }
    __syncthreads();
    for (int j = 0; j < nf; ++j) {
        // entry of the row entering the window at the end of this step
        // (row j + wn, column j + 1 + tid), loaded early
        const int rn = j + wn;
        const double anew = (tid < wn && rn < nf) ? patch_stiff(kappa, g, p, rn, j + 1 + tid) : 0.0;
        const double piv = win[(j % wn) * wn + j % wn];
        if (!(piv > 0.0) || !isfinite(piv)) {
            if (tid == 0) info[i] = j + 1;
            return;  // uniform: every thread read the same pivot
        }
        const double s = sqrt(piv);
        if (tid < wn) {
            const int r = j + tid;
            double l = 0.0;
            if (r < nf) {
                l = tid == 0 ? s : win[(r % wn) * wn + j % wn] / s;
                L[(long)r * wn + tid] = l;
            }
            col[tid] = l;
        }
        __syncthreads();
        // trailing update of rows j+1..j+bw (row j's slots are not touched)
        for (int idx = tid; idx < bw * bw; idx += 256) {
            const int a = idx / bw + 1, b = idx - (a - 1) * bw + 1;
            if (b <= a && j + a < nf) win[((j + a) % wn) * wn + (j + b) % wn] -= col[a] * col[b];
        }
        // the new row takes the retired row j's slots
        if (tid < wn && rn < nf) win[(rn % wn) * wn + (j + 1 + tid) % wn] = anew;
        __syncthreads();
    }
    if (tid == 0) info[i] = 0;
}

// 2. Y = L^-1 C^T, one thread per constraint column; the last wn rows of Y
// are kept in LDS for the band products. Y row r at Y + r * CEM_NAUX.
__global__ __launch_bounds__(CEM_NAUX) void k_cem_forward(const CemGeom g, const double* __restrict__ Lb,
                                                          const double* __restrict__ spsi, double* __restrict__ Yg) {
    __shared__ double yw[CEM_WN][CEM_NAUX];
    __shared__ double lrow[2][CEM_WN];
    const int i = blockIdx.x, q = threadIdx.x;
    const Patch p = patch_of(g, i);
    const int nf = p.nf, wn = p.wn;
    const double* L = Lb + (long)i * g.lb_stride;
    double* Y = Yg + (long)i * g.y_stride;
    const bool act = q < p.naux;
    int qa = 0, ql = 0;
    if (act) constraint_slot(g, p, q, &qa, &ql);
    // row 0 operands
    if (q < wn) lrow[0][q] = q == 0 ? L[0] : 0.0;
    double c = act ? constraint(spsi, g, p, qa, ql, 0) : 0.0;
    __syncthreads();
    for (int r = 0; r < nf; ++r) {
        const int cur = r & 1;
        // next row's operands, loaded before this row's arithmetic
        const int rn = r + 1;
        const double ln = (q < wn && rn < nf && q <= rn) ? L[(long)rn * wn + q] : 0.0;
        const double cn = (act && rn < nf) ? constraint(spsi, g, p, qa, ql, rn) : 0.0;
        if (act) {
            double s = c;
            const int dmax = min(p.bw, r);
            for (int d = 1; d <= dmax; ++d) s -= lrow[cur][d] * yw[(r - d) % wn][q];
            const double y = s / lrow[cur][0];
            yw[r % wn][q] = y;
            Y[(long)r * CEM_NAUX + q] = y;
        }
        if (q < wn) lrow[cur ^ 1][q] = ln;
        c = cn;
        __syncthreads();
    }
}

// 3. S = Y^T Y (naux x naux, stored CEM_NAUX x CEM_NAUX): 256 threads, each
// an 8 x 8 block; Y staged through LDS 16 rows at a time.
__global__ __launch_bounds__(256) void k_cem_gram(const CemGeom g, const double* __restrict__ Yg,
                                                  double* __restrict__ Sg) {
    constexpr int RB = 16;
    __shared__ double ys[RB][CEM_NAUX];
    const int i = blockIdx.x, tid = threadIdx.x;
    const Patch p = patch_of(g, i);
    const double* Y = Yg + (long)i * g.y_stride;
    const int ty = tid / 16, tx = tid % 16;
    double acc[8][8];
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int b = 0; b < 8; ++b) acc[a][b] = 0.0;
    for (int r0 = 0; r0 < p.nf; r0 += RB) {
        for (int idx = tid; idx < RB * CEM_NAUX; idx += 256) {
            const int rr = idx / CEM_NAUX, qq = idx % CEM_NAUX;
            ys[rr][qq] = (r0 + rr < p.nf && qq < p.naux) ? Y[(long)(r0 + rr) * CEM_NAUX + qq] : 0.0;
        }
        __syncthreads();
        for (int rr = 0; rr < RB; ++rr) {
            double va[8], vb[8];
#pragma unroll
            for (int a = 0; a < 8; ++a) va[a] = ys[rr][ty * 8 + a];
#pragma unroll
            for (int b = 0; b < 8; ++b) vb[b] = ys[rr][tx * 8 + b];
#pragma unroll
            for (int a = 0; a < 8; ++a)
#pragma unroll
                for (int b = 0; b < 8; ++b) acc[a][b] += va[a] * vb[b];
        }
        __syncthreads();
    }
    double* S = Sg + (long)i * CEM_NAUX * CEM_NAUX;
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int b = 0; b < 8; ++b) S[(long)(ty * 8 + a) * CEM_NAUX + tx * 8 + b] = acc[a][b];
}

// 4. Cholesky of S in LDS, z = S^-1 e_(ai, l) for l < J, w = Y z,
// phi = L^-T w; phi_l goes to row i * J + l of Psi^T at the fine interior
// node of every patch node. info[i] = -(1-based pivot) if S is not positive.
__global__ __launch_bounds__(256) void k_cem_finish(const CemGeom g, const double* __restrict__ Lb,
                                                    const double* __restrict__ Yg, const double* __restrict__ Sg,
                                                    double* __restrict__ PsiT, int* __restrict__ info) {
    __shared__ double sh[CEM_LDS_S];  // S, then w (nf x J)
    __shared__ double z[CEM_NAUX][8];
    __shared__ double phw[CEM_WN][8];
    __shared__ int bad;
    const int i = blockIdx.x, tid = threadIdx.x;
    const Patch p = patch_of(g, i);
    const int na = p.naux, J = p.jown, nf = p.nf, wn = p.wn;
    const long row0 = g.foff ? (long)g.foff[i] : (long)i * g.J;  // the element's first row of Psi^T
    const double* Sgl = Sg + (long)i * CEM_NAUX * CEM_NAUX;
    for (int idx = tid; idx < na * na; idx += 256) sh[idx] = Sgl[(long)(idx / na) * CEM_NAUX + idx % na];
    if (tid == 0) bad = 0;
    __syncthreads();
    // right-looking Cholesky, lower triangle of sh (na x na)
    for (int k = 0; k < na; ++k) {
        const double piv = sh[k * na + k];
        if (!(piv > 0.0) || !isfinite(piv)) {
            if (tid == 0) bad = k + 1;
            break;  // uniform
        }
        const double s = sqrt(piv);
        __syncthreads();
        for (int r = k + 1 + tid; r < na; r += 256) sh[r * na + k] /= s;
        if (tid == 0) sh[k * na + k] = s;
        __syncthreads();
        const int m = na - k - 1;
        for (int idx = tid; idx < m * m; idx += 256) {
            const int r = k + 1 + idx / m, c = k + 1 + idx % m;
            if (c <= r) sh[r * na + c] -= sh[r * na + k] * sh[c * na + k];
        }
        __syncthreads();
    }
    __syncthreads();  // bad is written by thread 0 inside the loop
    if (bad) {
        if (tid == 0) info[i] = -bad;
        return;  // uniform
    }
    // z = S^-1 e_(aoff + l): forward and backward substitution, thread l
    if (tid < J) {
        const int l = tid, e = p.aoff + l;
        for (int r = 0; r < na; ++r) {
            double v = r == e ? 1.0 : 0.0;
            for (int c = 0; c < r; ++c) v -= sh[r * na + c] * z[c][l];
            z[r][l] = v / sh[r * na + r];
        }
        for (int r = na - 1; r >= 0; --r) {
            double v = z[r][l];
            for (int c = r + 1; c < na; ++c) v -= sh[c * na + r] * z[c][l];
            z[r][l] = v / sh[r * na + r];
        }
    }
    __syncthreads();
    // w = Y z into sh (nf x J), one thread per row
    const double* Y = Yg + (long)i * g.y_stride;
    for (int r = tid; r < nf; r += 256) {
        double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int q = 0; q < na; ++q) {
            const double y = Y[(long)r * CEM_NAUX + q];
#pragma unroll
            for (int l = 0; l < 8; ++l) acc[l] += y * z[q][l];
        }
#pragma unroll
        for (int l = 0; l < 8; ++l)
            if (l < J) sh[r * J + l] = acc[l];
    }
    __syncthreads();
    // phi = L^-T w by a backward sweep on wave 0 alone (in-order LDS
    // traffic of one wave, no work-group barrier below): lane d - 1 holds
    // L[r + d][r] for d = 1..bw; the last wn rows of phi stay in phw
    if (tid >= 64) return;
    const int lane = tid, d = lane + 1;
    const double* L = Lb + (long)i * g.lb_stride;
    const int n1 = g.n_dof1;
    auto lval = [&](int r) { return (d <= p.bw && r + d < nf) ? L[(long)(r + d) * wn + d] : 0.0; };
    auto ldiag = [&](int r) { return L[(long)r * wn]; };
    double lc = lval(nf - 1), dg = ldiag(nf - 1);
    for (int r = nf - 1; r >= 0; --r) {
        const double ln = r > 0 ? lval(r - 1) : 0.0;
        const double dn = r > 0 ? ldiag(r - 1) : 1.0;
        const bool in = d <= p.bw && r + d < nf;
        double part[8];
#pragma unroll
        for (int l = 0; l < 8; ++l) part[l] = (in && l < J) ? lc * phw[(r + d) % wn][l] : 0.0;
#pragma unroll
        for (int l = 0; l < 8; ++l) {
            double v = part[l];
            for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
            part[l] = v;
        }
        // every lane holds the sums; lane l < J finishes column l
        double mine = part[0];
#pragma unroll
        for (int l = 1; l < 8; ++l)
            if (lane == l) mine = part[l];
        if (lane < J) {
            const double ph = (sh[r * J + lane] - mine) / dg;
            phw[r % wn][lane] = ph;
            const int ry = r / p.nx, rx = r - ry * p.nx;
            const long dof = (long)(p.gy0 + ry - 1) * n1 + (p.gx0 + rx - 1);
            PsiT[(row0 + lane) * g.ldp + dof] = ph;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        lc = ln;
        dg = dn;
    }
    if (lane == 0) info[i] = 0;
}

// M and K applied to rows of Psi^T by the Q1 stencils on the interior nodes
__global__ __launch_bounds__(256) void k_cem_stencil(const double* __restrict__ kappa, int n, long ldp,
                                                     const double* __restrict__ X, double* __restrict__ MX,
                                                     double* __restrict__ KX) {
    const int n1 = n - 1;
    const long nd = (long)n1 * n1;
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    const long row = blockIdx.y;
    if (t >= ldp) return;
    if (t >= nd) {  // padding columns stay zero
        MX[row * ldp + t] = 0.0;
        KX[row * ldp + t] = 0.0;
        return;
    }
    const int gy = (int)(t / n1) + 1, gx = (int)(t % n1) + 1;
    const double h = 1.0 / n, h2 = h * h;
    const double* x = X + row * ldp;
    double m = 0.0, k = 0.0;
    for (int dy = -1; dy <= 1; ++dy) {
        const int hy = gy + dy;
        if (hy < 1 || hy > n1) continue;
        for (int dx = -1; dx <= 1; ++dx) {
            const int hx = gx + dx;
            if (hx < 1 || hx > n1) continue;
            const double v = x[(long)(hy - 1) * n1 + (hx - 1)];
            const int ad = (dy != 0) + (dx != 0);
            // mass: 16/36 h^2 (same node), 2 cells x 2/36 h^2 (edge), 1/36 h^2 (diagonal)
            const double mc = ad == 0 ? 16.0 / 36.0 : ad == 1 ? 4.0 / 36.0 : 1.0 / 36.0;
            m += mc * h2 * v;
            k += q1_stiff(kappa, n, gy, gx, hy, hx) * v;
        }
    }
    MX[row * ldp + t] = m;
    KX[row * ldp + t] = k;
}

// loads (R x n_dof) into a zero-padded copy (R x ldp)
__global__ void k_cem_pad(const double* __restrict__ src, long nd, long ldp, long rows, double* __restrict__ dst) {
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t >= rows * ldp) return;
    const long r = t / ldp, c = t % ldp;
    dst[t] = c < nd ? src[r * nd + c] : 0.0;
}

// space index -> full index (element-major, J per element) of the V_H1 /
// V_H2 split; fmap (nullable) gives it as a table
__device__ inline int cem_full(int s, int d1, int J, int J1, const int* __restrict__ fmap) {
    if (fmap) return fmap[s];
    if (s < d1) return (s / J1) * J + s % J1;
    const int J2 = J - J1, t = s - d1;
    return (t / J2) * J + J1 + t % J2;
}

// blocks of eq. (3.8) from the Gram matrices of the unnormalised functions
__global__ void k_cem_blocks(const double* __restrict__ Gm, const double* __restrict__ Gk, int Dall, int d1,
                             int d2, int J, int J1, const int* __restrict__ fmap, double* __restrict__ M11, double* __restrict__ M12,
                             double* __restrict__ M22, double* __restrict__ A11, double* __restrict__ A12,
                             double* __restrict__ A22) {
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    const int D = d1 + d2;
    if (t >= (long)D * D) return;
    const int a = (int)(t / D), b = (int)(t % D);
    const int fa = cem_full(a, d1, J, J1, fmap), fb = cem_full(b, d1, J, J1, fmap);
    const double s = 1.0 / (sqrt(Gm[(long)fa * Dall + fa]) * sqrt(Gm[(long)fb * Dall + fb]));
    const double mab = Gm[(long)fa * Dall + fb] * s, mba = Gm[(long)fb * Dall + fa] * s;
    const double kab = Gk[(long)fa * Dall + fb] * s, kba = Gk[(long)fb * Dall + fa] * s;
    if (a < d1 && b < d1) {
        M11[(long)a * d1 + b] = 0.5 * (mab + mba);
        A11[(long)a * d1 + b] = 0.5 * (kab + kba);
    } else if (a < d1) {
        M12[(long)a * d2 + (b - d1)] = mab;
        A12[(long)a * d2 + (b - d1)] = kab;
    } else if (b >= d1) {
        M22[(long)(a - d1) * d2 + (b - d1)] = 0.5 * (mab + mba);
        A22[(long)(a - d1) * d2 + (b - d1)] = 0.5 * (kab + kba);
    }
}

// source factors G (D x R) and, optionally, the normalised basis (D x n_dof)
__global__ void k_cem_sources(const double* __restrict__ Gm, const double* __restrict__ GL, int Dall, int d1, int D,
                              int J, int J1, const int* __restrict__ fmap, int R, double* __restrict__ G) {
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t >= (long)D * R) return;
    const int a = (int)(t / R), c = (int)(t % R);
    const int fa = cem_full(a, d1, J, J1, fmap);
    G[t] = GL[(long)fa * R + c] / sqrt(Gm[(long)fa * Dall + fa]);
}

__global__ void k_cem_basis_out(const double* __restrict__ Gm, const double* __restrict__ PsiT, int Dall, int d1,
                                int D, int J, int J1, const int* __restrict__ fmap, long nd, long ldp,
                                double* __restrict__ out) {
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    if (t >= (long)D * nd) return;
    const int a = (int)(t / nd);
    const long c = t % nd;
    const int fa = cem_full(a, d1, J, J1, fmap);
    out[t] = PsiT[(long)fa * ldp + c] / sqrt(Gm[(long)fa * Dall + fa]);
}

// ---------------------------------------------------------------------------
// Local spectral problems of eq. (3.1): on every coarse element
// A_e psi = lambda S_e psi over the element's nodes not on the boundary of
// the domain (natural conditions on interior coarse edges), A_e the
// kappa-weighted Q1 stiffness and S_e the (kappa H^-2)-weighted Q1 mass over
// the element's cells. One work-group per element: S_e = L L^T (Cholesky in
// LDS), C = L^-1 A_e L^-T, cyclic Jacobi on C in LDS with the round-robin
// pair order (n/2 disjoint rotations per round, C <- R^T C R; the
// accumulated rotations V in global memory), the J smallest eigenvalues,
// psi = L^-T V[:, j] (S_e-orthonormal). Each psi is signed so that
// sum_f (f + 1) psi[f] > 0 over the free nodes f in local order (an
// eigenvector is fixed only up to sign).
// ---------------------------------------------------------------------------
constexpr int SPEC_N = 128;  // largest number of element nodes

// element matrix entry between nodes (gy, gx), (hy, hx) of element (ey, ex):
// sum over the element's cells containing both of kappa_c * (stiffness
// reference entry) or kappa_c * (mass reference entry)
__device__ inline void elem_pair(const double* __restrict__ kappa, int n, int m, int ey, int ex, int gy, int gx,
                                 int hy, int hx, double& a, double& s) {
    a = 0.0;
    s = 0.0;
    const int dy = hy - gy, dx = hx - gx;
    if (dy < -1 || dy > 1 || dx < -1 || dx > 1) return;
    const int ad = (dy != 0) + (dx != 0);
    const double ke = ad == 0 ? 4.0 / 6.0 : ad == 1 ? -1.0 / 6.0 : -2.0 / 6.0;
    const double me = ad == 0 ? 4.0 / 36.0 : ad == 1 ? 2.0 / 36.0 : 1.0 / 36.0;
    for (int cy = max(gy, hy) - 1; cy <= min(gy, hy); ++cy) {
        if (cy < ey * m || cy >= (ey + 1) * m) continue;
        for (int cx = max(gx, hx) - 1; cx <= min(gx, hx); ++cx) {
            if (cx < ex * m || cx >= (ex + 1) * m) continue;
            const double k = kappa[(long)cy * n + cx];
            a += k * ke;
            s += k * me;
        }
    }
}

// info[e]: 0, 1 (weighted mass not positive definite) or 2 (the Jacobi
// sweeps hit max_sweeps with the off-diagonal norm still above 1e-10 of the
// diagonal's)
__global__ __launch_bounds__(256) void k_spec_element(int n, int n_c, int J, const double* __restrict__ kappa,
                                                      double* __restrict__ Lg, double* __restrict__ Vg,
                                                      double* __restrict__ lam, double* __restrict__ psi,
                                                      double* __restrict__ spsi, int* __restrict__ info,
                                                      int max_sweeps) {
    __shared__ double C[SPEC_N * SPEC_N];
    __shared__ double cs[SPEC_N / 2], sn[SPEC_N / 2];
    __shared__ int pp[SPEC_N / 2], qq[SPEC_N / 2];
    __shared__ int node_of[SPEC_N];  // free index -> local node
    __shared__ int free_of[SPEC_N];  // local node -> free index or -1
    __shared__ double red[256];
    __shared__ int sel[8];
    __shared__ int nfree, bad;
    const int e = blockIdx.x, tid = threadIdx.x;
    const int m = n / n_c, ml = m + 1, nl = ml * ml;
    const int ey = e / n_c, ex = e % n_c;
    const double H = 1.0 / n_c, h = 1.0 / n, sw = h * h / (H * H);  // mass weight h^2 / H^2
    double* L = Lg + (long)e * SPEC_N * SPEC_N;
    double* V = Vg + (long)e * SPEC_N * SPEC_N;
    if (tid == 0) {
        int c = 0;
        for (int ln = 0; ln < nl; ++ln) {
            const int gy = ey * m + ln / ml, gx = ex * m + ln % ml;
            const bool fr = gy >= 1 && gy <= n - 1 && gx >= 1 && gx <= n - 1;
            free_of[ln] = fr ? c : -1;
            if (fr) node_of[c++] = ln;
        }
        nfree = c;
        bad = 0;
    }
    __syncthreads();
    const int nf = nfree;
    const int n2 = nf + (nf & 1);  // even size for the round-robin pairs
    auto gnode = [&](int f, int& gy, int& gx) {
        const int ln = node_of[f];
        gy = ey * m + ln / ml;
        gx = ex * m + ln % ml;
    };
    // S_e (free x free) in LDS, Cholesky in place (lower)
    for (int idx = tid; idx < nf * nf; idx += 256) {
        const int r = idx / nf, c = idx % nf;
        int gy, gx, hy, hx;
        gnode(r, gy, gx);
        gnode(c, hy, hx);
        double a, s;
        elem_pair(kappa, n, m, ey, ex, gy, gx, hy, hx, a, s);
        C[r * nf + c] = s * sw;
    }
    __syncthreads();
    for (int k = 0; k < nf; ++k) {
        const double piv = C[k * nf + k];
        if (!(piv > 0.0)) {
            if (tid == 0) bad = 1;
            break;  // uniform
        }
        const double sq = sqrt(piv);
        __syncthreads();
        for (int r = k + 1 + tid; r < nf; r += 256) C[r * nf + k] /= sq;
        if (tid == 0) C[k * nf + k] = sq;
        __syncthreads();
        const int w = nf - k - 1;
        for (int idx = tid; idx < w * w; idx += 256) {
            const int r = k + 1 + idx / w, c = k + 1 + idx % w;
            if (c <= r) C[r * nf + c] -= C[r * nf + k] * C[c * nf + k];
        }
        __syncthreads();
    }
    __syncthreads();
    if (bad) {
        if (tid == 0) info[e] = 1;
        return;  // uniform
    }
    for (int idx = tid; idx < nf * nf; idx += 256) {
        const int r = idx / nf, c = idx % nf;
        L[r * SPEC_N + c] = c <= r ? C[r * nf + c] : 0.0;
    }
    __syncthreads();
    // A_e into LDS (stride n2), then X = L^-1 A (thread per column) and
    // C = X L^-T (thread per row); pad row/column nf (odd nf) decoupled with
    // a diagonal above every eigenvalue
    for (int idx = tid; idx < n2 * n2; idx += 256) {
        const int r = idx / n2, c = idx % n2;
        double a = 0.0, s;
        if (r < nf && c < nf) {
            int gy, gx, hy, hx;
            gnode(r, gy, gx);
            gnode(c, hy, hx);
            elem_pair(kappa, n, m, ey, ex, gy, gx, hy, hx, a, s);
        }
        C[r * n2 + c] = a;
    }
    __syncthreads();
    if (tid < nf) {
        const int j = tid;
        for (int r = 0; r < nf; ++r) {
            double v = C[r * n2 + j];
            for (int c = 0; c < r; ++c) v -= L[r * SPEC_N + c] * C[c * n2 + j];
            C[r * n2 + j] = v / L[r * SPEC_N + r];
        }
    }
    __syncthreads();
    if (tid < nf) {
        const int i = tid;
        for (int c = 0; c < nf; ++c) {
            double v = C[i * n2 + c];
            for (int k = 0; k < c; ++k) v -= L[c * SPEC_N + k] * C[i * n2 + k];
            C[i * n2 + c] = v / L[c * SPEC_N + c];
        }
    }
    __syncthreads();
    // symmetrise, trace bound for the pad entry
    double part = 0.0;
    for (int idx = tid; idx < nf * nf; idx += 256) {
        const int r = idx / nf, c = idx % nf;
        if (c > r) {
            const double v = 0.5 * (C[r * n2 + c] + C[c * n2 + r]);
            C[r * n2 + c] = v;
            C[c * n2 + r] = v;
        }
        if (r == c) part += fabs(C[r * n2 + r]);
    }
    red[tid] = part;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) red[tid] += red[tid + o];
        __syncthreads();
    }
    // for a symmetric positive semi-definite C the trace bounds every
    // eigenvalue
    if (n2 > nf && tid == 0) C[nf * n2 + nf] = 2.0 * red[0] + 1.0;
    for (int idx = tid; idx < n2 * n2; idx += 256) V[(idx / n2) * SPEC_N + idx % n2] = (idx / n2 == idx % n2);
    __syncthreads();
    // cyclic Jacobi sweeps down to the rounding floor: once the off-diagonal
    // Frobenius norm is below 1e-10 of the diagonal's, stop at the first
    // sweep that no longer halves the off-diagonal mass (early sweeps may
    // reduce it by less; the eigenvectors need the floor, not a threshold)
    const int half = n2 / 2;
    double off_prev = -1.0;
    bool converged = false;
    double offs_last = 0.0, dgs_last = 0.0;
    for (int sweep = 0; sweep <= max_sweeps; ++sweep) {
        double off = 0.0, dg = 0.0;
        for (int idx = tid; idx < n2 * n2; idx += 256) {
            const int r = idx / n2, c = idx % n2;
            const double v = C[idx];
            if (r == c)
                dg += v * v;
            else
                off += v * v;
        }
        red[tid] = off;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (tid < o) red[tid] += red[tid + o];
            __syncthreads();
        }
        const double offs = red[0];
        __syncthreads();
        red[tid] = dg;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if (tid < o) red[tid] += red[tid + o];
            __syncthreads();
        }
        const double dgs = red[0];
        __syncthreads();
        offs_last = offs;
        dgs_last = dgs;
        if (offs != offs || dgs != dgs) break;  // NaN: reported as not converged
        if (!(offs > 0.0) || (offs < 1e-20 * dgs && off_prev >= 0.0 && offs > 0.5 * off_prev)) {
            converged = true;
            break;  // uniform
        }
        // the last pass only measures what max_sweeps sweeps left
        if (sweep == max_sweeps) break;
        off_prev = offs;
        for (int rd = 0; rd < n2 - 1; ++rd) {
            if (tid < half) {
                const int k = tid;
                const int a = k == 0 ? 0 : (k - 1 + rd) % (n2 - 1) + 1;
                const int b = (n2 - 2 - k + rd) % (n2 - 1) + 1;
                const int p = min(a, b), q = max(a, b);
                const double apq = C[p * n2 + q];
                double c = 1.0, s = 0.0;
                if (apq != 0.0) {
                    const double th = (C[q * n2 + q] - C[p * n2 + p]) / (2.0 * apq);
                    const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                    c = 1.0 / sqrt(t * t + 1.0);
                    s = t * c;
                }
                cs[k] = c;
                sn[k] = s;
                pp[k] = p;
                qq[k] = q;
            }
            __syncthreads();
            // columns p, q of C and V, four entries per thread at a time so
            // that their global loads of V are in flight together
            for (int base = tid; base < half * n2; base += 4 * 256) {
                int rr[4], pc[4], qc[4], kc[4];
                double x[4], y[4], vx[4], vy[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int idx = min(base + u * 256, half * n2 - 1);
                    kc[u] = idx / n2;
                    rr[u] = idx % n2;
                    pc[u] = pp[kc[u]];
                    qc[u] = qq[kc[u]];
                    vx[u] = V[rr[u] * SPEC_N + pc[u]];
                    vy[u] = V[rr[u] * SPEC_N + qc[u]];
                    x[u] = C[rr[u] * n2 + pc[u]];
                    y[u] = C[rr[u] * n2 + qc[u]];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (base + u * 256 >= half * n2) break;
                    const double c = cs[kc[u]], s = sn[kc[u]];
                    C[rr[u] * n2 + pc[u]] = c * x[u] - s * y[u];
                    C[rr[u] * n2 + qc[u]] = s * x[u] + c * y[u];
                    V[rr[u] * SPEC_N + pc[u]] = c * vx[u] - s * vy[u];
                    V[rr[u] * SPEC_N + qc[u]] = s * vx[u] + c * vy[u];
                }
            }
            __syncthreads();
            // rows p, q of C
            for (int idx = tid; idx < half * n2; idx += 256) {
                const int k = idx / n2, j = idx % n2;
                const int p = pp[k], q = qq[k];
                const double c = cs[k], s = sn[k];
                const double x = C[p * n2 + j], y = C[q * n2 + j];
                C[p * n2 + j] = c * x - s * y;
                C[q * n2 + j] = s * x + c * y;
            }
            __syncthreads();
        }
    }
    // the J smallest eigenvalues (ascending, ties by index)
    if (tid == 0) {
        for (int j = 0; j < J; ++j) {
            int best = -1;
            for (int i = 0; i < nf; ++i) {
                bool used = false;
                for (int u = 0; u < j; ++u) used |= sel[u] == i;
                if (used) continue;
                if (best < 0 || C[i * n2 + i] < C[best * n2 + best]) best = i;
            }
            sel[j] = best;
            lam[(long)e * J + j] = C[best * n2 + best];
        }
    }
    __syncthreads();
    // psi = L^-T u for the selected columns u of V, in LDS rows [f][j]
    // (the area of C is free now)
    double* W = C;
    if (tid < J) {
        const int j = tid, col = sel[j];
        for (int r = nf - 1; r >= 0; --r) {
            double v = V[r * SPEC_N + col];
            for (int c = r + 1; c < nf; ++c) v -= L[c * SPEC_N + r] * W[c * 8 + j];
            W[r * 8 + j] = v / L[r * SPEC_N + r];
        }
        double sg = 0.0;
        for (int r = 0; r < nf; ++r) sg += (r + 1) * W[r * 8 + j];
        if (sg < 0.0)
            for (int r = 0; r < nf; ++r) W[r * 8 + j] = -W[r * 8 + j];
    }
    __syncthreads();
    // psi on the element's local nodes (zero on the domain boundary) and
    // spsi = S_e psi over all local nodes (the element's full weighted mass)
    for (int idx = tid; idx < nl * J; idx += 256) {
        const int ln = idx / J, j = idx % J;
        const int f = free_of[ln];
        if (psi) psi[((long)e * nl + ln) * J + j] = f >= 0 ? W[f * 8 + j] : 0.0;
        const int gy = ey * m + ln / ml, gx = ex * m + ln % ml;
        double acc = 0.0;
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int ly = ln / ml + dy, lx = ln % ml + dx;
                if (ly < 0 || ly > m || lx < 0 || lx > m) continue;
                const int f2 = free_of[ly * ml + lx];
                if (f2 < 0) continue;
                double a, s;
                elem_pair(kappa, n, m, ey, ex, gy, gx, gy + dy, gx + dx, a, s);
                acc += s * sw * W[f2 * 8 + j];
            }
        spsi[((long)e * nl + ln) * J + j] = acc;
    }
    if (tid == 0) info[e] = (converged || offs_last < 1e-20 * dgs_last) ? 0 : 2;
}

}  // namespace
}  // namespace pe

using namespace pe;

namespace pe {
namespace {

// The set-up pipeline for constraint data with J slots per element: every
// element has J functions (cnt_h null; the J1 lowest span V_H1), or cnt_h[k]
// functions (host counts) placed in the blocks by fmap_h (host, D entries:
// space index -> element-major function index; the first d1 span V_H1).
pe_status spaces_impl(const char* who, int n, int n_c, int layers, int J, int J1, const double* kappa,
                      const double* spsi, const int* cnt_h, const int* fmap_h, int d1, int d2, int R,
                      const double* loads, double* M11, double* M12, double* M22, double* A11, double* A12,
                      double* A22, double* G, double* Psi, hipStream_t st) {
    const std::string tag = std::string(who) + ": ";
    const int m = n / n_c;
    if (m < 2) return set_error(PE_ERR_ARG, tag + "a coarse element needs at least 2 fine cells per side");
    const int span = std::min(2 * layers + 1, n_c);  // coarse elements per patch side, at most
    const int nx_max = span * m - 1, nf_max = nx_max * nx_max;
    if (nx_max + 2 > CEM_WN)
        return set_error(PE_ERR_ARG, tag + "patch rows of " + std::to_string(nx_max) +
                                         " nodes exceed the band window (at most " + std::to_string(CEM_WN - 2) +
                                         ")");
    const int n_elem = n_c * n_c;
    // constraints per patch (at most CEM_NAUX) and functions per element
    int naux_max = span * span * J, own_max = J, Dall = n_elem * J;
    std::vector<int> foff_h;
    if (cnt_h) {
        foff_h.assign(n_elem + 1, 0);
        own_max = 0;
        for (int k = 0; k < n_elem; ++k) {
            if (cnt_h[k] < 1 || cnt_h[k] > J)
                return set_error(PE_ERR_ARG, tag + "element " + std::to_string(k) + " has " +
                                                 std::to_string(cnt_h[k]) + " functions (1.." + std::to_string(J) +
                                                 ")");
            foff_h[k + 1] = foff_h[k] + cnt_h[k];
            own_max = std::max(own_max, cnt_h[k]);
        }
        Dall = foff_h[n_elem];
        naux_max = 0;
        for (int i = 0; i < n_elem; ++i) {
            const int ey = i / n_c, ex = i % n_c;
            int tot = 0;
            for (int ky = std::max(ey - layers, 0); ky <= std::min(ey + layers, n_c - 1); ++ky)
                for (int kx = std::max(ex - layers, 0); kx <= std::min(ex + layers, n_c - 1); ++kx)
                    tot += cnt_h[ky * n_c + kx];
            naux_max = std::max(naux_max, tot);
        }
    }
    if (naux_max > CEM_NAUX)
        return set_error(PE_ERR_ARG, tag + "more than " + std::to_string(CEM_NAUX) + " constraints per patch");
    if ((long)nf_max * own_max > CEM_LDS_S) return set_error(PE_ERR_ARG, tag + "patch too large for the final sweep");
    const int D = d1 + d2;
    if (D != Dall || d1 < 1) return set_error(PE_ERR_ARG, tag + "split sizes do not match the functions");
    const long nd = (long)(n - 1) * (n - 1);
    const long ldp = (nd + 7) / 8 * 8;

    CemGeom g;
    g.n = n;
    g.n_c = n_c;
    g.m = m;
    g.layers = layers;
    g.J = J;
    g.lb_stride = (long)nf_max * (nx_max + 2);
    g.y_stride = (long)nf_max * CEM_NAUX;
    g.ldp = ldp;
    g.n_dof1 = n - 1;

    std::vector<void*> bufs;
    auto alloc = [&](void** ptr, size_t bytes) {
        if (hipMalloc(ptr, bytes) != hipSuccess) {
            (void)hipGetLastError();
            *ptr = nullptr;
            return false;
        }
        bufs.push_back(*ptr);
        return true;
    };
    auto done = [&](pe_status s) {
        (void)hipStreamSynchronize(st);
        for (void* b : bufs) (void)hipFree(b);
        return s;
    };
    double *Lb, *Yb, *Sb, *PsiT, *MX, *KX, *Gm, *Gk, *Ld = nullptr, *GL = nullptr;
    int* info;
    int *cnt_d = nullptr, *foff_d = nullptr, *fmap_d = nullptr;
    if (cnt_h) {
        if (!alloc((void**)&cnt_d, sizeof(int) * n_elem) || !alloc((void**)&foff_d, sizeof(int) * (n_elem + 1)) ||
            !alloc((void**)&fmap_d, sizeof(int) * D))
            return done(set_error(PE_ERR_NOMEM, tag + "device memory"));
        if (hipMemcpyAsync(cnt_d, cnt_h, sizeof(int) * n_elem, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(foff_d, foff_h.data(), sizeof(int) * (n_elem + 1), hipMemcpyHostToDevice, st) !=
                hipSuccess ||
            hipMemcpyAsync(fmap_d, fmap_h, sizeof(int) * D, hipMemcpyHostToDevice, st) != hipSuccess)
            return done(set_error(PE_ERR_HIP, tag + "table upload"));
        g.cnt = cnt_d;
        g.foff = foff_d;
    }
    if (!alloc((void**)&Lb, sizeof(double) * g.lb_stride * n_elem) ||
        !alloc((void**)&Yb, sizeof(double) * g.y_stride * n_elem) ||
        !alloc((void**)&Sb, sizeof(double) * CEM_NAUX * CEM_NAUX * n_elem) ||
        !alloc((void**)&PsiT, sizeof(double) * ldp * Dall) || !alloc((void**)&MX, sizeof(double) * ldp * Dall) ||
        !alloc((void**)&KX, sizeof(double) * ldp * Dall) || !alloc((void**)&Gm, sizeof(double) * Dall * Dall) ||
        !alloc((void**)&Gk, sizeof(double) * Dall * Dall) || !alloc((void**)&info, sizeof(int) * n_elem) ||
        (R > 0 && (!alloc((void**)&Ld, sizeof(double) * ldp * R) || !alloc((void**)&GL, sizeof(double) * Dall * R))))
        return done(set_error(PE_ERR_NOMEM, tag + "device memory"));
    auto hip_ok = [&](hipError_t e, const char* what) -> pe_status {
        if (e == hipSuccess) return PE_OK;
        return set_error(PE_ERR_HIP, tag + what + ": " + hipGetErrorString(e));
    };
    pe_status s;
    if ((s = hip_ok(hipMemsetAsync(PsiT, 0, sizeof(double) * ldp * Dall, st), "clear")) != PE_OK) return done(s);
    if ((s = hip_ok(hipMemsetAsync(info, 0, sizeof(int) * n_elem, st), "clear")) != PE_OK) return done(s);
    hipLaunchKernelGGL(k_cem_band_chol, dim3(n_elem), dim3(256), 0, st, g, kappa, Lb, info);
    hipLaunchKernelGGL(k_cem_forward, dim3(n_elem), dim3(CEM_NAUX), 0, st, g, Lb, spsi, Yb);
    hipLaunchKernelGGL(k_cem_gram, dim3(n_elem), dim3(256), 0, st, g, Yb, Sb);
    if ((s = hip_ok(hipGetLastError(), "patch kernels")) != PE_OK) return done(s);
    // a failed band factorisation leaves its patch's later stages reading
    // finite garbage only; its status is reported below
    std::vector<int> hinfo(n_elem);
    if ((s = hip_ok(hipMemcpyAsync(hinfo.data(), info, sizeof(int) * n_elem, hipMemcpyDeviceToHost, st),
                    "status")) != PE_OK)
        return done(s);
    if ((s = hip_ok(hipStreamSynchronize(st), "patch factorisations")) != PE_OK) return done(s);
    for (int i = 0; i < n_elem; ++i)
        if (hinfo[i] != 0)
            return done(set_error(PE_ERR_NOT_SPD, tag + "patch " + std::to_string(i) +
                                                      " stiffness not positive definite at row " +
                                                      std::to_string(hinfo[i])));
    hipLaunchKernelGGL(k_cem_finish, dim3(n_elem), dim3(256), 0, st, g, Lb, Yb, Sb, PsiT, info);
    if ((s = hip_ok(hipGetLastError(), "basis kernel")) != PE_OK) return done(s);
    if ((s = hip_ok(hipMemcpyAsync(hinfo.data(), info, sizeof(int) * n_elem, hipMemcpyDeviceToHost, st),
                    "status")) != PE_OK)
        return done(s);
    if ((s = hip_ok(hipStreamSynchronize(st), "basis functions")) != PE_OK) return done(s);
    for (int i = 0; i < n_elem; ++i)
        if (hinfo[i] != 0)
            return done(set_error(PE_ERR_NOT_SPD, tag + "constraint Gram matrix of patch " +
                                                      std::to_string(i) + " not positive definite at row " +
                                                      std::to_string(-hinfo[i])));
    // projections
    const unsigned gx = (unsigned)((ldp + 255) / 256);
    hipLaunchKernelGGL(k_cem_stencil, dim3(gx, Dall), dim3(256), 0, st, kappa, n, ldp, PsiT, MX, KX);
    if (R > 0) {
        const long tot = (long)R * ldp;
        hipLaunchKernelGGL(k_cem_pad, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, loads, nd, ldp,
                           (long)R, Ld);
    }
    if ((s = hip_ok(hipGetLastError(), "stencil")) != PE_OK) return done(s);
    GemmWork ws;
    auto product = [&](const double* Bop, int Ns, double* C) -> pe_status {
        GemmShape sh;
        sh.Mr = Dall;
        sh.Ns = Ns;
        sh.A = PsiT;
        sh.lda = ldp;
        sh.B = Bop;
        sh.ldb = ldp;
        sh.s_split = Ns;
        sh.k0a = 0;
        sh.k1a = (int)ldp;
        sh.k0b = 0;
        sh.k1b = 0;
        Epi epi;
        epi.mode = EPI_STORE;
        epi.C = C;
        epi.ldc = Ns;
        TileCfg cfg = choose_tiles(sh, false, 256);
        const size_t need = gemm_part_bytes(sh, cfg, sizeof(double));
        if (need > ws.part_bytes) {
            if (ws.part) (void)hipFree(ws.part);
            ws.part = nullptr;
            ws.part_bytes = 0;
            if (hipMalloc(&ws.part, need) != hipSuccess) {
                (void)hipGetLastError();
                return set_error(PE_ERR_NOMEM, tag + "product workspace");
            }
            ws.part_bytes = need;
        }
        return hip_ok(gemm_launch<double>(sh, epi, cfg, ws, st), "Gram product");
    };
    s = product(MX, Dall, Gm);
    if (s == PE_OK) s = product(KX, Dall, Gk);
    if (s == PE_OK && R > 0) s = product(Ld, R, GL);
    if (s != PE_OK) {
        pe_status r = done(s);
        if (ws.part) (void)hipFree(ws.part);
        return r;
    }
    {
        const long tot = (long)D * D;
        hipLaunchKernelGGL(k_cem_blocks, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, Gm, Gk, Dall, d1,
                           d2, J, J1, fmap_d, M11, M12, M22, A11, A12, A22);
    }
    if (R > 0) {
        const long tot = (long)D * R;
        hipLaunchKernelGGL(k_cem_sources, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, Gm, GL, Dall, d1,
                           D, J, J1, fmap_d, R, G);
    }
    if (Psi) {
        const long tot = (long)D * nd;
        hipLaunchKernelGGL(k_cem_basis_out, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, Gm, PsiT, Dall,
                           d1, D, J, J1, fmap_d, nd, ldp, Psi);
    }
    s = hip_ok(hipGetLastError(), "block kernels");
    pe_status r = done(s);
    if (ws.part) (void)hipFree(ws.part);
    return r;
}

}  // namespace
}  // namespace pe

extern "C" pe_status pe_cem_spaces(int n, int n_c, int layers, int J, int J1, const double* kappa,
                                   const double* spsi, int R, const double* loads, double* M11, double* M12,
                                   double* M22, double* A11, double* A12, double* A22, double* G, double* Psi,
                                   void* hip_stream) {
    if (n <= 0 || n_c <= 0 || n % n_c != 0 || layers < 0 || J <= 0 || J > 8 || J1 <= 0 || J1 > J || !kappa ||
        !spsi || R < 0 || (R > 0 && (!loads || !G)) || !M11 || !M22 || !A11 || !A22 ||
        (J1 < J && (!M12 || !A12)))
        return set_error(PE_ERR_ARG, "pe_cem_spaces: bad arguments");
    const int n_elem = n_c * n_c;
    return spaces_impl("pe_cem_spaces", n, n_c, layers, J, J1, kappa, spsi, nullptr, nullptr, n_elem * J1,
                       n_elem * (J - J1), R, loads, M11, M12, M22, A11, A12, A22, G, Psi, (hipStream_t)hip_stream);
}

extern "C" pe_status pe_nlmc_spaces(int n, int n_c, int layers, int J, const int* counts, const double* kappa,
                                    const double* rdata, int R, const double* loads, double* M11, double* M12,
                                    double* M22, double* A11, double* A12, double* A22, double* G, double* Psi,
                                    void* hip_stream) {
    if (n <= 0 || n_c <= 0 || n % n_c != 0 || layers < 0 || J <= 1 || J > 8 || !counts || !rdata || !kappa ||
        R < 0 || (R > 0 && (!loads || !G)) || !M11 || !M12 || !M22 || !A11 || !A12 || !A22)
        return set_error(PE_ERR_ARG, "pe_nlmc_spaces: bad arguments");
    const int n_elem = n_c * n_c;
    // V_H1: the fracture functions (slots 1.. of every element), V_H2: the
    // matrix functions (slot 0), both element-major
    std::vector<int> fmap;
    int off = 0, d1 = 0;
    std::vector<int> first(n_elem);
    for (int k = 0; k < n_elem; ++k) {
        if (counts[k] < 1 || counts[k] > J)
            return set_error(PE_ERR_ARG, "pe_nlmc_spaces: element " + std::to_string(k) + " has " +
                                             std::to_string(counts[k]) + " regions (1.." + std::to_string(J) + ")");
        first[k] = off;
        for (int l = 1; l < counts[k]; ++l) fmap.push_back(off + l);
        d1 += counts[k] - 1;
        off += counts[k];
    }
    if (d1 < 1) return set_error(PE_ERR_ARG, "pe_nlmc_spaces: no fracture function");
    for (int k = 0; k < n_elem; ++k) fmap.push_back(first[k]);
    return spaces_impl("pe_nlmc_spaces", n, n_c, layers, J, 0, kappa, rdata, counts, fmap.data(), d1, n_elem, R,
                       loads, M11, M12, M22, A11, A12, A22, G, Psi, (hipStream_t)hip_stream);
}

extern "C" pe_status pe_local_spectral(int n, int n_c, int J, const double* kappa, double* lam, double* psi,
                                       double* spsi, void* hip_stream) {
    hipStream_t st = (hipStream_t)hip_stream;
    if (n <= 0 || n_c <= 0 || n % n_c != 0 || J <= 0 || J > 8 || !kappa || !lam || !spsi)
        return set_error(PE_ERR_ARG, "pe_local_spectral: bad arguments");
    const int m = n / n_c;
    if ((m + 1) * (m + 1) > SPEC_N)
        return set_error(PE_ERR_ARG, "pe_local_spectral: more than " + std::to_string(SPEC_N) +
                                         " nodes per coarse element");
    // every element keeps at least (m - 1)^2 nodes off the boundary
    if (m < 2 || J > (m - 1) * (m - 1)) return set_error(PE_ERR_ARG, "pe_local_spectral: J exceeds the element's nodes");
    const int n_elem = n_c * n_c;
    double *Lg = nullptr, *Vg = nullptr;
    int* info = nullptr;
    auto done = [&](pe_status s) {
        (void)hipStreamSynchronize(st);
        for (void* b : {(void*)Lg, (void*)Vg, (void*)info})
            if (b) (void)hipFree(b);
        return s;
    };
    const size_t mat = sizeof(double) * SPEC_N * SPEC_N * n_elem;
    if (hipMalloc((void**)&Lg, mat) != hipSuccess || hipMalloc((void**)&Vg, mat) != hipSuccess ||
        hipMalloc((void**)&info, sizeof(int) * n_elem) != hipSuccess) {
        (void)hipGetLastError();
        return done(set_error(PE_ERR_NOMEM, "pe_local_spectral: device memory"));
    }
    // sweep cap (PE_SPECTRAL_SWEEPS overrides the default 30, e.g. to test
    // the non-convergence report)
    int max_sweeps = 30;
    if (const char* ms = getenv("PE_SPECTRAL_SWEEPS")) {
        const int v = atoi(ms);
        if (v >= 0 && v <= 1000) max_sweeps = v;
    }
    hipLaunchKernelGGL(k_spec_element, dim3(n_elem), dim3(256), 0, st, n, n_c, J, kappa, Lg, Vg, lam, psi, spsi,
                       info, max_sweeps);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return done(set_error(PE_ERR_HIP, std::string("pe_local_spectral: ") + hipGetErrorString(e)));
    std::vector<int> hinfo(n_elem);
    if (hipMemcpyAsync(hinfo.data(), info, sizeof(int) * n_elem, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return done(set_error(PE_ERR_HIP, "pe_local_spectral: status read-back"));
    for (int i = 0; i < n_elem; ++i) {
        if (hinfo[i] == 2)
            return done(set_error(PE_ERR_NUMERIC, "pe_local_spectral: the Jacobi sweeps of element " +
                                                      std::to_string(i) + " did not converge in " +
                                                      std::to_string(max_sweeps) + " sweeps"));
        if (hinfo[i] != 0)
            return done(set_error(PE_ERR_NOT_SPD, "pe_local_spectral: weighted mass of element " +
                                                      std::to_string(i) + " not positive definite"));
    }
    return done(PE_OK);
}
