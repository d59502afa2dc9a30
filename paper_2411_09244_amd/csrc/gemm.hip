// MFMA GEMM for gfx950 with the fused epilogues of the splitting-scheme step.
//
// C[r][s] = epi( sum_k A[r][k] * B[s][k] ), A and B both K-contiguous.
// Work-group: 256 threads = 4 wave64, arranged 2 x 2 over a BR x BS tile;
// each wave owns a (BR/2) x (BS/2) sub-tile made of 16x16 MFMA blocks
// (v_mfma_f32_16x16x4f32 for FP32, v_mfma_f64_16x16x4f64 for FP64).
// Operand tiles are staged through LDS (BK deep, padded rows, register
// prefetch of the next K tile). With split-K, every work-group writes its
// partial tile into the plane of its split; a second, element-parallel kernel
// sums the planes in split order (a fixed order, so results are bitwise
// reproducible) and runs the epilogue. Products with at most 4 state columns
// (the coarse sweep) use a row-parallel GEMV kernel instead.
#include "pe_internal.h"

#include <hip/hip_cooperative_groups.h>

#include <cstdlib>
#include <type_traits>

namespace pe {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct MfmaOp;

template <>
struct MfmaOp<float> {
    typedef f32x4 acc_t;
    typedef float4 vec_t;  // 16-byte global/LDS vector
    static constexpr int BK = 32;
    __device__ static inline acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // row of accumulator element q held by `lane` (column is lane % 16)
    __device__ static inline int row(int lane, int q) { return 4 * (lane >> 4) + q; }
};

template <>
struct MfmaOp<double> {
    typedef f64x4 acc_t;
    typedef double2 vec_t;
    static constexpr int BK = 16;
    __device__ static inline acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // the FP64 block interleaves rows: element q of `lane` is row lane/16 + 4q
    __device__ static inline int row(int lane, int q) { return (lane >> 4) + 4 * q; }
};

// ---------------------------------------------------------------------------
// epilogue
// ---------------------------------------------------------------------------
__device__ inline double source_value_p(const Epi& e, int r, int s, int p_step) {
    if (e.src_kind == 0) return 0.0;
    if (e.rows_per_p > 0) {
        p_step += r / e.rows_per_p;
        r = e.col_off + r % e.rows_per_p;
    }
    int b, n;
    if (e.n_fixed >= 0) {
        b = r;
        n = e.n_fixed;
    } else {
        b = r / e.cols_per_b;
        n = r - b * e.cols_per_b;
    }
    if (e.src_kind == 2) return e.Fint[((long)b * e.N + n) * e.ldf + s];
    const long tau = (e.time_mode == 0) ? (long)n * e.P + p_step : (long)n;
    const double* g = e.Gs + (long)s * e.R;
    const double* h = e.Hs + (long)b * e.R * e.Tlen + tau;
    // blocks of QB terms: all loads of a block (indices clamped, surplus
    // terms weighted by zero) before any use, so a block costs one round trip
    constexpr int QB = 8;
    double v = 0.0;
    for (int q0 = 0; q0 < e.R; q0 += QB) {
        double gq[QB], hq[QB];
#pragma unroll
        for (int q = 0; q < QB; ++q) {
            const int qq = min(q0 + q, e.R - 1);
            gq[q] = g[qq];
            hq[q] = h[(long)qq * e.Tlen];
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) v = fma(q0 + q < e.R ? gq[q] : 0.0, hq[q], v);
    }
    return v;
}

__device__ inline double source_value(const Epi& e, int r, int s) { return source_value_p(e, r, s, e.p_step); }

// fused fine step (EPI_FSTEP) with the step index and state buffers given
// explicitly: increment d = Z F(t) - base - acc, then the state/history
// update from din into dout (layout per column: [du_prev | u - u_a | w - w_a | dw_prev])
__device__ inline void fstep_apply(const Epi& e, int r, int s, double acc, int p_step, const double* __restrict__ din,
                                   double* __restrict__ dout, float* __restrict__ dout32, double* __restrict__ traj) {
    double v = source_value_p(e, r, s, p_step) - acc;
    if (e.base) v -= e.base[(long)r * e.ldb + s];
    const double* di = din + (long)r * e.ldd;
    double* d = dout + (long)r * e.ldd;
    float* d32 = dout32 ? dout32 + (long)r * e.ldd : nullptr;
    double full_dev;
    if (s < e.d1p) {
        const double u = di[e.d1p + s] + v;
        d[s] = v;
        d[e.d1p + s] = u;
        if (d32) {
            d32[s] = (float)v;
            d32[e.d1p + s] = (float)u;
        }
        full_dev = u;
    } else {
        const int j = s - e.d1p;
        const long ow = 2L * e.d1p + j, oh = 2L * e.d1p + e.d2p + j;
        const double w = di[ow] + v;
        d[ow] = w;
        d[oh] = v;
        if (d32) {
            d32[ow] = (float)w;
            d32[oh] = (float)v;
        }
        full_dev = w;
    }
    if (traj) traj[(long)r * e.ldtraj + s] = e.xa[(long)r * (e.d1p + e.d2p) + s] + full_dev;
}

// Each epilogue is split into a load phase (everything it reads besides the
// accumulated value) and a finish phase. Kernels whose accumulation is short
// (the split-K reduction, the coarse-step matrix-vector products) issue the
// load phase together with their operand loads, so an output costs one memory
// round trip instead of two. The arithmetic, and its order, is the same as
// in a single-phase epilogue.
struct EpiIn {
    double a = 0.0, b = 0.0, c = 0.0, d = 0.0;
    bool ok = true;
};

template <int MODE>
__device__ inline EpiIn epi_load(const Epi& e, int r, int s) {
    EpiIn in;
    if constexpr (MODE == EPI_STORE) {
        if (e.beta != 0.0) in.a = e.C0[(long)r * e.ldc0 + s];
    } else if constexpr (MODE == EPI_RESID) {
        if (e.base) in.b = e.base[(long)r * e.ldb + s];
        if (e.dres) in.c = e.dres[(long)r * e.lddres + s];
        in.a = source_value(e, r, s);
    } else if constexpr (MODE == EPI_FSTEP) {
        // branch-free load first, the source term (branches, waits) last
        in.c = e.din[(long)r * e.ldd + (s < e.d1p ? e.d1p + s : 2L * e.d1p + (s - e.d1p))];
        if (e.vr && s >= e.d1p) in.d = e.din[(long)r * e.ldd + 2L * e.d1p + e.d2p + (s - e.d1p)];
        if (e.base) in.b = e.base[(long)r * e.ldb + s];
        in.a = source_value_p(e, r, s, e.p_step);
    } else if constexpr (MODE == EPI_FCORR) {
        const double* d = e.dev64 + (long)r * e.ldd;
        const long o0 = s < e.d1p ? (long)s : 2L * e.d1p + (s - e.d1p);
        const long o1 = s < e.d1p ? (long)e.d1p + s : 2L * e.d1p + e.d2p + (s - e.d1p);
        in.a = d[o0];
        in.b = d[o1];
        if (e.traj) in.c = e.traj[(long)r * e.ldtraj + s];
    } else if constexpr (MODE == EPI_COARSE_INIT) {
        if (e.cs) in.a = e.cs[(long)r * e.ldcs + s];
    } else if constexpr (MODE == EPI_COARSE_DELTA) {
        in.ok = !(e.active && !e.active[r]);
        in.a = e.fbuf[(long)r * e.ldfb + s];
        in.b = e.xprev[(long)r * e.ldxo + s];
    } else if constexpr (MODE == EPI_ADJ_STATE) {
        const long D = e.ldr;
        const int j = s < D ? s : (int)(s - D);
        in.a = e.s_cur[(long)r * 2 * D + j];
        if (e.inj) in.b = e.inj[(long)r * e.ldinj + j];
        if (s >= D && e.sacc) in.c = e.sacc[(long)r * D + j];
    }
    return in;
}

template <int MODE>
__device__ inline void epi_finish(const Epi& e, int r, int s, double acc, const EpiIn& in) {
    if constexpr (MODE == EPI_STORE) {
        double v = e.alpha * acc;
        if (e.beta != 0.0) v += e.beta * in.a;
        if (e.diag_add != 0.0 && r == s + e.diag_off) v += e.diag_add;
        e.C[(long)r * e.ldc + s] = v;
        if (e.C32) e.C32[(long)r * e.ldc + s] = (float)v;
    } else if constexpr (MODE == EPI_RESID) {
        double v = in.a - acc;
        if (e.base) v -= in.b;
        if (e.dres) v -= e.cres * in.c;
        if (e.R64) e.R64[(long)r * e.ldr + s] = v;
        if (e.R32) e.R32[(long)r * e.ldr + s] = (float)v;
    } else if constexpr (MODE == EPI_FSTEP) {
        // increment d = Z F(t) - base - acc, then the state/history update
        // (layout per column: [du_prev | u - u_a | w - w_a | dw_prev])
        double v = in.a - acc;
        if (e.base) v -= in.b;
        double* d = e.dev64 + (long)r * e.ldd;
        float* d32 = e.dev32 ? e.dev32 + (long)r * e.ldd : nullptr;
        double full_dev;
        if (s < e.d1p) {
            const double u = in.c + v;
            d[s] = v;
            d[e.d1p + s] = u;
            if (d32) {
                d32[s] = (float)v;
                d32[e.d1p + s] = (float)u;
            }
            full_dev = u;
            if (e.vr) {
                double* q = e.vr + (long)r * e.ldd;
                q[s] = u;
                q[e.d1p + 2L * e.d2p + s] = v;
            }
        } else {
            const int j = s - e.d1p;
            const long ow = 2L * e.d1p + j, oh = 2L * e.d1p + e.d2p + j;
            const double w = in.c + v;
            d[ow] = w;
            d[oh] = v;
            if (d32) {
                d32[ow] = (float)w;
                d32[oh] = (float)v;
            }
            full_dev = w;
            if (e.vr) {
                double* q = e.vr + (long)r * e.ldd;
                q[e.d1p + j] = in.c;
                q[e.d1p + e.d2p + j] = in.d;
            }
        }
        if (e.traj) e.traj[(long)r * e.ldtraj + s] = e.xa[(long)r * (e.d1p + e.d2p) + s] + full_dev;
    } else if constexpr (MODE == EPI_FCORR) {
        // the correction c = acc of the step's increment: du (or dw) and the
        // state u - u_a (or w - w_a) both move by c
        double* d = e.dev64 + (long)r * e.ldd;
        float* d32 = e.dev32 ? e.dev32 + (long)r * e.ldd : nullptr;
        const long o0 = s < e.d1p ? (long)s : 2L * e.d1p + (s - e.d1p);
        const long o1 = s < e.d1p ? (long)e.d1p + s : 2L * e.d1p + e.d2p + (s - e.d1p);
        // o0 holds du (u rows) or w - w_a (w rows); o1 holds u - u_a or dw
        const double a = in.a + acc, b = in.b + acc;
        d[o0] = a;
        d[o1] = b;
        if (d32) {
            d32[o0] = (float)a;
            d32[o1] = (float)b;
        }
        if (e.traj) e.traj[(long)r * e.ldtraj + s] = in.c + acc;
    } else if constexpr (MODE == EPI_COARSE_INIT) {
        double x = acc;
        if (e.cs) x += in.a;
        e.xout[(long)r * e.ldxo + s] = x;
    } else if constexpr (MODE == EPI_COARSE_DELTA) {
        if (!in.ok) return;
        const double x = in.a + acc;
        e.xout[(long)r * e.ldxo + s] = x;
        const double d = x - in.b;
        if (e.dl64) e.dl64[(long)r * e.ldl + s] = d;
        if (e.dl32) e.dl32[(long)r * e.ldl + s] = (float)d;
    } else if constexpr (MODE == EPI_ADJ_STATE) {
        const long D = e.ldr;
        const int j = s < D ? s : (int)(s - D);
        double v = in.a - acc;
        if (e.inj) v += in.b;
        e.s_nxt[(long)r * 2 * D + s] = v;
        if (s >= D) {
            if (e.nu32) e.nu32[(long)r * D + j] = (float)v;
            if (e.sacc) e.sacc[(long)r * D + j] = in.c + v;
            if (e.rho_all) e.rho_all[((long)r * e.P + e.m_step) * D + j] = v;
        }
    }
}

// one epilogue per mode (the product kernel emits one unrolled store loop per
// mode, which keeps each loop small enough to unroll with static accumulator
// indexing)
template <int MODE>
__device__ inline void epi_apply(const Epi& e, int r, int s, double acc) {
    epi_finish<MODE>(e, r, s, acc, epi_load<MODE>(e, r, s));
}

// call f(integral_constant<mode>) for the runtime mode
template <typename F>
__device__ inline void epi_dispatch(int mode, F&& f) {
    switch (mode) {
        case EPI_STORE: f(std::integral_constant<int, EPI_STORE>{}); break;
        case EPI_RESID: f(std::integral_constant<int, EPI_RESID>{}); break;
        case EPI_FSTEP: f(std::integral_constant<int, EPI_FSTEP>{}); break;
        case EPI_COARSE_INIT: f(std::integral_constant<int, EPI_COARSE_INIT>{}); break;
        case EPI_COARSE_DELTA: f(std::integral_constant<int, EPI_COARSE_DELTA>{}); break;
        case EPI_ADJ_STATE: f(std::integral_constant<int, EPI_ADJ_STATE>{}); break;
        case EPI_FCORR: f(std::integral_constant<int, EPI_FCORR>{}); break;
        default: break;
    }
}

__device__ inline void epilogue(const Epi& e, int r, int s, double acc) {
    epi_dispatch(e.mode, [&](auto m) { epi_apply<decltype(m)::value>(e, r, s, acc); });
}

// ---------------------------------------------------------------------------
// kernel
// ---------------------------------------------------------------------------
// one BR x BS output tile (or its split-K part) of C = epi(A B^T)
template <typename T, int BR, int BS, int BK>
__device__ __forceinline__ void gemm_tile(const GemmShape& sh, const Epi& epi, const int tiles_r, const int tile,
                                          const int split, const int splitk, T* __restrict__ part,
                                          const bool planes_only = false) {
    using Op = MfmaOp<T>;
    using acc_t = typename Op::acc_t;
    using vec_t = typename Op::vec_t;
    constexpr int VW = 16 / sizeof(T);      // elements per 16-byte vector
    constexpr int LDT = BK;                 // LDS row (elements), 16-byte chunks XOR-swizzled
    constexpr int KV = BK / VW;             // vectors per tile row
    constexpr int R2 = (256 / (KV * 16)) > 0 ? (256 / (KV * 16)) : 1;  // rows per 256-byte bank line
    constexpr int AV = BR * KV / 256;       // A vectors per thread
    constexpr int BV = BS * KV / 256;       // B vectors per thread
    constexpr int MI = BR / 32, MJ = BS / 32;
    static_assert(AV >= 1 && BV >= 1, "tile too small for 256 threads");
    static_assert(BR % 32 == 0 && BS % 32 == 0 && BK % 16 == 0, "bad tile");

    // two LDS stages: the next K tile is stored while the current one is used
    __shared__ __align__(16) T As[2][BR * LDT];
    __shared__ __align__(16) T Bs[2][BS * LDT];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = wave & 1, wsi = wave >> 1;
    const int tr = tile % tiles_r, ts = tile / tiles_r;
    const int r0 = tr * BR, s0 = ts * BS;
    const int s1 = min(s0 + BS, sh.Ns);
    // 16 x 16 blocks of this wave's quarter that hold rows and columns of
    // the product: i < ni, j < nj. Blocks wholly in the padding past Mr or
    // Ns (a ragged last tile) are not sent to the matrix cores.
    const int ni = min(MI, max(0, (sh.Mr - (r0 + wr * (BR / 2)) + 15) / 16));
    const int nj = min(MJ, max(0, (sh.Ns - (s0 + wsi * (BS / 2)) + 15) / 16));
    const bool full = ni == MI && nj == MJ;

    int k0, k1;
    if (s1 <= sh.s_split) {
        k0 = sh.k0a;
        k1 = sh.k1a;
    } else if (s0 >= sh.s_split) {
        k0 = sh.k0b;
        k1 = sh.k1b;
    } else {
        k0 = min(sh.k0a, sh.k0b);
        k1 = max(sh.k1a, sh.k1b);
    }
    const int nkt = (k1 > k0) ? (k1 - k0 + BK - 1) / BK : 0;
    const int per = (nkt + splitk - 1) / splitk;
    const int kt0 = min(nkt, split * per);
    const int kt1 = min(nkt, kt0 + per);

    const T* __restrict__ A = (const T*)sh.A;
    const T* __restrict__ B = (const T*)sh.B;

    acc_t acc[MI][MJ];
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < MJ; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

    vec_t ra[AV], rb[BV];
    auto gload = [&](int kbase) {
#pragma unroll
        for (int v = 0; v < AV; ++v) {
            const int idx = tid + v * 256;
            const int row = idx / KV, kk = (idx % KV) * VW;
            const int r = r0 + row, k = kbase + kk;
            if (r < sh.Mr && k < k1)
                ra[v] = *(const vec_t*)(A + (long)r * sh.lda + k);
            else
                ra[v] = vec_t{};
        }
#pragma unroll
        for (int v = 0; v < BV; ++v) {
            const int idx = tid + v * 256;
            const int row = idx / KV, kk = (idx % KV) * VW;
            const int s = s0 + row, k = kbase + kk;
            if (s < sh.Ns && k < k1)
                rb[v] = *(const vec_t*)(B + (long)s * sh.ldb + k);
            else
                rb[v] = vec_t{};
        }
    };
    // physical chunk of logical chunk c in row r: c ^ ((r / R2) % KV), so
    // the 16 rows one MFMA operand read spans fall in distinct banks
    auto sstore = [&](int stage) {
#pragma unroll
        for (int v = 0; v < AV; ++v) {
            const int idx = tid + v * 256;
            const int row = idx / KV, c = idx % KV;
            *(vec_t*)(&As[stage][row * LDT + ((c ^ ((row / R2) % KV)) * VW)]) = ra[v];
        }
#pragma unroll
        for (int v = 0; v < BV; ++v) {
            const int idx = tid + v * 256;
            const int row = idx / KV, c = idx % KV;
            *(vec_t*)(&Bs[stage][row * LDT + ((c ^ ((row / R2) % KV)) * VW)]) = rb[v];
        }
    };

    int stage = 0;
    if (kt0 < kt1) {
        gload(k0 + kt0 * BK);
        sstore(0);
        __syncthreads();
    }
    // the products of one staged K tile; FULL: every block of the quarter
    // is live (no per-block conditions in the unrolled loop)
    auto kstep = [&](auto full_c, const T* Asc, const T* Bsc) {
        constexpr bool FULL = decltype(full_c)::value;
#pragma unroll
        for (int kk = 0; kk < BK; kk += 16) {
            T a[MI][4], b[MJ][4];
            // four consecutive k of this lane: element offset koff in the
            // row, inside one 16-byte chunk (VW = 4: the whole chunk; VW =
            // 2: chunks koff / 2 and koff / 2 + 1)
            const int koff = kk + 4 * (lane >> 4);
#pragma unroll
            for (int i = 0; i < MI; ++i) {
                if (!FULL && i >= ni) continue;
                const int row = wr * (BR / 2) + i * 16 + (lane & 15);
                const T* pr = Asc + row * LDT;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int e = koff + q, c = e / VW;
                    a[i][q] = pr[((c ^ ((row / R2) % KV)) * VW) + e % VW];
                }
            }
#pragma unroll
            for (int j = 0; j < MJ; ++j) {
                if (!FULL && j >= nj) continue;
                const int row = wsi * (BS / 2) + j * 16 + (lane & 15);
                const T* pr = Bsc + row * LDT;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int e = koff + q, c = e / VW;
                    b[j][q] = pr[((c ^ ((row / R2) % KV)) * VW) + e % VW];
                }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int i = 0; i < MI; ++i)
#pragma unroll
                    for (int j = 0; j < MJ; ++j)
                        if (FULL || (i < ni && j < nj)) acc[i][j] = Op::mma(a[i][q], b[j][q], acc[i][j]);
        }
    };

    for (int kt = kt0; kt < kt1; ++kt) {
        const bool more = kt + 1 < kt1;
        if (more) gload(k0 + (kt + 1) * BK);
        if (full)
            kstep(std::true_type{}, As[stage], Bs[stage]);
        else if (ni > 0 && nj > 0)
            kstep(std::false_type{}, As[stage], Bs[stage]);
        if (more) sstore(stage ^ 1);
        __syncthreads();
        stage ^= 1;
    }

    // output coordinates of this lane: 16x16 block (i, j), element q ->
    // row Op::row(lane, q), column lane % 16 of the block
    if (splitk == 1 && !planes_only) {
        epi_dispatch(epi.mode, [&](auto m) {
            constexpr int MODE = decltype(m)::value;
#pragma unroll
            for (int i = 0; i < MI; ++i)
#pragma unroll
                for (int j = 0; j < MJ; ++j)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int r = r0 + wr * (BR / 2) + i * 16 + Op::row(lane, q);
                        const int s = s0 + wsi * (BS / 2) + j * 16 + (lane & 15);
                        if (r < sh.Mr && s < sh.Ns) epi_apply<MODE>(epi, r, s, (double)acc[i][j][q]);
                    }
        });
        return;
    }

    // split-K: write the partial tile into this split's plane (Mr x Ns)
    T* plane = part + (long)split * sh.Mr * sh.Ns;
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < MJ; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = r0 + wr * (BR / 2) + i * 16 + Op::row(lane, q);
                const int s = s0 + wsi * (BS / 2) + j * 16 + (lane & 15);
                if (r < sh.Mr && s < sh.Ns) plane[(long)r * sh.Ns + s] = acc[i][j][q];
            }
}

template <typename T, int BR, int BS, int BK>
__global__ __launch_bounds__(256) void gemm_nt_kernel(const GemmShape sh, const Epi epi, const int tiles_r,
                                                      const int splitk, T* __restrict__ part) {
    gemm_tile<T, BR, BS, BK>(sh, epi, tiles_r, blockIdx.x, blockIdx.y, splitk, part);
}

// ---------------------------------------------------------------------------
// Wave-split-K product for skinny outputs (all state columns of a product in
// one 64-row tile, as in the fine steps of one sample): each of the W waves
// of a work-group computes the whole 64 x BS output tile over its own slice
// of K. A wave reads its MFMA operands straight from global memory into
// registers in the MFMA lane layout (lane l holds rows l % 16 + 16 i and the
// four consecutive k values 4 (l / 16) .. +3 of each 16-deep step), keeping
// PF steps in flight: there is no LDS staging and no barrier in the K loop,
// so each wave streams its slice at its own pace. At the end the W partial
// tiles are added through LDS in wave order (bitwise reproducible) and the
// sum goes to the epilogue (one split) or to the split's plane, which the
// split-K reduction kernel adds in split order.
// ---------------------------------------------------------------------------
template <typename T>
struct Quad4 {
    T v[4];
};

// elements k .. k+3 of a row, read at min(k, k1 - 4) so that the address
// stays inside the row's K range [.., k1) (k1 a multiple of 16 / sizeof(T));
// the caller zeroes a quad with k >= k1 when it uses it. Loads are never
// skipped or post-processed here, so that the compiler can keep them in
// flight across loop iterations.
template <typename T>
__device__ __forceinline__ Quad4<T> load_quad(const T* row, int k, int k1);

template <>
__device__ __forceinline__ Quad4<float> load_quad<float>(const float* row, int k, int k1) {
    const float4 x = *(const float4*)(row + min(k, k1 - 4));
    return Quad4<float>{{x.x, x.y, x.z, x.w}};
}

template <>
__device__ __forceinline__ Quad4<double> load_quad<double>(const double* row, int k, int k1) {
    const double2 a = *(const double2*)(row + min(k, k1 - 2));
    const double2 b = *(const double2*)(row + min(k + 2, k1 - 2));
    return Quad4<double>{{a.x, a.y, b.x, b.y}};
}

template <typename T, int BS, int W, int PF>
__global__ __launch_bounds__(W * 64) void gemm_wsk_kernel(const GemmShape sh, const Epi epi, const int tiles_r,
                                                          const int splitk, T* __restrict__ part) {
    using Op = MfmaOp<T>;
    using acc_t = typename Op::acc_t;
    constexpr int BR = 64, MI = BR / 16, MJ = BS / 16;
    constexpr int LDR = BS + 4;  // padded row of the LDS partial tiles
    static_assert(BS % 16 == 0, "bad tile");
    __shared__ __align__(16) T red[W][BR * LDR];

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int tile = blockIdx.x, split = blockIdx.y;
    const int tr = tile % tiles_r, ts = tile / tiles_r;
    const int r0 = tr * BR, s0 = ts * BS;
    const int s1 = min(s0 + BS, sh.Ns);

    int k0, k1;
    if (s1 <= sh.s_split) {
        k0 = sh.k0a;
        k1 = sh.k1a;
    } else if (s0 >= sh.s_split) {
        k0 = sh.k0b;
        k1 = sh.k1b;
    } else {
        k0 = min(sh.k0a, sh.k0b);
        k1 = max(sh.k1a, sh.k1b);
    }
    // this wave's slice: steps [st0, st0 + n) of 16 K values, piece
    // split * W + wave of splitk * W equal pieces
    const int nst = (k1 > k0) ? (k1 - k0 + 15) / 16 : 0;
    const int pieces = splitk * W;
    const int per = (nst + pieces - 1) / pieces;
    const int st0 = min(nst, (split * W + wave) * per);
    const int n = min(nst, st0 + per) - st0;

    const T* __restrict__ A = (const T*)sh.A;
    const T* __restrict__ B = (const T*)sh.B;
    const int kl = k0 + 4 * (lane >> 4);  // this lane's first k
    // operand rows of this lane; a row out of range reads row 0 instead (its
    // outputs are never stored, and no valid output depends on it)
    const T* pa[MI];
    const T* pb[MJ];
#pragma unroll
    for (int i = 0; i < MI; ++i) {
        const int r = r0 + i * 16 + (lane & 15);
        pa[i] = A + (long)(r < sh.Mr ? r : 0) * sh.lda;
    }
#pragma unroll
    for (int j = 0; j < MJ; ++j) {
        const int s = s0 + j * 16 + (lane & 15);
        pb[j] = B + (long)(s < sh.Ns ? s : 0) * sh.ldb;
    }

    acc_t acc[MI][MJ];
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < MJ; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

    // ring of PF steps in registers; a step index past the slice repeats its
    // last step (loaded, never used)
    Quad4<T> qa[PF][MI], qb[PF][MJ];
    auto load = [&](Quad4<T>(&xa)[MI], Quad4<T>(&xb)[MJ], int step) {
        const int k = kl + (st0 + min(step, n - 1)) * 16;
#pragma unroll
        for (int i = 0; i < MI; ++i) xa[i] = load_quad<T>(pa[i], k, k1);
#pragma unroll
        for (int j = 0; j < MJ; ++j) xb[j] = load_quad<T>(pb[j], k, k1);
    };
    // step `step` of the slice: the operator quads past k1 (only in a last,
    // partial step of the K range) are zeroed, which zeroes their products
    auto mma_step = [&](const Quad4<T>(&xa)[MI], const Quad4<T>(&xb)[MJ], int step) {
        const int k = kl + (st0 + step) * 16;
        const bool z_lo = k >= k1, z_hi = k + 2 >= k1;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const bool z = q < 2 ? z_lo : z_hi;
#pragma unroll
            for (int i = 0; i < MI; ++i)
#pragma unroll
                for (int j = 0; j < MJ; ++j)
                    acc[i][j] = Op::mma(xa[i].v[q], z ? T(0) : xb[j].v[q], acc[i][j]);
        }
    };
    if (n > 0) {
#pragma unroll
        for (int u = 0; u < PF; ++u) load(qa[u], qb[u], u);
        int t = 0;
        // full rounds: step t + u is used, then its slot is refilled with
        // step t + u + PF (same load sequence on every path)
        for (; t + PF < n; t += PF) {
#pragma unroll
            for (int u = 0; u < PF; ++u) {
                mma_step(qa[u], qb[u], t + u);
                // keep the refill between this step's and the next step's
                // products (the scheduler would otherwise sink every load
                // of the round below the last product)
                __builtin_amdgcn_sched_barrier(0);
                load(qa[u], qb[u], t + u + PF);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        // last round: no more loads
#pragma unroll
        for (int u = 0; u < PF; ++u)
            if (t + u < n) mma_step(qa[u], qb[u], t + u);
    }

    // partial tiles through LDS, added in wave order
    T* mine = red[wave];
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < MJ; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                mine[(i * 16 + Op::row(lane, q)) * LDR + j * 16 + (lane & 15)] = acc[i][j][q];
    __syncthreads();
    auto tile_sum = [&](int o) {
        const int idx = (o / BS) * LDR + (o % BS);
        T v = red[0][idx];
#pragma unroll
        for (int w = 1; w < W; ++w) v += red[w][idx];
        return v;
    };
    if (splitk == 1) {
        epi_dispatch(epi.mode, [&](auto m) {
            constexpr int MODE = decltype(m)::value;
            for (int o = threadIdx.x; o < BR * BS; o += W * 64) {
                const int r = r0 + o / BS, s = s0 + o % BS;
                if (r < sh.Mr && s < sh.Ns) epi_apply<MODE>(epi, r, s, (double)tile_sum(o));
            }
        });
        return;
    }
    T* plane = part + (long)split * sh.Mr * sh.Ns;
    for (int o = threadIdx.x; o < BR * BS; o += W * 64) {
        const int r = r0 + o / BS, s = s0 + o % BS;
        if (r < sh.Mr && s < sh.Ns) plane[(long)r * sh.Ns + s] = tile_sum(o);
    }
}

// Persistent fine sweep: every fused step of one sweep in one cooperative
// launch, for products whose state columns fit one row tile (Mr <= BR).
// Step p: the work-groups compute the split-K partial tiles of Z W dev into
// the planes, the grid synchronises, every thread sums its elements' planes
// in split order (bitwise reproducible) and runs the step epilogue (state
// ping-pong: even steps read state buffer a, odd steps b), and the grid
// synchronises again. Step 0 has no product (zero deviation).
template <typename T, int BR, int BS, int BK>
__global__ __launch_bounds__(256) void fine_sweep_persistent_kernel(const GemmShape sh, const void* A1, const Epi epi,
                                                                    double* d64a, double* d64b, float* d32a,
                                                                    float* d32b, double* traj, const int P,
                                                                    const int n_tiles, const int splitk,
                                                                    T* __restrict__ part) {
    namespace cg = cooperative_groups;
    cg::grid_group grid = cg::this_grid();
    const long total = (long)sh.Mr * sh.Ns;
    const int G = gridDim.x;
    const long nthreads = (long)G * blockDim.x;
    const int Dp = epi.d1p + epi.d2p;
    for (int p = 0; p < P; ++p) {
        const int c = p & 1;
        if (p > 0) {
            GemmShape s2 = sh;
            if (c) s2.A = A1;
            for (int item = blockIdx.x; item < n_tiles * splitk; item += G)
                gemm_tile<T, BR, BS, BK>(s2, epi, 1, item % n_tiles, item / n_tiles, splitk, part, true);
            grid.sync();
        }
        const double* din = c ? d64b : d64a;
        double* dout = c ? d64a : d64b;
        float* dout32 = c ? d32a : d32b;
        double* tr = traj ? traj + (long)p * Dp : nullptr;
        for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < total; i += nthreads) {
            double v = 0.0;
            if (p > 0)
                for (int sp = 0; sp < splitk; ++sp) v += (double)part[(long)sp * total + i];
            const int r = (int)(i / sh.Ns), s = (int)(i - (long)r * sh.Ns);
            fstep_apply(epi, r, s, v, p, din, dout, dout32, tr);
        }
        grid.sync();
    }
}

// grouped products: work-group w computes tile wg_tile[w] of product
// wg_item[w] (each product with its own shape, operands and epilogue)
template <typename T, int BR, int BS, int BK>
__global__ __launch_bounds__(256) void gemm_grouped_kernel(const GemmItem* __restrict__ items,
                                                           const int* __restrict__ wg_item,
                                                           const int* __restrict__ wg_tile) {
    const int item = wg_item[blockIdx.x];
    if (item < 0) return;  // padding of an XCD-aware table
    const GemmItem& it = items[item];
    gemm_tile<T, BR, BS, BK>(it.sh, it.epi, it.tiles_r, wg_tile[blockIdx.x], 0, 1, nullptr);
}

// split-K reduction with the epilogue: out[i] = epi(sum_sp part[sp][i]),
// partial tiles summed in split order (bitwise reproducible). The epilogue's
// loads are issued together with the SK plane loads.
template <typename T, int MODE, int SK>
__global__ __launch_bounds__(256) void splitk_epilogue_kernel(const int Mr, const int Ns, const int splitk,
                                                              const T* __restrict__ part, const Epi epi) {
    const long total = (long)Mr * Ns;
    const long stride = (long)gridDim.x * blockDim.x;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < total; i += stride) {
        const int r = (int)(i / Ns), s = (int)(i - (long)r * Ns);
        double v = 0.0;
        if constexpr (SK > 0) {
            // plane loads first (no branches), then the epilogue's loads
            T pv[SK];
#pragma unroll
            for (int sp = 0; sp < SK; ++sp) pv[sp] = part[(long)sp * total + i];
            const EpiIn in = epi_load<MODE>(epi, r, s);
#pragma unroll
            for (int sp = 0; sp < SK; ++sp) v += (double)pv[sp];
            epi_finish<MODE>(epi, r, s, v, in);
        } else {
            const EpiIn in = epi_load<MODE>(epi, r, s);
            for (int sp = 0; sp < splitk; ++sp) v += (double)part[(long)sp * total + i];
            epi_finish<MODE>(epi, r, s, v, in);
        }
    }
}

// y[r][s] = sum_k A[r][k] B[s][k] for MR <= 4 state columns: two waves per
// operator row (two rows per work-group), each wave taking every other
// 64-lane chunk of K with 16-byte loads. A lane loads CH chunks before it
// multiplies any of them (addresses clamped into the operands, chunks past
// the end zeroed by a select, so no load sits under a branch), and the lane
// that runs the epilogue requests the epilogue's inputs first: at the
// 2000-row size every load of the kernel is in flight at once. Wave
// reductions, then the two partial sums are added in wave order (bitwise
// reproducible) and the epilogue runs once per (r, s).
template <typename T, int MR, int MODE>
__global__ __launch_bounds__(256) void gemv_kernel(const GemmShape sh, const Epi epi) {
    using vec_t = typename MfmaOp<T>::vec_t;
    constexpr int VW = 16 / sizeof(T);
    constexpr int WPR = 2, CH = 4;
    __shared__ double red[4][MR];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int sub = wave % WPR;
    const int s = blockIdx.x * (4 / WPR) + wave / WPR;
    const bool epi_lane = lane == 0 && sub == 0 && s < sh.Ns;
    EpiIn in[MR];
    if (epi_lane) {
#pragma unroll
        for (int r = 0; r < MR; ++r)
            if (r < sh.Mr) in[r] = epi_load<MODE>(epi, r, s);
    }
    double acc[MR];
#pragma unroll
    for (int r = 0; r < MR; ++r) acc[r] = 0.0;
    if (s < sh.Ns) {
        const int k0 = s < sh.s_split ? sh.k0a : sh.k0b;
        const int k1 = s < sh.s_split ? sh.k1a : sh.k1b;
        const T* __restrict__ B = (const T*)sh.B + (long)s * sh.ldb;
        const T* __restrict__ A = (const T*)sh.A;
        constexpr int step = 64 * VW * WPR;
        for (int kb = k0 + VW * (lane + 64 * sub); kb < k1; kb += CH * step) {
            vec_t w[CH], x[CH][MR];
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const int kc = min(kb + c * step, k1 - VW);
                w[c] = *(const vec_t*)(B + kc);
#pragma unroll
                for (int r = 0; r < MR; ++r) x[c][r] = *(const vec_t*)(A + (long)min(r, sh.Mr - 1) * sh.lda + kc);
            }
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const bool ok = kb + c * step < k1;
                const T* wp = (const T*)&w[c];
#pragma unroll
                for (int r = 0; r < MR; ++r) {
                    const T* xp = (const T*)&x[c][r];
#pragma unroll
                    for (int q = 0; q < VW; ++q) acc[r] = fma(ok ? (double)wp[q] : 0.0, (double)xp[q], acc[r]);
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < MR; ++r)
        for (int off = 32; off > 0; off >>= 1) acc[r] += __shfl_xor(acc[r], off, 64);
    if (lane == 0)
#pragma unroll
        for (int r = 0; r < MR; ++r) red[wave][r] = acc[r];
    __syncthreads();
    if (epi_lane) {
#pragma unroll
        for (int r = 0; r < MR; ++r) {
            if (r >= sh.Mr) break;
            double v = red[wave][r];
            for (int w = 1; w < WPR; ++w) v += red[wave + w][r];
            epi_finish<MODE>(epi, r, s, v, in[r]);
        }
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

static int k_extent(const GemmShape& sh) {
    const int la = sh.k1a - sh.k0a, lb = sh.k1b - sh.k0b;
    return la > lb ? la : lb;
}

size_t gemm_part_bytes(const GemmShape& sh, const TileCfg& cfg, size_t elem) {
    if (cfg.splitk <= 1 || sh.Mr <= 4) return 0;
    return (size_t)cfg.splitk * sh.Mr * sh.Ns * elem;
}

TileCfg choose_tiles(const GemmShape& sh, bool fp32, int n_cu) {
    TileCfg c;
    c.br = sh.Mr <= 32 ? 32 : 64;
    c.bs = 64;
    const long tiles = (long)cdiv(sh.Mr, c.br) * cdiv(sh.Ns, c.bs);
    const int bk = fp32 ? 32 : 16;
    const int nkt = cdiv(k_extent(sh), bk);
    const long target = 2L * n_cu;
    int sk = 1;
    if (tiles < target && nkt > 1) {
        sk = (int)((target + tiles - 1) / tiles);
        const int max_sk = nkt / 2 > 1 ? nkt / 2 : 1;   // keep >= 2 K tiles per split
        if (sk > max_sk) sk = max_sk;
        if (sk > 32) sk = 32;
        if (sk < 1) sk = 1;
    }
    c.splitk = sk;
    return c;
}

// split-K reduction launch for one epilogue mode, with the split count as a
// compile-time constant for the common counts
template <typename T, int MODE>
static void launch_reduce(dim3 g, dim3 b, hipStream_t stream, const GemmShape& sh, int splitk, const T* part,
                          const Epi& epi) {
    switch (splitk) {
        case 2: hipLaunchKernelGGL((splitk_epilogue_kernel<T, MODE, 2>), g, b, 0, stream, sh.Mr, sh.Ns, splitk, part, epi); break;
        case 4: hipLaunchKernelGGL((splitk_epilogue_kernel<T, MODE, 4>), g, b, 0, stream, sh.Mr, sh.Ns, splitk, part, epi); break;
        case 8: hipLaunchKernelGGL((splitk_epilogue_kernel<T, MODE, 8>), g, b, 0, stream, sh.Mr, sh.Ns, splitk, part, epi); break;
        case 16: hipLaunchKernelGGL((splitk_epilogue_kernel<T, MODE, 16>), g, b, 0, stream, sh.Mr, sh.Ns, splitk, part, epi); break;
        default: hipLaunchKernelGGL((splitk_epilogue_kernel<T, MODE, 0>), g, b, 0, stream, sh.Mr, sh.Ns, splitk, part, epi); break;
    }
}

// split-K reduction of the partial planes in ws.part and the epilogue
template <typename T>
static hipError_t launch_splitk_reduce(const GemmShape& sh, const Epi& epi, int splitk, GemmWork& ws,
                                       hipStream_t stream) {
    if (ws.between) ws.between(ws.between_arg);
    const long total = (long)sh.Mr * sh.Ns;
    long blocks = (total + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    const dim3 g((unsigned)blocks), b(256);
    const T* part = (const T*)ws.part;
    switch (epi.mode) {
        case EPI_STORE: launch_reduce<T, EPI_STORE>(g, b, stream, sh, splitk, part, epi); break;
        case EPI_RESID: launch_reduce<T, EPI_RESID>(g, b, stream, sh, splitk, part, epi); break;
        case EPI_FSTEP: launch_reduce<T, EPI_FSTEP>(g, b, stream, sh, splitk, part, epi); break;
        case EPI_COARSE_INIT: launch_reduce<T, EPI_COARSE_INIT>(g, b, stream, sh, splitk, part, epi); break;
        case EPI_COARSE_DELTA: launch_reduce<T, EPI_COARSE_DELTA>(g, b, stream, sh, splitk, part, epi); break;
        case EPI_ADJ_STATE: launch_reduce<T, EPI_ADJ_STATE>(g, b, stream, sh, splitk, part, epi); break;
        case EPI_FCORR: launch_reduce<T, EPI_FCORR>(g, b, stream, sh, splitk, part, epi); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int BR, int BS, int BK>
static hipError_t launch_cfg(const GemmShape& sh, const Epi& epi, int splitk, GemmWork& ws,
                             hipStream_t stream) {
    const int tr = cdiv(sh.Mr, BR), tsn = cdiv(sh.Ns, BS);
    dim3 grid(tr * tsn, splitk);
    if (splitk > 1) {
        const size_t need = (size_t)splitk * sh.Mr * sh.Ns * sizeof(T);
        if (need > ws.part_bytes) return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL((gemm_nt_kernel<T, BR, BS, BK>), grid, dim3(256), 0, stream, sh, epi, tr, splitk,
                       (T*)ws.part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || splitk == 1) return e;
    return launch_splitk_reduce<T>(sh, epi, splitk, ws, stream);
}

// wave-split-K kernel: W waves per work-group, PF steps in flight per wave
template <typename T, int BS, int W>
static hipError_t launch_wsk(const GemmShape& sh, const Epi& epi, int splitk, GemmWork& ws, hipStream_t stream) {
    constexpr int PF = sizeof(T) == 4 ? 4 : 2;
    const int tr = cdiv(sh.Mr, 64), tsn = cdiv(sh.Ns, BS);
    dim3 grid(tr * tsn, splitk);
    if (splitk > 1) {
        const size_t need = (size_t)splitk * sh.Mr * sh.Ns * sizeof(T);
        if (need > ws.part_bytes) return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL((gemm_wsk_kernel<T, BS, W, PF>), grid, dim3(W * 64), 0, stream, sh, epi, tr, splitk,
                       (T*)ws.part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || splitk == 1) return e;
    return launch_splitk_reduce<T>(sh, epi, splitk, ws, stream);
}

template <typename T, int MODE>
static void launch_gemv_m(const GemmShape& sh, const Epi& epi, hipStream_t stream) {
    const dim3 grid((unsigned)cdiv(sh.Ns, 2));
    switch (sh.Mr) {
        case 1: hipLaunchKernelGGL((gemv_kernel<T, 1, MODE>), grid, dim3(256), 0, stream, sh, epi); break;
        case 2: hipLaunchKernelGGL((gemv_kernel<T, 2, MODE>), grid, dim3(256), 0, stream, sh, epi); break;
        default: hipLaunchKernelGGL((gemv_kernel<T, 4, MODE>), grid, dim3(256), 0, stream, sh, epi); break;
    }
}

template <typename T>
static hipError_t launch_gemv(const GemmShape& sh, const Epi& epi, hipStream_t stream) {
    switch (epi.mode) {
        case EPI_STORE: launch_gemv_m<T, EPI_STORE>(sh, epi, stream); break;
        case EPI_RESID: launch_gemv_m<T, EPI_RESID>(sh, epi, stream); break;
        case EPI_FSTEP: launch_gemv_m<T, EPI_FSTEP>(sh, epi, stream); break;
        case EPI_COARSE_INIT: launch_gemv_m<T, EPI_COARSE_INIT>(sh, epi, stream); break;
        case EPI_COARSE_DELTA: launch_gemv_m<T, EPI_COARSE_DELTA>(sh, epi, stream); break;
        case EPI_ADJ_STATE: launch_gemv_m<T, EPI_ADJ_STATE>(sh, epi, stream); break;
        case EPI_FCORR: launch_gemv_m<T, EPI_FCORR>(sh, epi, stream); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

bool gemm_shape_ok(const GemmShape& sh, size_t elem) {
    const long vw = 16 / (long)elem;
    return !((sh.lda % vw) || (sh.ldb % vw) || (sh.k0a % vw) || (sh.k0b % vw) || (sh.k1a % vw) ||
             (sh.k1b % vw) || (((uintptr_t)sh.A) % 16) || (((uintptr_t)sh.B) % 16));
}

template <typename T>
hipError_t gemm_launch(const GemmShape& sh, const Epi& epi, const TileCfg& cfg, GemmWork& ws,
                       hipStream_t stream) {
    if (sh.Mr <= 0 || sh.Ns <= 0) return hipSuccess;
    if (!gemm_shape_ok(sh, sizeof(T))) return hipErrorInvalidValue;
    if (sh.Mr <= 4) return launch_gemv<T>(sh, epi, stream);
    const int sk = cfg.splitk < 1 ? 1 : cfg.splitk;
    constexpr int B0 = MfmaOp<T>::BK;  // base K depth: 32 (FP32), 16 (FP64)
    if (cfg.wsk > 0) {
        if (cfg.bs == 32 && cfg.wsk == 4) return launch_wsk<T, 32, 4>(sh, epi, sk, ws, stream);
        if (cfg.bs == 32 && cfg.wsk == 8) return launch_wsk<T, 32, 8>(sh, epi, sk, ws, stream);
        if (cfg.bs == 16 && cfg.wsk == 4) return launch_wsk<T, 16, 4>(sh, epi, sk, ws, stream);
        if (cfg.bs == 16 && cfg.wsk == 8) return launch_wsk<T, 16, 8>(sh, epi, sk, ws, stream);
        return hipErrorInvalidValue;
    }
    const bool deep = cfg.bk2 != 0;
#define PE_CFG(R, S)                                                                 \
    if (cfg.br == R && cfg.bs == S)                                                  \
        return deep ? launch_cfg<T, R, S, 2 * B0>(sh, epi, sk, ws, stream)           \
                    : launch_cfg<T, R, S, B0>(sh, epi, sk, ws, stream);
    PE_CFG(32, 64)
    PE_CFG(64, 32)
    PE_CFG(64, 64)
    PE_CFG(64, 128)
    PE_CFG(128, 64)
    PE_CFG(128, 128)
#undef PE_CFG
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t gemm_grouped_launch(const GemmItem* items, const int* wg_item, const int* wg_tile, int n_wg,
                               const TileCfg& cfg, hipStream_t stream) {
    if (n_wg <= 0) return hipSuccess;
    constexpr int B0 = MfmaOp<T>::BK;
    const bool deep = cfg.bk2 != 0;
#define PE_GCFG(R, S)                                                                                      \
    if (cfg.br == R && cfg.bs == S) {                                                                     \
        if (deep)                                                                                          \
            hipLaunchKernelGGL((gemm_grouped_kernel<T, R, S, 2 * B0>), dim3((unsigned)n_wg), dim3(256), 0, \
                               stream, items, wg_item, wg_tile);                                           \
        else                                                                                               \
            hipLaunchKernelGGL((gemm_grouped_kernel<T, R, S, B0>), dim3((unsigned)n_wg), dim3(256), 0,     \
                               stream, items, wg_item, wg_tile);                                           \
        return hipGetLastError();                                                                          \
    }
    PE_GCFG(64, 64)
    PE_GCFG(32, 64)
    PE_GCFG(64, 128)
    PE_GCFG(128, 64)
#undef PE_GCFG
    return hipErrorInvalidValue;
}

// grouped coarse step: one wave per operator row of one problem, its samples
// in chunks of 4, wave reduction, epilogue by lane 0
template <typename T>
__global__ __launch_bounds__(256) void coarse_grouped_kernel(const CoarseItem* __restrict__ items,
                                                             const int* __restrict__ wg_item,
                                                             const int* __restrict__ wg_row, const int n,
                                                             const int delta, const int c) {
    using vec_t = typename MfmaOp<T>::vec_t;
    constexpr int VW = 16 / sizeof(T);
    const CoarseItem& it = items[wg_item[blockIdx.x]];
    if (n >= it.N) return;
    const int lane = threadIdx.x & 63;
    const int s = wg_row[blockIdx.x] * 4 + (threadIdx.x >> 6);
    if (s >= it.Dp) return;
    const int Dp = it.Dp;
    const T* __restrict__ Phi = (const T*)(sizeof(T) == 4 ? (const void*)it.Phi32 : (const void*)it.Phi64) +
                                (long)s * Dp;
    const T* Dl = (const T*)(sizeof(T) == 4 ? (const void*)it.Dl32[c] : (const void*)it.Dl64[c]);
    for (int b0 = 0; b0 < it.B; b0 += 4) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int k = VW * lane; k < Dp; k += 64 * VW) {
            const vec_t w = *(const vec_t*)(Phi + k);
            const T* wp = (const T*)&w;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int b = b0 + r;
                if (b < it.B) {
                    const T* v = delta ? Dl + (long)b * Dp : (const T*)(it.Xk + (long)b * it.ldX + (long)n * Dp);
                    const vec_t x = *(const vec_t*)(v + k);
                    const T* xp = (const T*)&x;
#pragma unroll
                    for (int q = 0; q < VW; ++q) acc[r] += (double)wp[q] * (double)xp[q];
                }
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
            for (int off = 32; off > 0; off >>= 1) acc[r] += __shfl_xor(acc[r], off, 64);
        if (lane == 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int b = b0 + r;
                if (b >= it.B) break;
                const long ox = (long)b * it.ldX + (long)(n + 1) * Dp + s;
                const long of = ((long)b * it.N + n) * Dp + s;
                if (!delta) {
                    it.Xk[ox] = acc[r] + (it.cs ? it.cs[of] : 0.0);
                } else {
                    if (it.active && !it.active[b]) continue;
                    const double x = it.Fbuf[of] + acc[r];
                    it.Xk[ox] = x;
                    const double d = x - it.Xprev[ox];
                    if (sizeof(T) == 4)
                        it.Dl32[1 - c][(long)b * Dp + s] = (float)d;
                    else
                        it.Dl64[1 - c][(long)b * Dp + s] = d;
                }
            }
        }
    }
}

template <typename T>
hipError_t coarse_grouped_launch(const CoarseItem* items, const int* wg_item, const int* wg_row, int n_wg, int n,
                                 int delta, int c, hipStream_t stream) {
    if (n_wg <= 0) return hipSuccess;
    hipLaunchKernelGGL((coarse_grouped_kernel<T>), dim3((unsigned)n_wg), dim3(256), 0, stream, items, wg_item,
                       wg_row, n, delta, c);
    return hipGetLastError();
}

template <typename T>
static auto persistent_fn() {
    return fine_sweep_persistent_kernel<T, 64, 32, 2 * MfmaOp<T>::BK>;
}

template <typename T>
int fine_sweep_persistent_grid() {
    int per_cu = 0, n_cu = 0, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, persistent_fn<T>(), 256, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    int coop = 0;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop) {
        (void)hipGetLastError();
        return 0;
    }
    return per_cu * n_cu;
}

template <typename T>
hipError_t fine_sweep_persistent(const GemmShape& sh, const void* A1, const Epi& epi, double* d64a, double* d64b,
                                 float* d32a, float* d32b, double* traj, int P, int grid, int splitk, void* part,
                                 size_t part_bytes, hipStream_t stream) {
    if (sh.Mr > 64 || sh.Mr <= 0 || grid <= 0 || splitk < 1) return hipErrorInvalidValue;
    if (!gemm_shape_ok(sh, sizeof(T)) || (((uintptr_t)A1) % 16)) return hipErrorInvalidValue;
    if ((size_t)splitk * sh.Mr * sh.Ns * sizeof(T) > part_bytes) return hipErrorInvalidValue;
    int n_tiles = cdiv(sh.Ns, 32);
    GemmShape s0 = sh;
    const void* a1 = A1;
    Epi e = epi;
    T* pt = (T*)part;
    void* args[] = {(void*)&s0, (void*)&a1, (void*)&e, (void*)&d64a, (void*)&d64b, (void*)&d32a, (void*)&d32b,
                    (void*)&traj, (void*)&P, (void*)&n_tiles, (void*)&splitk, (void*)&pt};
    return hipLaunchCooperativeKernel((const void*)persistent_fn<T>(), dim3((unsigned)grid), dim3(256), args, 0,
                                      stream);
}

template int fine_sweep_persistent_grid<float>();
template int fine_sweep_persistent_grid<double>();
template hipError_t fine_sweep_persistent<float>(const GemmShape&, const void*, const Epi&, double*, double*, float*,
                                                 float*, double*, int, int, int, void*, size_t, hipStream_t);
template hipError_t fine_sweep_persistent<double>(const GemmShape&, const void*, const Epi&, double*, double*,
                                                  float*, float*, double*, int, int, int, void*, size_t, hipStream_t);

template hipError_t gemm_grouped_launch<float>(const GemmItem*, const int*, const int*, int, const TileCfg&,
                                               hipStream_t);
template hipError_t gemm_grouped_launch<double>(const GemmItem*, const int*, const int*, int, const TileCfg&,
                                                hipStream_t);
template hipError_t coarse_grouped_launch<float>(const CoarseItem*, const int*, const int*, int, int, int, int,
                                                 hipStream_t);
template hipError_t coarse_grouped_launch<double>(const CoarseItem*, const int*, const int*, int, int, int, int,
                                                  hipStream_t);

template hipError_t gemm_launch<float>(const GemmShape&, const Epi&, const TileCfg&, GemmWork&,
                                       hipStream_t);
template hipError_t gemm_launch<double>(const GemmShape&, const Epi&, const TileCfg&, GemmWork&,
                                        hipStream_t);

}  // namespace pe
