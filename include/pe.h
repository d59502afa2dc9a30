/*
 * pe.h - C ABI of libpe: parareal for the partially explicit temporal
 * splitting scheme in CEM-GMsFEM multiscale spaces, on one MI355X (gfx950).
 *
 * Method (Wang, Yang, Leung, "Parallel in time partially explicit splitting
 * scheme for high contrast linear multiscale diffusion problems"):
 *   - the splitting scheme of eqs. (2.4)-(2.5): u in V_H1 implicit, w in
 *     V_H2 explicit, step h, with mass-coupling differences of the previous
 *     step;
 *   - the coarse propagator G = one step of size dt_coarse, the fine
 *     propagator F = P = dt_coarse/dt_fine steps of size dt_fine (the exact
 *     solution of the all-at-once fine system of Section 4.2 on one coarse
 *     interval), every propagator call starting with a fresh history;
 *   - the parareal update of eq. (2.7) and the stopping test of eq. (2.8)
 *     (Algorithm 1), iteration k applying F to iterate k-1.
 *
 * Conventions shared by every call:
 *   - Matrices and state arrays are dense, row-major, FP64, contiguous.
 *     "device" pointers are HIP device memory of the current device;
 *     "host" pointers are ordinary host memory.
 *   - State vectors are x = [u; w] with u in R^d1 (coefficients in the basis
 *     of V_H1) and w in R^d2 (V_H2), D = d1 + d2.
 *   - Input buffers are borrowed for the duration of the call only: the
 *     library copies what it keeps. Output buffers are caller-allocated.
 *   - All GPU work is ordered on the stream given at problem creation.
 *     Calls that return results to the host synchronise that stream.
 *   - Return value: 0 = success, > 0 = warning, < 0 = error. No exception
 *     crosses the ABI. pe_last_error() gives a message for the calling
 *     thread's last failing call. Handles are not thread-safe.
 */
#ifndef PE_H
#define PE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef int pe_status;
typedef struct pe_problem_s* pe_problem;

enum {
    PE_OK = 0,
    PE_WARN_NOT_CONVERGED = 1, /* k_max reached before the stopping test held */
    PE_ERR_ARG = -1,           /* invalid argument (sizes, step ratio, symmetry) */
    PE_ERR_NOT_SPD = -2,       /* a Cholesky factorisation met a non-positive pivot */
    PE_ERR_NONFINITE = -3,     /* NaN or Inf in a parareal jump */
    PE_ERR_STATE = -4,         /* call order violated (e.g. solve before source) */
    PE_ERR_HIP = -5,           /* HIP runtime error */
    PE_ERR_NOMEM = -6,         /* device allocation failed */
    PE_ERR_NUMERIC = -7        /* an iteration of the set-up pipeline did not converge */
};

/* precision of the fine propagator */
enum {
    PE_FP64 = 0,  /* every product in FP64 on FP64 MFMA */
    PE_MIXED = 1, /* fine-step products in FP32 on MFMA with FP32 accumulation,
                     applied to the deviation from an FP64 anchor state taken at
                     each interval start; FP64 state accumulation, FP64
                     factorisations, coarse propagator and jump norms */
    PE_MIXED_REFINE = 2 /* PE_MIXED plus one refinement of the implicit V_H1 solve
                     of every fine step (eq. (2.4)): the residual
                     r = F1 - A11 u' - A12 w - M12 (w - w_prev)/dt_fine - M11 (u' - u)/dt_fine
                     of the FP32 step's u' is formed in FP64 from the FP64
                     state, and the FP32 correction Z[:, u] r (Z the step's
                     solve operator, formed in FP64) is added to the
                     increments of u and w. Applied in the fine sweeps taken
                     at the state's scale (the first parareal iteration's
                     sweep, pe_fine_propagate, the adjoint's trajectory
                     recomputation); the later sweeps, which propagate only
                     the iterate change, run unrefined (their FP32 rounding
                     scales with that change) unless PE_REFINE_ALL=1 is in
                     the environment at creation. The transposed (adjoint)
                     sweeps are not refined. */
};

/* time layout of the source amplitudes */
enum {
    PE_T_FINE = 0,     /* H[b][r][m], m = n*P + p: amplitude at t_n + (p+1) dt_fine */
    PE_T_INTERVAL = 1  /* H[b][r][n]: amplitude constant on (t_n, t_{n+1}] */
};

/* stopping test of eq. (2.8), norm |e|_M = sqrt(e^T M e), M the full
   projected mass matrix (the L2(Omega) norm of the coarse function) */
enum {
    PE_NORM_M_ABS = 0, /* stop when max_n |x_n^k - x_n^{k-1}|_M <= tol */
    PE_NORM_M_REL = 1  /* ... <= tol * max_n |x_n^0|_M (x^0 = initial coarse sweep) */
};

/*
 * pe_problem_create - set up the operators of one multiscale problem
 * (Algorithm 1 "Require": the coarse matrices of eq. (3.8)).
 *   d1, d2      dimensions of V_H1 and V_H2 (d1 >= 1, d2 >= 0).
 *   M11 (d1 x d1), M12 (d1 x d2, NULL means zero), M22 (d2 x d2),
 *   A11 (d1 x d1), A12 (d1 x d2), A21 (d2 x d1, NULL means A12^T),
 *   A22 (d2 x d2): device pointers to the projected mass and stiffness
 *               blocks. M11, M22, A11, A22 must be symmetric and A21 = A12^T
 *               (relative tolerance 1e-12), else PE_ERR_ARG.
 *   dt_coarse   coarse step Delta t = T/N (> 0).
 *   dt_fine     fine step delta t; P = dt_coarse/dt_fine must be an integer
 *               within 1e-12 relative, else PE_ERR_ARG.
 *   N           number of coarse intervals (>= 1).
 *   precision   PE_FP64, PE_MIXED or PE_MIXED_REFINE.
 *   hip_stream  hipStream_t for all work of this handle. NULL: the handle
 *               creates and owns a non-blocking stream (the caller then
 *               orders its own producers/consumers by the blocking calls).
 * On the GPU: FP64 Cholesky factorisations of M11/dt_fine + A11,
 * M11/dt_coarse + A11 and M22 (PE_ERR_NOT_SPD names the block and pivot),
 * the inverses formed from the factors, and the step operators.
 * On success *out owns all device memory it needs until pe_problem_destroy.
 */
pe_status pe_problem_create(pe_problem* out, int d1, int d2,
                            const double* M11, const double* M12, const double* M22,
                            const double* A11, const double* A12, const double* A21,
                            const double* A22, double dt_coarse, double dt_fine, int N,
                            int precision, void* hip_stream);

/*
 * pe_source_set - source term f(x, t) = sum_r g_r(x) h_r(t) in projected
 * form (F_i^n of eq. (3.8)), taken at the new time level of every step.
 *   B           number of samples (independent right-hand sides, >= 1).
 *   R           number of spatial modes (>= 0; 0 means f = 0).
 *   G           device, D x R: column r = [Psi1^T b_r; Psi2^T b_r].
 *   H           device, B x R x T_len amplitudes, T_len = N*P for PE_T_FINE
 *               (requires R <= 64) and N for PE_T_INTERVAL.
 * The coarse step of interval n uses the amplitude at t_{n+1}
 * (PE_T_FINE: index n*P + P - 1; PE_T_INTERVAL: index n).
 */
pe_status pe_source_set(pe_problem p, int B, int R, const double* G, const double* H,
                        int time_mode);

/*
 * pe_solve - parareal (Algorithm 1) for B samples that share the problem.
 *   B           must equal the B of the last pe_source_set (or any B >= 1
 *               when no source was set: f = 0).
 *   x0          device, B x D initial states (x_0^k = x0 for every k).
 *   tol, norm_mode   stopping test (see PE_NORM_*); tol >= 0.
 *   k_max       maximum number of parareal iterations, 0 <= k_max <= N
 *               (k_max = N reproduces the sequential fine solution).
 *   X           device, B x (N+1) x D output: the last iterate of each
 *               sample (samples stop updating once their own test holds).
 *   iters       host, B ints (nullable): iterations taken per sample.
 *   jump_hist   host, B x k_max doubles (nullable): max_n |x_n^k - x_n^{k-1}|_M
 *               for k = 1..k_max (unused entries 0).
 * Blocks until done; one scalar read-back per iteration. After the first
 * call for a given B, each sweep (fine sweep, coarse sweep + stopping-test
 * products) is replayed from a captured HIP graph (PE_GRAPHS=0 in the
 * environment at problem creation keeps every launch eager). With B = 1, a
 * fresh history and N >= 4 the coarse sweeps run as doubling scans over the
 * intervals (ceil(log2 N) products with powers of the coarse step matrix,
 * formed at the first such call; PE_COARSE_SCAN=0 at problem creation keeps
 * the sequential sweeps); the results agree with the sequential sweeps up
 * to rounding order.
 * Returns PE_WARN_NOT_CONVERGED if some sample did not meet the test.
 */
pe_status pe_solve(pe_problem p, int B, const double* x0, double tol, int norm_mode,
                   int k_max, double* X, int* iters, double* jump_hist);

/*
 * pe_fine_propagate - the fine propagator F of Algorithm 1 (its parallel
 * step) applied to B*N states at once: Y[b][n] = F(Xin[b][n]) over interval
 * n with the source of sample b.
 *   Xin, Y      device, B x N x D (may not alias).
 */
pe_status pe_fine_propagate(pe_problem p, int B, const double* Xin, double* Y);

/*
 * pe_coarse_propagate - the coarse propagator G (one step of dt_coarse)
 * applied to B*N states at once: Y[b][n] = G(Xin[b][n]) over interval n.
 *   Xin, Y      device, B x N x D (may not alias).
 */
pe_status pe_coarse_propagate(pe_problem p, int B, const double* Xin, double* Y);

/*
 * pe_coarse_propagate_noalloc - pe_coarse_propagate for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same G with the same kernels and
 * results, but its workspace (packed input, residual, increment, split-K
 * planes) is a 64 MiB array in the library's device memory, one per GPU,
 * held until the process ends. No hipMalloc, hipFree or allocating library
 * routine is called.
 *   Xin, Y      device, B x N x D (may not alias), as pe_coarse_propagate.
 * Limit: 3 * B * N * D_pad * 8 bytes <= 64 MiB (D_pad = D rounded up to
 * whole multiples of 8 per block), else PE_ERR_ARG naming the size.
 * The handle's device must be current (PE_ERR_ARG otherwise); restarting
 * history only (PE_ERR_STATE otherwise). Every call on a GPU shares that
 * GPU's array: calls that overlap in time on one GPU (other streams, other
 * threads) race and must be ordered by the caller.
 */
pe_status pe_coarse_propagate_noalloc(pe_problem p, int B, const double* Xin, double* Y);

/*
 * pe_mass_norms - |x|_M for `count` states (the norm of eq. (2.8)).
 *   X           device, count x D;  out  host, count doubles.
 */
pe_status pe_mass_norms(pe_problem p, int count, const double* X, double* out);

/*
 * pe_adjoint - gradients of a loss L of the sequential fine solution (the
 * limit of parareal, eq. (2.7)) with respect to the initial states and the
 * source amplitudes. The transposed splitting scheme of eqs. (2.4)-(2.5) is
 * run backward in time, itself parallel across the intervals by parareal:
 *     lambda_N = Xbar_N,
 *     lambda_n^k = Xbar_n + F_n^T lambda_{n+1}^{k-1}
 *                  + Phi_G^T (lambda_{n+1}^k - lambda_{n+1}^{k-1}),
 * with F_n^T the transposed fine propagator (every fine step transposed,
 * forward states never needed: the scheme is linear) and Phi_G the linear
 * part of the coarse step G. lambda_n is the adjoint of the state X_n.
 *   B           samples (the B of the last pe_source_set when a source is set).
 *   Xbar        device, B x (N+1) x D: dL/dX_n at the coarse boundaries
 *               (nullable: zero).
 *   beta        >= 0: weight of a fine-step tracking term
 *                   1/2 beta sum_{m=1}^{N*P} dt_fine |y_m|_M^2
 *               in L, where y is a trajectory of the scheme given by its
 *               coarse-boundary states Ybnd and source amplitudes dH; its
 *               fine levels are recomputed inside each interval from Ybnd
 *               (for the tracking error x - x_ref of two solves of the same
 *               problem, Ybnd = X - X_ref and dH = H - H_ref). 0: no term.
 *   Ybnd        device, B x (N+1) x D (required when beta > 0, else unused).
 *   dH          device, B x R x T_len in the layout of pe_source_set
 *               (nullable: y has no source).
 *   tol, k_max  stop when max_{n<N} |lambda_n^k - lambda_n^{k-1}|_2 <=
 *               tol * max_n |lambda_n^0|_2 (Euclidean: lambda is a dual
 *               vector), or after k_max <= N iterations (k_max = N gives the
 *               exact transposed sequential solution).
 *   x0bar       device, B x D out: dL/dx0 = lambda_0.
 *   Hbar        device, B x R x T_len out (nullable): dL/dH for the
 *               handle's G and time layout.
 *   Lam         device, B x (N+1) x D out (nullable): lambda_n.
 *   iters, jump_hist   host, as in pe_solve (nullable).
 * Works independently of pe_solve (the loss's dependence on the forward
 * solution enters only through Xbar and Ybnd). Returns
 * PE_WARN_NOT_CONVERGED if some sample did not meet the test.
 */
pe_status pe_adjoint(pe_problem p, int B, const double* Xbar, double beta, const double* Ybnd,
                     const double* dH, double tol, int k_max, double* x0bar, double* Hbar,
                     double* Lam, int* iters, double* jump_hist);

/*
 * pe_tracking - the fine-step tracking term of pe_adjoint,
 *     J_b = 1/2 beta sum_{m=1}^{N*P} dt_fine |y_m|_M^2,
 * for the trajectory y with coarse-boundary states Ybnd (device,
 * B x (N+1) x D) and source amplitudes dH (device, nullable), every fine
 * level recomputed by the fine propagator. J: host, B doubles.
 */
pe_status pe_tracking(pe_problem p, int B, const double* Ybnd, const double* dH, double beta, double* J);

/*
 * pe_fine_wr - the fine propagator computed by the paper's waveform
 * relaxation with the alpha-circulant diagonalisation in time (Sections 4.1
 * and 4.2), FP64 in the caller's coordinates whatever the handle's precision.
 * On every interval n of every sample b, from the start state x_n, K0
 * iterations of:
 *   (1) the V_H1 part at all P fine levels at once: the all-at-once system
 *       of eq. (4.12) with the alpha-circulant matrix of eq. (4.4), whose
 *       right-hand side (eq. (4.8)) uses the previous iterate's V_H2 part,
 *       solved by the diagonalisation of eqs. (4.5)-(4.7): a scaled discrete
 *       Fourier transform along time, one (d_k M11 + A11) solve per
 *       frequency, the inverse transform;
 *   (2) the V_H2 part sequentially in time (eq. (4.9)) with the new V_H1
 *       levels.
 * The history is reset at the interval start (as for the propagators of
 * pe_solve) and the first iterate continues the start state in time. The
 * iteration's fixed point is pe_fine_propagate's F (P steps of
 * eqs. (2.4)-(2.5)); the error contracts by about gamma^2 per iteration
 * (gamma of eq. (4.15)), and a smaller alpha converges faster but scales
 * rounding errors by about 1/alpha.
 *   B        samples (must equal the source's sample count when a source is set).
 *   Xin      device, B x N x D: row b*N + n is the start state of interval n
 *            of sample b (the layout of pe_fine_propagate).
 *   alpha    in (0, 1).
 *   K0       iterations, >= 0 (0 returns the start states).
 *   Fout     device, B x N x D out: the end state of interval n after K0
 *            iterations in row b*N + n.
 * Operators (one complex-shifted inverse per frequency, P/2 + 1 of them,
 * built by two Cholesky factorisations each) are built at the first call for
 * an alpha and kept until the next alpha or source. Needs P <= 128.
 * Errors: PE_ERR_ARG for bad arguments, PE_ERR_NOMEM, PE_ERR_NOT_SPD (only
 * for a mass or stiffness block that is not positive definite), PE_ERR_HIP.
 */
pe_status pe_fine_wr(pe_problem p, int B, const double* Xin, double alpha, int K0, double* Fout);

/*
 * pe_set_fine_solver - the fine propagator F that pe_solve uses in the
 * parareal update (eq. (2.7)):
 *   PE_FINE_STEP (default): P steps of eqs. (2.4)-(2.5);
 *   PE_FINE_WR: K0 >= 1 iterations of waveform relaxation with alpha in
 *     (0, 1), exactly as pe_fine_wr (Algorithm 1 with the paper's fine
 *     solver, Section 4.3). PE_FP64 handles only; parareal then converges
 *     to the sequential composition of this F.
 * pe_fine_propagate, pe_adjoint and pe_tracking always use P steps of the
 * scheme. Errors: PE_ERR_ARG.
 */
enum { PE_FINE_STEP = 0, PE_FINE_WR = 1 };
pe_status pe_set_fine_solver(pe_problem p, int kind, double alpha, int K0);

/*
 * pe_set_history - what the two-step scheme (2.4)-(2.5) uses as the previous
 * level at the start of each propagator call (the paper passes only the
 * state between the intervals of Algorithm 1 and leaves this open):
 *   PE_HIST_RESTART (default): a fresh history, u_{-1} = u_0, w_{-1} = w_0 at
 *     every interval start (the coupling differences vanish on the first
 *     step); states are x = [u; w] of D entries.
 *   PE_HIST_CARRY: the history travels with the state. Every state of the
 *     iteration is [x; delta] (2D entries), delta = x - x_prev the change
 *     over the last fine step of size dt_fine. F starts its first step from
 *     x_prev = x - delta and returns [x_P; x_P - x_{P-1}]; the coarse step G
 *     stays the one-step propagator with a fresh history (it reads x only)
 *     and returns [x'; (x' - x)/P], its change at the fine-step rate. The
 *     parareal limit is then one uninterrupted run of N*P fine steps from x0
 *     (delta = 0 at t = 0). The carried change couples the intervals through
 *     a slowly decaying mode of the two-step scheme that G cannot represent:
 *     parareal contracts more slowly than with PE_HIST_RESTART (finite
 *     termination at k = N still holds).
 * With PE_HIST_CARRY: pe_solve takes x0 as B x D and writes X as
 * B x (N+1) x 2D ([x_n; delta_n] per row; its stopping test measures the
 * change of x only, as eq. (2.8)); pe_fine_propagate and pe_coarse_propagate
 * take and return B x N x 2D. pe_adjoint, pe_tracking, pe_fine_wr, the
 * waveform-relaxation fine solver and batches return PE_ERR_STATE.
 * Changing the mode releases the iteration workspace (regrown at the next
 * call). Errors: PE_ERR_ARG (unknown mode), PE_ERR_STATE (waveform-relaxation
 * fine solver selected).
 */
enum { PE_HIST_RESTART = 0, PE_HIST_CARRY = 1 };
pe_status pe_set_history(pe_problem p, int mode);

/*
 * pe_probe_peaks - measured peaks of the part the library runs on, for the
 * rooflines the benchmark reports: out3[0] FP32 and out3[1] FP64 matrix-core
 * throughput (TFLOP/s; 2048 work-groups of 4 waves, each wave 16 independent
 * chains of 16x16x4 products with register operands, 2000 rounds) and
 * out3[2] HBM bandwidth (TB/s; read + write bytes of a 512 MiB device copy
 * with 16-byte vectors). Best of three timed runs after a warm-up, HIP events
 * on hip_stream (NULL: the default stream). Allocates ~1 GiB of device memory
 * for the call. Errors: PE_ERR_ARG, PE_ERR_NOMEM, PE_ERR_HIP.
 */
pe_status pe_probe_peaks(void* hip_stream, double* out3);

/*
 * pe_local_spectral - the local spectral problems of eq. (3.1) on the GPU:
 * on every coarse element A_e psi = lambda S_e psi over the element's nodes
 * not on the domain boundary (natural conditions on interior coarse edges),
 * A_e the kappa-weighted Q1 stiffness and S_e the (kappa H^-2)-weighted Q1
 * mass over the element's cells (same medium and grids as pe_cem_spaces,
 * m = n/n_c cells per element side, (m+1)^2 <= 128). Outputs, per element
 * e, its J smallest eigenvalues lam (n_c^2 x J, ascending), the
 * S_e-orthonormal eigenvectors psi (nullable; n_c^2 x (m+1)^2 x J on the
 * local nodes, row-major, zero on the domain boundary) and spsi = S_e psi
 * over all local nodes (the constraint data pe_cem_spaces takes). An
 * eigenvector is fixed up to sign: each is signed so that sum_f (f+1) psi_f
 * > 0 over the free nodes f in local order; within an eigenvalue of
 * multiplicity > 1 the vectors are one orthonormal basis of the eigenspace
 * (the one the rotations reach). Dense per element: Cholesky of S_e, cyclic
 * Jacobi on L^-1 A_e L^-T (sweeps down to the rounding floor: once the
 * off-diagonal Frobenius norm is below 1e-10 of the diagonal's, until a sweep
 * no longer halves it; at most 30, or PE_SPECTRAL_SWEEPS from the
 * environment). All pointers are device
 * memory; work on hip_stream, returns when done. Allocates 256 KiB per
 * element for the call. Errors: PE_ERR_ARG, PE_ERR_NOT_SPD (an element's
 * weighted mass), PE_ERR_NUMERIC (an element's sweeps stopped at the cap with
 * the off-diagonal norm above 1e-10 of the diagonal's; the message names the
 * element), PE_ERR_NOMEM, PE_ERR_HIP.
 */
pe_status pe_local_spectral(int n, int n_c, int J, const double* kappa, double* lam, double* psi, double* spsi,
                            void* hip_stream);

/*
 * pe_cem_spaces - the set-up pipeline on the GPU: CEM-GMsFEM basis
 * functions (Section 3.1, eq. (3.2)) and the Galerkin blocks of eq. (3.8).
 * Medium: Q1 elements on the unit square with n x n cells of side 1/n,
 * zero boundary values, kappa one value per cell (row-major, cell (cy, cx)
 * at cy*n + cx). Coarse grid: n_c x n_c elements of m = n/n_c cells per
 * side; the oversampled patch of element i is the element plus `layers`
 * coarse layers, clipped to the domain. For every element i and j < J the
 * basis function phi_j^(i) minimises a(phi, phi) over functions vanishing
 * outside the patch's interior nodes, subject to s(phi, psi_l^(k)) =
 * delta_{(k,l),(i,j)} for the J auxiliary functions of every element k of
 * the patch (eq. (3.2)); the constraint data are spsi = S_k psi_l^(k), the
 * local spectral eigenvectors of eq. (3.1) multiplied by the element's
 * kappa H^-2-weighted mass, given per element on its (m+1)^2 local nodes
 * (row-major) as n_c^2 x (m+1)^2 x J. Functions j < J1 of every element
 * span V_H1 (d1 = n_c^2 J1, ordered element-major), j >= J1 span V_H2
 * (d2 = n_c^2 (J - J1)); each is scaled to unit L2 norm.
 * Outputs (caller-allocated, row-major): M11 (d1 x d1), M12 (d1 x d2),
 * M22, A11, A12, A22 (the mass and kappa-weighted stiffness Gram blocks,
 * the diagonal blocks symmetrised); with R > 0 the source factors
 * G = [Psi1^T b; Psi2^T b] (D x R) of the fine-grid load vectors loads
 * (R x (n-1)^2, one per interior node, row-major); Psi (nullable) the
 * normalised basis, D x (n-1)^2 (one function per row, V_H1 first).
 * All pointers are device memory; inputs are borrowed for the call. Work is
 * ordered on hip_stream and the call returns after it finished. Allocates
 * its workspace for the call (about 3 D (n-1)^2 doubles, plus about 450 K
 * doubles per patch at 49 x 49 patch nodes).
 * Limits: J <= 8, at most 128 constraints per patch, at most 62 interior
 * nodes along a patch row. Errors: PE_ERR_ARG, PE_ERR_NOT_SPD (a patch
 * stiffness or constraint Gram matrix without a positive pivot, the patch
 * named in the message), PE_ERR_NOMEM, PE_ERR_HIP.
 */
pe_status pe_cem_spaces(int n, int n_c, int layers, int J, int J1, const double* kappa, const double* spsi,
                        int R, const double* loads, double* M11, double* M12, double* M22, double* A11,
                        double* A12, double* A22, double* G, double* Psi, void* hip_stream);

/*
 * pe_nlmc_spaces - the set-up pipeline for the NLMC spaces of Section 3.2
 * (eqs. (3.4)-(3.6)), split by continuum: every coarse element k has
 * counts[k] regions, its matrix region (slot 0) and its fracture pieces
 * (slots 1..counts[k]-1); the basis function of region (k, l) minimises
 * a(psi, psi) over functions vanishing outside the oversampled patch's
 * interior nodes subject to int_r psi = delta_{r,(k,l)} for every region r
 * of every element of the patch (eq. (3.6)). The constraint data rdata
 * (device, n_c^2 x (m+1)^2 x J, as pe_cem_spaces' spsi) hold, for region
 * slot l of element k on its local node (row-major), the region's integral
 * of the Q1 function of that node: h^2/4 for every region cell the node is
 * a corner of; slots at or beyond counts[k] are not read. counts: host
 * array of n_c^2 entries, 1 <= counts[k] <= J <= 8. V_H1 = the fracture
 * functions (d1 = sum_k (counts[k] - 1), element-major), V_H2 = the matrix
 * functions (d2 = n_c^2, element-major); each scaled to unit L2 norm. The
 * medium, grids, outputs, workspace, limits and errors are those of
 * pe_cem_spaces (the constraint limit counts regions); no fracture function
 * at all is PE_ERR_ARG. The paper's own V_H2 (with the mean function psi_bar
 * of eq. (3.7) and the s-orthogonalised fracture functions) is not built here.
 */
pe_status pe_nlmc_spaces(int n, int n_c, int layers, int J, const int* counts, const double* kappa,
                         const double* rdata, int R, const double* loads, double* M11, double* M12, double* M22,
                         double* A11, double* A12, double* A22, double* G, double* Psi, void* hip_stream);

/*
 * Batches of different problems (different d1, d2, N, sources and sample
 * counts; same precision and step ratio P), solved together: every
 * product of a fine step runs as one grouped MFMA launch over all problems'
 * interval columns, every coarse step n as one grouped launch over the
 * problems with N > n, and each sweep is replayed from a captured HIP graph
 * after its first visits. Each problem keeps its own stopping test
 * (eq. (2.8)) and iteration count; finished samples are frozen.
 *
 * pe_batch_create - borrow `count` problem handles (they must outlive the
 *   batch and keep their sources; a later pe_source_set or a pe_solve with
 *   more samples is picked up at the next pe_batch_solve). hip_stream: the
 *   stream for all batch work (NULL: the batch creates its own).
 *   Launch options read from the environment at creation: PE_BATCH_TILE=
 *   "br bs bk2" the grouped products' tile (32 64, 64 64 (default), 64 128
 *   or 128 64; bk2 = 1 twice the K depth); PE_BATCH_XCD the work-group order
 *   (2, the default: the row tiles of each operator column tile on one XCD;
 *   1 or 3: every tile of a product on one XCD; 0: plain); PE_BATCH_SCAN=0
 *   keeps the sequential coarse sweeps of the mixed path (the default runs
 *   the initial sweep and the corrections as doubling scans). Results are
 *   bitwise reproducible for a fixed tile; the work-group order does not
 *   change them.
 * pe_batch_solve - Algorithm 1 for every problem of the batch.
 *   x0          host array of `count` device pointers, x0[i]: B_i x D_i
 *               (B_i the sample count of problem i's source, 1 without one).
 *   tol, norm_mode   as in pe_solve, per sample.
 *   k_max       maximum iterations (each problem also stops at its own N).
 *   X           host array of `count` device pointers, X[i]: B_i x (N_i+1) x D_i.
 *   iters       host, sum_i B_i ints (problem-major, nullable).
 *   Returns PE_WARN_NOT_CONVERGED if some sample did not meet its test.
 * pe_batch_destroy - release the batch (not the problems).
 */
typedef struct pe_batch_s* pe_batch;
pe_status pe_batch_create(pe_batch* out, int count, const pe_problem* problems, void* hip_stream);
pe_status pe_batch_solve(pe_batch b, const double* const* x0, double tol, int norm_mode, int k_max,
                         double* const* X, int* iters);
pe_status pe_batch_destroy(pe_batch b);

/* pe_batch_profile / pe_batch_profile_read - launch timing of a batch's
   grouped launches by class (PE_PROF_*), as pe_profile / pe_profile_read:
   HIP event pairs on the batch's stream; sweeps run eagerly while enabled. */
pe_status pe_batch_profile(pe_batch b, int enable);
pe_status pe_batch_profile_read(pe_batch b, int kind, double* total_ms, long long* launches);

/* launch classes timed by pe_profile */
enum {
    PE_PROF_FINE_STEP = 0,      /* fine step (steps 2..P): the increment
                                   Z F - (Z A) x_a - (Z W) dev as one product,
                                   with the state/history update fused        */
    PE_PROF_FINE_FIRST = 1,     /* fine step 1 (zero deviation: source and anchor) */
    PE_PROF_ANCHOR = 2,         /* fine sweep anchors: Z A x_a and coordinate changes */
    PE_PROF_COARSE = 3,         /* coarse step + parareal correction              */
    PE_PROF_NORM = 4,           /* mass products of the stopping test             */
    PE_PROF_SPLITK_REDUCE = 5,  /* split-K reduction + epilogue kernels of the above */
    PE_PROF_ADJ_STEP = 6,       /* transposed fine step: [a; nu] <- a - ([A; A + Mh] Z^T) nu
                                   as one product                                 */
    PE_PROF_FINE_SWEEP = 7,     /* persistent fine sweep: all P fused steps of a sweep
                                   in one cooperative launch with grid barriers
                                   between them; used when PE_PERSISTENT=1 is in the
                                   environment at problem creation and the N*B
                                   interval columns fit one 64-row tile (by default
                                   each step is its own launch, replayed from a graph) */
    PE_PROF_WR_RHS = 8,         /* waveform relaxation: the right-hand-side products
                                   of eqs. (4.8) and (4.9) over all fine levels  */
    PE_PROF_WR_SOLVE = 9,       /* waveform relaxation: one complex-shifted solve
                                   (d_k M11 + A11)^-1 per frequency, as a product
                                   with its real 2 d1 x 2 d1 form                */
    PE_PROF_WR_WSTEP = 10,      /* waveform relaxation: one sequential V_H2 step   */
    PE_PROF_REFINE = 11,        /* PE_MIXED_REFINE: the FP64 residual product and the
                                   FP32 correction product of a fine step        */
    PE_PROF_KINDS = 12
};

/*
 * pe_profile - enable (1) or disable (0) launch timing and reset the totals.
 * When enabled, every launch of the classes above is bracketed by a pair of
 * HIP events recorded on the handle's stream (GPU time from the start to
 * the end of that launch); a product that splits K launches a second,
 * reduction kernel, which is bracketed separately (PE_PROF_SPLITK_REDUCE).
 * Sweeps then run with eager launches (no graph replay).
 */
pe_status pe_profile(pe_problem p, int enable);

/*
 * pe_profile_read - accumulated GPU milliseconds and number of launches of
 * class `kind` since the last pe_profile call (host out-pointers, nullable).
 * Synchronises the handle's stream.
 */
pe_status pe_profile_read(pe_problem p, int kind, double* total_ms, long long* launches);

/*
 * pe_autotune - choose the tile configuration (tile shape, K depth per LDS
 * stage, split-K) of each product of the fine sweep and of the stopping test
 * for B samples, by timing candidates on this problem's operands; the
 * choices are kept in the handle (and appended to the file named by the
 * environment variable PE_TUNE_CACHE, which later handles read back). The
 * same happens lazily at the first use of a shape unless PE_AUTOTUNE=0.
 * Shapes listed in the read-only file named by PE_TUNE_DB (a database of
 * configurations measured on MI355X) are not re-tuned. PE_FORCE_WSK=
 * "bs,waves,splitk" at problem creation runs every product of at most 64
 * state columns on the wave-split-K kernel with that configuration (for
 * tests; operator tiles of 16 or 32 rows, 4 or 8 waves). PE_FORCE_TILES=
 * "br,bs,bk2,splitk" at problem creation runs every product of more than 4
 * state columns with that tile configuration (for tests: tile shapes 32x64,
 * 64x32, 64x64, 64x128, 128x64, 128x128, K depth flag 0/1, 1..64 splits).
 * Results are bitwise reproducible for fixed configurations.
 */
pe_status pe_autotune(pe_problem p, int B);

/*
 * pe_last_tiles - tile configuration of the last product launched in class
 * `kind` (PE_PROF_*): tiles4 = {rows of the state tile, rows of the operator
 * tile, K depth per LDS stage, split-K count}; all 0 for the GEMV kernel or
 * if the class has not run. For the wave-split-K kernel (every wave of a
 * work-group takes its own slice of K, no LDS staging) tiles4[2] is minus
 * the number of waves per work-group. tiles4: host, 4 ints.
 */
pe_status pe_last_tiles(pe_problem p, int kind, int* tiles4);

/* pe_problem_info - d1, d2, N, P (host ints, each nullable). */
pe_status pe_problem_info(pe_problem p, int* d1, int* d2, int* N, int* P);

/* pe_problem_destroy - release all device memory of the handle (NULL ok). */
pe_status pe_problem_destroy(pe_problem p);

/* message of the calling thread's last failing call ("" if none) */
const char* pe_last_error(void);

/* library version as an integer (major*10000 + minor*100 + patch) */
int pe_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PE_H */
