"""Pins for the FP64 oracle of the splitting scheme and parareal, against
facts fixed by the paper and by mathematics: exact scalar recursions,
brute-force fine-grid backward Euler, the Galerkin steady state, the
semi-discrete ODE limit, a space-time all-at-once solve of the same
equations, and the parareal exactness property (x_n^k = X*_n for n <= k).
A planted sign error in the oracle is caught (last test)."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle.scheme as S
from oracle.finebe import fine_backward_euler
from problem import build_problem, full_mass, full_stiffness
from problem.fem import FineGrid


def _blocks_from(M11, M12, M22, A11, A12, A22, dt, P, N=1):
    return S.Blocks(M11, M12, M22, A11, A12, A22, dt, dt / P, N)


def _moderate_problem():
    cfg = dict(n=20, n_c=2, layers=1, J1=2, J2=3, medium="channels", n_h=1, n_v=1,
               contrast=10.0, seed=21, source="one", u0="sine2", N=4, P=4, T=None, B=1)
    return build_problem(cfg)


def test_fine_be_sine_recursion():
    """kappa = 1, f = sin(pi x) sin(pi y) e^-t, u0 = 0: fine BE reduces to
    a_{m+1} = (a_m + dt e^{-t_{m+1}}) / (1 + dt lam_h) exactly."""
    n, dt, steps = 16, 1e-2, 25
    fine = FineGrid(np.ones((n, n)))
    s = fine.nodal(lambda x, y: np.sin(np.pi * x) * np.sin(np.pi * y))
    b = fine.load_smooth(lambda x, y: np.sin(np.pi * x) * np.sin(np.pi * y))
    U = fine_backward_euler(fine.M, fine.A, np.zeros(fine.n_dof), dt, steps,
                            lambda m: b * np.exp(-(m + 1) * dt))
    h = 1.0 / n
    lam = 12 * (1 - np.cos(np.pi * h)) / (h * h * (2 + np.cos(np.pi * h)))
    a = 0.0
    for m in range(steps):
        a = (a + dt * np.exp(-(m + 1) * dt)) / (1 + dt * lam)
        np.testing.assert_allclose(U[m + 1], a * s, rtol=0, atol=1e-13)
    # and the continuum limit a(t) = (e^-t - e^{-2 pi^2 t}) / (2 pi^2 - 1)
    t = steps * dt
    assert abs(a - (np.exp(-t) - np.exp(-2 * np.pi ** 2 * t)) / (2 * np.pi ** 2 - 1)) < 0.05 * a


def test_full_space_scheme_equals_fine_be():
    """V_H1 = whole Q1 space, V_H2 = {0}: the scheme is fine BE (O16)."""
    n, dt, P = 10, 5e-3, 7
    rng = np.random.default_rng(2)
    fine = FineGrid(np.exp(rng.standard_normal((n, n))))
    M, A = fine.M.toarray(), fine.A.toarray()
    z = np.zeros((fine.n_dof, 0))
    bl = S.Blocks(M, z, np.zeros((0, 0)), A, z, np.zeros((0, 0)), dt * P, dt, 1)
    b = fine.load_smooth(lambda x, y: x * (1 - x) * np.cos(3 * y))
    src = S.Source(b[:, None], np.cos(np.arange(P) * 0.3)[None, None, :], S.TIME_FINE, 1, P)
    u0 = rng.standard_normal(fine.n_dof)
    x = S.fine_propagator(bl, src, u0, 0)
    U = fine_backward_euler(fine.M, fine.A, u0, dt, P, lambda m: b * np.cos(m * 0.3))
    np.testing.assert_allclose(x, U[-1], rtol=1e-12, atol=1e-12 * np.abs(U[-1]).max())


def test_decoupled_eigenpair_recursions():
    """Psi1 = [sine(1,1)], Psi2 = [sine(2,1)] on kappa = 1: the blocks are
    diagonal (M12 = A12 = 0 up to roundoff) and the scheme splits into a
    scalar backward-Euler recursion for u and a scalar forward-Euler
    recursion for w."""
    n = 24
    fine = FineGrid(np.ones((n, n)))
    s1 = fine.nodal(lambda x, y: np.sin(np.pi * x) * np.sin(np.pi * y))
    s2 = fine.nodal(lambda x, y: np.sin(2 * np.pi * x) * np.sin(np.pi * y))
    P = np.stack([s1, s2], axis=1)
    M = P.T @ (fine.M @ P)
    A = P.T @ (fine.A @ P)
    assert abs(M[0, 1]) < 1e-14 * M[0, 0] and abs(A[0, 1]) < 1e-12 * A[0, 0]
    m1, m2, a1, a2 = M[0, 0], M[1, 1], A[0, 0], A[1, 1]
    h, steps = 1.0 / (3 * a2 / m2), 12   # explicit part stable: h a2/m2 = 1/3
    bl = _blocks_from(M[:1, :1], M[:1, 1:], M[1:, 1:], A[:1, :1], A[:1, 1:], A[1:, 1:], h * steps, steps)
    g = np.array([0.7, -0.4])
    src = S.Source(g[:, None], np.exp(-np.arange(steps) * h)[None, None, :] + 0.5, S.TIME_FINE, 1, steps)
    x0 = np.array([0.3, 1.1])
    x = S.fine_propagator(bl, src, x0, 0)
    u, w = x0
    for m in range(steps):
        f = np.exp(-m * h) + 0.5
        u = (m1 * u / h + g[0] * f) / (m1 / h + a1)
        w = w + h * (g[1] * f - a2 * w) / m2
    np.testing.assert_allclose(x, [u, w], rtol=1e-12)


def test_steady_state_is_galerkin_solution():
    """Time-constant source: the scheme's fixed point solves A x = F
    (both equations with the coupling differences gone)."""
    p = _moderate_problem()
    bl = S.Blocks.from_problem(p)
    F = p["G"][:, 0]
    Afull = full_stiffness(p)
    xs = np.linalg.solve(Afull, F)
    d1 = bl.d1
    u, w = p["x0"][0][:d1].copy(), p["x0"][0][d1:].copy()
    up, wp = u.copy(), w.copy()
    for _ in range(20000):
        un, wn = S.step(bl, bl.dt, u, w, up, wp, F)
        up, wp, u, w = u, w, un, wn
    x = np.concatenate([u, w])
    assert np.linalg.norm(x - xs) < 1e-9 * np.linalg.norm(xs)


def _ode_error(bl, F, x0, T, steps):
    """Error at time T of one run of the scheme (history kept across all
    steps) against the exact solution of M x' + A x = F."""
    M, A = bl.M, np.block([[bl.A11, bl.A12], [bl.A12.T, bl.A22]])
    xs = np.linalg.solve(A, F)
    xe = xs + sla.expm(-np.linalg.solve(M, A) * T) @ (x0 - xs)
    h = T / steps
    d1 = bl.d1
    u, w = x0[:d1].copy(), x0[d1:].copy()
    up, wp = u.copy(), w.copy()
    for _ in range(steps):
        un, wn = S.step(bl, h, u, w, up, wp, F)
        up, wp, u, w = u, w, un, wn
    return np.sqrt((np.concatenate([u, w]) - xe) @ M @ (np.concatenate([u, w]) - xe))


def test_first_order_convergence_to_semidiscrete_ode():
    """The scheme is a first-order discretisation of M x' + A x = F in V_H
    (full M including M12): halving the step halves the error."""
    p = _moderate_problem()
    bl = S.Blocks.from_problem(p)
    F = p["G"][:, 0]
    x0 = p["x0"][0]
    T = 200 * p["dt"]
    e = [_ode_error(bl, F, x0, T, s) for s in (400, 800, 1600)]
    r1, r2 = e[0] / e[1], e[1] / e[2]
    assert 1.8 < r1 < 2.2 and 1.8 < r2 < 2.2, (e, r1, r2)


def _all_at_once(bl, x0, F_of_m, h, steps):
    """Space-time solve of eqs. (2.4)-(2.5) for `steps` steps: one sparse
    linear system for all levels 1..steps, history at level -1 equal to
    level 0. Unknown ordering [u_1, w_1, u_2, w_2, ...]."""
    d1, d2, D = bl.d1, bl.d2, bl.D
    M11, M12, M22 = bl.M11, bl.M12, bl.M22
    A11, A12, A22 = bl.A11, bl.A12, bl.A22
    blocks = [[None] * steps for _ in range(steps)]
    rhs = np.zeros(steps * D)
    u0, w0 = x0[:d1], x0[d1:]
    for m in range(steps):     # equations producing level m+1
        Fm = F_of_m(m)
        # eq. (2.4): M11 (u_{m+1}-u_m)/h + M12 (w_m - w_{m-1})/h + A11 u_{m+1} + A12 w_m = F1
        # eq. (2.5): M22 (w_{m+1}-w_m)/h + M21 (u_m - u_{m-1})/h + A21 u_{m+1} + A22 w_m = F2
        diag = np.block([[M11 / h + A11, np.zeros((d1, d2))], [A12.T, M22 / h]])
        blocks[m][m] = sp.csr_matrix(diag)
        cur = np.block([[-M11 / h, M12 / h + A12], [M12.T / h, -M22 / h + A22]])   # level m
        prev = np.block([[np.zeros((d1, d1)), -M12 / h], [-M12.T / h, np.zeros((d2, d2))]])  # level m-1
        r = np.array(Fm, dtype=float)
        if m >= 1:
            blocks[m][m - 1] = sp.csr_matrix(cur)
        else:
            r -= cur @ x0
        if m >= 2:
            blocks[m][m - 2] = sp.csr_matrix(prev)
        else:
            r -= prev @ x0   # level m-1 is level 0 (m = 1) or the reset history (m = 0)
        rhs[m * D:(m + 1) * D] = r
    Z = sp.bmat(blocks, format="csc")
    return spla.spsolve(Z, rhs).reshape(steps, D)


def test_all_at_once_space_time_solve_equals_stepping():
    p = build_problem("t1")
    bl = S.Blocks.from_problem(p)
    src = S.Source.from_problem(p)
    x0 = p["x0"][0] + 0.01 * np.random.default_rng(3).standard_normal(bl.D)
    n = 2
    X = _all_at_once(bl, x0, lambda m: src.at_fine(0, n, m), bl.dt_fine, bl.P)
    x = S.fine_propagator(bl, src, x0, n)
    np.testing.assert_allclose(x, X[-1], rtol=0, atol=1e-10 * np.abs(X[-1]).max())


def test_fine_propagator_linear_and_affine():
    p = build_problem("t1")
    bl = S.Blocks.from_problem(p)
    zero = S.Source(None, None, S.TIME_FINE, bl.N, bl.P)
    rng = np.random.default_rng(4)
    x, y = rng.standard_normal(bl.D), rng.standard_normal(bl.D)
    Fx, Fy = S.fine_propagator(bl, zero, x, 0), S.fine_propagator(bl, zero, y, 0)
    Fxy = S.fine_propagator(bl, zero, 2.5 * x - 0.5 * y, 0)
    np.testing.assert_allclose(Fxy, 2.5 * Fx - 0.5 * Fy, rtol=1e-10, atol=1e-12 * np.abs(Fxy).max())
    # column form equals one-column form
    src = S.Source.from_problem(p)
    cols = S.fine_propagator_cols(bl, src, np.stack([x, y], 1), [1, 3], [0, 0])
    np.testing.assert_allclose(cols[:, 0], S.fine_propagator(bl, src, x, 1), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(cols[:, 1], S.fine_propagator(bl, src, y, 3), rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("name", ["t0", "t1", "c0"])
def test_parareal_exact_after_k_iterations(name):
    """x_n^k equals the sequential fine solution for n <= k, and x^N = X*
    (finite termination, Section 5.1)."""
    p = build_problem(name)
    bl = S.Blocks.from_problem(p)
    src = S.Source.from_problem(p)
    x0 = p["x0"][0]
    Xs = S.fine_composition(bl, src, x0)
    r = S.parareal(bl, src, x0, tol=0.0, k_max=bl.N)
    assert r["K"] == bl.N and len(r["X"]) == bl.N + 1
    scale = max(S.m_norm(bl, Xs[n]) for n in range(bl.N + 1))
    for k, X in enumerate(r["X"]):
        for n in range(min(k, bl.N) + 1):
            assert S.m_norm(bl, X[n] - Xs[n]) <= 1e-12 * scale, (k, n)
    # the error does not grow with k and is tiny at k = N
    errs = [S.rel_l2_M(bl, X, Xs) for X in r["X"]]
    assert errs[-1] < 1e-13
    assert errs[1] < errs[0]


def test_parareal_p1_converges_in_one_iteration():
    p = build_problem("t1")
    bl = S.Blocks(p["M11"], p["M12"], p["M22"], p["A11"], p["A12"], p["A22"], p["dt"], p["dt"], p["N"])
    src = S.Source(p["G"], p["H"][:, :, p["P"] - 1::p["P"]], S.TIME_INTERVAL, bl.N, 1)
    r = S.parareal(bl, src, p["x0"][0], tol=1e-13, rel=True)
    # F == G here, so the first correction only moves x by rounding
    assert r["K"] == 1 and r["J"][0] <= r["threshold"]


def test_parareal_jumps_decay_fast():
    p = build_problem("c0")
    bl = S.Blocks.from_problem(p)
    src = S.Source.from_problem(p)
    r = S.parareal(bl, src, p["x0"][0], tol=0.0, k_max=6)
    J = r["J"]
    ratios = J[1:] / J[:-1]
    assert np.all(ratios < 0.1)          # contraction well below the paper's R_p = -0.5 slope
    assert np.all(np.diff(np.log10(J)) < -1.0)


def test_mass_norm_is_fine_l2_norm():
    p = build_problem("t0", use_cache=False, keep_spaces=True)
    bl = S.Blocks.from_problem(p)
    rng = np.random.default_rng(5)
    e = rng.standard_normal(bl.D)
    u = p["Psi1"] @ e[:bl.d1] + p["Psi2"] @ e[bl.d1:]
    assert abs(S.m_norm(bl, e) - np.sqrt(u @ (p["fine"].M @ u))) < 1e-12 * S.m_norm(bl, e)


def test_planted_sign_error_is_caught(monkeypatch):
    """Flip the sign of the M12 coupling inside the oracle: the space-time
    pin and the ODE-limit pin both fail."""
    p = _moderate_problem()
    bl = S.Blocks.from_problem(p)
    F = p["G"][:, 0]
    good = _ode_error(bl, F, p["x0"][0], 200 * p["dt"], 800)
    orig = S.step

    def wrong_step(bl_, h, u, w, u_prev, w_prev, Fv):
        d1 = bl_.d1
        Fv = np.zeros((bl_.D,) + u.shape[1:]) if np.ndim(Fv) == 0 else np.asarray(Fv)
        rhs_u = bl_.M11 @ u / h + bl_.M12 @ (w - w_prev) / h - bl_.A12 @ w + Fv[:d1]
        u_new = sla.cho_solve(bl_.chol(h), rhs_u)
        rhs_w = bl_.M22 @ w - bl_.M12.T @ (u - u_prev) - h * (bl_.A12.T @ u_new) - h * (bl_.A22 @ w) + h * Fv[d1:]
        return u_new, sla.cho_solve(bl_._m22, rhs_w)

    monkeypatch.setattr(S, "step", wrong_step)
    bad = _ode_error(bl, F, p["x0"][0], 200 * p["dt"], 800)
    assert bad > 20 * good
    p1 = build_problem("t1")
    b1 = S.Blocks.from_problem(p1)
    s1 = S.Source.from_problem(p1)
    x0 = p1["x0"][0] + 0.01
    X = _all_at_once(b1, x0, lambda m: s1.at_fine(0, 0, m), b1.dt_fine, b1.P)
    x = S.fine_propagator(b1, s1, x0, 0)
    assert np.abs(x - X[-1]).max() > 1e-6 * np.abs(X[-1]).max()
    monkeypatch.setattr(S, "step", orig)
