"""Pins of the waveform-relaxation oracle (Sections 4.1-4.2): the
alpha-circulant eigenvalues against a general eigensolver, the diagonalised
all-at-once solve against the dense Kronecker system, the fixed point against
the sequential fine propagator, finite termination of the alpha = 0
iteration, the d2 = 0 closed-form recursion, the convergence factor of the
theorem of Section 4.2, affinity, and parareal with the WR fine solver
(finite termination at the WR composition; the plain parareal iterates once
WR has converged)."""
import numpy as np
import pytest

import oracle.scheme as S
import oracle.wr as WR
from problem import build_problem


@pytest.fixture(scope="module")
def c0():
    p = build_problem("c0")
    return S.Blocks.from_problem(p), S.Source.from_problem(p)


@pytest.mark.parametrize("P,alpha", [(8, 0.1), (16, 0.01), (5, 0.3), (64, 1e-3)])
def test_circulant_eigenvalues(P, alpha):
    # eq. (4.5): every eigenvalue of B (general eigensolver) has a closed-form
    # partner d_k, and vice versa
    h = 0.01
    ev = np.linalg.eigvals(WR.circulant_matrix(P, alpha, h))
    d = WR.circulant_eigs(P, alpha, h)
    scale = np.max(np.abs(d))
    assert max(np.min(np.abs(ev - x)) for x in d) < 1e-9 * scale
    assert max(np.min(np.abs(d - x)) for x in ev) < 1e-9 * scale


@pytest.mark.parametrize("alpha", [0.5, 0.05, 1e-3, 0.0])
def test_all_at_once_solve_matches_kronecker(c0, alpha):
    # eqs. (4.6)-(4.7) and (4.12)-(4.13): the diagonalised solve equals a dense
    # solve of (B (x) M11 + I (x) A11) U = R
    bl, _ = c0
    P, d1 = 6, bl.d1
    R = np.random.default_rng(1).standard_normal((P, d1, 3))
    h = bl.dt_fine
    if alpha == 0.0:
        U = WR.sequential_solve(bl.M11, bl.A11, R, h)
    else:
        U = WR.all_at_once_solve(bl.M11, bl.A11, R, alpha, h)
    K = np.kron(WR.circulant_matrix(P, alpha, h), bl.M11) + np.kron(np.eye(P), bl.A11)
    Uk = np.linalg.solve(K, R.reshape(P * d1, 3)).reshape(P, d1, 3)
    assert np.max(np.abs(U - Uk)) <= 1e-12 * np.max(np.abs(Uk)) / max(alpha, 1e-2)


@pytest.mark.parametrize("alpha", [0.0, 1e-3, 1e-2])
def test_fixed_point_is_the_fine_propagator(c0, alpha):
    # the WR fixed point solves eqs. (4.8)-(4.9) with equal iterates, i.e. the
    # sequential scheme (2.4)-(2.5): F
    bl, src = c0
    X = np.random.default_rng(2).standard_normal((bl.D, 4))
    ns, bs = [0, 3, 5, 7], [0] * 4
    ref = S.fine_propagator_cols(bl, src, X, ns, bs)
    got = WR.wr_fine_cols(bl, src, X, ns, bs, alpha, 40)
    assert np.linalg.norm(got - ref) <= 1e-12 / max(alpha, 1e-2) * np.linalg.norm(ref)


def test_alpha_zero_terminates_after_P_iterations(c0):
    # with alpha = 0 the u-part at level s uses w up to level s-1 of the
    # previous iterate, so after iteration j every level <= j is exact: the
    # iterate equals F after at most P iterations, and not after one
    bl, src = c0
    X = np.random.default_rng(3).standard_normal((bl.D, 3))
    ns, bs = [1, 4, 6], [0] * 3
    ref = S.fine_propagator_cols(bl, src, X, ns, bs)
    _, ends = WR.wr_fine_cols(bl, src, X, ns, bs, 0.0, bl.P, history=True)
    rel = [np.linalg.norm(e - ref) / np.linalg.norm(ref) for e in ends]
    assert rel[-1] < 1e-13
    assert rel[0] > 1e-6


@pytest.mark.parametrize("alpha", [0.3, 0.05])
def test_d2_zero_closed_form_alpha_recursion(c0, alpha):
    # with no V_H2 part one WR iteration is backward Euler from the start
    # u_0 + alpha (u_P^j - u_P^{j-1}); the end-state error e_j = u_P^j - u*
    # obeys e_j = alpha Phi (e_j - e_{j-1}), Phi = ((M11/h + A11)^-1 M11/h)^P,
    # e_0 = u_0 - u*
    bl, src = c0
    d1 = bl.d1
    z = np.zeros((d1, 0))
    bl0 = S.Blocks(bl.M11, z, np.zeros((0, 0)), bl.A11, z, np.zeros((0, 0)), bl.dt, bl.dt_fine, bl.N)
    src0 = S.Source(src.G[:d1] if src.G is not None else None, src.H, src.mode, src.N, src.P)
    x = np.random.default_rng(4).standard_normal(d1)
    ust = S.fine_propagator(bl0, src0, x, 2)
    h = bl.dt_fine
    Phi = np.linalg.matrix_power(np.linalg.solve(bl.M11 / h + bl.A11, bl.M11 / h), bl.P)
    _, ends = WR.wr_fine_cols(bl0, src0, x[:, None], [2], [0], alpha, 5, history=True)
    e = x - ust
    for end in ends:
        e = np.linalg.solve(np.eye(d1) - alpha * Phi, -alpha * Phi @ e)
        assert np.linalg.norm(end[:, 0] - ust - e) <= 1e-12 * np.linalg.norm(ust)


def test_contraction_within_theorem_bound(c0):
    # theorem of Section 4.2: the error contracts by gamma^2 per iteration
    # (gamma of eq. (4.15)); checked on the alpha = 0 iteration before it
    # terminates
    bl, src = c0
    g2 = WR.gamma_sq(bl)
    assert 0.0 < g2 < 1.0
    X = np.random.default_rng(5).standard_normal((bl.D, 2))
    ns, bs = [2, 5], [0, 0]
    ref = S.fine_propagator_cols(bl, src, X, ns, bs)
    _, ends = WR.wr_fine_cols(bl, src, X, ns, bs, 0.0, bl.P // 2, history=True)
    err = [np.linalg.norm(e - ref) for e in ends]
    for a, b in zip(err, err[1:]):
        assert b <= g2 * a


def test_affine_in_the_start_state(c0):
    bl, src = c0
    rng = np.random.default_rng(6)
    x, y = rng.standard_normal(bl.D), rng.standard_normal(bl.D)

    def f(v):
        return WR.wr_fine(bl, src, v, 3, 0.05, 4)

    lhs = f(x + y) - f(x) - f(y) + f(np.zeros(bl.D))
    assert np.linalg.norm(lhs) <= 1e-10 * np.linalg.norm(f(x))


def test_parareal_with_wr_terminates_at_the_wr_composition(c0):
    # parareal reproduces the sequential composition of the fine solver it
    # uses after N iterations (the first k intervals are exact after k
    # iterations), here with F = K0 WR iterations
    bl, src = c0
    x0 = np.random.default_rng(7).standard_normal(bl.D)
    r = WR.parareal_wr(bl, src, x0, 0.0, 0.05, 2, k_max=bl.N)
    ref = WR.wr_composition(bl, src, x0, 0.05, 2)
    assert r["K"] == bl.N
    assert np.linalg.norm(r["X"][-1] - ref) <= 1e-11 * np.linalg.norm(ref)
    # and after k iterations the first k+1 boundary states are exact
    k = 3
    assert np.linalg.norm(r["X"][k][:k + 1] - ref[:k + 1]) <= 1e-11 * np.linalg.norm(ref)


def test_parareal_with_converged_wr_is_plain_parareal(c0):
    bl, src = c0
    x0 = np.random.default_rng(8).standard_normal(bl.D)
    a = WR.parareal_wr(bl, src, x0, 0.0, 0.01, 40, k_max=3)
    b = S.parareal(bl, src, x0, 0.0, k_max=3)
    for Xa, Xb in zip(a["X"], b["X"]):
        assert np.linalg.norm(Xa - Xb) <= 1e-10 * np.linalg.norm(Xb)
