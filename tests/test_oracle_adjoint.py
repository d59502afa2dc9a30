"""Pins for the oracle's discrete adjoint: the dot-product identity of the
linear map (x0, H) -> X, central finite differences of a quadratic loss
(exact up to rounding), and the transpose of a single fine propagator
against its explicitly formed matrix."""
import numpy as np
import pytest

import oracle.adjoint as ADJ
import oracle.scheme as S
from problem import build_problem


@pytest.mark.parametrize("name", ["t0", "t1", "t2"])
def test_dot_product_identity(name):
    p = build_problem(name)
    bl, src = S.Blocks.from_problem(p), S.Source.from_problem(p)
    rng = np.random.default_rng(11)
    x0 = rng.standard_normal(bl.D)
    H = rng.standard_normal(p["H"].shape[1:])
    Xbar = rng.standard_normal((bl.N + 1, bl.D))
    X = ADJ.forward_linear(bl, p["G"], p["time_mode"], x0, H)
    sbar = S.Source(p["G"], H[None], p["time_mode"], bl.N, bl.P)
    x0b, Hb, lam = ADJ.adjoint(bl, sbar, Xbar)
    lhs = np.sum(X * Xbar)
    rhs = np.sum(x0 * x0b) + np.sum(H * Hb)
    assert abs(lhs - rhs) <= 1e-11 * (np.abs(X * Xbar).sum() + np.abs(x0 * x0b).sum() + np.abs(H * Hb).sum())


def test_fine_propagator_transpose_matches_matrix():
    """F_hom as an explicit matrix (columns = F_hom of unit vectors) and its
    transpose applied to a vector equals the adjoint sweep."""
    p = build_problem("t0")
    bl = S.Blocks.from_problem(p)
    zero = S.Source(None, None, S.TIME_FINE, bl.N, bl.P)
    Phi = np.stack([S.fine_propagator(bl, zero, e, 0) for e in np.eye(bl.D)], axis=1)
    lam = np.random.default_rng(3).standard_normal(bl.D)
    back, _ = ADJ.fine_propagator_adjoint(bl, lam)
    np.testing.assert_allclose(back, Phi.T @ lam, rtol=1e-10, atol=1e-12 * np.abs(Phi.T @ lam).max())


@pytest.mark.parametrize("name", ["t1", "t2"])
def test_finite_differences_quadratic_loss(name):
    """L = 1/2 |X_N - ref|_M^2 + 1/2 sum_n dt |X_n - ref_n|_M^2 is quadratic
    in (x0, H): central differences have no truncation error."""
    p = build_problem(name)
    bl = S.Blocks.from_problem(p)
    rng = np.random.default_rng(5)
    scale = 1e-3
    x0 = scale * rng.standard_normal(bl.D)
    H = rng.standard_normal(p["H"].shape[1:])
    ref = ADJ.forward_linear(bl, p["G"], p["time_mode"], 0 * x0, H + 0.3 * rng.standard_normal(H.shape))
    M = bl.M

    def loss(X):
        e = X - ref
        q = np.einsum("nd,de,ne->n", e, M, e)
        return 0.5 * q[-1] + 0.5 * bl.dt * q.sum()

    X = ADJ.forward_linear(bl, p["G"], p["time_mode"], x0, H)
    e = X - ref
    Xbar = (bl.dt * e) @ M
    Xbar[-1] += e[-1] @ M
    sbar = S.Source(p["G"], H[None], p["time_mode"], bl.N, bl.P)
    x0b, Hb, _ = ADJ.adjoint(bl, sbar, Xbar)
    dirs = []
    for _ in range(4):
        dx, dH = rng.standard_normal(bl.D), rng.standard_normal(H.shape)
        nrm = np.sqrt(np.sum(dx ** 2) + np.sum(dH ** 2))
        dirs.append((dx / nrm, dH / nrm))
    for i in range(3):  # coordinate directions of H
        dH = np.zeros(H.shape)
        dH.flat[rng.integers(H.size)] = 1.0
        dirs.append((np.zeros(bl.D), dH))
    fd, ad = ADJ.fd_check(bl, p["G"], p["time_mode"], x0, H, loss, x0b, Hb, dirs, h=1e-3)
    np.testing.assert_allclose(fd, ad, rtol=1e-6, atol=1e-9 * np.abs(ad).max())


def test_fine_trajectory_boundaries_are_the_fine_composition():
    p = build_problem("t1")
    bl, src = S.Blocks.from_problem(p), S.Source.from_problem(p)
    x0 = np.random.default_rng(2).standard_normal(bl.D)
    Y = ADJ.fine_trajectory(bl, src, x0)
    X = S.fine_composition(bl, src, x0)
    assert Y.shape == (bl.N * bl.P + 1, bl.D)
    np.testing.assert_array_equal(Y[::bl.P], X)


@pytest.mark.parametrize("name", ["t1", "t2"])
def test_dot_product_identity_fine_levels(name):
    """<x_fine(x0, H), Xbar_fine> + <X(x0, H), Xbar> = <x0, x0bar> + <H, Hbar>."""
    p = build_problem(name)
    bl = S.Blocks.from_problem(p)
    rng = np.random.default_rng(13)
    x0 = rng.standard_normal(bl.D)
    H = rng.standard_normal(p["H"].shape[1:])
    Xf = ADJ.forward_fine_linear(bl, p["G"], p["time_mode"], x0, H)
    Xbar = rng.standard_normal((bl.N + 1, bl.D))
    Xbar_f = rng.standard_normal(Xf.shape)
    sbar = S.Source(p["G"], H[None], p["time_mode"], bl.N, bl.P)
    x0b, Hb, _ = ADJ.adjoint(bl, sbar, Xbar, Xbar_fine=Xbar_f)
    lhs = np.sum(Xf * Xbar_f) + np.sum(Xf[::bl.P] * Xbar)
    rhs = np.sum(x0 * x0b) + np.sum(H * Hb)
    scale = np.abs(Xf * Xbar_f).sum() + np.abs(x0 * x0b).sum() + np.abs(H * Hb).sum()
    assert abs(lhs - rhs) <= 1e-11 * scale


@pytest.mark.parametrize("name", ["t1", "t2"])
def test_finite_differences_fine_tracking_loss(name):
    """Terminal plus fine-step tracking loss
    L = 1/2 |x_NP - r_NP|_M^2 + 1/2 beta sum_{m>=1} dt_fine |x_m - r_m|_M^2,
    r the fine trajectory of a reference (x0_ref, H_ref): quadratic, so
    central differences are exact up to rounding. The tracking cotangents
    come from the trajectory of the difference (linearity of the scheme)."""
    p = build_problem(name)
    bl = S.Blocks.from_problem(p)
    rng = np.random.default_rng(7)
    beta = 1.0
    H_ref = rng.standard_normal(p["H"].shape[1:])
    ref = ADJ.forward_fine_linear(bl, p["G"], p["time_mode"], np.zeros(bl.D), H_ref)
    H = H_ref + 0.1 * rng.standard_normal(H_ref.shape)
    x0 = 0.1 * rng.standard_normal(bl.D) / np.sqrt(bl.D)
    M = bl.M

    def loss(Xf):
        e = Xf - ref
        q = np.einsum("nd,de,ne->n", e, M, e)
        return 0.5 * q[-1] + 0.5 * beta * bl.dt_fine * q[1:].sum()

    Y = ADJ.forward_fine_linear(bl, p["G"], p["time_mode"], x0, H - H_ref)  # x - r
    Xbar = np.zeros((bl.N + 1, bl.D))
    Xbar[-1] = M @ Y[-1]
    sbar = S.Source(p["G"], H[None], p["time_mode"], bl.N, bl.P)
    x0b, Hb, _ = ADJ.adjoint(bl, sbar, Xbar, Xbar_fine=ADJ.tracking_cotangents(bl, Y, beta))
    dirs = []
    for _ in range(4):
        dx, dH = rng.standard_normal(bl.D), rng.standard_normal(H.shape)
        nrm = np.sqrt(np.sum(dx ** 2) + np.sum(dH ** 2))
        dirs.append((dx / nrm, dH / nrm))
    fd, ad = ADJ.fd_check(bl, p["G"], p["time_mode"], x0, H, loss, x0b, Hb, dirs, h=1e-3, fine=True)
    np.testing.assert_allclose(fd, ad, rtol=1e-6, atol=1e-9 * np.abs(ad).max())


def test_planted_tracking_mistake_is_caught():
    """A tracking cotangent injected one fine level late (an off-by-one a
    GPU sweep could make) breaks the finite-difference agreement."""
    p = build_problem("t1")
    bl = S.Blocks.from_problem(p)
    rng = np.random.default_rng(9)
    H = rng.standard_normal(p["H"].shape[1:])
    x0 = rng.standard_normal(bl.D)
    M = bl.M

    def loss(Xf):
        q = np.einsum("nd,de,ne->n", Xf, M, Xf)
        return 0.5 * bl.dt_fine * q[1:].sum()

    Y = ADJ.forward_fine_linear(bl, p["G"], p["time_mode"], x0, H)
    Xf = ADJ.tracking_cotangents(bl, Y, 1.0)
    shifted = np.zeros_like(Xf)
    shifted[2:] = Xf[1:-1]
    sbar = S.Source(p["G"], H[None], p["time_mode"], bl.N, bl.P)
    dirs = [(rng.standard_normal(bl.D) / np.sqrt(bl.D), np.zeros(H.shape))]
    Xbar0 = np.zeros((bl.N + 1, bl.D))
    good = ADJ.adjoint(bl, sbar, Xbar0, Xbar_fine=Xf)
    bad = ADJ.adjoint(bl, sbar, Xbar0, Xbar_fine=shifted)
    fd, ad = ADJ.fd_check(bl, p["G"], p["time_mode"], x0, H, loss, good[0], good[1], dirs, h=1e-3, fine=True)
    np.testing.assert_allclose(fd, ad, rtol=1e-6)
    fd, ad = ADJ.fd_check(bl, p["G"], p["time_mode"], x0, H, loss, bad[0], bad[1], dirs, h=1e-3, fine=True)
    assert abs(fd[0] - ad[0]) > 1e-4 * abs(fd[0])


def test_finite_differences_h_1e6_directions_and_coordinates():
    """Central differences at h = 1e-6 of the terminal + fine-step tracking
    loss along 8 random unit directions and 16 random coordinates of
    (x0, H): the loss is quadratic, so the only FD error is rounding,
    about eps |L| / h."""
    p = build_problem("t2")
    bl = S.Blocks.from_problem(p)
    rng = np.random.default_rng(15)
    H_ref = rng.standard_normal(p["H"].shape[1:])
    ref = ADJ.forward_fine_linear(bl, p["G"], p["time_mode"], np.zeros(bl.D), H_ref)
    H = H_ref + 0.1 * rng.standard_normal(H_ref.shape)
    x0 = 0.1 * rng.standard_normal(bl.D) / np.sqrt(bl.D)
    M = bl.M

    def loss(Xf):
        e = Xf - ref
        q = np.einsum("nd,de,ne->n", e, M, e)
        return 0.5 * q[-1] + 0.5 * bl.dt_fine * q[1:].sum()

    Y = ADJ.forward_fine_linear(bl, p["G"], p["time_mode"], x0, H - H_ref)
    Xbar = np.zeros((bl.N + 1, bl.D))
    Xbar[-1] = M @ Y[-1]
    sbar = S.Source(p["G"], H[None], p["time_mode"], bl.N, bl.P)
    x0b, Hb, _ = ADJ.adjoint(bl, sbar, Xbar, Xbar_fine=ADJ.tracking_cotangents(bl, Y, 1.0))
    dirs = []
    for _ in range(8):
        dx, dH = rng.standard_normal(bl.D), rng.standard_normal(H.shape)
        nrm = np.sqrt(np.sum(dx ** 2) + np.sum(dH ** 2))
        dirs.append((dx / nrm, dH / nrm))
    n_x0, n_h = bl.D, H.size
    for idx in rng.choice(n_x0 + n_h, size=16, replace=False):
        dx, dH = np.zeros(bl.D), np.zeros(H.shape)
        if idx < n_x0:
            dx[idx] = 1.0
        else:
            dH.flat[idx - n_x0] = 1.0
        dirs.append((dx, dH))
    fd, ad = ADJ.fd_check(bl, p["G"], p["time_mode"], x0, H, loss, x0b, Hb, dirs, h=1e-6, fine=True)
    L = loss(ADJ.forward_fine_linear(bl, p["G"], p["time_mode"], x0, H))
    np.testing.assert_allclose(fd, ad, rtol=1e-5, atol=1e3 * np.finfo(float).eps * abs(L) / 1e-6)


def test_gradient_vanishes_at_the_reference():
    """At (x0, H) = (x0_ref, H_ref) the tracking error is zero, so every
    cotangent and the gradient are exactly zero."""
    p = build_problem("t1")
    bl = S.Blocks.from_problem(p)
    rng = np.random.default_rng(21)
    H_ref = rng.standard_normal(p["H"].shape[1:])
    x0_ref = rng.standard_normal(bl.D)
    Y = ADJ.forward_fine_linear(bl, p["G"], p["time_mode"], x0_ref - x0_ref, H_ref - H_ref)
    assert not Y.any()
    Xbar = np.zeros((bl.N + 1, bl.D))
    Xbar[-1] = bl.M @ Y[-1]
    sbar = S.Source(p["G"], H_ref[None], p["time_mode"], bl.N, bl.P)
    x0b, Hb, lam = ADJ.adjoint(bl, sbar, Xbar, Xbar_fine=ADJ.tracking_cotangents(bl, Y, 1.0))
    assert not x0b.any() and not Hb.any() and not lam.any()
