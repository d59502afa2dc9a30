"""FP64 CPU oracle: discrete adjoint of the sequential fine solution.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The forward map (x0, H) -> X = (X*_0, ..., X*_N), X*_{n+1} = F(X*_n) (the
limit of parareal, eq. (2.7)), is linear in (x0, H) jointly, and so is the
map to every fine time level of that solution. Given the cotangents
Xbar_n = dL/dX*_n at the coarse boundaries and, optionally, cotangents at
the fine levels (a tracking term), the adjoint returns dL/dx0 and dL/dH by
running the transpose of every fine step of eqs. (2.4)-(2.5) backward in
time: the transposed implicit solve with M11/h + A11, the transposed
explicit solve with M22, the history copies, and the fresh history at every
interval start (whose transpose adds the history adjoint to the state
adjoint there).
"""
import numpy as np
import scipy.linalg as sla

from .scheme import TIME_FINE


def _step_adjoint(bl, h, ub, wb, upb, wpb):
    """Transpose of one step. Forward (see scheme.step):
        u' = K^-1 (M11 u/h - M12 (w - w_p)/h - A12 w + F1)
        w' = M22^-1 (M22 w - M21 (u - u_p) - h A21 u' - h A22 w + h F2)
        (u_p', w_p') = (u, w)
    Input: adjoints of (u', w', u_p', w_p'). Output: adjoints of
    (u, w, u_p, w_p) and of (F1, F2)."""
    # history copy
    u_b = upb.copy()
    w_b = wpb.copy()
    up_b = np.zeros_like(ub)
    wp_b = np.zeros_like(wb)
    F2_b = np.zeros_like(wb)
    u_new_b = ub.copy()
    if bl.d2:
        eta = sla.cho_solve(bl._m22, wb)
        w_b += bl.M22 @ eta - h * (bl.A22 @ eta)
        u_b -= bl.M12 @ eta
        up_b += bl.M12 @ eta
        u_new_b -= h * (bl.A12 @ eta)
        F2_b = h * eta
    xi = sla.cho_solve(bl.chol(h), u_new_b)
    u_b += bl.M11 @ xi / h
    w_b -= bl.M12.T @ xi / h + bl.A12.T @ xi
    wp_b += bl.M12.T @ xi / h
    F1_b = xi
    return u_b, w_b, up_b, wp_b, np.concatenate([F1_b, F2_b])


def fine_propagator_adjoint(bl, lam, inj=None):
    """Transpose of the linear part of F over one interval, plus the
    adjoints of the P step sources. lam: adjoint of F's output (D,) or
    (D, ncol). inj (optional, (P, D)): extra cotangents of the states after
    steps p = 0..P-1 of the interval (inj[P-1] is at F's output). Returns
    (adjoint of the interval-start state, list of the source adjoints of
    steps p = 0..P-1)."""
    d1 = bl.d1
    ub, wb = lam[:d1].copy(), lam[d1:].copy()
    upb, wpb = np.zeros_like(ub), np.zeros_like(wb)
    srcb = [None] * bl.P
    for p in reversed(range(bl.P)):
        if inj is not None:
            ub += inj[p][:d1]
            wb += inj[p][d1:]
        ub, wb, upb, wpb, fb = _step_adjoint(bl, bl.dt_fine, ub, wb, upb, wpb)
        srcb[p] = fb
    # fresh history at the interval start: u_p = u, w_p = w
    return np.concatenate([ub + upb, wb + wpb]), srcb


def adjoint(bl, src, Xbar, b=0, Xbar_fine=None):
    """Gradients of L with dL/dX*_n = Xbar[n] (n = 0..N) for sample b and,
    if given, dL/dx_m = Xbar_fine[m] at the fine levels m = 0..N*P (x_m the
    state at time m*dt_fine of the sequential fine solution; level n*P is
    X*_n, level 0 is x0). Returns (x0bar (D,), Hbar shaped like src.H[b]
    (R, T_len), lam (N+1, D)) where lam[n] = Xbar[n] + (transpose of F over
    interval n, including that interval's fine-level cotangents) lam[n+1]."""
    N, P = bl.N, bl.P
    lam = np.zeros((N + 1, bl.D))
    lam[N] = Xbar[N]
    R = 0 if src.G is None else src.G.shape[1]
    Hbar = np.zeros((R, src.H.shape[2])) if R else None
    for n in reversed(range(N)):
        inj = None if Xbar_fine is None else Xbar_fine[n * P + 1:(n + 1) * P + 1]
        back, srcb = fine_propagator_adjoint(bl, lam[n + 1], inj)
        lam[n] = Xbar[n] + back
        if R:
            for p, fb in enumerate(srcb):
                tau = n * bl.P + p if src.mode == TIME_FINE else n
                Hbar[:, tau] += src.G.T @ fb
    x0bar = lam[0] if Xbar_fine is None else lam[0] + Xbar_fine[0]
    return x0bar, Hbar, lam


def fine_trajectory(bl, src, x0, b=0):
    """Every fine time level of the sequential fine solution: row m is the
    state at t = m dt_fine, m = 0..N*P (row n*P is X*_n). Each interval
    starts with a fresh history, as F does."""
    from .scheme import step
    N, P, d1 = bl.N, bl.P, bl.d1
    X = np.zeros((N * P + 1, bl.D))
    X[0] = x0
    for n in range(N):
        u, w = X[n * P, :d1].copy(), X[n * P, d1:].copy()
        u_prev, w_prev = u.copy(), w.copy()
        for p in range(P):
            u_new, w_new = step(bl, bl.dt_fine, u, w, u_prev, w_prev, src.at_fine(b, n, p))
            u_prev, w_prev, u, w = u, w, u_new, w_new
            X[n * P + p + 1] = np.concatenate([u, w])
    return X


def tracking_cotangents(bl, Y, beta):
    """Cotangents of the fine-step tracking term
        1/2 beta sum_{m=1}^{N*P} dt_fine |y_m|_M^2
    of a fine trajectory y (rows m = 0..N*P): beta dt_fine M y_m, zero at
    m = 0 (the initial level is not tracked)."""
    Xf = beta * bl.dt_fine * (Y @ bl.M)
    Xf[0] = 0.0
    return Xf


def forward_linear(bl, src_G, src_mode, x0, H):
    """X*(x0, H) with source amplitudes H (R, T_len) for one sample."""
    from .scheme import Source, fine_composition
    s = Source(src_G, H[None], src_mode, bl.N, bl.P)
    return fine_composition(bl, s, x0, 0)


def forward_fine_linear(bl, src_G, src_mode, x0, H):
    """Fine trajectory (N*P+1, D) with source amplitudes H for one sample."""
    from .scheme import Source
    s = Source(src_G, H[None], src_mode, bl.N, bl.P)
    return fine_trajectory(bl, s, x0, 0)


def fd_check(bl, src_G, src_mode, x0, H, loss, grad_x0, grad_H, directions, h=1e-6, fine=False):
    """Central differences of the scalar loss(X) along the given unit
    directions (dx0, dH); X is the coarse-boundary solution, or the fine
    trajectory if fine. Returns (fd values, adjoint values)."""
    fwd = forward_fine_linear if fine else forward_linear
    fd, ad = [], []
    for dx0, dH in directions:
        lp = loss(fwd(bl, src_G, src_mode, x0 + h * dx0, H + h * dH))
        lm = loss(fwd(bl, src_G, src_mode, x0 - h * dx0, H - h * dH))
        fd.append((lp - lm) / (2 * h))
        ad.append(float(np.sum(dx0 * grad_x0) + (np.sum(dH * grad_H) if grad_H is not None else 0.0)))
    return np.array(fd), np.array(ad)
