"""FP64 CPU oracle: discrete adjoint of the sequential fine solution.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The forward map (x0, H) -> X = (X*_0, ..., X*_N), X*_{n+1} = F(X*_n) (the
limit of parareal, eq. (2.7)), is linear in (x0, H) jointly. Given the
cotangents Xbar_n = dL/dX*_n, the adjoint returns dL/dx0 and dL/dH by running
the transpose of every fine step of eqs. (2.5)-(2.6) backward in time: the
transposed implicit solve with M11/h + A11, the transposed explicit solve
with M22, the history copies, and the fresh history at every interval start
(whose transpose adds the history adjoint to the state adjoint there).
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


def fine_propagator_adjoint(bl, lam):
    """Transpose of the linear part of F over one interval, plus the
    adjoints of the P step sources. lam: adjoint of F's output (D,) or
    (D, ncol). Returns (adjoint of the interval-start state, list of the
    source adjoints of steps p = 0..P-1)."""
    d1 = bl.d1
    ub, wb = lam[:d1].copy(), lam[d1:].copy()
    upb, wpb = np.zeros_like(ub), np.zeros_like(wb)
    srcb = [None] * bl.P
    for p in reversed(range(bl.P)):
        ub, wb, upb, wpb, fb = _step_adjoint(bl, bl.dt_fine, ub, wb, upb, wpb)
        srcb[p] = fb
    # fresh history at the interval start: u_p = u, w_p = w
    return np.concatenate([ub + upb, wb + wpb]), srcb


def adjoint(bl, src, Xbar, b=0):
    """Gradients of L with dL/dX*_n = Xbar[n] (n = 0..N) for sample b.
    Returns (x0bar (D,), Hbar shaped like src.H[b] (R, T_len), lam (N+1, D))
    where lam[n] is the adjoint of X*_n."""
    N = bl.N
    lam = np.zeros((N + 1, bl.D))
    lam[N] = Xbar[N]
    R = 0 if src.G is None else src.G.shape[1]
    Hbar = np.zeros((R, src.H.shape[2])) if R else None
    for n in reversed(range(N)):
        back, srcb = fine_propagator_adjoint(bl, lam[n + 1])
        lam[n] = Xbar[n] + back
        if R:
            for p, fb in enumerate(srcb):
                tau = n * bl.P + p if src.mode == TIME_FINE else n
                Hbar[:, tau] += src.G.T @ fb
    return lam[0], Hbar, lam


def forward_linear(bl, src_G, src_mode, x0, H):
    """X*(x0, H) with source amplitudes H (R, T_len) for one sample."""
    from .scheme import Source, fine_composition
    s = Source(src_G, H[None], src_mode, bl.N, bl.P)
    return fine_composition(bl, s, x0, 0)


def fd_check(bl, src_G, src_mode, x0, H, loss, grad_x0, grad_H, directions, h=1e-6):
    """Central differences of the scalar loss(X) along the given unit
    directions (dx0, dH); returns (fd values, adjoint values)."""
    fd, ad = [], []
    for dx0, dH in directions:
        lp = loss(forward_linear(bl, src_G, src_mode, x0 + h * dx0, H + h * dH))
        lm = loss(forward_linear(bl, src_G, src_mode, x0 - h * dx0, H - h * dH))
        fd.append((lp - lm) / (2 * h))
        ad.append(float(np.sum(dx0 * grad_x0) + (np.sum(dH * grad_H) if grad_H is not None else 0.0)))
    return np.array(fd), np.array(ad)
