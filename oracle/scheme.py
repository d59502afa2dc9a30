"""FP64 CPU oracle: the partially explicit splitting scheme, the fine and
coarse propagators, the sequential fine solution and plain parareal.

TEST INFRASTRUCTURE ONLY. Nothing in the library or its Python binding may
import this package; only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it. It is written directly from the paper and shares no
code with the GPU path.

Scheme (paper eqs. (2.4)-(2.5)) in matrix form, step size h, state (u, w) at
level n and history (u_prev, w_prev) at level n-1:
    M11 (u' - u)/h + M12 (w - w_prev)/h + A11 u' + A12 w = F1
    M22 (w' - w)/h + M21 (u - u_prev)/h + A21 u' + A22 w = F2
with M21 = M12^T, A21 = A12^T (symmetric forms a(.,.) and (.,.)).
Readings:
  * the source is taken at the new time level t_{n+1}, as in eqs. (4.8)-(4.9)
    and in backward Euler (2.3);
  * every propagator call starts a fresh history: u_prev = u, w_prev = w at
    the first step of an interval (the coupling differences vanish there);
    the coarse propagator G is then one step of size Delta t;
  * the parareal update follows eq. (2.7): iteration k applies F to the
    iterate k-1; x_0^k = x_0 for all k;
  * the stopping test (2.8) measures the full state change in the L2 norm of
    the coarse function, |e|_M = sqrt(e^T M e) with M the full projected mass,
    absolute, "<="; at most N iterations.
The oracle solves the implicit equation for u' by a Cholesky factorisation
of (M11/h + A11) in the non-increment form written above (a different
algebraic route from the GPU path, which works with residuals and
increments).
"""
import numpy as np
import scipy.linalg as sla

TIME_FINE = 0
TIME_INTERVAL = 1


class Blocks:
    """Projected blocks of eq. (3.8) plus step sizes. Arrays are FP64."""

    def __init__(self, M11, M12, M22, A11, A12, A22, dt, dt_fine, N):
        self.M11 = np.asarray(M11, dtype=np.float64)
        self.M12 = np.asarray(M12, dtype=np.float64)
        self.M22 = np.asarray(M22, dtype=np.float64)
        self.A11 = np.asarray(A11, dtype=np.float64)
        self.A12 = np.asarray(A12, dtype=np.float64)
        self.A22 = np.asarray(A22, dtype=np.float64)
        self.d1 = self.M11.shape[0]
        self.d2 = self.M22.shape[0]
        self.D = self.d1 + self.d2
        self.dt = float(dt)
        self.dt_fine = float(dt_fine)
        self.N = int(N)
        self.P = int(round(dt / dt_fine))
        self._chol = {}
        self._m22 = sla.cho_factor(self.M22) if self.d2 else None  # d2 = 0: no V_H2
        self.M = np.block([[self.M11, self.M12], [self.M12.T, self.M22]])

    @classmethod
    def from_problem(cls, prob):
        return cls(prob["M11"], prob["M12"], prob["M22"], prob["A11"], prob["A12"],
                   prob["A22"], prob["dt"], prob["dt_fine"], prob["N"])

    def chol(self, h):
        if h not in self._chol:
            self._chol[h] = sla.cho_factor(self.M11 / h + self.A11)
        return self._chol[h]


class Source:
    """f = sum_r G[:, r] h_r(t) (projected onto V_H1 x V_H2)."""

    def __init__(self, G, H, time_mode, N, P):
        self.G = None if G is None else np.asarray(G, dtype=np.float64)
        self.H = None if H is None else np.asarray(H, dtype=np.float64)
        self.mode = int(time_mode)
        self.N, self.P = N, P

    @classmethod
    def from_problem(cls, prob):
        return cls(prob["G"], prob["H"], prob["time_mode"], prob["N"], prob["P"])

    def at_fine(self, b, n, p):
        """Source at fine time t_n + (p+1) dt_fine of interval n, sample b."""
        if self.G is None or self.G.shape[1] == 0:
            return 0.0
        if self.mode == TIME_FINE:
            return self.G @ self.H[b, :, n * self.P + p]
        return self.G @ self.H[b, :, n]

    def at_coarse(self, b, n):
        """Source used by the coarse step of interval n (time t_{n+1})."""
        if self.G is None or self.G.shape[1] == 0:
            return 0.0
        if self.mode == TIME_FINE:
            return self.G @ self.H[b, :, n * self.P + self.P - 1]
        return self.G @ self.H[b, :, n]


def step(bl, h, u, w, u_prev, w_prev, F):
    """One step of eqs. (2.4)-(2.5) with step size h. u, w (and the history)
    are vectors or (d, ncol) arrays of independent columns; F is 0 or has
    the shape of the stacked state [u; w]."""
    d1 = bl.d1
    F = np.zeros((bl.D,) + u.shape[1:]) if np.ndim(F) == 0 else np.asarray(F, dtype=np.float64)
    F1, F2 = F[:d1], F[d1:]
    rhs_u = bl.M11 @ u / h - bl.M12 @ (w - w_prev) / h - bl.A12 @ w + F1
    u_new = sla.cho_solve(bl.chol(h), rhs_u)
    if bl.d2 == 0:
        return u_new, w.copy()
    rhs_w = bl.M22 @ w - bl.M12.T @ (u - u_prev) - h * (bl.A12.T @ u_new) - h * (bl.A22 @ w) + h * F2
    w_new = sla.cho_solve(bl._m22, rhs_w)
    return u_new, w_new


def fine_propagator(bl, src, x, n, b=0):
    """F: P steps of size dt_fine over interval n from state x (history reset
    at the interval start). x has shape (D,)."""
    d1 = bl.d1
    u, w = x[:d1].copy(), x[d1:].copy()
    u_prev, w_prev = u.copy(), w.copy()
    for p in range(bl.P):
        u_new, w_new = step(bl, bl.dt_fine, u, w, u_prev, w_prev, src.at_fine(b, n, p))
        u_prev, w_prev, u, w = u, w, u_new, w_new
    return np.concatenate([u, w])


def fine_propagator_cols(bl, src, X, ns, bs):
    """F applied to many columns at once: X is (D, ncol); column c belongs to
    interval ns[c] and sample bs[c]. Same arithmetic as fine_propagator, with
    the columns carried through library matrix products together."""
    d1 = bl.d1
    u, w = X[:d1].copy(), X[d1:].copy()
    u_prev, w_prev = u.copy(), w.copy()
    for p in range(bl.P):
        F = np.stack([np.broadcast_to(src.at_fine(b, n, p), (bl.D,)) for n, b in zip(ns, bs)], axis=1)
        u_new, w_new = step(bl, bl.dt_fine, u, w, u_prev, w_prev, F)
        u_prev, w_prev, u, w = u, w, u_new, w_new
    return np.concatenate([u, w])


def coarse_propagator(bl, src, x, n, b=0):
    """G: one step of size dt over interval n (history reset)."""
    d1 = bl.d1
    u, w = x[:d1], x[d1:]
    u_new, w_new = step(bl, bl.dt, u, w, u, w, src.at_coarse(b, n))
    return np.concatenate([u_new, w_new])


def fine_composition(bl, src, x0, b=0):
    """Sequential fine solution X*_{n+1} = F(X*_n), X*_0 = x0: the limit of
    parareal. Returns (N+1, D)."""
    X = np.zeros((bl.N + 1, bl.D))
    X[0] = x0
    for n in range(bl.N):
        X[n + 1] = fine_propagator(bl, src, X[n], n, b)
    return X


def m_norm(bl, e):
    """L2(Omega) norm of the coarse function with coefficients e."""
    e = np.asarray(e, dtype=np.float64)
    return float(np.sqrt(max(e @ (bl.M @ e), 0.0)))


def parareal(bl, src, x0, tol, k_max=None, b=0, columns=True, rel=False, fine_cols=None):
    """Plain parareal (Algorithm 1 with the update of eq. (2.7) and the stop
    test of eq. (2.8)). Returns dict with all iterates X[k] (k = 0..K, each
    (N+1, D)), the jump history J[k] (k = 1..K) and K.
    With rel=True the tolerance is scaled by max_n |x_n^0|_M.
    fine_cols (optional) replaces the fine propagator: called as
    fine_cols(X, ns, bs) with the start states as columns of X (D, N)."""
    N = bl.N
    k_max = N if k_max is None else min(int(k_max), N)
    X = np.zeros((N + 1, bl.D))
    X[0] = x0
    g_old = np.zeros((N, bl.D))
    for n in range(N):
        g_old[n] = coarse_propagator(bl, src, X[n], n, b)
        X[n + 1] = g_old[n]
    iterates = [X.copy()]
    jumps = []
    thr = tol
    if rel:
        thr = tol * max(m_norm(bl, X[n]) for n in range(N + 1))
    k = 0
    while k < k_max:
        k += 1
        if fine_cols is not None:
            f = fine_cols(X[:N].T.copy(), list(range(N)), [b] * N).T
        elif columns:
            f = fine_propagator_cols(bl, src, X[:N].T.copy(), list(range(N)), [b] * N).T
        else:
            f = np.stack([fine_propagator(bl, src, X[n], n, b) for n in range(N)])
        Xn = np.zeros_like(X)
        Xn[0] = x0
        for n in range(N):
            g = coarse_propagator(bl, src, Xn[n], n, b)
            Xn[n + 1] = g + f[n] - g_old[n]
            g_old[n] = g
        J = max(m_norm(bl, Xn[n] - X[n]) for n in range(1, N + 1))
        X = Xn
        iterates.append(X.copy())
        jumps.append(J)
        if J <= thr:
            break
    return dict(X=iterates, J=np.array(jumps), K=k, threshold=thr)


def rel_l2_M(bl, X, Xref):
    """sqrt(sum_n |X_n - Xref_n|_M^2) / sqrt(sum_n |Xref_n|_M^2) over the
    coarse boundary states n = 0..N (rows of X)."""
    num = sum(m_norm(bl, X[n] - Xref[n]) ** 2 for n in range(X.shape[0]))
    den = sum(m_norm(bl, Xref[n]) ** 2 for n in range(Xref.shape[0]))
    return float(np.sqrt(num / den)) if den > 0 else float(np.sqrt(num))


# ---------------------------------------------------------------------------
# History carried across intervals (the alternative reading of the two-step
# scheme at interval starts). The scheme (2.4)-(2.5) couples the two spaces
# through the difference quotients (u_n - u_{n-1})/h and (w_n - w_{n-1})/h of
# the previous step. Instead of restarting that history at every interval
# start, the state carries it: y = [x; delta] with delta = x - x_prev the
# change over the last step of size dt_fine (the rate times dt_fine). A fine
# step starts from x_prev = x - delta. The coarse step (one step of size
# Delta t = P dt_fine, as in Algorithm 1) starts with a fresh history as
# before and hands back the rate of its own step, delta' = (x' - x)/P. The
# fine composition of this propagator is one uninterrupted run of N*P steps
# of size dt_fine; the parareal limit depends on F only, so the choice of G
# changes the convergence, not the limit.
# ---------------------------------------------------------------------------
def fine_propagator_carry(bl, src, y, n, b=0):
    """F with carried history: P steps of size dt_fine over interval n from
    y = [x; delta] (shape (2D,)). Returns [x_P; x_P - x_{P-1}]."""
    d1, D = bl.d1, bl.D
    u, w = y[:d1].copy(), y[d1:D].copy()
    u_prev, w_prev = u - y[D:D + d1], w - y[D + d1:]
    for p in range(bl.P):
        u_new, w_new = step(bl, bl.dt_fine, u, w, u_prev, w_prev, src.at_fine(b, n, p))
        u_prev, w_prev, u, w = u, w, u_new, w_new
    return np.concatenate([u, w, u - u_prev, w - w_prev])


def coarse_propagator_carry(bl, src, y, n, b=0):
    """G on carried states: one step of size dt over interval n from x with a
    fresh history (the carried change is not used); returns [x'; (x' - x)/P],
    the change of one fine step at the coarse step's rate."""
    d1, D, P = bl.d1, bl.D, bl.P
    u, w = y[:d1], y[d1:D]
    u_new, w_new = step(bl, bl.dt, u, w, u, w, src.at_coarse(b, n))
    return np.concatenate([u_new, w_new, (u_new - u) / P, (w_new - w) / P])


def fine_composition_carry(bl, src, x0, b=0):
    """Y*_{n+1} = F(Y*_n) with carried history from Y*_0 = [x0; 0] (no
    history before t = 0). Returns (N+1, 2D)."""
    Y = np.zeros((bl.N + 1, 2 * bl.D))
    Y[0, :bl.D] = x0
    for n in range(bl.N):
        Y[n + 1] = fine_propagator_carry(bl, src, Y[n], n, b)
    return Y


def sequential_run(bl, src, x0, b=0):
    """N*P steps of the scheme of size dt_fine without any restart (x_{-1} =
    x_0), the history always taken from the previous step. Returns the states
    at the coarse boundaries with their last change, (N+1, 2D)."""
    d1, D, P = bl.d1, bl.D, bl.P
    u, w = np.array(x0[:d1], dtype=np.float64), np.array(x0[d1:], dtype=np.float64)
    u_prev, w_prev = u.copy(), w.copy()
    out = np.zeros((bl.N + 1, 2 * D))
    out[0, :D] = x0
    for n in range(bl.N):
        for p in range(P):
            u_new, w_new = step(bl, bl.dt_fine, u, w, u_prev, w_prev, src.at_fine(b, n, p))
            u_prev, w_prev, u, w = u, w, u_new, w_new
        out[n + 1] = np.concatenate([u, w, u - u_prev, w - w_prev])
    return out


def parareal_carry(bl, src, x0, tol, k_max=None, b=0, rel=False):
    """Parareal (update (2.7), stop test (2.8)) on the history-carrying states
    y = [x; delta]; y_0^k = [x0; 0]. The stopping test measures the change of
    x only, |x_n^k - x_n^{k-1}|_M, as (2.8) does. Returns the iterates
    (each (N+1, 2D)), the jumps and K, as parareal()."""
    N, D = bl.N, bl.D
    k_max = N if k_max is None else min(int(k_max), N)
    Y = np.zeros((N + 1, 2 * D))
    Y[0, :D] = x0
    g_old = np.zeros((N, 2 * D))
    for n in range(N):
        g_old[n] = coarse_propagator_carry(bl, src, Y[n], n, b)
        Y[n + 1] = g_old[n]
    iterates = [Y.copy()]
    jumps = []
    thr = tol
    if rel:
        thr = tol * max(m_norm(bl, Y[n, :D]) for n in range(N + 1))
    k = 0
    while k < k_max:
        k += 1
        f = np.stack([fine_propagator_carry(bl, src, Y[n], n, b) for n in range(N)])
        Yn = np.zeros_like(Y)
        Yn[0] = Y[0]
        for n in range(N):
            g = coarse_propagator_carry(bl, src, Yn[n], n, b)
            Yn[n + 1] = g + f[n] - g_old[n]
            g_old[n] = g
        J = max(m_norm(bl, Yn[n, :D] - Y[n, :D]) for n in range(1, N + 1))
        Y = Yn
        iterates.append(Y.copy())
        jumps.append(J)
        if J <= thr:
            break
    return dict(X=iterates, J=np.array(jumps), K=k, threshold=thr)
