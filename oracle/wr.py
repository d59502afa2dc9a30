"""FP64 CPU oracle: the paper's own fine solver, waveform relaxation (WR) with
the alpha-circulant diagonalisation in time (Sections 4.1 and 4.2).

TEST INFRASTRUCTURE ONLY. Nothing in the library or its Python binding may
import this package; only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it. It is written from the paper and shares no code with
the GPU path.

Inside one coarse interval with P fine steps of size h (levels s = 0..P, s = 0
the interval start x = (u_0, w_0)), iteration j of WR does:

  1. the V_H1 part at all levels at once (eq. (4.8) as the all-at-once system
     (4.12)): for s = 1..P
        M11 (u_s - u_{s-1})/h + A11 u_s
            = F1_s - M12 (w_{s-1} - w_{s-2})/h - A12 w_{s-1}      (w = w^{j-1})
     with the periodic-like start u_0 + alpha (u_P^j - u_P^{j-1}); in matrix
     form (B (x) M11 + I (x) A11) U = R, B the alpha-circulant matrix of
     eq. (4.4), R_1 carrying + M11 (u_0 - alpha u_P^{j-1})/h;
  2. the V_H2 part sequentially in time (eq. (4.9)), with U = U^j:
        M22 (w_s - w_{s-1})/h + M21 (u_{s-1} - u_{s-2})/h + A21 u_s + A22 w_{s-1}
            = F2_s.

Step 1 is solved as in eqs. (4.5)-(4.7) and (4.13): B = S D S^-1 with
S^-1 = F Gamma (Gamma = diag(alpha^{q/P}), F the discrete Fourier matrix),
D = diag(d_k), d_k = (1 - alpha^{1/P} e^{-2 pi i k/P})/h, so that
U = Gamma^-1 F^-1 [(d_k M11 + A11)^-1 (F Gamma R)_k]_k.

Readings (beyond those of the scheme oracle):
  * the history terms follow eq. (4.8) (w_{s-1} - w_{s-2}, A12 w_{s-1}) with
    the interval-start reset w_{-1} = w_0, u_{-1} = u_0, as for the sequential
    fine propagator;
  * initial waveform: w_s^0 = w_0 at every level and u_P^0 = u_0 (the start
    state continued as a constant);
  * the fixed point of the iteration is the sequential fine propagator F
    (P steps of eqs. (2.4)-(2.5)); the theorem of Section 4.2 bounds the
    error after j iterations by a factor gamma^(2(j-1)), gamma the cosine of
    eq. (4.15) (continuous time, alpha -> 0).
"""
import numpy as np
import scipy.linalg as sla

from .scheme import Source  # noqa: F401  (type of `src`)


def circulant_eigs(P, alpha, h):
    """Eigenvalues d_k of the alpha-circulant matrix B of eq. (4.4), in the
    order matching numpy's forward FFT (eq. (4.5))."""
    k = np.arange(P)
    return (1.0 - alpha ** (1.0 / P) * np.exp(-2j * np.pi * k / P)) / h


def circulant_matrix(P, alpha, h):
    """B of eq. (4.4) written out (for checks on small sizes)."""
    B = np.eye(P) - np.eye(P, k=-1)
    B[0, P - 1] = -alpha
    return B / h


def all_at_once_solve(M11, A11, R, alpha, h):
    """Solve (B (x) M11 + I (x) A11) U = R through the diagonalisation of
    eqs. (4.5)-(4.7): R and U are (P, d1, ncol). Step (a) scales by Gamma
    and transforms along time, step (b) solves the P shifted systems
    (d_k M11 + A11) (complex, one LU each), step (c) transforms back."""
    P = R.shape[0]
    gam = alpha ** (np.arange(P) / P)
    Rh = np.fft.fft(gam[:, None, None] * R, axis=0)                 # (a)
    d = circulant_eigs(P, alpha, h)
    key = (id(M11), id(A11), M11.shape[0], float(alpha), float(h), P)
    if _LU.get("key") != key:   # factorisations reused across iterations
        _LU.clear()
        _LU["key"] = key
        _LU["refs"] = (M11, A11)  # held, so that the ids in the key stay unique
        _LU["f"] = [sla.lu_factor(d[k] * M11 + A11) for k in range(P)]
    Uh = np.empty_like(Rh)
    for k in range(P):                                               # (b)
        Uh[k] = sla.lu_solve(_LU["f"][k], Rh[k])
    U = np.fft.ifft(Uh, axis=0) / gam[:, None, None]                 # (c)
    return U.real


_LU = {}


def sequential_solve(M11, A11, R, h):
    """The same all-at-once system with alpha = 0 (B lower bidiagonal),
    solved by forward substitution in time: the classical WR sweep."""
    P = R.shape[0]
    c = sla.cho_factor(M11 / h + A11)
    U = np.empty_like(R)
    prev = np.zeros_like(R[0])
    for s in range(P):
        U[s] = sla.cho_solve(c, R[s] + M11 @ prev / h)
        prev = U[s]
    return U


def _sources(bl, src, ns, bs):
    """F at the fine levels s = 1..P of each column's interval: (P, D, ncol)."""
    P = bl.P
    F = np.zeros((P, bl.D, len(ns)))
    for c, (n, b) in enumerate(zip(ns, bs)):
        for p in range(P):
            F[p, :, c] = src.at_fine(b, n, p)
    return F


def wr_fine_cols(bl, src, X, ns, bs, alpha, K0, history=False):
    """K0 iterations of WR (Section 4.2) on many intervals at once: X is
    (D, ncol), column c the start state of interval ns[c], sample bs[c].
    Returns the state at the interval end after K0 iterations, (D, ncol);
    with history=True also the list of end states after iterations 1..K0.
    alpha = 0 uses the sequential solve for step 1 (no diagonalisation)."""
    d1, d2, h, P = bl.d1, bl.d2, bl.dt_fine, bl.P
    u0, w0 = X[:d1].copy(), X[d1:].copy()
    F = _sources(bl, src, ns, bs)
    F1, F2 = F[:, :d1], F[:, d1:]
    W = np.repeat(w0[None], P + 1, axis=0)   # levels 0..P of w^{j-1}
    uP_old = u0.copy()
    ends = []
    for _ in range(K0):
        # step 1: right-hand sides of eq. (4.8) at s = 1..P
        w_prev = W[:P]                                              # w_{s-1}
        w_prev2 = np.concatenate([W[:1], W[:P - 1]], axis=0)        # w_{s-2}, w_{-1} = w_0
        R = F1 - np.einsum("ij,sjc->sic", bl.M12, w_prev - w_prev2) / h \
            - np.einsum("ij,sjc->sic", bl.A12, w_prev)
        R[0] += bl.M11 @ (u0 - alpha * uP_old) / h
        if alpha == 0.0:
            U = sequential_solve(bl.M11, bl.A11, R, h)
        else:
            U = all_at_once_solve(bl.M11, bl.A11, R, alpha, h)
        # step 2: eq. (4.9) sequentially in time with U^j
        Ul = np.concatenate([u0[None], U], axis=0)                  # levels 0..P
        Wn = np.empty_like(W)
        Wn[0] = w0
        for s in range(1, P + 1):
            du = Ul[s - 1] - (Ul[s - 2] if s >= 2 else u0)           # u_{-1} = u_0
            rhs = bl.M22 @ Wn[s - 1] - bl.M12.T @ du - h * (bl.A12.T @ Ul[s]) \
                - h * (bl.A22 @ Wn[s - 1]) + h * F2[s - 1]
            Wn[s] = sla.cho_solve(bl._m22, rhs) if d2 else Wn[s - 1]
        W = Wn
        uP_old = U[P - 1].copy()
        end = np.concatenate([U[P - 1], W[P]])
        if history:
            ends.append(end.copy())
    out = np.concatenate([U[P - 1], W[P]]) if K0 > 0 else X.copy()
    return (out, ends) if history else out


def wr_fine(bl, src, x, n, alpha, K0, b=0, history=False):
    """WR fine propagator on one interval, x of shape (D,)."""
    r = wr_fine_cols(bl, src, x[:, None], [n], [b], alpha, K0, history)
    if history:
        return r[0][:, 0], [e[:, 0] for e in r[1]]
    return r[:, 0]


def parareal_wr(bl, src, x0, tol, alpha, K0, k_max=None, b=0, rel=False):
    """Algorithm 1 with the paper's fine solver: the parareal update of
    eq. (2.7) where F is K0 iterations of WR on every interval (Section 4.3
    uses WR as the fine propagator inside parareal)."""
    from .scheme import parareal
    return parareal(bl, src, x0, tol, k_max=k_max, b=b, rel=rel,
                    fine_cols=lambda X, ns, bs: wr_fine_cols(bl, src, X, ns, bs, alpha, K0))


def wr_composition(bl, src, x0, alpha, K0, b=0):
    """X_{n+1} = F_WR(X_n), X_0 = x0: the limit of parareal with the WR fine
    solver (the sequential composition of the fine solver it uses)."""
    X = np.zeros((bl.N + 1, bl.D))
    X[0] = x0
    for n in range(bl.N):
        X[n + 1] = wr_fine(bl, src, X[n], n, alpha, K0, b)
    return X


def gamma_sq(bl):
    """gamma^2 of eq. (4.15) for the discrete spaces: the largest generalised
    eigenvalue of (M21 M11^-1 M12, M22) (the squared cosine of the largest
    angle-free pair between V_H1 and V_H2 in L2)."""
    X = sla.cho_solve(sla.cho_factor(bl.M11), bl.M12)
    ev = sla.eigh(bl.M12.T @ X, bl.M22, eigvals_only=True)
    return float(ev[-1])
