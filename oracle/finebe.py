"""Brute-force fine-grid backward Euler, paper eq. (2.3) with V_H replaced by
the full Q1 space: (M_f/dt + A_f) u' = M_f u/dt + b(t'), solved by a sparse
LU factorisation. TEST INFRASTRUCTURE ONLY."""
import numpy as np
import scipy.sparse.linalg as spla


def fine_backward_euler(M, A, u0, dt, n_steps, load):
    """load(m) returns the load vector at time level m+1 (t_{m+1})."""
    lu = spla.splu((M / dt + A).tocsc())
    u = np.array(u0, dtype=np.float64)
    out = [u.copy()]
    for m in range(n_steps):
        u = lu.solve(M @ u / dt + load(m))
        out.append(u.copy())
    return np.array(out)
