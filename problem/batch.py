"""Seeded ragged batch of independent solves (the batched workload): every
solve has its own medium, coarse grid, contrast, interval count and source.

Solve b draws, from numpy.random.default_rng(base_seed + b) in this order:
n_c ~ U{8..32} (fine grid n = 10 n_c), N ~ U{16..128} intervals of P = 32
fine steps, contrast c = 10^U(4,6), a medium kappa = 1 with floor(n_c/4)
horizontal and floor(n_c/4) vertical full-span one-cell channels of value c
(at most one per coarse row / column, `media.straight_channels`), and a
source f = sum_{m=1..8} a_m sin(p_m pi x) sin(q_m pi y) with (p_m, q_m) ~
U{1..4}^2 and a_m ~ N(0,1), constant in time; u0 = 0.

The multiscale spaces are CEM-GMsFEM's (Section 3.1, J = 5 local functions
per coarse element, 2 layers of oversampling, V_H1 = the first two,
d1 = 2 n_c^2, d2 = 3 n_c^2). On the GPU they are built by the library's
set-up pipeline (`pe_local_spectral`, `pe_cem_spaces`: eqs. (3.1), (3.2),
(3.8)); `cpu_problem` builds the same solve with the CPU generator, which
checks the GPU-built blocks on a seeded subset.

The coarse step is half the largest stable one, dt = (1 - gamma^2) /
(2 lambda2) (the stability condition of Section 3.2; lambda2 = largest
eigenvalue of (A22, M22), gamma^2 = squared largest cosine between V_H1 and
V_H2 in L2). On the GPU these two eigenvalues are computed with
torch.linalg from the mass Cholesky factors; this is part of the input
recipe (how the step size is chosen), not of the parareal path.

This module produces inputs only: no time stepping, no propagator, no
parareal update and no convergence test.
"""
import numpy as np

from . import media
from .fem import FineGrid

P_FINE = 32
J_LOCAL, J1_LOCAL, LAYERS = 5, 2, 2


def solve_spec(b, base_seed=1000):
    """Seeded description of solve b (no spaces yet)."""
    rng = np.random.default_rng(base_seed + b)
    n_c = int(rng.integers(8, 33))
    N = int(rng.integers(16, 129))
    contrast = float(10 ** rng.uniform(4, 6))
    n = 10 * n_c
    kappa, _, _ = media.straight_channels(n, n_c, n_c // 4, n_c // 4, contrast, rng)
    pq = rng.integers(1, 5, size=(8, 2))
    a = rng.standard_normal(8)
    return dict(b=b, n_c=n_c, n=n, N=N, P=P_FINE, contrast=contrast, kappa=kappa, pq=pq, a=a)


_grids = {}


def mode_loads(n, pq):
    """Fine-grid load vectors (8 x (n-1)^2) of the modes sin(p pi x) sin(q pi y)
    (consistent mass times the nodal interpolant; the mass matrix does not
    depend on kappa, so one unit-coefficient grid per n serves every solve)."""
    if n not in _grids:
        _grids[n] = FineGrid(np.ones((n, n)))
    fine = _grids[n]
    return np.stack([fine.load_smooth(lambda x, y, p=p, q=q: np.sin(p * np.pi * x) * np.sin(q * np.pi * y))
                     for p, q in pq])


def amplitudes(spec):
    """Time amplitudes H (1 x 8 x N) of the source: a_m on every interval."""
    return np.repeat(spec["a"][None, :, None], spec["N"], axis=2)


def stable_step(M11, M12, M22, A22):
    """(lambda2, gamma2, dt_max) of the stability condition from device
    FP64 blocks (torch tensors): lambda2 = largest eigenvalue of
    L2^-1 A22 L2^-T, gamma2 = largest eigenvalue of Y Y^T with
    Y = L1^-1 M12 L2^-T (M11 = L1 L1^T, M22 = L2 L2^T). gamma2 is within about
    3e-5 of 1 for the CEM split, so it is taken from a dense symmetric
    eigensolver (not an iteration), which fixes it to rounding level."""
    import torch
    L1 = torch.linalg.cholesky(M11)
    L2 = torch.linalg.cholesky(M22)
    X = torch.linalg.solve_triangular(L2, A22, upper=False)
    C = torch.linalg.solve_triangular(L2, X.T.contiguous(), upper=False)
    C = 0.5 * (C + C.T)
    lam2 = float(torch.linalg.eigvalsh(C)[-1])
    Y = torch.linalg.solve_triangular(L1, M12, upper=False)          # L1^-1 M12
    Y = torch.linalg.solve_triangular(L2, Y.T.contiguous(), upper=False).T  # L1^-1 M12 L2^-T
    S = Y @ Y.T
    g2 = float(torch.linalg.eigvalsh(0.5 * (S + S.T))[-1])
    return lam2, g2, (1.0 - g2) / lam2


def gpu_problem(spec, device="cuda"):
    """Blocks (device tensors), source factors and step sizes of one solve,
    built by the library's GPU set-up pipeline."""
    import time

    import torch

    import paper_2411_09244_amd as pe
    t0 = time.perf_counter()
    loads = mode_loads(spec["n"], spec["pq"])
    t1 = time.perf_counter()
    out = pe.cem_spaces(spec["kappa"], None, spec["n_c"], LAYERS, J1_LOCAL, loads=loads, device=device,
                        J=J_LOCAL)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    lam2, g2, dt_max = stable_step(out["M11"], out["M12"], out["M22"], out["A22"])
    t3 = time.perf_counter()
    dt = 0.5 * dt_max
    prob = {k: out[k] for k in ("M11", "M12", "M22", "A11", "A12", "A22")}
    prob.update(G=out["G"], H=amplitudes(spec), time_mode=1, N=spec["N"], P=spec["P"], dt=dt,
                dt_fine=dt / spec["P"], d1=out["M11"].shape[0], d2=out["M22"].shape[0],
                diag=dict(lambda2=lam2, gamma2=g2, dt_max=dt_max),
                seconds=dict(loads=t1 - t0, spaces=t2 - t1, stable_step=t3 - t2))
    return prob


def cpu_problem(spec):
    """The same solve from the CPU generator (spaces, blocks, source
    factors; step sizes from its own diagnostics), with the local spectral
    data spsi and eigenvalues lam it used. On the elements of these media
    that hold no channel (kappa = 1) the local eigenvalues are multiple, so
    which functions of an eigenspace a solver returns, and with them the
    spaces, depend on the solver: the GPU pipeline reproduces the CPU
    generator's spaces when it is given the same spsi."""
    from .build import diagnostics, project_blocks
    from .cem import CoarseGrid, cem_basis, local_spectral, split_spaces
    fine = FineGrid(spec["kappa"])
    cg = CoarseGrid(fine, spec["n_c"])
    lam, _, spsi = local_spectral(cg, J_LOCAL)
    phis = cem_basis(cg, J_LOCAL, LAYERS, spsi)
    Psi1, Psi2 = split_spaces(cg, phis, J1_LOCAL, J_LOCAL - J1_LOCAL)
    bl = project_blocks(fine, Psi1, Psi2)
    loads = mode_loads(spec["n"], spec["pq"])
    G = np.concatenate([Psi1.T @ loads.T, Psi2.T @ loads.T])
    diag = diagnostics(bl, with_cond=False)
    dt = 0.5 * diag["dt_max"]
    prob = dict(bl)
    prob.update(G=G, H=amplitudes(spec), time_mode=1, N=spec["N"], P=spec["P"], dt=dt, dt_fine=dt / spec["P"],
                d1=Psi1.shape[1], d2=Psi2.shape[1], diag=diag, spsi=spsi, lam=lam)
    return prob
