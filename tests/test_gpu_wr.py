"""GPU parity of the waveform-relaxation fine solver (pe_fine_wr, Sections 4.1
and 4.2) against the oracle's WR at equal iteration counts, and of its fixed
point against the sequential fine propagator.

Bar: both sides compute in FP64 by different algebraic routes (the oracle:
numpy's FFT and one complex LU per frequency; the GPU: a real transform
matrix and the real 2x2 block form of each complex inverse through an SPD
Schur complement). Both round at about kappa * eps * (1/alpha) with kappa
the condition number of the shifted blocks (the scaling alpha^(q/P) of the
transform is undone by its inverse, which amplifies rounding by up to
1/alpha); with kappa <= 1e5, eps = 1.1e-16 and alpha >= 0.01 that is
<= 1.1e-9, so the bar is 1e-9 relative (Euclidean over all columns)."""
import numpy as np
import pytest
import torch

import oracle.scheme as S
import oracle.wr as WR
from problem import build_problem

pytestmark = pytest.mark.gpu

TOL = 1e-9

RAGGED = dict(n=30, n_c=3, layers=1, J1=2, J2=3, medium="channels", n_h=1, n_v=1, contrast=1e5,
              seed=31, source="sine_exp", u0="sine2", N=5, P=7, T=None, B=1)
ELEM = dict(n=50, n_c=5, layers=2, J1=2, J2=3, medium="channels", n_h=1, n_v=1, contrast=1e5,
            seed=21, source="elem_interval", u0="zero", N=6, P=5, T=None, B=2, src_seed=21)
CFGS = {"ragged": RAGGED, "elem": ELEM}


def _pe():
    import paper_2411_09244_amd as pe
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return pe


def _setup(name, seed=0):
    p = build_problem(CFGS.get(name, name))
    bl, src = S.Blocks.from_problem(p), S.Source.from_problem(p)
    B = p["H"].shape[0] if p.get("H") is not None else 1
    X = np.random.default_rng(seed).standard_normal((B, bl.N, bl.D))
    return p, bl, src, B, X


def _oracle(bl, src, X, alpha, K0):
    B, N, D = X.shape
    cols = X.reshape(B * N, D).T
    ns = [c % N for c in range(B * N)]
    bs = [c // N for c in range(B * N)]
    out = WR.wr_fine_cols(bl, src, cols, ns, bs, alpha, K0)
    return out.T.reshape(B, N, D)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("name", ["c0", "t1", "ragged", "elem", "t2"])
@pytest.mark.parametrize("K0", [1, 3])
def test_wr_matches_oracle(name, K0):
    pe = _pe()
    p, bl, src, B, X = _setup(name)
    alpha = 0.05
    ref = _oracle(bl, src, X, alpha, K0)
    pr = pe.problem_from(p, "fp64", device="cuda:0")
    got = pr.fine_wr(X, alpha, K0).cpu().numpy()
    err = _rel(got, ref)
    print(f"{name} K0={K0}: rel err vs oracle WR {err:.3e}")
    assert err < TOL
    pr.close()


def test_wr_mixed_handle_runs_fp64():
    # the WR path is FP64 in the caller's coordinates whatever the handle's precision
    pe = _pe()
    p, bl, src, B, X = _setup("t1", seed=1)
    ref = _oracle(bl, src, X, 0.02, 2)
    pr = pe.problem_from(p, "mixed", device="cuda:0")
    got = pr.fine_wr(X, 0.02, 2).cpu().numpy()
    assert _rel(got, ref) < TOL
    pr.close()


@pytest.mark.parametrize("name", ["c0", "ragged"])
def test_wr_fixed_point_is_the_fine_propagator(name):
    pe = _pe()
    p, bl, src, B, X = _setup(name, seed=2)
    pr = pe.problem_from(p, "fp64", device="cuda:0")
    exact = pr.fine(torch.tensor(X, device="cuda:0")).cpu().numpy()
    cols = X.reshape(B * bl.N, bl.D).T
    ref = S.fine_propagator_cols(bl, src, cols, [c % bl.N for c in range(B * bl.N)],
                                 [c // bl.N for c in range(B * bl.N)]).T.reshape(B, bl.N, bl.D)
    got = pr.fine_wr(X, 0.01, 60).cpu().numpy()
    e1, e2 = _rel(got, ref), _rel(got, exact)
    print(f"{name}: WR(60) vs oracle F {e1:.3e}, vs GPU F {e2:.3e}")
    assert e1 < TOL and e2 < TOL
    pr.close()


def test_wr_d2_zero():
    # no V_H2 part: one WR iteration is the alpha-periodic backward Euler solve
    pe = _pe()
    from problem.fem import FineGrid
    n, P, N = 10, 6, 3
    rng = np.random.default_rng(7)
    fine = FineGrid(np.exp(2 * rng.standard_normal((n, n))))
    M, A = fine.M.toarray(), fine.A.toarray()
    d1 = M.shape[0]
    dt = 1e-2
    z = np.zeros((d1, 0))
    bl = S.Blocks(M, z, np.zeros((0, 0)), A, z, np.zeros((0, 0)), dt, dt / P, N)
    G = fine.load_smooth(lambda x, y: np.sin(np.pi * x) * y)[:, None]
    H = rng.standard_normal((1, 1, N))
    src = S.Source(G, H, S.TIME_INTERVAL, N, P)
    X = rng.standard_normal((1, N, d1))
    pr = pe.Problem(dict(M11=M, M12=z, M22=np.zeros((0, 0)), A11=A, A12=z, A22=np.zeros((0, 0))),
                    dt, dt / P, N, "fp64")
    pr.set_source(G, H, "interval")
    for K0 in (1, 4):
        ref = _oracle(bl, src, X, 0.1, K0)
        got = pr.fine_wr(X, 0.1, K0).cpu().numpy()
        assert _rel(got, ref) < TOL, K0
    pr.close()


def test_wr_graph_replay_bitwise():
    # iterations after the first replay a captured graph; with profiling on
    # every launch is eager: the results must agree bit for bit
    pe = _pe()
    p, bl, src, B, X = _setup("t2", seed=3)
    pr = pe.problem_from(p, "fp64", device="cuda:0")
    a = pr.fine_wr(X, 0.05, 4).cpu().numpy()
    b = pr.fine_wr(X, 0.05, 4).cpu().numpy()
    pr.profile(True)
    c = pr.fine_wr(X, 0.05, 4).cpu().numpy()
    prof = pr.profile_read()
    pr.profile(False)
    assert np.array_equal(a, b) and np.array_equal(a, c)
    assert prof["wr_solve"][1] == 4          # the P/2 + 1 frequency solves: one grouped launch
    assert prof["wr_wstep"][1] == 4 * bl.P
    pr.close()


def test_wr_alpha_change_and_zero_iterations():
    pe = _pe()
    p, bl, src, B, X = _setup("c0", seed=4)
    pr = pe.problem_from(p, "fp64", device="cuda:0")
    assert np.array_equal(pr.fine_wr(X, 0.3, 0).cpu().numpy(), X)
    for alpha in (0.3, 0.02, 0.3):
        ref = _oracle(bl, src, X, alpha, 2)
        assert _rel(pr.fine_wr(X, alpha, 2).cpu().numpy(), ref) < TOL, alpha
    pr.close()


def test_wr_errors():
    pe = _pe()
    p, bl, src, B, X = _setup("c0", seed=5)
    pr = pe.problem_from(p, "fp64", device="cuda:0")
    for alpha, K0 in ((0.0, 1), (1.0, 1), (-0.1, 1), (0.5, -1)):
        with pytest.raises(Exception):
            pr.fine_wr(X, alpha, K0)
    pt, blt, srct, Bt, Xt = _setup("t2", seed=5)
    prt = pe.problem_from(pt, "fp64", device="cuda:0")
    with pytest.raises(Exception):
        prt.fine_wr(Xt[:1], 0.1, 1)   # B differs from the source's B
    pr.close()
    prt.close()


def test_wr_full_size_sampled():
    # the 200x200 workload (d1 = 800, d2 = 1200, P = 64): all 64 intervals on the
    # GPU, two of them on the oracle
    pe = _pe()
    p = build_problem("c1")
    bl, src = S.Blocks.from_problem(p), S.Source.from_problem(p)
    X = np.random.default_rng(6).standard_normal((1, bl.N, bl.D))
    pr = pe.problem_from(p, "fp64", device="cuda:0")
    got = pr.fine_wr(X, 0.02, 2).cpu().numpy()
    for n in (0, 37):
        ref = WR.wr_fine(bl, src, X[0, n], n, 0.02, 2)
        err = _rel(got[0, n], ref)
        print(f"c1 interval {n}: rel err vs oracle WR {err:.3e}")
        assert err < TOL
    pr.close()


def test_parareal_with_wr_fine_solver():
    # Algorithm 1 with the paper's fine solver: iterates against the oracle's
    # parareal with F = K0 WR iterations, the limit at k = N against the
    # sequential WR composition, then back to the scheme's F
    pe = _pe()
    p = build_problem("t1")
    bl, src = S.Blocks.from_problem(p), S.Source.from_problem(p)
    x0 = p["x0"][0]
    pr = pe.problem_from(p, "fp64", device="cuda:0")
    pr.set_fine_solver("wr", 0.05, 3)
    X, iters, hist, st = pr.solve(p["x0"], tol=0.0, k_max=3)
    ref = WR.parareal_wr(bl, src, x0, 0.0, 0.05, 3, k_max=3)
    e3 = S.rel_l2_M(bl, X[0].cpu().numpy(), ref["X"][3])
    ej = np.max(np.abs(hist[0, :3] - ref["J"][:3]) / np.abs(ref["J"][:3]))
    X, iters, hist, st = pr.solve(p["x0"], tol=0.0, k_max=bl.N)
    eN = S.rel_l2_M(bl, X[0].cpu().numpy(), WR.wr_composition(bl, src, x0, 0.05, 3))
    pr.set_fine_solver("step")
    X, iters, hist, st = pr.solve(p["x0"], tol=0.0, k_max=3)
    es = S.rel_l2_M(bl, X[0].cpu().numpy(), S.parareal(bl, src, x0, 0.0, k_max=3)["X"][3])
    print(f"parareal with WR: k=3 {e3:.3e} (jumps {ej:.3e}), k=N vs WR composition {eN:.3e}; scheme F {es:.3e}")
    assert e3 < TOL and ej < 1e-8 and eN < TOL and es < 1e-10
    pr.close()


def test_set_fine_solver_errors():
    pe = _pe()
    p = build_problem("t1")
    pm = pe.problem_from(p, "mixed", device="cuda:0")
    with pytest.raises(Exception):
        pm.set_fine_solver("wr", 0.05, 2)          # FP64 handles only
    pm.close()
    pr = pe.problem_from(p, "fp64", device="cuda:0")
    for alpha, K0 in ((0.0, 2), (1.5, 2), (0.1, 0)):
        with pytest.raises(Exception):
            pr.set_fine_solver("wr", alpha, K0)
    pr.close()


def test_wr_converges_fast_on_nlmc_spaces():
    # with the NLMC fracture/matrix split gamma^2 = 0.23 (Section 3.2): WR
    # reaches the sequential F to rounding within 25 iterations, and its error
    # after 1..6 iterations contracts at about gamma^2 or faster
    pe = _pe()
    p, bl, src, B, X = _setup("t1n", seed=9)
    pr = pe.problem_from(p, "fp64", device="cuda:0")
    exact = pr.fine(torch.tensor(X, device="cuda:0")).cpu().numpy()
    errs = [_rel(pr.fine_wr(X, 0.05, k).cpu().numpy(), exact) for k in range(1, 7)]
    final = _rel(pr.fine_wr(X, 0.05, 25).cpu().numpy(), exact)
    print("t1n WR errors", " ".join(f"{e:.2e}" for e in errs), f"K0=25: {final:.2e}")
    assert final < TOL
    g2 = WR.gamma_sq(bl)
    assert errs[-1] <= errs[0] * (1.5 * g2) ** 5
    pr.close()
