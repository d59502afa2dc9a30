"""GPU parity of the history-carrying mode (pe_set_history(PE_HIST_CARRY)):
states [x; delta] with delta the change over the last fine step, against
the oracle's carrying propagators and parareal on the same seeded inputs.
Bars: FP64 path 1e-10 relative (M-norm), mixed path 1e-6 for x; the carried
change delta is measured against its own scale (FP64 1e-10, mixed 1e-5: it
is one step's increment, a difference of two states, so the FP32 rounding
of the state is a larger fraction of it); the coarse step is FP64 in both
paths (1e-12)."""
import numpy as np
import pytest
import torch

import oracle.scheme as S
from problem import build_problem

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOLMIX = 1e-6
TOLMIX_DELTA = 1e-5

RAGGED = dict(n=30, n_c=3, layers=1, J1=2, J2=3, medium="channels", n_h=1, n_v=1, contrast=1e5,
              seed=31, source="sine_exp", u0="sine2", N=5, P=7, T=None, B=1)


def _pe():
    import paper_2411_09244_amd as pe
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return pe


def _prob(name):
    return build_problem(RAGGED if name == "ragged" else name)


def _carry_problem(pe, p, prec):
    pr = pe.problem_from(p, prec)
    pr.set_history("carry")
    return pr


def _rel_parts(bl, Y, Yref):
    """(x error, delta error): max over rows of |.|_M of the difference over
    the max |.|_M of the reference rows, for the x and delta halves."""
    D = bl.D
    out = []
    for sl in (slice(0, D), slice(D, 2 * D)):
        scale = max(S.m_norm(bl, y[sl]) for y in Yref) or 1.0
        out.append(max(S.m_norm(bl, a[sl] - b[sl]) for a, b in zip(Y, Yref)) / scale)
    return out


def _random_carry_states(p, seed, B, N):
    rng = np.random.default_rng(seed)
    D = p["d1"] + p["d2"]
    x = 1e-3 * rng.standard_normal((B, N, D))
    d = 1e-5 * rng.standard_normal((B, N, D))
    return np.concatenate([x, d], axis=2)


@pytest.mark.parametrize("name", ["t0", "t1", "c0", "t2", "ragged"])
@pytest.mark.parametrize("prec,tol,tol_d", [("fp64", TOL64, TOL64), ("mixed", TOLMIX, TOLMIX_DELTA)])
def test_fine_propagator_carry(name, prec, tol, tol_d):
    pe = _pe()
    p = _prob(name)
    bl, src = S.Blocks.from_problem(p), S.Source.from_problem(p)
    B, N = p["B"], p["N"]
    Yin = _random_carry_states(p, 3, B, N)
    pr = _carry_problem(pe, p, prec)
    Y = pr.fine(Yin).cpu().numpy()
    assert Y.shape == (B, N, 2 * bl.D)
    for b in range(B):
        ref = np.stack([S.fine_propagator_carry(bl, src, Yin[b, n], n, b) for n in range(N)])
        ex, ed = _rel_parts(bl, Y[b], ref)
        print(f"{name} {prec} b={b}: F carry x {ex:.3e} delta {ed:.3e}")
        assert ex < tol and ed < tol_d, (name, prec, b, ex, ed)


@pytest.mark.parametrize("name", ["t0", "t1", "c0", "t2", "ragged"])
def test_coarse_propagator_carry(name):
    pe = _pe()
    p = _prob(name)
    bl, src = S.Blocks.from_problem(p), S.Source.from_problem(p)
    B, N = p["B"], p["N"]
    Yin = _random_carry_states(p, 2, B, N)
    for prec in ("fp64", "mixed"):
        pr = _carry_problem(pe, p, prec)
        Y = pr.coarse(Yin).cpu().numpy()
        for b in range(B):
            ref = np.stack([S.coarse_propagator_carry(bl, src, Yin[b, n], n, b) for n in range(N)])
            ex, ed = _rel_parts(bl, Y[b], ref)
            assert ex < 1e-12 and ed < 1e-12, (name, prec, b, ex, ed)


@pytest.mark.parametrize("name", ["t0", "t1", "c0", "t2", "ragged"])
@pytest.mark.parametrize("prec,tol,tol_d", [("fp64", TOL64, TOL64), ("mixed", TOLMIX, TOLMIX_DELTA)])
def test_solve_carry_equal_iteration(name, prec, tol, tol_d):
    """GPU iterate k vs the oracle's carrying parareal at iteration k."""
    pe = _pe()
    p = _prob(name)
    bl, src = S.Blocks.from_problem(p), S.Source.from_problem(p)
    k = min(3, p["N"])
    pr = _carry_problem(pe, p, prec)
    X, iters, hist, st = pr.solve(p["x0"], tol=0.0, k_max=k)
    X = X.cpu().numpy()
    assert X.shape == (p["B"], p["N"] + 1, 2 * bl.D)
    assert (iters == k).all()
    for b in range(p["B"]):
        r = S.parareal_carry(bl, src, p["x0"][b], 0.0, k_max=k, b=b)
        ex, ed = _rel_parts(bl, X[b], r["X"][k])
        print(f"{name} {prec} b={b}: parareal carry k={k} x {ex:.3e} delta {ed:.3e}")
        assert ex < tol and ed < tol_d, (name, prec, b, ex, ed)
        scale = max(S.m_norm(bl, x[:bl.D]) for x in r["X"][k])
        assert np.abs(hist[b] - r["J"]).max() <= tol * scale, (hist[b], r["J"])


@pytest.mark.parametrize("name", ["t1", "c0"])
def test_solve_carry_ends_at_uninterrupted_run(name):
    """k = N reproduces one run of N*P fine steps without restarts."""
    pe = _pe()
    p = _prob(name)
    bl, src = S.Blocks.from_problem(p), S.Source.from_problem(p)
    run = S.sequential_run(bl, src, p["x0"][0])
    pr = _carry_problem(pe, p, "fp64")
    X, iters, hist, st = pr.solve(p["x0"], tol=0.0, k_max=p["N"])
    ex, ed = _rel_parts(bl, X[0].cpu().numpy(), run)
    print(f"{name}: parareal carry at k = N vs uninterrupted run x {ex:.3e} delta {ed:.3e}")
    assert ex < TOL64 and ed < TOL64


@pytest.mark.parametrize("name,tol", [("t1", 1e-3), ("c0", 1e-4), ("t2", 1e-3)])
def test_carry_stopping_test_iterations_match_oracle(name, tol):
    """Same iteration count as the oracle under the relative stopping test
    (tolerances at which the carried-history iteration stops before k = N)."""
    pe = _pe()
    p = _prob(name)
    bl, src = S.Blocks.from_problem(p), S.Source.from_problem(p)
    refs = [S.parareal_carry(bl, src, p["x0"][b], tol, b=b, rel=True) for b in range(p["B"])]
    assert all(r["J"][-1] <= r["threshold"] for r in refs)
    for prec in ("fp64", "mixed"):
        pr = _carry_problem(pe, p, prec)
        X, iters, hist, st = pr.solve(p["x0"], tol=tol, norm="rel")
        assert st == 0
        for b, r in enumerate(refs):
            assert iters[b] == r["K"], (prec, b, iters[b], r["K"], hist[b])
            ex, _ = _rel_parts(bl, X[b].cpu().numpy(), r["X"][r["K"]])
            assert ex < (TOL64 if prec == "fp64" else TOLMIX), (prec, b, ex)


def test_mode_switch_keeps_the_restarting_path():
    """restart -> carry -> restart on one handle: the restarting results are
    bitwise unchanged (the workspace is regrown with the state stride)."""
    pe = _pe()
    p = _prob("t2")
    for prec in ("fp64", "mixed"):
        pr = pe.problem_from(p, prec)
        X1 = pr.solve(p["x0"], tol=0.0, k_max=3)[0].clone()
        pr.set_history("carry")
        Xc = pr.solve(p["x0"], tol=0.0, k_max=3)[0]
        assert Xc.shape[-1] == 2 * X1.shape[-1]
        pr.set_history("restart")
        X2 = pr.solve(p["x0"], tol=0.0, k_max=3)[0]
        assert torch.equal(X1, X2), prec


def test_carry_unsupported_calls_refuse():
    pe = _pe()
    from paper_2411_09244_amd import _lib
    p = _prob("t1")
    pr = _carry_problem(pe, p, "fp64")
    D, N = pr.D, pr.N
    with pytest.raises(pe.PeError) as ei:
        pr.adjoint(Xbar=np.zeros((1, N + 1, D)))
    assert ei.value.status == _lib.PE_ERR_STATE
    with pytest.raises(pe.PeError) as ei:
        pr.fine_wr(np.zeros((1, N, D)), 0.05, 2)
    assert ei.value.status == _lib.PE_ERR_STATE
    with pytest.raises(pe.PeError) as ei:
        pr.set_fine_solver("wr", 0.05, 2)
    assert ei.value.status == _lib.PE_ERR_STATE
    with pytest.raises(pe.PeError) as ei:
        pe.Batch([pr])
    assert ei.value.status == _lib.PE_ERR_STATE
