"""Pins for the oracle's history-carrying propagators (the reading in which
the two-step scheme (2.4)-(2.5) keeps its previous-step differences across
interval starts instead of restarting them).

What fixes them independently of their own code:
  * the uninterrupted run of N*P steps equals one space-time solve of the
    same equations over all N*P levels (a sparse all-at-once system), and
    the fine composition with carried history equals that run;
  * with no history (delta = 0) the carrying propagators reduce to the
    restarting ones, and the coarse step never reads the carried change;
  * P = 1 and delta = 0: fine and coarse propagator are the same step;
  * parareal with carried history is exact at n <= k and ends at the fine
    composition, i.e. at the uninterrupted run, which the restarting
    parareal does not reach when M12 != 0;
  * the Galerkin steady state with zero rate is a fixed point of both.
A planted error in the carried history is caught (last test)."""
import numpy as np
import pytest

import oracle.scheme as S
from problem import build_problem
from test_oracle_pins import _all_at_once


def _prob(name="t1"):
    p = build_problem(name)
    return p, S.Blocks.from_problem(p), S.Source.from_problem(p)


def _rand_state(bl, seed, scale_delta=1e-2):
    rng = np.random.default_rng(seed)
    y = np.concatenate([rng.standard_normal(bl.D), scale_delta * rng.standard_normal(bl.D)])
    return y


def test_uninterrupted_run_equals_space_time_solve():
    p, bl, src = _prob("t1")
    x0 = p["x0"][0] + 0.01 * np.random.default_rng(5).standard_normal(bl.D)
    NP = bl.N * bl.P
    X = _all_at_once(bl, x0, lambda m: src.at_fine(0, m // bl.P, m % bl.P), bl.dt_fine, NP)
    run = S.sequential_run(bl, src, x0)
    scale = np.abs(X).max()
    for n in range(1, bl.N + 1):
        m = n * bl.P - 1            # level n*P is row m of X (levels 1..NP)
        np.testing.assert_allclose(run[n, :bl.D], X[m], rtol=0, atol=1e-10 * scale)
        prev = X[m - 1] if m >= 1 else x0
        np.testing.assert_allclose(run[n, bl.D:], X[m] - prev, rtol=0, atol=1e-10 * scale)


@pytest.mark.parametrize("name", ["t0", "t1", "c0"])
def test_carry_composition_is_uninterrupted_run(name):
    p, bl, src = _prob(name)
    x0 = p["x0"][0] + 0.01 * np.random.default_rng(6).standard_normal(bl.D)
    Y = S.fine_composition_carry(bl, src, x0)
    run = S.sequential_run(bl, src, x0)
    np.testing.assert_allclose(Y, run, rtol=0, atol=1e-12 * np.abs(run).max())


def test_zero_history_reduces_to_restart():
    p, bl, src = _prob("t1")
    y = _rand_state(bl, 7)
    y[bl.D:] = 0.0
    for n in (0, 3):
        f = S.fine_propagator_carry(bl, src, y, n)
        np.testing.assert_allclose(f[:bl.D], S.fine_propagator(bl, src, y[:bl.D], n), rtol=1e-13, atol=1e-14)
        g = S.coarse_propagator_carry(bl, src, y, n)
        g0 = S.coarse_propagator(bl, src, y[:bl.D], n)
        np.testing.assert_allclose(g[:bl.D], g0, rtol=1e-13, atol=1e-14)
        np.testing.assert_allclose(g[bl.D:], (g0 - y[:bl.D]) / bl.P, rtol=1e-13, atol=1e-14)


def test_coarse_step_ignores_the_carried_change():
    """G starts with a fresh history: its x part is the restarting G for any
    carried change, its delta part that step's change at the fine-step
    rate."""
    p, bl, src = _prob("t1")
    y = _rand_state(bl, 8)
    for n in (1, 6):
        g = S.coarse_propagator_carry(bl, src, y, n)
        g0 = S.coarse_propagator(bl, src, y[:bl.D], n)
        np.testing.assert_allclose(g[:bl.D], g0, rtol=1e-13, atol=1e-14)
        np.testing.assert_allclose(g[bl.D:], (g0 - y[:bl.D]) / bl.P, rtol=1e-13, atol=1e-14)
    # the fine propagator does read it (M12 != 0 in this space)
    z = np.concatenate([y[:bl.D], np.zeros(bl.D)])
    f, f0 = S.fine_propagator_carry(bl, src, y, 2), S.fine_propagator_carry(bl, src, z, 2)
    assert np.abs(f[:bl.D] - f0[:bl.D]).max() > 1e-6 * np.abs(f[:bl.D]).max()


def test_p1_fine_equals_coarse():
    p, bl, _ = _prob("t1")
    bl1 = S.Blocks(p["M11"], p["M12"], p["M22"], p["A11"], p["A12"], p["A22"], p["dt"], p["dt"], bl.N)
    src = S.Source(p["G"], p["H"][:, :, ::bl.P] if p["time_mode"] == S.TIME_FINE else p["H"],
                   p["time_mode"], bl.N, 1)
    y = _rand_state(bl1, 9)
    y[bl1.D:] = 0.0
    for n in (0, 5):
        np.testing.assert_allclose(S.fine_propagator_carry(bl1, src, y, n), S.coarse_propagator_carry(bl1, src, y, n),
                                   rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("name", ["t0", "t1", "c0"])
def test_parareal_carry_exact_and_ends_at_uninterrupted_run(name):
    p, bl, src = _prob(name)
    x0 = p["x0"][0]
    run = S.sequential_run(bl, src, x0)
    out = S.parareal_carry(bl, src, x0, tol=0.0, k_max=bl.N)
    scale = np.abs(run).max()
    for k, Yk in enumerate(out["X"]):
        np.testing.assert_allclose(Yk[:k + 1], run[:k + 1], rtol=0, atol=1e-11 * scale)
    np.testing.assert_allclose(out["X"][-1], run, rtol=0, atol=1e-11 * scale)
    # the restarting parareal ends elsewhere: the restart changes the solution
    r0 = S.parareal(bl, src, x0, tol=0.0, k_max=bl.N)["X"][-1]
    assert np.abs(r0[-1] - run[-1, :bl.D]).max() > 1e-8 * scale


def test_steady_state_with_zero_rate_is_fixed():
    p, bl, _ = _prob("t1")
    rng = np.random.default_rng(10)
    Fc = rng.standard_normal(bl.D)
    A = np.block([[bl.A11, bl.A12], [bl.A12.T, bl.A22]])
    xs = np.linalg.solve(A, Fc)
    src = S.Source(Fc[:, None], np.ones((1, 1, bl.N * bl.P)), S.TIME_FINE, bl.N, bl.P)
    y = np.concatenate([xs, np.zeros(bl.D)])
    for fn in (S.fine_propagator_carry, S.coarse_propagator_carry):
        out = fn(bl, src, y, 2)
        np.testing.assert_allclose(out[:bl.D], xs, rtol=0, atol=1e-9 * np.abs(xs).max())
        assert np.abs(out[bl.D:]).max() < 1e-9 * np.abs(xs).max()


def test_planted_history_error_is_caught(monkeypatch):
    """Starting the fine propagator from x_prev = x + delta (sign flip) must
    break the uninterrupted-run pin."""
    p, bl, src = _prob("t1")
    orig = S.fine_propagator_carry

    def wrong(bl_, src_, y, n, b=0):
        z = y.copy()
        z[bl_.D:] *= -1.0
        return orig(bl_, src_, z, n, b)

    monkeypatch.setattr(S, "fine_propagator_carry", wrong)
    x0 = p["x0"][0]
    Y = S.fine_composition_carry(bl, src, x0)
    run = S.sequential_run(bl, src, x0)
    assert np.abs(Y - run).max() > 1e-8 * np.abs(run).max()
