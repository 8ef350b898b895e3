"""Property tests of the FP64 oracle on random small problems (hypothesis):
random grids of 2^3 to 6^3 cells, degree 0-2 and per-cell coefficients with
ratios up to 1e3, on the CPU. Each property is fixed by the mathematics of
the discretisation or of the method, not by the oracle's own formulas."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
import synth

SETTINGS = dict(max_examples=12, deadline=None, derandomize=True,
                suppress_health_check=[HealthCheck.too_slow])


@st.composite
def problems(draw):
    n = draw(st.sampled_from([2, 4, 6]))
    p = draw(st.integers(0, 2))
    seed = draw(st.integers(0, 2 ** 31 - 1))
    rng = np.random.default_rng(seed)
    nu = 10.0 ** rng.uniform(0.0, 3.0, n ** 3)
    levels = 2 if n % 2 == 0 else 1
    return synth.make_problem(n, p, n_levels=levels), nu, seed


@settings(**SETTINGS)
@given(problems())
def test_operator_spd_and_homogeneous(case):
    """A is symmetric positive definite; A(c nu) = c A(nu) exactly in exact
    arithmetic (every term carries one coefficient); the Galerkin coarse
    operator P^T A P is symmetric."""
    prob, nu, _ = case
    A = oracle.Oracle.from_sip(prob, nu).scipy_matrix(0).toarray()
    assert np.abs(A - A.T).max() <= 1e-12 * np.abs(A).max()
    assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() > 0.0
    A3 = oracle.Oracle.from_sip(prob, 3.0 * nu).scipy_matrix(0).toarray()
    assert np.abs(A3 - 3.0 * A).max() <= 1e-12 * np.abs(A3).max()
    if prob.n_levels > 1:
        Ac = oracle.Oracle.from_sip(prob, nu).scipy_matrix(1).toarray()
        assert np.abs(Ac - Ac.T).max() <= 1e-12 * np.abs(Ac).max()


@settings(**SETTINGS)
@given(problems(), st.sampled_from(["sync", "overlap", "hybrid"]))
def test_solve_properties(case, variant):
    """Every configuration stops with the recursive residual at 1e-10 (the
    stopping rule), the finest-level residual never increases, the recursive
    residual stays within 1e-10 ||b|| of the true one (rounding drift of the
    updates r -= alpha w), and x lies within kappa times the true relative
    residual of the dense solution."""
    prob, nu, seed = case
    o = oracle.Oracle.from_sip(prob, nu, variant=variant, s_pre=1, s_post=1)
    b = synth.rhs(prob.n_dofs, seed % 1000)
    x = o.solve(b)
    rep = o.last_report
    A = o.scipy_matrix(0).toarray()
    assert rep["rel_res_rec"] <= 1.0001e-10
    true = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    assert abs(true - rep["rel_res_rec"]) <= 1e-10
    rn = o.trace()[:, 1]
    assert np.all(rn[1:] <= rn[:-1] * (1 + 1e-14))
    xs = np.linalg.solve(A, b)
    ev = np.linalg.eigvalsh(A)
    kappa = ev.max() / ev.min()
    assert np.linalg.norm(x - xs) <= 1.1 * kappa * true * np.linalg.norm(xs)

