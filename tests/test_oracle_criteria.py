"""Pins of the oracle's level-local stopping rules (Sec. 4.2), of its
nonzero-initial-guess path, of its breakdown rule and of the visit structure
of the multiplicative cycle (Algorithm 2), all read from the per-visit
residual log (level, iterations, ||r0||, ||r|| after each iteration)."""
import numpy as np
import pytest

import oracle
import synth


def sip(n, p, n_levels=None, nu=None, **opts):
    prob = synth.make_problem(n, p, n_levels=n_levels)
    if nu is None:
        nu = synth.nu_sphere(n, n, n, prob.h)
    return prob, nu, oracle.Oracle.from_sip(prob, nu, **opts)


def check_rule(log, crit, n_levels, tol, bn):
    """Every visit ended at the FIRST iteration whose residual met its level's
    test, or at the iteration cap: level 0 at ||r|| <= tol ||b||; level l >= 1
    at ||r|| <= rel_l ||r0|| or after max_l iterations (Sec. 4.2)."""
    for l, it, r0, rns in log:
        assert 0 <= l < n_levels - 1
        assert it == len(rns) and it >= 1
        if l == 0:
            hit = rns <= tol * bn
            assert hit[-1], "the finest level ended without meeting the tolerance"
            assert not hit[:-1].any(), "the finest level went on after meeting the tolerance"
            continue
        rel, mx = crit[l - 1]
        hit = (rns <= rel * r0) if rel >= 0 else np.zeros(it, bool)
        assert it <= mx
        assert not hit[:-1].any(), f"level {l} went on after ||r|| <= {rel} ||r0||"
        assert hit[-1] or it == mx, f"level {l} stopped early"


def check_tree(visits, n_levels):
    """Completion-order visit log of Algorithm 2: a level-l visit with `it`
    iterations is preceded by exactly `it` complete level-(l+1) visits (one
    coarse-grid correction per iteration) unless l+1 is the coarsest level."""
    pos = [len(visits) - 1]

    def parse(level):
        l, it = visits[pos[0]]
        assert l == level
        pos[0] -= 1
        if level + 1 < n_levels - 1:
            for _ in range(it):
                parse(level + 1)

    parse(0)
    assert pos[0] == -1


DEFAULT = [(0.1, 20), (0.5, 2)] + [(-1.0, 1)] * 14


def test_sec42_default_rule_every_visit():
    """Four levels: level 1 stops at 0.1 ||r0|| or 20 iterations, level 2 at
    0.5 ||r0|| or 2, the finest level at the tolerance; swapping any two
    thresholds or caps breaks one of the checks (both kinds of exit occur)."""
    prob, nu, o = sip(16, 1, n_levels=4)
    b = synth.rhs(prob.n_dofs, 0)
    o.solve(b, tol=1e-10)
    log = o.visit_norms()
    check_rule(log, DEFAULT, 4, 1e-10, np.linalg.norm(b))
    check_tree(o.visits(), 4)
    lv1 = [(it, rns[-1] / r0) for l, it, r0, rns in log if l == 1]
    lv2 = [(it, rns[-1] / r0) for l, it, r0, rns in log if l == 2]
    # both exits of each level's test are taken somewhere in this solve
    assert any(it == 20 for it, _ in lv1) or any(q <= 0.1 for _, q in lv1)
    assert any(it < 2 for it, q in lv2) and any(it == 2 for it, q in lv2)
    # level-2 visits that used both iterations did not reach 0.5 after the first
    assert all(q <= 0.5 for it, q in lv2 if it == 1)


def test_sec42_custom_rule_is_followed():
    """The thresholds are options: with level 1 at (0.5, 3) and level 2 at
    (0.1, 5) every visit follows those instead."""
    crit = [(0.5, 3), (0.1, 5)] + [(-1.0, 1)] * 14
    prob, nu, o = sip(16, 1, n_levels=4, crit=crit)
    b = synth.rhs(prob.n_dofs, 0)
    o.solve(b, tol=1e-10)
    check_rule(o.visit_norms(), crit, 4, 1e-10, np.linalg.norm(b))
    check_tree(o.visits(), 4)


def test_deeper_levels_take_one_iteration():
    prob, nu, o = sip(16, 1, n_levels=5)
    b = synth.rhs(prob.n_dofs, 0)
    o.solve(b, tol=1e-10)
    log = o.visit_norms()
    check_rule(log, DEFAULT, 5, 1e-10, np.linalg.norm(b))
    assert all(it == 1 for l, it, _, _ in log if l == 3)
    check_tree(o.visits(), 5)


def test_logged_norms_are_residual_norms():
    """The finest level's logged norms are the residual after each cycle: the
    residual trace at every third RM (end of an Algorithm 2 cycle), starting
    from ||b||, and the final one is the reported recursive residual."""
    prob, nu, o = sip(8, 1, n_levels=3)
    b = synth.rhs(prob.n_dofs, 3)
    o.solve(b, tol=1e-10)
    (l, it, r0, rns), = [v for v in o.visit_norms() if v[0] == 0]
    tr = o.trace()
    assert r0 == tr[0, 1] and r0 == pytest.approx(np.linalg.norm(b), rel=1e-14)
    ends = tr[1:1 + 3 * it, 1][2::3]
    assert np.array_equal(ends, rns)
    assert rns[-1] / r0 == pytest.approx(o.last_report["rel_res_rec"], rel=1e-15)
    lv1 = [v for v in o.visit_norms() if v[0] == 1]
    assert len(lv1) == it and all(v[2] > 0 for v in lv1)


def test_nonzero_initial_guess():
    """x0 != 0: the solve stops at ||b - A x|| <= tol ||b|| (not relative to
    ||b - A x0||). From x0 = the dense solution it takes no cycle and returns
    x0; from x0 = x* + d with ||A d|| = 100 tol ||b|| it needs only the
    reduction by 100 (a few cycles), reaches the tolerance and is not driven
    far below it."""
    prob, nu, o = sip(8, 1, n_levels=2)
    A = o.scipy_matrix().toarray()
    b = synth.rhs(prob.n_dofs, 0)
    xs = np.linalg.solve(A, b)
    bn = np.linalg.norm(b)
    x = o.solve(b, x0=xs, tol=1e-10)
    assert o.last_report["iters_fine"] == 0
    assert np.array_equal(x, xs)
    d = np.random.default_rng(4).standard_normal(prob.n_dofs)
    d *= 100 * 1e-10 * bn / np.linalg.norm(A @ d)
    x = o.solve(b, x0=xs + d, tol=1e-10)
    it_x0 = o.last_report["iters_fine"]
    rt = np.linalg.norm(b - A @ x) / bn
    assert rt <= 1.0001e-10 and rt >= 1e-13
    o.solve(b, tol=1e-10)
    it_0 = o.last_report["iters_fine"]
    assert 1 <= it_x0 <= it_0 // 2


def test_breakdown_keeps_zero_slots():
    """A direction whose orthogonalised w falls to `breakdown` times its start
    is dropped: W and Z hold a zero vector in its slot, the residual does not
    change at that RM, the slot counts as a stored direction (three per
    Algorithm 2 cycle on the finest level) and the kept directions stay
    orthonormal."""
    prob, nu, o = sip(8, 1, n_levels=2, breakdown=0.35, max_iter=400)
    b = synth.rhs(prob.n_dofs, 0)
    o.solve(b, tol=1e-8, check=False)
    rep = o.last_report
    assert rep["n_breakdowns"] > 0
    assert rep["n_dirs_fine"] == 3 * rep["iters_fine"]
    W, Z = o.dirs(0)
    zero = np.all(W == 0, axis=1)
    assert zero.sum() >= 1 and np.all(Z[zero] == 0)
    Wk = W[~zero]
    assert np.abs(Wk @ Wk.T - np.eye(len(Wk))).max() < 1e-12
    tr = o.trace()[:, 1]
    steps = np.flatnonzero(zero) + 1          # trace entry after the RM of slot j
    assert np.all(tr[steps] == tr[steps - 1])
    assert np.all(tr[1:] <= tr[:-1] * (1 + 1e-14))


def test_breakdown_counts_toward_m_max():
    """With m_max restarts a dropped slot counts like a kept one: after R RMs
    on the finest level the level holds ((R - 1) mod m_max) + 1 slots."""
    m = 7
    prob, nu, o = sip(8, 1, n_levels=2, breakdown=0.35, m_max=m, max_iter=400)
    b = synth.rhs(prob.n_dofs, 0)
    o.solve(b, tol=1e-8, check=False)
    rep = o.last_report
    assert rep["n_breakdowns"] > 0
    R = 3 * rep["iters_fine"]
    assert rep["n_dirs_fine"] == (R - 1) % m + 1


def test_restarted_cycle_amplifies_rounding():
    """With m_max = 5 on 8^3 P2 (three levels) the restarted K-cycle is
    sensitive: perturbing b by 1e-15 relative changes the finest level's
    residual history by far more than 1e-15 within 50 cycles and the cycle
    count by several, while the converged solutions still agree to 1e-9.
    (This is why two correct implementations with different summation orders
    take different cycle counts on this case.) Without restarts the same
    perturbation stays at rounding level."""
    prob = synth.make_problem(8, 2, n_levels=3)
    nu = synth.nu_sphere(8, 8, 8, prob.h)
    b = synth.rhs(prob.n_dofs, 0)
    bp = b * (1 + 1e-15 * np.random.default_rng(5).standard_normal(len(b)))
    runs = []
    for mm in (5, 0):
        for bb in (b, bp):
            o = oracle.Oracle.from_sip(prob, nu, s_post=2, m_max=mm, max_iter=2000)
            x = o.solve(bb)
            (_, it, r0, rns), = [v for v in o.visit_norms() if v[0] == 0]
            runs.append((x, it, rns / r0))
    (x1, it1, q1), (x2, it2, q2), (x3, it3, q3), (x4, it4, q4) = runs
    n = min(len(q1), len(q2))
    assert np.abs(q2[:n] / q1[:n] - 1).max() > 1e-3 and it1 != it2
    assert np.linalg.norm(x2 - x1) <= 1e-9 * np.linalg.norm(x1)
    assert it3 == it4 and np.abs(q4 / q3 - 1).max() < 1e-5
