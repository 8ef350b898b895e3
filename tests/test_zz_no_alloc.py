"""The allocation-free RM step (omg_rm_step_noalloc: caller arrays, the
library's fixed device scratch) against the existing RM step entry point
(omg_level_rm_step, the level's own storage) and the sequential MGS step in
numpy, on two calls in a row, the second with fewer entries and
directions, and with a dropped (broken-down) direction; sizes beyond the
scratch are rejected."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def omg():
    import paper_2512_08728_amd as m
    return m


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def reference(W, w, r):
    w = w.copy()
    betas = []
    for Wi in W:
        b = Wi @ w
        betas.append(b)
        w -= b * Wi
    gamma = 1.0 / np.linalg.norm(w)
    wk = gamma * w
    alpha = wk @ r
    return np.array(betas), gamma, wk, alpha, r - alpha * wk


def solver(n, p):
    prob = synth.make_problem(n, p, n_levels=2)
    nu = synth.nu_sphere(n, n, n, prob.h)
    return prob, omg().Solver.from_sip(omg().Solver.make_grid(n, n, n, p, 2, prob.h), dev(nu))


def check_same(a, b, w, r, what):
    (Wk1, rn1, b1, g1, al1), (Wk2, rn2, b2, g2, al2) = a, b
    assert np.abs(b1 - b2).max(initial=0) <= 1e-12 * np.abs(w).max(), what
    assert abs(g1 - g2) <= 1e-12 * abs(g2), what
    assert abs(al1 - al2) <= 1e-12 * np.linalg.norm(r), what
    assert (Wk1 - Wk2).abs().max().item() <= 1e-12, what
    assert (rn1 - rn2).abs().max().item() <= 1e-12 * np.abs(r).max(), what


def test_noalloc_step_matches_level_step_twice():
    m = omg()
    rng = np.random.default_rng(41)
    # first call: 16^3 P2 (40,960 entries) with 40 directions; second: 8^3 P1
    # (2,048 entries) with 5 directions, on the scratch the first call left
    for (n, p, k) in ((16, 2, 40), (8, 1, 5)):
        prob, g = solver(n, p)
        N = prob.n_dofs
        W = np.linalg.qr(rng.standard_normal((N, k)))[0].T.copy()
        w, z, r = (rng.standard_normal(N) for _ in range(3))
        Wd, wd, zd, rd = dev(W), dev(w), dev(z), dev(r)
        a = m.rm_step_noalloc(Wd, wd, zd, rd)
        b = g.rm_step(0, Wd, wd, zd, rd)
        check_same(a, b, w, r, f"{n}^3 P{p} k={k}")
        betas, gamma, wk, alpha, rn = reference(W, w, r)
        assert np.abs(a[2] - betas).max() <= 1e-12 * np.abs(w).max()
        assert abs(a[3] - gamma) <= 1e-12 * gamma and abs(a[4] - alpha) <= 1e-12 * np.linalg.norm(r)
        assert np.abs(a[0].cpu().numpy() - wk).max() <= 1e-12
        assert np.abs(a[1].cpu().numpy() - rn).max() <= 1e-12 * np.abs(r).max()
        assert torch.equal(rd, dev(r))  # r is not written when r_new is another array


def test_noalloc_breakdown_in_place_and_limits():
    m = omg()
    rng = np.random.default_rng(42)
    N, k = 3000, 6   # not a multiple of any grid: a ragged tail
    W = np.linalg.qr(rng.standard_normal((N, k)))[0].T.copy()
    w = W[2].copy()
    z, r = rng.standard_normal(N), rng.standard_normal(N)
    rd = dev(r)
    Wk, rn, betas, gamma, alpha = m.rm_step_noalloc(dev(W), dev(w), dev(z), rd, r_new=rd)
    assert gamma == 0.0 and alpha == 0.0 and not torch.any(Wk != 0)
    assert np.array_equal(rd.cpu().numpy(), r)
    ref = reference(W, w, r)[0]
    assert np.abs(betas - ref).max() <= 1e-12
    x = dev(np.ones(8))
    for kk, NN in ((257, 8), (1, 5242881)):   # beyond the scratch: rejected before any launch
        with pytest.raises(m.OmgError) as e:
            st = m.lib().omg_rm_step_noalloc(NN, kk, m._ptr(x), m._ptr(x), m._ptr(x), m._ptr(x), 1e-14,
                                             m._stream(), m._ptr(x), m._ptr(x), np.zeros(300).ctypes.data)
            m._check(st, "rm_step_noalloc")
        assert e.value.status == m.EINVAL
