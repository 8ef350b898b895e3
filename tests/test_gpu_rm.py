"""The persistent residual-minimisation kernel (Algorithm 1 after w = A z) in
every co-resident launch configuration (entries per thread, directions per
grid exchange, exchange form, exchange wave, lag, grid) against the
sequential modified Gram-Schmidt step written out in numpy (FP64): MGS
coefficients beta_i = W_i . w (w updated after each), gamma = 1/||w||, the
new direction gamma w, alpha = w_k . r and the updated residual. k covers no
direction, fewer directions than one exchange block, partial last blocks,
and (on the smallest level) more directions than the kernel's pointer table
holds at once. The
exchange-wave form with four compute waves sums in the same order as the
plain form, so the two are compared bit for bit."""
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


@pytest.mark.parametrize("n,p", [(8, 1), (16, 2)])
def test_rm_step_every_configuration(n, p):
    prob = synth.make_problem(n, p, n_levels=2)
    nu = synth.nu_sphere(n, n, n, prob.h)
    g = omg().Solver.from_sip(omg().Solver.make_grid(n, n, n, p, 2, prob.h), torch.tensor(nu, device="cuda"))
    N = prob.n_dofs
    rng = np.random.default_rng(7)
    configs = g.rm_configs(0)
    assert configs, "finest level uses the persistent kernel"
    # 1100 directions: the lagged form's pointer ring is refilled twice
    for k in (0, 1, 4, 7, 40) + ((1100,) if n == 8 else ()):
        W = np.linalg.qr(rng.standard_normal((N, k)))[0].T.copy() if k else np.zeros((0, N))
        w = rng.standard_normal(N)
        z = rng.standard_normal(N)
        r = rng.standard_normal(N)
        betas, gamma, wk, alpha, rn = reference(W, w, r)
        dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
        for cfg in configs:
            Wk, rn_g, b_g, gm_g, al_g = g.rm_step(0, dev(W) if k else None, dev(w), dev(z), dev(r), cfg)
            Wk, rn_g = Wk.cpu().numpy(), rn_g.cpu().numpy()
            what = f"k={k} config={cfg}"
            assert np.abs(b_g - betas).max(initial=0) <= 1e-12 * np.abs(w).max(), what
            assert abs(gm_g - gamma) <= 1e-12 * gamma, what
            assert abs(al_g - alpha) <= 1e-12 * np.linalg.norm(r), what
            assert np.abs(Wk - wk).max() <= 1e-12, what
            assert np.abs(rn_g - rn).max() <= 1e-12 * np.abs(r).max(), what


@pytest.mark.parametrize("n,p", [(8, 2), (16, 2)])
def test_rm_step_exchange_wave_is_bitwise_plain(n, p):
    prob = synth.make_problem(n, p, n_levels=2)
    nu = synth.nu_sphere(n, n, n, prob.h)
    g = omg().Solver.from_sip(omg().Solver.make_grid(n, n, n, p, 2, prob.h), torch.tensor(nu, device="cuda"))
    N = prob.n_dofs
    rng = np.random.default_rng(8)
    configs = g.rm_configs(0)
    pairs = [(c, c[:4] + (0, 0)) for c in configs if c[4] == 4 and c[5] == 0 and c[:4] + (0, 0) in configs]
    assert pairs, "some configuration has both forms"
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    for k in (0, 3, 9, 33):
        W = np.linalg.qr(rng.standard_normal((N, k)))[0].T.copy() if k else np.zeros((0, N))
        w, z, r = (rng.standard_normal(N) for _ in range(3))
        for cw, plain in pairs:
            a = g.rm_step(0, dev(W) if k else None, dev(w), dev(z), dev(r), cw)
            b = g.rm_step(0, dev(W) if k else None, dev(w), dev(z), dev(r), plain)
            what = f"k={k} config={cw}"
            assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]), what
            assert np.array_equal(a[2], b[2]) and a[3] == b[3] and a[4] == b[4], what


@pytest.mark.parametrize("n,p", [(8, 1), (16, 2)])
def test_rm_step_breakdown_drops_direction(n, p):
    """A new vector already in span(W) (here a stored direction itself):
    after MGS ||w_out|| <= 1e-14 ||w_in||, so every configuration drops it:
    gamma = alpha = 0, the new direction is zero and r is unchanged bit for
    bit; the MGS coefficients are still the sequential ones."""
    prob = synth.make_problem(n, p, n_levels=2)
    nu = synth.nu_sphere(n, n, n, prob.h)
    g = omg().Solver.from_sip(omg().Solver.make_grid(n, n, n, p, 2, prob.h), torch.tensor(nu, device="cuda"))
    N = prob.n_dofs
    rng = np.random.default_rng(9)
    k = 6
    W = np.linalg.qr(rng.standard_normal((N, k)))[0].T.copy()
    w = W[2].copy()
    z = rng.standard_normal(N)
    r = rng.standard_normal(N)
    betas, _, _, _, _ = reference(W, w, r)
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    for cfg in g.rm_configs(0):
        Wk, rn_g, b_g, gm_g, al_g = g.rm_step(0, dev(W), dev(w), dev(z), dev(r), cfg)
        what = f"config={cfg}"
        assert gm_g == 0.0 and al_g == 0.0, what
        assert not torch.any(Wk != 0), what
        assert np.array_equal(rn_g.cpu().numpy(), r), what
        assert np.abs(b_g - betas).max() <= 1e-12, what


@pytest.mark.parametrize("n,p,lv", [(8, 1, 3), (16, 2, 2), (16, 1, 4)])
def test_every_rm_form_in_whole_solves(n, p, lv):
    """Whole Algorithm 2 solves with each RM form forced on the finest level
    (plain blocks, exchange wave, lagged with one or two exchanges in flight,
    each with the smallest and largest grid available): the lagged forms'
    Gram-entry corrections are exercised on the directions the solve itself
    produces. Same visit log as the oracle, solution within 1e-9."""
    import oracle
    prob = synth.make_problem(n, p, n_levels=lv)
    nu = synth.nu_sphere(n, n, n, prob.h)
    o = oracle.Oracle.from_sip(prob, nu, s_pre=2, s_post=2)
    b = synth.rhs(prob.n_dofs, 0)
    x_o = o.solve(b)
    g = omg().Solver.from_sip(omg().Solver.make_grid(n, n, n, p, lv, prob.h), torch.tensor(nu, device="cuda"),
                              s_pre=2, s_post=2)
    forms = {}
    for c in g.rm_configs(0):
        forms.setdefault((c[2], c[4], c[5]), []).append(c)
    assert any(key[2] > 0 for key in forms), "lagged forms are candidates"
    for key, cs in sorted(forms.items()):
        for cfg in {cs[0], cs[-1]}:
            g.set_rm_config(0, cfg)
            x_g = g.solve(torch.tensor(b, device="cuda")).cpu().numpy()
            what = f"config {cfg}"
            assert np.array_equal(g.visits(), o.visits()), what
            assert np.linalg.norm(x_g - x_o) <= 1e-9 * np.linalg.norm(x_o), what
