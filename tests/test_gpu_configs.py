"""GPU checks at the workload sizes (64^3 P2, 48^3 P2, 96^3 P1), where the
oracle cannot run whole solves in seconds: per-kernel outputs against the
oracle, properties of the solves (true FP64 residual by the oracle's own
SpMV) under every cycle configuration and smoother, mixed precision at
coefficient ratios 1e3 and 1e6, and gradients against finite differences."""
import time

import numpy as np
import pytest

import oracle
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


def grid_of(prob):
    return omg().Solver.make_grid(prob.nx, prob.ny, prob.nz, prob.p, prob.n_levels, prob.h, prob.penalty_c)


def cuda(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def big():
    """64^3 P2, 4 levels, sphere r = 0.3, ratio 1000 (the benchmark workload)."""
    prob = synth.make_problem(64, 2)
    nu = synth.nu_sphere(64, 64, 64, prob.h)
    t = time.time()
    o = oracle.Oracle.from_sip(prob, nu, s_pre=2, s_post=2)
    say(f"oracle setup 64^3 P2: {time.time() - t:.1f} s")
    g = omg().Solver.from_sip(grid_of(prob), cuda(nu), s_pre=2, s_post=2)
    return prob, nu, o, g


def test_fullsize_operators(big):
    """Device assembly and Galerkin coarse operators at 64^3 P2 equal the
    oracle's quadrature assembly and triple products on every level."""
    prob, nu, o, g = big
    for l in range(prob.n_levels):
        rp, ci, v = o.matrix(l)
        grp, gci, gv = g.level_matrix(l)
        assert np.array_equal(rp, grp) and np.array_equal(ci, gci)
        err = np.abs(gv - v).max() / np.abs(v).max()
        say(f"level {l}: {len(ci)} blocks, max rel. difference {err:.2e}")
        assert err < 1e-13


def test_fullsize_kernels(big):
    prob, nu, o, g = big
    rng = np.random.default_rng(11)
    x = rng.standard_normal(prob.n_dofs)
    b = rng.standard_normal(prob.n_dofs)
    scale = np.abs(o.spmv(np.abs(x))).max()
    assert np.abs(host(g.level_spmv(0, cuda(x), cuda(b))) - o.spmv(x, 0, b)).max() <= 1e-14 * scale
    ref = o.smoother(b, 2, 0)
    assert np.abs(host(g.level_smoother(0, cuda(b), 2)) - ref).max() <= 1e-12 * np.abs(ref).max()
    rc = o.restrict(x, 0)
    assert np.abs(host(g.level_restrict(0, cuda(x))) - rc).max() <= 1e-14 * np.abs(rc).max()
    n3 = (64 >> 3) ** 3 * prob.bs
    bc = rng.standard_normal(n3)
    ref = o.coarse_solve(bc)
    assert np.abs(host(g.coarse_solve(cuda(bc))) - ref).max() <= 1e-10 * np.abs(ref).max()


def test_fullsize_fp32_kernels(big):
    """The single-precision SpMV, block-Jacobi, restriction and prolongation
    of the mixed forms on the finest 64^3 P2 level against the oracle's FP32
    emulation: within twice the float rounding bound of the exact result on
    the rounded data (element by element for SpMV); errors printed."""
    import scipy.sparse as sp
    prob, nu, o, g = big
    rng = np.random.default_rng(12)
    eps = float(np.finfo(np.float32).eps)
    f32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    x = rng.standard_normal(prob.n_dofs)
    b = rng.standard_normal(prob.n_dofs)
    rp, ci, v = o.matrix(0)
    absA = sp.bsr_matrix((np.abs(f32(v)), ci, rp), shape=(prob.n_dofs, prob.n_dofs))
    bnd = 2 * (7 * prob.bs + 2) * eps * (absA @ np.abs(f32(x)) + np.abs(f32(b)))
    del absA, v
    yo = o.spmv(x, 0, b, fp32=True)
    yg = host(g.level_spmv(0, cuda(x), cuda(b), fp32=True))
    say(f"64^3 P2 FP32 SpMV: max rel. difference {np.abs(yg - yo).max() / np.abs(yo).max():.2e}")
    assert np.all(np.abs(yg - yo) <= bnd)
    for sw in (1, 2):
        so = o.smoother(b, sw, 0, fp32=True)
        err = np.abs(host(g.level_smoother(0, cuda(b), sw, fp32=True)) - so).max() / np.abs(so).max()
        say(f"64^3 P2 FP32 block-Jacobi, {sw} iteration(s): max rel. difference {err:.2e}")
        assert err <= 2e-5
    ro = o.restrict(x, 0, fp32=True)
    err = np.abs(host(g.level_restrict(0, cuda(x), fp32=True)) - ro).max() / np.abs(ro).max()
    say(f"64^3 P2 FP32 restriction: max rel. difference {err:.2e}")
    assert err <= 2 * (8 * prob.bs + 2) * eps * 8
    zc = rng.standard_normal(len(ro))
    po = o.prolong(zc, 0, fp32=True)
    err = np.abs(host(g.level_prolong(0, cuda(zc), fp32=True)) - po).max() / np.abs(po).max()
    say(f"64^3 P2 FP32 prolongation: max rel. difference {err:.2e}")
    assert err <= 2 * (prob.bs + 2) * eps * 8


def test_fullsize_rm_step_every_configuration(big):
    """One residual-minimisation step (Algorithm 1 after w = A z) of the
    finest 64^3 P2 level (N = 2,621,440) in every co-resident launch
    configuration of the persistent kernel -- including the grids of more
    than 256 blocks, where the exchange words are gathered in several passes
    -- for k = 0, 1, 40 and 64 orthonormal directions, against the
    sequential MGS step in numpy: coefficients, gamma, alpha, the new
    direction and the residual to 1e-12."""
    prob, nu, o, g = big
    N = prob.n_dofs
    rng = np.random.default_rng(31)
    configs = g.rm_configs(0)
    say(f"64^3 P2 finest level: {len(configs)} co-resident RM configurations, "
        f"grids {sorted(set(c[0] for c in configs))}")
    assert any(c[0] > 256 for c in configs)
    # the tuner reports configurations it dropped for an expired wait (none
    # here: every candidate below also completes its bounded waits)
    dropped = [g.rm_dropped(l) for l in range(prob.n_levels - 1)]
    say(f"RM configurations dropped by the tuner per level: {dropped}")
    assert all(d == 0 for d in dropped)
    Wall = np.linalg.qr(rng.standard_normal((N, 64)))[0].T.copy()
    Wdev = cuda(Wall)
    for k in (0, 1, 40, 64):
        W = Wall[:k]
        w, z, r = (rng.standard_normal(N) for _ in range(3))
        ww = w.copy()
        betas = []
        for Wi in W:
            bb = Wi @ ww
            betas.append(bb)
            ww -= bb * Wi
        gamma = 1.0 / np.linalg.norm(ww)
        wk = gamma * ww
        alpha = wk @ r
        rn = r - alpha * wk
        wk_d, rn_d, w_d, z_d, r_d = cuda(wk), cuda(rn), cuda(w), cuda(z), cuda(r)
        Wk_arg = Wdev[:k].contiguous() if k else None
        rscale = np.abs(r).max()
        for cfg in configs:
            Wk, rn_g, b_g, gm_g, al_g = g.rm_step(0, Wk_arg, w_d, z_d, r_d, cfg)
            what = f"k={k} config={cfg}"
            assert np.abs(b_g - np.array(betas)).max(initial=0) <= 1e-12 * np.abs(w).max(), what
            assert abs(gm_g - gamma) <= 1e-12 * gamma, what
            assert abs(al_g - alpha) <= 1e-12 * np.linalg.norm(r), what
            assert (Wk - wk_d).abs().max().item() <= 1e-12, what
            assert (rn_g - rn_d).abs().max().item() <= 1e-12 * rscale, what


def _visit_divergence(log_a, log_b):
    """Per visit, while the two logs agree on (level, iterations): the
    largest difference of the residual ratios ||r_i|| / ||r_0|| (and, on the
    finest level, of ||r_0|| itself, relative)."""
    dq = []
    for (la, ia, r0a, ra), (lb, ib, r0b, rb) in zip(log_a, log_b):
        if (la, ia) != (lb, ib):
            break
        dq.append(max(abs(r0a / r0b - 1) if la == 0 else 0.0, np.abs(ra / r0a - rb / r0b).max(initial=0.0)))
    return np.array(dq)


def test_fullsize_replay_matches_oracle_golden(big):
    """The 64^3 P2 plain-method solve (2+2 block-Jacobi sweeps, tolerance
    1e-10, b from seed 0) with the oracle's visit log imposed on the GPU,
    against the oracle's solve of this workload
    (tests/golden/make_oracle_64cubed_p2.py).

    At this size two correct runs of the method do not agree to 1e-9: the
    same oracle with b perturbed by 1e-15 relative (the --perturb solve of
    the same script) follows the same visit sequence but its per-visit
    residual ratios drift from the unperturbed ones from visit ~125 on
    (1e-12), pass 1e-9 at visit ~380 and reach 0.58; it stops after 241
    cycles instead of 256 and its solution differs by 1.1e-8 at the sampled
    entries. The GPU's rounding differs from the oracle's at every reduction,
    so the bar is that envelope: the running maximum of the GPU's per-visit
    divergence from the oracle stays within 10x that of the perturbed
    oracle (plus 1e-12), and the solution differences stay within 5x the
    perturbed oracle's. Same visits, cycles and directions;
    true residual within 2e-10 after the oracle's 256 cycles."""
    import json
    import os
    here = os.path.join(os.path.dirname(__file__), "golden")
    path = os.path.join(here, "oracle_64cubed_p2.npz")
    path_p = os.path.join(here, "oracle_64cubed_p2_perturbed.npz")
    if not (os.path.exists(path) and os.path.exists(path_p)):
        pytest.skip("golden files not generated (tests/golden/make_oracle_64cubed_p2.py [--perturb])")
    gd = np.load(path, allow_pickle=False)
    gp = np.load(path_p, allow_pickle=False)
    rep_o = json.loads(str(gd["report"]))
    prob, nu, o, g = big
    b = synth.rhs(prob.n_dofs, 0)
    g.set_replay(gd["visits"])
    t = time.time()
    x = host(g.solve(cuda(b), tol=1e-10))
    g.set_replay([])
    rep = g.last_report
    say(f"replayed 64^3 P2 solve: {time.time() - t:.1f} s, {rep['iters_fine']} cycles "
        f"(oracle {rep_o['iters_fine']}), {rep['n_dirs_fine']} directions (oracle {rep_o['n_dirs_fine']})")
    assert np.array_equal(g.visits(), gd["visits"])
    assert rep["iters_fine"] == rep_o["iters_fine"] and rep["n_dirs_fine"] == rep_o["n_dirs_fine"]
    log_o = oracle.parse_visit_norms(gd["vnorm"])
    log_g = g.visit_norms()
    assert [(l, i) for l, i, _, _ in log_g] == [(l, i) for l, i, _, _ in log_o]
    d_g = _visit_divergence(log_g, log_o)
    d_p = _visit_divergence(oracle.parse_visit_norms(gp["vnorm"]), log_o)
    n = len(d_p)
    env_g = np.maximum.accumulate(d_g[:n])
    env_p = np.maximum.accumulate(d_p)
    worst = int(np.argmax(env_g / (env_p + 1e-12)))
    say(f"per-visit divergence: GPU first > 1e-9 at visit {int(np.argmax(d_g > 1e-9))}, perturbed oracle at "
        f"{int(np.argmax(d_p > 1e-9))}; largest envelope ratio {env_g[worst] / (env_p[worst] + 1e-12):.2f} "
        f"at visit {worst}")
    assert np.all(env_g <= 10 * env_p + 1e-12)
    idx = gd["idx"]
    xs = gd["x_idx"]
    e_s = np.linalg.norm(x[idx] - xs) / np.linalg.norm(xs)
    u = synth.rhs(prob.n_dofs, 8)
    xn = float(gd["x_norm"])
    e_n = abs(np.linalg.norm(x) / xn - 1)
    # |x.v - x*.v| <= ||x - x*|| ||v|| (Cauchy-Schwarz): relative to ||x*|| ||v||
    e_b = abs(x @ b - float(gd["x_dot_b"])) / (xn * np.linalg.norm(b))
    e_u = abs(x @ u - float(gd["x_dot_u"])) / (xn * np.linalg.norm(u))
    p_s = np.linalg.norm(gp["x_idx"] - xs) / np.linalg.norm(xs)
    p_n = abs(float(gp["x_norm"]) / xn - 1)
    p_u = abs(float(gp["x_dot_u"]) - float(gd["x_dot_u"])) / (xn * np.linalg.norm(u))
    say(f"solution vs oracle: sampled {e_s:.2e} (perturbed oracle {p_s:.2e}), ||x|| {e_n:.2e} ({p_n:.2e}), "
        f"x.u {e_u:.2e} ({p_u:.2e}), x.b {e_b:.2e}; true residual {rep['rel_res_true']:.3e}")
    # | ||x|| - ||x*|| | <= ||x - x*||: the norm is held to the sampled bound
    assert e_s <= 5 * p_s and e_n <= 5 * p_s and e_u <= 5 * p_u and e_b <= 5 * p_u
    assert rep["rel_res_true"] <= 2e-10


def test_fullsize_solve_true_residual(big):
    """The benchmark solve reaches ||b - A x|| <= 1e-10 ||b|| with A the
    oracle's own operator; the recursive residual agrees with the true one."""
    prob, nu, o, g = big
    b = synth.rhs(prob.n_dofs, 0)
    t = time.time()
    x = host(g.solve(cuda(b), tol=1e-10))
    rep = g.last_report
    say(f"64^3 P2 FP64 solve: {time.time() - t:.1f} s, {rep['iters_fine']} cycles, {rep['n_dirs_fine']} directions")
    r = o.spmv(x, 0, b)
    rel = np.linalg.norm(r) / np.linalg.norm(b)
    assert rel <= 1.0001e-10, rel
    assert abs(rep["rel_res_true"] - rel) <= 1e-3 * rel


@pytest.mark.parametrize("opts", [dict(variant="hybrid"), dict(variant="overlap", n_s_max=10),
                                  dict(variant="overlap", n_s_max=10, precision="mixed_flex"),
                                  dict(smoother="schwarz", s_pre=2, s_post=2, omega=0.1, precision="mixed_flex")],
                         ids=["hybrid", "adaptive", "adaptive-mixed_flex", "schwarz-mixed_flex"])
def test_fullsize_other_configurations(big, opts):
    """The benchmark workload under the hybrid configuration of Table 1, the
    timing-adaptive loops of Sec. 4.3 (FP64 and mixed) and the additive
    Schwarz smoother with single-precision local solves: each reaches
    ||b - A x|| <= 1e-10 ||b|| with A the oracle's own operator."""
    prob, nu, o, _ = big
    o2 = dict(s_pre=2, s_post=2)
    o2.update(opts)
    g = omg().Solver.from_sip(grid_of(prob), cuda(nu), **o2)
    b = synth.rhs(prob.n_dofs, 0)
    t = time.time()
    x = host(g.solve(cuda(b), tol=1e-10))
    rep = g.last_report
    rel = np.linalg.norm(o.spmv(x, 0, b)) / np.linalg.norm(b)
    say(f"{opts}: {time.time() - t:.1f} s, {rep['iters_fine']} cycles, true residual {rel:.2e}")
    assert rel <= 1.0001e-10, rel
    g.close()


@pytest.mark.parametrize("ratio", [1e3, 1e6])
def test_mixed_precision_ratios(ratio):
    """FP32 inner OrthoMG with FP64 iterative refinement reaches the FP64
    residual 1e-10 at coefficient ratios 1e3 and 1e6 (64^3 P2); the
    difference to the FP64 solution is reported."""
    prob = synth.make_problem(64, 2)
    nu = synth.nu_sphere(64, 64, 64, prob.h, nu_out=ratio)
    b = synth.rhs(prob.n_dofs, 0)
    g64 = omg().Solver.from_sip(grid_of(prob), cuda(nu), s_pre=2, s_post=2)
    gm = omg().Solver.from_sip(grid_of(prob), cuda(nu), s_pre=2, s_post=2, precision="mixed_ir")
    t = time.time()
    xm = host(gm.solve(cuda(b), tol=1e-10))
    tm = time.time() - t
    rm = gm.last_report
    t = time.time()
    x64 = host(g64.solve(cuda(b), tol=1e-10))
    t64 = time.time() - t
    r64 = g64.last_report
    diff = np.linalg.norm(xm - x64) / np.linalg.norm(x64)
    say(f"ratio {ratio:g}: FP64 {t64:.1f} s ({r64['iters_fine']} cycles), mixed {tm:.1f} s "
        f"({rm['iters_fine']} inner cycles, {rm['outer_iters']} refinements), rel. diff {diff:.2e}, "
        f"true residuals {r64['rel_res_true']:.2e} / {rm['rel_res_true']:.2e}")
    assert rm["rel_res_true"] <= 1.0001e-10 and r64["rel_res_true"] <= 1.0001e-10
    g64.close()
    gm.close()


def _delta(prob, s0, nu1, u0, tol):
    """u(nu1) - u(nu0) = A(nu1)^-1 (A(nu0) - A(nu1)) u0 with s0 the solver of
    nu0, solved directly so its accuracy is relative to the (small)
    difference itself."""
    s1 = omg().Solver.from_sip(grid_of(prob), cuda(nu1))
    rhs = s0.level_spmv(0, cuda(u0)) - s1.level_spmv(0, cuda(u0))
    d = host(s1.solve(rhs, tol=tol))
    s1.close()
    return d


@pytest.fixture(scope="module")
def grad48():
    """48^3 P2 (ratio 1000): forward solve, adjoint gradient of
    L = 0.5 ||u - u_t||^2 with respect to f and log(nu)."""
    prob = synth.make_problem(48, 2)
    nu = synth.nu_sphere(48, 48, 48, prob.h)
    f = synth.rhs(prob.n_dofs, 0)
    ut = synth.rhs(prob.n_dofs, 1)
    s = omg().Solver.from_sip(grid_of(prob), cuda(nu))
    t = time.time()
    u = host(s.solve(cuda(f), tol=1e-12))
    g_f, g_nu = s.backward(cuda(u), cuda(u - ut), tol=1e-12)
    say(f"48^3 P2 forward + adjoint: {time.time() - t:.1f} s")
    cells = np.random.default_rng(3).choice(prob.n_cells, size=20, replace=False)
    yield prob, nu, f, ut, u, host(g_f), host(g_nu) * nu, s, cells
    s.close()


def test_gradient_48p2_euler_identity(grad48):
    """nu -> c nu scales A by c, so sum_K dL/dlog nu_K = -lambda^T A u = -lambda^T f."""
    prob, nu, f, ut, u, g_f, g_lognu, s, cells = grad48
    lam_f = g_f @ f
    assert abs(g_lognu.sum() + lam_f) <= 1e-8 * abs(lam_f)


@pytest.mark.parametrize("chunk", [0, 1, 2, 3])
def test_gradient_48p2_finite_differences(grad48, chunk):
    """dL/dlog nu on 20 random cells (5 per chunk) against central finite
    differences (h = 1e-6): u(nu e^{+-h}) - u(nu) solved directly to 1e-11.
    Bound: |fd - adj| <= 1e-5 |fd| + 1e-9 max|adj|. The absolute term is
    the adjoint gradient's own accuracy (forward and adjoint solved to
    1e-12): on the sampled cell with the smallest gradient (2.4e-4 of the
    largest) the difference is 4-8e-14 (2-3e-9 of the largest gradient) whether
    h is 1e-4, 1e-5 or 1e-6 (1.4e-5, 1.1e-5, 7.8e-6 relative), so it does not
    come from the finite differences."""
    prob, nu, f, ut, u, g_f, g_lognu, s, cells = grad48
    h = 1e-6
    gmax = np.abs(g_lognu).max()
    t = time.time()
    for c in cells[5 * chunk: 5 * chunk + 5]:
        nup, num = nu.copy(), nu.copy()
        nup[c] *= np.exp(h)
        num[c] *= np.exp(-h)
        dp = _delta(prob, s, nup, u, 1e-11)
        dm = _delta(prob, s, num, u, 1e-11)
        fd = ((dp - dm) @ (u - ut) + 0.5 * (dp @ dp - dm @ dm)) / (2 * h)
        err = abs(fd - g_lognu[c])
        say(f"cell {c}: adjoint {g_lognu[c]:.9e}, finite difference {fd:.9e}, rel. {err / abs(fd):.1e}")
        assert err <= 1e-5 * abs(fd) + 1e-9 * gmax, (c, fd, g_lognu[c])
    say(f"chunk {chunk}: {time.time() - t:.1f} s")


def test_forward_96p1_checkpointed():
    """96^3 P1 (3.54M DOFs, 5 levels) forward solve through the autograd
    Function, which keeps only (f, log nu, u) and frees the hierarchy."""
    prob = synth.make_problem(96, 1)
    assert prob.n_levels == 5 and prob.n_dofs == 3538944
    nu = synth.nu_sphere(96, 96, 96, prob.h)
    f = cuda(synth.rhs(prob.n_dofs, 0)).requires_grad_(True)
    lognu = cuda(np.log(nu)).requires_grad_(True)
    fn = omg().solve_fn()
    t = time.time()
    u = fn.apply(f, lognu, grid_of(prob), 1e-10, None)
    torch.cuda.synchronize()
    say(f"96^3 P1 checkpointed forward: {time.time() - t:.1f} s")
    assert u.grad_fn is not None
    o = oracle.Oracle.from_sip(prob, nu)
    r = o.spmv(host(u), 0, host(f.detach()))
    assert np.linalg.norm(r) <= 1.0001e-10 * np.linalg.norm(host(f.detach()))
