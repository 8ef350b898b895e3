"""Batched solves on the GPU against the FP64 CPU oracle.

Multi-right-hand-side level operations (matrix-core block products: SpMV,
block-Jacobi, coarsest solve) column by column against the oracle's
single-vector operations, with ragged column counts (1, 7, 16, 19, 32) that
cover a partial first tile, exactly one tile, a partial second tile and two
full tiles. Lockstep batched solves: every column has the oracle's iteration
count for that right-hand side alone and its solution within 1e-9."""
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


def pair(n, p, n_levels=None, **opts):
    prob = synth.make_problem(n, p, n_levels=n_levels)
    nu = synth.nu_sphere(n, n, n, prob.h)
    o = oracle.Oracle.from_sip(prob, nu, **opts)
    g = omg().Solver.from_sip(grid_of(prob), torch.tensor(nu, device="cuda"), **opts)
    return prob, nu, o, g


def cuda(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


NRHS = [1, 7, 16, 19, 32]


@pytest.mark.parametrize("n,p,lv", [(8, 1, 3), (8, 2, 2)])
def test_multi_rhs_level_operations(n, p, lv):
    m = omg()
    prob, nu, o, g = pair(n, p, lv)
    rng = np.random.default_rng(5)
    for l in range(lv - 1):
        nl = (n >> l) ** 3 * prob.bs
        for nr in NRHS:
            X = rng.standard_normal((nl, nr))
            B = rng.standard_normal((nl, nr))
            Y = host(g.level_multi(l, m.MR_SPMV, cuda(X)))
            Yb = host(g.level_multi(l, m.MR_SPMV, cuda(X), cuda(B)))
            Y32 = host(g.level_multi(l, m.MR_SPMV, cuda(X), cuda(B), fp32=True))
            for j in range(nr):
                ref = o.spmv(X[:, j], l)
                scale = np.abs(o.spmv(np.abs(X[:, j]), l)).max()
                assert np.abs(Y[:, j] - ref).max() <= 1e-14 * scale, (l, nr, j)
                refb = o.spmv(X[:, j], l, B[:, j])
                assert np.abs(Yb[:, j] - refb).max() <= 1e-14 * scale, (l, nr, j)
                assert np.abs(Y32[:, j] - refb).max() <= 1e-5 * scale, (l, nr, j)
            for s in (1, 2, 3):
                Z = host(g.level_multi(l, m.MR_SMOOTHER, cuda(B), sweeps=s))
                Z32 = host(g.level_multi(l, m.MR_SMOOTHER, cuda(B), sweeps=s, fp32=True))
                for j in range(nr):
                    ref = o.smoother(B[:, j], s, l)
                    sc = np.abs(ref).max()
                    assert np.abs(Z[:, j] - ref).max() <= 1e-12 * sc, (l, nr, s, j)
                    assert np.abs(Z32[:, j] - ref).max() <= 1e-4 * sc, (l, nr, s, j)
    nc = (n >> (lv - 1)) ** 3 * prob.bs
    for nr in NRHS:
        Bc = rng.standard_normal((nc, nr))
        Xc = host(g.level_multi(lv - 1, m.MR_COARSE, cuda(Bc)))
        for j in range(nr):
            ref = o.coarse_solve(Bc[:, j])
            assert np.abs(Xc[:, j] - ref).max() <= 1e-10 * np.abs(ref).max(), (nr, j)


def _oracle_columns(o, B, tol=1e-10):
    xs, its = [], []
    for j in range(B.shape[1]):
        xs.append(o.solve(B[:, j], tol=tol))
        its.append(o.last_report["iters_fine"])
    return np.stack(xs, 1), its


@pytest.mark.parametrize("n,p,lv,nr,variant", [(8, 2, 3, 17, "sync"), (16, 1, 4, 5, "sync"),
                                              (8, 1, 2, 3, "overlap")])
def test_lockstep_columns_match_oracle(n, p, lv, nr, variant):
    opts = dict(s_pre=2, s_post=2, variant=variant, n_s=1)
    prob, nu, o, g = pair(n, p, lv, **opts)
    B = synth.multi_rhs(prob.n_dofs, nr, seed=3)
    xs, reps = omg().solve_batched([g], [cuda(B)], nrhs=nr)
    X = host(xs[0])
    Xo, its = _oracle_columns(o, B)
    for j in range(nr):
        assert reps[j]["status"] == 0 and reps[j]["rel_res_true"] <= 1.0001e-10, (j, reps[j])
        assert reps[j]["iters_fine"] == its[j], (j, reps[j]["iters_fine"], its[j])
        assert np.linalg.norm(X[:, j] - Xo[:, j]) <= 1e-9 * np.linalg.norm(Xo[:, j]), j


def test_lockstep_more_than_one_group_and_zero_column():
    """33 columns (groups of 32 and 1), one of them zero; a nonzero initial
    guess of the solution's magnitude (the recursive residual then starts
    near ||b||); every column equals the single solve from the same x0; the
    solver's own single solve is unaffected afterwards."""
    prob, nu, o, g = pair(4, 1, 2)
    B = synth.multi_rhs(prob.n_dofs, 33, seed=4)
    B[:, 5] = 0.0
    scale = np.abs(o.solve(B[:, 0])).max()
    X0 = scale * synth.multi_rhs(prob.n_dofs, 33, seed=6)
    xs, reps = omg().solve_batched([g], [cuda(B)], [cuda(X0)], nrhs=33)
    X = host(xs[0])
    assert np.all(X[:, 5] == 0.0)
    A = o.scipy_matrix(0)
    for j in range(33):
        if j == 5:
            continue
        assert np.linalg.norm(B[:, j] - A @ X[:, j]) <= 1.0001e-10 * np.linalg.norm(B[:, j]), j
        xj = host(g.solve(cuda(B[:, j]), x=cuda(X0[:, j])))
        assert np.linalg.norm(X[:, j] - xj) <= 1e-9 * np.linalg.norm(xj), j
        assert reps[j]["iters_fine"] == g.last_report["iters_fine"], j
    b = synth.rhs(prob.n_dofs, 0)
    assert np.linalg.norm(host(g.solve(cuda(b))) - o.solve(b)) <= 1e-9 * np.linalg.norm(o.solve(b))


def test_lockstep_mixed_precision():
    """FP32 inner work per column with FP64 refinement: every column reaches
    the true FP64 residual 1e-10."""
    prob, nu, o, _ = pair(8, 2, 3)
    g = omg().Solver.from_sip(grid_of(prob), cuda(nu), precision="mixed_ir")
    B = synth.multi_rhs(prob.n_dofs, 6, seed=7)
    xs, reps = omg().solve_batched([g], [cuda(B)], nrhs=6)
    X = host(xs[0])
    A = o.scipy_matrix(0)
    Xo, _ = _oracle_columns(o, B)
    for j in range(6):
        assert reps[j]["rel_res_true"] <= 1.0001e-10
        assert np.linalg.norm(B[:, j] - A @ X[:, j]) <= 1.0001e-10 * np.linalg.norm(B[:, j])
        err = np.linalg.norm(X[:, j] - Xo[:, j]) / np.linalg.norm(Xo[:, j])
        print(f"column {j}: {reps[j]['outer_iters']} refinements, rel. difference to FP64 oracle {err:.2e}")
        assert err < 1e-4


def _instance_set(sizes, count, p, seed=2, **opts):
    """Uneven instances (random sphere, centre and ratio per instance) on
    small grids; level counts differ between instances."""
    out = []
    for inst in synth.instances(count=count, seed=seed, sizes=sizes):
        lv = {4: 2, 8: 3, 16: 3}[inst.n]
        prob = synth.make_problem(inst.n, p, n_levels=lv)
        nu = synth.nu_sphere(inst.n, inst.n, inst.n, prob.h, center=inst.center, radius=inst.radius,
                             nu_out=inst.ratio)
        b = synth.rhs(prob.n_dofs, inst.seed)
        out.append((prob, nu, b))
    return out


def test_instances_lockstep_match_oracle():
    """Six uneven instances in one batched call (grouped launches, per-instance
    RM): each has the oracle's iteration count and solution within 1e-9."""
    sets = _instance_set((4, 8), 6, 2)
    gs = [omg().Solver.from_sip(grid_of(pr), cuda(nu), s_pre=2, s_post=2) for pr, nu, _ in sets]
    xs, reps = omg().solve_batched(gs, [cuda(b).reshape(-1, 1) for _, _, b in sets], nrhs=1)
    for i, (pr, nu, b) in enumerate(sets):
        o = oracle.Oracle.from_sip(pr, nu, s_pre=2, s_post=2)
        xo = o.solve(b)
        x = host(xs[i]).reshape(-1)
        assert reps[i]["status"] == 0 and reps[i]["rel_res_true"] <= 1.0001e-10, (i, reps[i])
        assert reps[i]["iters_fine"] == o.last_report["iters_fine"], i
        assert np.linalg.norm(x - xo) <= 1e-9 * np.linalg.norm(xo), i


@pytest.mark.parametrize("precision", ["fp64", "mixed_ir"])
def test_instances_lockstep_equal_single_solves(precision):
    """The batched instance path runs the single-instance arithmetic: results
    and iteration counts equal separate omg_solve calls bit for bit."""
    sets = _instance_set((4, 8, 16), 5, 2, seed=9)
    mk = lambda pr, nu: omg().Solver.from_sip(grid_of(pr), cuda(nu), s_pre=2, s_post=2, precision=precision)
    gs = [mk(pr, nu) for pr, nu, _ in sets]
    xs, reps = omg().solve_batched(gs, [cuda(b).reshape(-1, 1) for _, _, b in sets], nrhs=1)
    for i, (pr, nu, b) in enumerate(sets):
        s1 = mk(pr, nu)
        x1 = host(s1.solve(cuda(b)))
        assert np.array_equal(host(xs[i]).reshape(-1), x1), i
        assert reps[i]["iters_fine"] == s1.last_report["iters_fine"], i
        assert reps[i]["outer_iters"] == s1.last_report["outer_iters"], i
        assert reps[i]["rel_res_true"] <= 1.0001e-10
