"""Caller-supplied agglomeration hierarchies through the C ABI (omg_setup
with parent/slot maps and embedding blocks, the R and P of Algorithm 2):
renumbered cells on every level, coarse cells with fewer than eight finer
cells, the explicit Cartesian hierarchy equal to the default one, and
malformed hierarchies rejected."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth
from tests.test_oracle_hierarchy import cartesian_maps

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2512_08728_amd  # noqa: F401


def omg():
    import paper_2512_08728_amd as m
    return m


def cuda(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def relmax(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def test_renumbered_hierarchy_matches_oracle():
    """The 8^3 P1 operator with its cells renumbered at random on all three
    levels (matrix, maps and right-hand side): same visit log as the oracle
    on the original numbering and the permuted solution within 1e-9."""
    m = omg()
    prob = synth.make_problem(8, 1, n_levels=3)
    nu = synth.nu_sphere(8, 8, 8, prob.h)
    o = oracle.Oracle.from_sip(prob, nu)
    A = o.scipy_matrix(0)
    bs = prob.bs
    nc, par, sl = cartesian_maps(8, 8, 8, 3)
    rng = np.random.default_rng(21)
    perms = [rng.permutation(n) for n in nc]
    inv = [np.argsort(p) for p in perms]
    dof = (inv[0][:, None] * bs + np.arange(bs)).reshape(-1)
    Ap = sp.bsr_matrix(A[dof][:, dof], blocksize=(bs, bs))
    Ap.sort_indices()
    par_p = [perms[l + 1][par[l][inv[l]]] for l in range(2)]
    sl_p = [sl[l][inv[l]] for l in range(2)]
    H = m.Hierarchy(nc, par_p, sl_p, oracle.embedding(1))
    g = m.Solver.from_bsr(Ap.indptr, Ap.indices, Ap.data, H)
    b = synth.rhs(prob.n_dofs, 0)
    x_o = o.solve(b)
    x_g = host(g.solve(cuda(b[dof])))
    assert np.array_equal(g.visits(), o.visits())
    assert np.linalg.norm(x_g - x_o[dof]) <= 1e-9 * np.linalg.norm(x_o)


def test_partial_coarse_cells_match_oracle():
    """6^3 P1 -> 3^3 -> 2^3 (coarse cells with one, two, four or eight finer
    cells): Galerkin levels within 1e-13 of the oracle's, same visit log,
    solution within 1e-9."""
    m = omg()
    prob = synth.Problem(nx=6, ny=6, nz=6, p=1, n_levels=1, h=1.0 / 6)
    nu = synth.nu_sphere(6, 6, 6, prob.h)
    rp, ci, v = oracle.Oracle.from_sip(prob, nu).matrix(0)
    nc, par, sl = cartesian_maps(6, 6, 6, 3)
    E = oracle.embedding(1)
    o = oracle.Oracle.from_bsr_hierarchy(rp, ci, v, nc, par, sl, E, s_pre=2, s_post=2)
    g = m.Solver.from_bsr(rp, ci, v, m.Hierarchy(nc, par, sl, E), s_pre=2, s_post=2)
    for l in range(3):
        a, b_ = o.matrix(l), g.level_matrix(l)
        assert np.array_equal(a[0], b_[0]) and np.array_equal(a[1], b_[1]) and relmax(b_[2], a[2]) < 1e-13, l
    b = synth.rhs(prob.n_dofs, 2)
    x_o = o.solve(b)
    x_g = host(g.solve(cuda(b)))
    assert np.array_equal(g.visits(), o.visits())
    assert np.linalg.norm(x_g - x_o) <= 1e-9 * np.linalg.norm(x_o)
    assert g.last_report["rel_res_true"] <= 1.0001e-10


def test_explicit_grid_hierarchy_equals_default():
    m = omg()
    prob = synth.make_problem(8, 2, n_levels=3)
    nu = synth.nu_sphere(8, 8, 8, prob.h)
    grid = m.Solver.make_grid(8, 8, 8, 2, 3, prob.h)
    g1 = m.Solver.from_sip(grid, cuda(nu))
    g2 = m.Solver.from_sip(grid, cuda(nu), hierarchy=m.Hierarchy.of_grid(grid))
    b = cuda(synth.rhs(prob.n_dofs, 0))
    assert torch.equal(g1.solve(b), g2.solve(b))
    assert np.array_equal(oracle.embedding(2).shape, m.Hierarchy.of_grid(grid).embed.shape)
    assert np.abs(m.Hierarchy.of_grid(grid).embed - oracle.embedding(2)).max() < 1e-14


def test_malformed_hierarchies_rejected():
    m = omg()
    prob = synth.make_problem(4, 1, n_levels=2)
    nu = synth.nu_sphere(4, 4, 4, prob.h)
    rp, ci, v = oracle.Oracle.from_sip(prob, nu).matrix(0)
    nc, par, sl = cartesian_maps(4, 4, 4, 2)
    E = oracle.embedding(1)
    bad = []
    p2 = par[0].copy(); p2[5] = 8
    bad.append(m.Hierarchy(nc, [p2], sl, E))                       # parent out of range
    s2 = sl[0].copy(); s2[3] = 8
    bad.append(m.Hierarchy(nc, par, [s2], E))                      # slot out of range
    p3 = par[0].copy(); p3[p3 == 7] = 6
    bad.append(m.Hierarchy(nc, [p3], sl, E))                       # coarse cell 7 without finer cells
    bad.append(m.Hierarchy([32, 8], [par[0][:32]], [sl[0][:32]], E))  # level 0 size differs from A
    E2 = E.copy(); E2[0, 0, 0] = np.nan
    bad.append(m.Hierarchy(nc, par, sl, E2))                       # non-finite embedding
    for H in bad:
        with pytest.raises(m.OmgError) as e:
            m.Solver.from_bsr(rp, ci, v, H)
        assert e.value.status == m.EINVAL
    with pytest.raises(m.OmgError) as e:
        m.Solver.from_bsr(rp, ci, v[:, :2, :2].copy(), m.Hierarchy(nc, par, sl, E[:, :2, :2].copy()))
    assert e.value.status in (m.EUNSUPPORTED, m.EINVAL)
