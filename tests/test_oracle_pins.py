"""Pins of the FP64 CPU oracle against facts fixed by the paper and by
mathematics (closed forms, invariants, special cases, brute force on tiny
inputs). None of these re-type the oracle's own formulas."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spl

import oracle
import synth
from tests import basis_ref as br


def sip(n, p, n_levels=None, nu=None, **opts):
    prob = synth.make_problem(n, p, n_levels=n_levels)
    if nu is None:
        nu = synth.nu_sphere(n, n, n, prob.h)
    return prob, nu, oracle.Oracle.from_sip(prob, nu, **opts)


def P_matrix(E, nx, ny, nz):
    """Prolongation as a scipy matrix from the 8 embedding blocks."""
    bs = E.shape[1]
    rows, cols, vals = [], [], []
    cx, cy = nx // 2, ny // 2
    for c in range(nx * ny * nz):
        i, j, k = c % nx, (c // nx) % ny, c // (nx * ny)
        I = i // 2 + cx * (j // 2 + cy * (k // 2))
        s = (i % 2) + 2 * (j % 2) + 4 * (k % 2)
        rr, cc = np.meshgrid(np.arange(bs), np.arange(bs), indexing="ij")
        rows.append((c * bs + rr).ravel())
        cols.append((I * bs + cc).ravel())
        vals.append(E[s].ravel())
    nc = (nx // 2) * (ny // 2) * (nz // 2)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(nx * ny * nz * bs, nc * bs))


# --------------------------------------------------------------------------
# Embedding (hierarchy of Sec. 3.1: R^lambda, P^lambda between levels)
# --------------------------------------------------------------------------
def test_embedding_closed_form_1d():
    """1D left-child embedding for p=2 equals the closed form; right child has
    signs (-1)^(n+m)."""
    E = oracle.embedding(2)
    idx = {o: i for i, o in enumerate(br.orders(2))}
    eL = np.zeros((3, 3))
    eR = np.zeros((3, 3))
    for n in range(3):
        for m in range(3):
            # 3D entry with y,z degrees 0 factors as e_nm * (1/sqrt2)^2
            eL[n, m] = E[0][idx[(n, 0, 0)], idx[(m, 0, 0)]] / 0.5 if (m <= 2) else 0
            eR[n, m] = E[1][idx[(n, 0, 0)], idx[(m, 0, 0)]] / 0.5
    closed = np.array([[1 / math.sqrt(2), -math.sqrt(6) / 4, 0.0],
                       [0.0, 1 / (2 * math.sqrt(2)), -math.sqrt(30) / 8],
                       [0.0, 0.0, math.sqrt(2) / 8]])
    assert np.allclose(eL, closed, atol=1e-14)
    sgn = np.array([[(-1) ** (n + m) for m in range(3)] for n in range(3)])
    assert np.allclose(eR, sgn * closed, atol=1e-14)


@pytest.mark.parametrize("p", [0, 1, 2, 3])
def test_embedding_reproduces_polynomials(p):
    """E_s maps coarse coefficients to the child coefficients of the same
    polynomial (evaluated pointwise with an independent basis), and
    sum_s E_s^T E_s = I (P^T P = I)."""
    E = oracle.embedding(p)
    rng = np.random.default_rng(0)
    uc = rng.standard_normal(E.shape[2])
    pts = rng.uniform(0, 1, size=(50, 3))
    h = 0.25
    for s in range(8):
        off = np.array([s & 1, (s >> 1) & 1, (s >> 2) & 1], dtype=float)
        coarse_xi = (pts + off) / 2.0              # the same physical points in the coarse frame
        vc = br.eval_cell(p, 2 * h, coarse_xi) @ uc
        vf = br.eval_cell(p, h, pts) @ (E[s] @ uc)
        assert np.allclose(vc, vf, rtol=1e-12, atol=1e-12)
    assert np.allclose(sum(E[s].T @ E[s] for s in range(8)), np.eye(E.shape[1]), atol=1e-14)


# --------------------------------------------------------------------------
# Discretisation (Sec. 2: SIP; configs' weighted average / harmonic penalty)
# --------------------------------------------------------------------------
def test_p0_is_graph_laplacian():
    """p = 0: only penalty terms survive: 12 nu_F / h^2 times the 7-point graph
    Laplacian plus 12 nu_K / h^2 per boundary face on the diagonal."""
    n = 4
    prob = synth.make_problem(n, 0, n_levels=1)
    nu = np.random.default_rng(3).uniform(1, 10, n ** 3)
    o = oracle.Oracle.from_sip(prob, nu)
    A = o.scipy_matrix().toarray()
    h = prob.h
    ref = np.zeros((n ** 3, n ** 3))
    for c in range(n ** 3):
        ijk = (c % n, (c // n) % n, c // (n * n))
        for d, st in enumerate((1, n, n * n)):
            for side in (-1, 1):
                nb = ijk[d] + side
                if 0 <= nb < n:
                    e = c + side * st
                    nf = 2 * nu[c] * nu[e] / (nu[c] + nu[e])
                    ref[c, c] += 12 * nf / h ** 2
                    ref[c, e] -= 12 * nf / h ** 2
                else:
                    ref[c, c] += 12 * nu[c] / h ** 2
    assert np.allclose(A, ref, rtol=1e-13, atol=1e-9)


@pytest.mark.parametrize("p", [1, 2])
def test_h_scaling(p):
    """A(h) = h^-2 A_hat(nu): every term scales as h^-2 with this basis."""
    S1, F1, B1 = oracle.element(p, 1.0)
    S2, F2, B2 = oracle.element(p, 0.125)
    assert np.allclose(S2, S1 / 0.125 ** 2, rtol=1e-12, atol=1e-9)
    assert np.allclose(F2, F1 / 0.125 ** 2, rtol=1e-12, atol=1e-9)
    assert np.allclose(B2, B1 / 0.125 ** 2, rtol=1e-12, atol=1e-9)


@pytest.mark.parametrize("p", [1, 2])
def test_volume_matrix_closed_form(p):
    """Volume stiffness of the orthonormal Legendre basis:
    int_0^1 psi_m' psi_n' = 2 sqrt((2m+1)(2n+1)) * k(k+1) * [m+n even], k = min(m,n)
    (from int_{-1}^1 P_m' P_n' = k(k+1) for m+n even and the map t = (s+1)/2);
    3D is the tensor sum."""
    def d1(m, n):
        if (m + n) % 2:
            return 0.0
        k = min(m, n)
        return 2 * math.sqrt((2 * m + 1) * (2 * n + 1)) * k * (k + 1)
    o = br.orders(p)
    S = oracle.element(p, 1.0)[0]
    ref = np.zeros_like(S)
    for i, (a, b, c) in enumerate(o):
        for j, (a2, b2, c2) in enumerate(o):
            ref[i, j] = (d1(a, a2) * (b == b2) * (c == c2) + d1(b, b2) * (a == a2) * (c == c2)
                         + d1(c, c2) * (a == a2) * (b == b2))
    assert np.allclose(S, ref, atol=1e-12)


def test_symmetric_positive_definite():
    _, _, o = sip(4, 2, n_levels=2)
    A = o.scipy_matrix().toarray()
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    assert np.linalg.eigvalsh(A)[0] > 0


def _manufactured(n, p, nu1=1.0, nu2=1000.0, penalty_c=4.0):
    """u = sin(2 pi x)/nu(x) sin(pi y) sin(pi z), -div(nu grad u) = 6 pi^2 sin(2pi x)
    sin(pi y) sin(pi z) with nu = nu1 for x < 1/2 and nu2 otherwise; u is
    continuous, nu du/dx is continuous and u = 0 on the boundary."""
    h = 1.0 / n
    # keep the coarsest (dense) level small: only the fine operator is used here
    prob = synth.Problem(n, n, n, p, synth.default_levels(n, n, n, 64), h, penalty_c=penalty_c)
    cs = np.arange(n ** 3)
    ijk = np.stack([cs % n, (cs // n) % n, cs // (n * n)], axis=1)
    nu = np.where((ijk[:, 0] + 0.5) * h < 0.5, nu1, nu2)
    o = oracle.Oracle.from_sip(prob, nu)
    A = o.scipy_matrix().tocsc()
    pts, wts = br.tensor_points(p + 4)
    Phi = br.eval_cell(p, h, pts)
    X = ijk[:, None, :] * h + pts[None] * h          # (cells, q, 3)
    S = np.sin(2 * np.pi * X[..., 0]) * np.sin(np.pi * X[..., 1]) * np.sin(np.pi * X[..., 2])
    b = ((6 * np.pi ** 2 * S * wts) @ Phi * h ** 3).reshape(-1)
    uh = spl.spsolve(A, b).reshape(n ** 3, -1)
    U = S / nu[:, None]
    return math.sqrt(np.sum(wts * (U - uh @ Phi.T) ** 2) * h ** 3)


def test_manufactured_solution_convergence_p2_jump():
    """Consistency of the SIP assembly with a coefficient jump of 1000 (interface
    on a cell face): the L2 error of a smooth-per-phase exact solution drops at
    about the optimal rate p+1 = 3."""
    e1 = _manufactured(4, 2)
    e2 = _manufactured(8, 2)
    assert math.log2(e1 / e2) > 2.6, (e1, e2)


def test_manufactured_solution_convergence_p1():
    """P1 on hexahedra with a large penalty is pre-asymptotic on coarse grids
    (near-locking of total-degree P1); with penalty constant 1 the rate between
    8^3 and 16^3 is already above 1.5 and increasing toward 2."""
    e4 = _manufactured(4, 1, 1.0, 1.0, penalty_c=1.0)
    e8 = _manufactured(8, 1, 1.0, 1.0, penalty_c=1.0)
    e16 = _manufactured(16, 1, 1.0, 1.0, penalty_c=1.0)
    r1, r2 = math.log2(e4 / e8), math.log2(e8 / e16)
    assert r2 > 1.5 and r2 > r1, (e4, e8, e16)


# --------------------------------------------------------------------------
# Galerkin coarse operators, transfers, smoother, coarse solve
# --------------------------------------------------------------------------
def test_galerkin_matches_sparse_triple_product():
    prob, nu, o = sip(8, 1, n_levels=3)
    E = o.embedding()
    for l in range(2):
        n = 8 >> l
        A = o.scipy_matrix(l)
        Ac = o.scipy_matrix(l + 1)
        P = P_matrix(E, n, n, n)
        G = (P.T @ A @ P).toarray()
        Acd = Ac.toarray()
        assert np.abs(G - Acd).max() <= 1e-13 * np.abs(G).max()
        assert np.abs(Acd - Acd.T).max() <= 1e-14 * np.abs(Acd).max()
        assert np.linalg.eigvalsh(Acd)[0] > 0


def test_transfers_are_P_and_PT():
    prob, nu, o = sip(8, 2, n_levels=2)
    E = o.embedding()
    P = P_matrix(E, 8, 8, 8)
    rng = np.random.default_rng(5)
    r = rng.standard_normal(P.shape[0])
    zc = rng.standard_normal(P.shape[1])
    assert np.allclose(o.restrict(r), P.T @ r, rtol=1e-14, atol=1e-13)
    assert np.allclose(o.prolong(zc), P @ zc, rtol=1e-14, atol=1e-13)


def test_block_jacobi_smoother_matches_dense():
    """Algorithm 4 from x0 = 0 with s iterations, omega-damped, versus a dense
    numpy implementation with numpy block inverses."""
    prob, nu, o = sip(4, 2, n_levels=2, omega=0.7)
    A = o.scipy_matrix().toarray()
    bs = prob.bs
    Dinv = np.zeros_like(A)
    for c in range(prob.n_cells):
        sl = slice(c * bs, (c + 1) * bs)
        Dinv[sl, sl] = np.linalg.inv(A[sl, sl])
    r = np.random.default_rng(1).standard_normal(prob.n_dofs)
    for s in (1, 2, 3):
        x = np.zeros_like(r)
        for _ in range(s):
            x = x + 0.7 * Dinv @ (r - A @ x)
        assert np.allclose(o.smoother(r, s), x, rtol=1e-12, atol=1e-14 * np.abs(x).max())


def test_coarse_direct_solve():
    prob, nu, o = sip(8, 1, n_levels=2)
    Ac = o.scipy_matrix(1).toarray()
    b = np.random.default_rng(2).standard_normal(Ac.shape[0])
    x = o.coarse_solve(b)
    xs = np.linalg.solve(Ac, b)
    kappa = np.linalg.cond(Ac)
    assert np.linalg.norm(x - xs) <= 10 * kappa * 1e-16 * np.linalg.norm(xs)


# --------------------------------------------------------------------------
# Residual minimisation (Algorithm 1) and OrthoMG (Algorithms 2 and 5)
# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def solved_8p1():
    prob, nu, o = sip(8, 1, n_levels=2, s_pre=1, s_post=1, omega=0.7)
    b = synth.rhs(prob.n_dofs, 0)
    x = o.solve(b, tol=1e-10)
    return prob, nu, o, b, x


def test_dense_direct_solve(solved_8p1):
    """Pin 1: ||x - x*|| / ||x*|| <= kappa_2(A) ||r|| / ||b||."""
    prob, nu, o, b, x = solved_8p1
    A = o.scipy_matrix().toarray()
    xs = np.linalg.solve(A, b)
    ev = np.linalg.eigvalsh(A)
    kappa = ev[-1] / ev[0]
    rel_res = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    assert rel_res <= 1e-10
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= kappa * rel_res


def test_orthonormal_directions(solved_8p1):
    """Pin 3: |W^T W - I| < 1e-12 and A Z = W."""
    prob, nu, o, b, x = solved_8p1
    A = o.scipy_matrix()
    W, Z = o.dirs(0)
    assert W.shape[0] > 10
    assert np.abs(W @ W.T - np.eye(W.shape[0])).max() < 1e-12
    assert np.linalg.norm((A @ Z.T).T - W) / np.linalg.norm(W) < 1e-12


def test_rm_optimality(solved_8p1):
    """Pin 2: x = Z c with c = argmin ||b - A Z c||, and W^T r = 0."""
    prob, nu, o, b, x = solved_8p1
    A = o.scipy_matrix()
    W, Z = o.dirs(0)
    AZ = (A @ Z.T)
    c, *_ = np.linalg.lstsq(AZ, b, rcond=None)
    assert np.linalg.norm(Z.T @ c - x) <= 1e-10 * np.linalg.norm(x)
    r = o.residual(0)
    assert np.abs(W @ r).max() <= 1e-12 * np.linalg.norm(b)


def test_monotone_residual_and_pythagoras(solved_8p1):
    """Pin 4: the residual never increases; ||r_j||^2 - ||r_{j+1}||^2 = alpha^2
    with alpha = w_{j+1} . r_j (W orthonormal)."""
    prob, nu, o, b, x = solved_8p1
    tr = o.trace()
    rn = tr[:, 1]
    assert np.all(rn[1:] <= rn[:-1] * (1 + 1e-14))
    # the trace logs one entry per RM on the finest level (types 1 and 2)
    W, Z = o.dirs(0)
    A = o.scipy_matrix()
    r = b.copy()
    for j in range(W.shape[0]):
        a = W[j] @ r
        rn_next = np.linalg.norm(r - a * W[j])
        assert abs((np.linalg.norm(r) ** 2 - rn_next ** 2) - a * a) <= 1e-10 * np.linalg.norm(r) ** 2
        r = r - a * W[j]


def test_recursive_vs_true_residual(solved_8p1):
    """Pin 5: ||(b - A x) - r|| <= 1e-12 ||b||."""
    prob, nu, o, b, x = solved_8p1
    A = o.scipy_matrix()
    r = o.residual(0)
    assert np.linalg.norm((b - A @ x) - r) <= 1e-12 * np.linalg.norm(b)


def test_mgs2_mode():
    """Oracle option: MGS with one DGKS re-orthogonalisation pass (repeat
    the sweep when ||w_out|| < ||w_in|| / sqrt(2)). It keeps W orthonormal to
    1e-13, reaches the residual 1e-10 and, on this well-converged problem,
    agrees with plain MGS to 1e-8 relative."""
    prob, nu, o2 = sip(8, 1, n_levels=2, gs="mgs2")
    _, _, o1 = sip(8, 1, n_levels=2)
    b = synth.rhs(prob.n_dofs, 0)
    x2 = o2.solve(b)
    x1 = o1.solve(b)
    assert o2.last_report["rel_res_true"] <= 1.0001e-10
    W, _ = o2.dirs(0)
    assert np.abs(W @ W.T - np.eye(W.shape[0])).max() < 1e-13
    assert np.linalg.norm(x2 - x1) <= 1e-8 * np.linalg.norm(x1)


def test_literal_alpha_agrees():
    """Ambiguity: alpha from r0 (literal Algorithm 1) vs from the current r."""
    prob, nu, o = sip(4, 1, n_levels=2)
    _, _, o2 = sip(4, 1, n_levels=2, alpha_mode=1)
    b = synth.rhs(prob.n_dofs, 3)
    x1 = o.solve(b)
    x2 = o2.solve(b)
    assert np.linalg.norm(x1 - x2) <= 1e-10 * np.linalg.norm(x1)


def _dense_parts(o, prob):
    A = o.scipy_matrix().toarray()
    bs = prob.bs
    Dinv = np.zeros_like(A)
    for c in range(prob.n_cells):
        sl = slice(c * bs, (c + 1) * bs)
        Dinv[sl, sl] = np.linalg.inv(A[sl, sl])
    P = P_matrix(o.embedding(), prob.nx, prob.ny, prob.nz).toarray()
    Ac = P.T @ A @ P
    return A, Dinv, P, Ac


def _lsq_update(A, Zs, b):
    AZ = A @ np.stack(Zs, axis=1)
    c, *_ = np.linalg.lstsq(AZ, b, rcond=None)
    x = np.stack(Zs, axis=1) @ c
    return x, b - A @ x


def test_first_sync_cycle_structure():
    """Algorithm 2, first cycle with 2 levels and s = 1: after the cycle,
    x minimises ||b - A x|| over span{z1, z2, z3} with z1 = omega D^-1 b,
    z2 = P Ac^-1 P^T r1, z3 = omega D^-1 r2 (r_j the residual after j RMs)."""
    prob, nu, o = sip(4, 1, n_levels=2, max_iter=1, s_pre=1, s_post=1)
    b = synth.rhs(prob.n_dofs, 7)
    x = o.solve(b, check=False)
    A, Dinv, P, Ac = _dense_parts(o, prob)
    z1 = 0.7 * Dinv @ b
    _, r1 = _lsq_update(A, [z1], b)
    z2 = P @ np.linalg.solve(Ac, P.T @ r1)
    _, r2 = _lsq_update(A, [z1, z2], b)
    z3 = 0.7 * Dinv @ r2
    xr, _ = _lsq_update(A, [z1, z2, z3], b)
    assert np.linalg.norm(x - xr) <= 1e-9 * np.linalg.norm(xr)


def test_first_overlap_cycle_structure():
    """Deterministic Algorithm 5, first cycle with 2 levels: the coarse
    correction is computed from the residual at the start of the cycle
    (z_cor = P Ac^-1 P^T b), the smoother side adds z1 = omega D^-1 b, and x
    minimises the residual over span{z1, z_cor}."""
    prob, nu, o = sip(4, 1, n_levels=2, variant="overlap", max_iter=1, s_post=1, n_s=1)
    b = synth.rhs(prob.n_dofs, 8)
    x = o.solve(b, check=False)
    A, Dinv, P, Ac = _dense_parts(o, prob)
    zc = P @ np.linalg.solve(Ac, P.T @ b)
    z1 = 0.7 * Dinv @ b
    xr, _ = _lsq_update(A, [z1, zc], b)
    assert np.linalg.norm(x - xr) <= 1e-9 * np.linalg.norm(xr)


def test_overlap_variant_converges_monotone():
    prob, nu, o = sip(8, 1, n_levels=2, variant="overlap", s_post=1, n_s=1)
    b = synth.rhs(prob.n_dofs, 0)
    x = o.solve(b)
    rep = o.last_report
    assert rep["rel_res_true"] <= 1.0001e-10
    rn = o.trace()[:, 1]
    assert np.all(rn[1:] <= rn[:-1] * (1 + 1e-14))


def _block_inv(A, bs):
    D = np.zeros_like(A)
    for c in range(A.shape[0] // bs):
        sl = slice(c * bs, (c + 1) * bs)
        D[sl, sl] = np.linalg.inv(A[sl, sl])
    return D


def test_first_hybrid_cycle_structure():
    """Hybrid configuration of Table 1, first cycle on 3 levels with s = 1 and
    one level-1 iteration: the finest level follows Algorithm 2 (pre-smoothing
    z1 = omega D0^-1 b, coarse correction from the residual after it,
    post-smoothing), the level-1 solve follows the Algorithm 5 form (its
    smoother direction and its coarse correction both from the restricted
    residual r_c, combined by RM), so z2 = P0 argmin ||r_c - A1 y|| over
    span{omega D1^-1 r_c, P1 A2^-1 P1^T r_c}. The multiplicative level-1
    cycle would take its coarse correction from an updated residual and give
    a different z2 (checked to differ)."""
    prob, nu, o = sip(8, 1, n_levels=3, variant="hybrid", max_iter=1, s_pre=1, s_post=1, n_s=1,
                      crit=[(-1.0, 1)])
    b = synth.rhs(prob.n_dofs, 9)
    x = o.solve(b, check=False)
    A0 = o.scipy_matrix().toarray()
    E = o.embedding()
    P0 = P_matrix(E, 8, 8, 8).toarray()
    P1 = P_matrix(E, 4, 4, 4).toarray()
    A1 = P0.T @ A0 @ P0
    A2 = P1.T @ A1 @ P1
    bs = prob.bs
    D0, D1 = _block_inv(A0, bs), _block_inv(A1, bs)

    def level1(rc, additive):
        za = 0.7 * D1 @ rc
        if additive:
            zb = P1 @ np.linalg.solve(A2, P1.T @ rc)
            y, _ = _lsq_update(A1, [za, zb], rc)
            return y
        _, r1 = _lsq_update(A1, [za], rc)
        zb = P1 @ np.linalg.solve(A2, P1.T @ r1)
        _, r2 = _lsq_update(A1, [za, zb], rc)
        zc = 0.7 * D1 @ r2
        y, _ = _lsq_update(A1, [za, zb, zc], rc)
        return y

    def cycle(additive):
        z1 = 0.7 * D0 @ b
        _, r1 = _lsq_update(A0, [z1], b)
        z2 = P0 @ level1(P0.T @ r1, additive)
        _, r2 = _lsq_update(A0, [z1, z2], b)
        z3 = 0.7 * D0 @ r2
        xr, _ = _lsq_update(A0, [z1, z2, z3], b)
        return xr

    xr = cycle(additive=True)
    assert np.linalg.norm(x - xr) <= 1e-9 * np.linalg.norm(xr)
    assert np.linalg.norm(x - cycle(additive=False)) > 1e-6 * np.linalg.norm(xr)


def test_step_schedule_first_overlap_cycle():
    """Adaptive loops (Sec. 4.3) replayed with two smoother steps in the
    first cycle (2 levels): the coarse correction comes from the residual at
    the start of the cycle, the smoother steps are multiplicative (the second
    one smooths the residual left by the first RM), and x minimises the
    residual over span{z1, z2, z_cor}."""
    prob, nu, o = sip(4, 1, n_levels=2, variant="overlap", max_iter=1, s_post=1, n_s=1)
    o.set_step_schedule([2])
    b = synth.rhs(prob.n_dofs, 10)
    x = o.solve(b, check=False)
    A, Dinv, P, Ac = _dense_parts(o, prob)
    zc = P @ np.linalg.solve(Ac, P.T @ b)
    z1 = 0.7 * Dinv @ b
    _, r1 = _lsq_update(A, [z1], b)
    z2 = 0.7 * Dinv @ r1
    xr, _ = _lsq_update(A, [z1, z2, zc], b)
    assert np.linalg.norm(x - xr) <= 1e-9 * np.linalg.norm(xr)


def test_step_schedule_hybrid_level1_and_default():
    """The schedule of the hybrid configuration applies to the cycles of
    level 1: with counts [2] the first level-1 iteration takes two smoother
    steps (dense least squares over its three directions); a schedule of n_s
    everywhere equals running without one, bit for bit."""
    prob, nu, o = sip(8, 1, n_levels=3, variant="hybrid", max_iter=1, s_pre=1, s_post=1, n_s=1,
                      crit=[(-1.0, 1)])
    o.set_step_schedule([2])
    b = synth.rhs(prob.n_dofs, 9)
    x = o.solve(b, check=False)
    A0 = o.scipy_matrix().toarray()
    E = o.embedding()
    P0 = P_matrix(E, 8, 8, 8).toarray()
    P1 = P_matrix(E, 4, 4, 4).toarray()
    A1 = P0.T @ A0 @ P0
    A2 = P1.T @ A1 @ P1
    D0, D1 = _block_inv(A0, prob.bs), _block_inv(A1, prob.bs)
    z1 = 0.7 * D0 @ b
    _, r1 = _lsq_update(A0, [z1], b)
    rc = P0.T @ r1
    za = 0.7 * D1 @ rc
    _, rca = _lsq_update(A1, [za], rc)
    zb = 0.7 * D1 @ rca
    zcor = P1 @ np.linalg.solve(A2, P1.T @ rc)
    y, _ = _lsq_update(A1, [za, zb, zcor], rc)
    z2 = P0 @ y
    _, r2 = _lsq_update(A0, [z1, z2], b)
    z3 = 0.7 * D0 @ r2
    xr, _ = _lsq_update(A0, [z1, z2, z3], b)
    assert np.linalg.norm(x - xr) <= 1e-9 * np.linalg.norm(xr)
    prob, nu, o1 = sip(8, 1, n_levels=3, variant="hybrid", s_post=2, n_s=1)
    b = synth.rhs(prob.n_dofs, 0)
    x1 = o1.solve(b)
    o1.set_step_schedule([1] * 500)
    assert np.array_equal(o1.solve(b), x1)
    with pytest.raises(oracle.OracleError):
        o1.set_step_schedule([1, 0])


def test_hybrid_two_levels_is_sync():
    """With two levels no level runs the Algorithm 5 form, so the hybrid
    configuration is Algorithm 2 exactly (bit for bit)."""
    prob, nu, o1 = sip(8, 1, n_levels=2, variant="hybrid")
    _, _, o2 = sip(8, 1, n_levels=2, variant="sync")
    b = synth.rhs(prob.n_dofs, 0)
    assert np.array_equal(o1.solve(b), o2.solve(b))
    assert o1.last_report["iters_fine"] == o2.last_report["iters_fine"]


@pytest.mark.parametrize("variant", ["hybrid", "add_sync"])
def test_table1_variants_converge(variant):
    """Hybrid and additive synchronous solves on 4 levels reach the true
    residual 1e-10 with a monotone finest-level residual; additive
    synchronous runs the deterministic Algorithm 5 order, i.e. it equals the
    overlap variant of this sequential code bit for bit."""
    prob, nu, o = sip(16, 1, n_levels=4, variant=variant, s_post=2)
    b = synth.rhs(prob.n_dofs, 0)
    x = o.solve(b)
    assert o.last_report["rel_res_true"] <= 1.0001e-10
    rn = o.trace()[:, 1]
    assert np.all(rn[1:] <= rn[:-1] * (1 + 1e-14))
    if variant == "add_sync":
        _, _, o2 = sip(16, 1, n_levels=4, variant="overlap", s_post=2)
        assert np.array_equal(x, o2.solve(b))
    v = o.visits()
    assert np.all(v[v[:, 0] == 1][:, 1] <= 20) and np.all(v[v[:, 0] == 2][:, 1] <= 2)


def _dense_schwarz(A, bs):
    """sum_i P_i (R_i A P_i)^-1 R_i with subdomain i = cell i and the cells
    its block row couples to (dense, numpy)."""
    n = A.shape[0] // bs
    M = np.zeros_like(A)
    for c in range(n):
        row = A[c * bs:(c + 1) * bs]
        cells = [c] + [d for d in range(n) if d != c and np.any(row[:, d * bs:(d + 1) * bs] != 0.0)]
        idx = np.concatenate([np.arange(d * bs, (d + 1) * bs) for d in cells])
        M[np.ix_(idx, idx)] += np.linalg.inv(A[np.ix_(idx, idx)])
    return M


@pytest.mark.parametrize("p", [1, 2])
def test_schwarz_smoother_matches_dense(p):
    """Additive Schwarz (Algorithm 3) with one cell per subdomain and a one-cell
    overlap: one sweep is omega sum_i P_i A_i^-1 R_i r, a second sweep adds
    omega M (r - A x); checked against dense inverses of the patch matrices,
    on the finest and on a Galerkin level."""
    prob, nu, o = sip(4, p, n_levels=3, smoother="schwarz")
    for l in (0, 1):
        A = o.scipy_matrix(l).toarray()
        M = _dense_schwarz(A, prob.bs)
        r = np.random.default_rng(l).standard_normal(A.shape[0])
        x1 = 0.7 * M @ r
        assert np.abs(o.smoother(r, 1, l) - x1).max() <= 1e-12 * np.abs(x1).max()
        x2 = x1 + 0.7 * M @ (r - A @ x1)
        assert np.abs(o.smoother(r, 2, l) - x2).max() <= 1e-11 * np.abs(x2).max()
        assert np.abs(M - M.T).max() <= 1e-10 * np.abs(M).max() and np.linalg.eigvalsh(M).min() > 0


def test_schwarz_without_overlap_is_block_jacobi():
    """Block-diagonal operator: every subdomain is a single cell, so the
    additive Schwarz sweep equals the block-Jacobi sweep."""
    rng = np.random.default_rng(4)
    n, bs = 8, 4
    blocks = []
    for _ in range(n):
        B = rng.standard_normal((bs, bs))
        blocks.append(B @ B.T + bs * np.eye(bs))
    rp, ci, v = np.arange(n + 1), np.arange(n), np.stack(blocks)
    oa = oracle.Oracle.from_bsr(rp, ci, v, 2, 2, 2, 1, 2, smoother="schwarz")
    ob = oracle.Oracle.from_bsr(rp, ci, v, 2, 2, 2, 1, 2)
    r = rng.standard_normal(n * bs)
    for s in (1, 2):
        xa, xb = oa.smoother(r, s), ob.smoother(r, s)
        assert np.abs(xa - xb).max() <= 1e-13 * np.abs(xb).max()


def test_schwarz_solve_converges_and_single_precision_local_solves():
    prob, nu, o = sip(8, 1, n_levels=3, smoother="schwarz", s_pre=1, s_post=1)
    _, _, ob = sip(8, 1, n_levels=3, s_pre=1, s_post=1)
    b = synth.rhs(prob.n_dofs, 0)
    o.solve(b)
    rep = o.last_report
    assert rep["rel_res_true"] <= 1.0001e-10
    rn = o.trace()[:, 1]
    assert np.all(rn[1:] <= rn[:-1] * (1 + 1e-14))
    ob.solve(b)
    print(f"cycles: additive Schwarz {rep['iters_fine']}, block-Jacobi {ob.last_report['iters_fine']}")
    # mixed forms: single-precision local solves (Sec. 3.2) within float
    # rounding of the dense FP64 sweep, and FP64 refinement still reaches 1e-10
    _, _, om = sip(4, 2, n_levels=2, smoother="schwarz", precision="mixed_ir")
    A = om.scipy_matrix(0).toarray()
    M = _dense_schwarz(A, 10)
    r = np.random.default_rng(2).standard_normal(A.shape[0])
    x1 = 0.7 * M @ r
    y = om.smoother(r, 1, 0, fp32=True)
    err = np.abs(y - x1).max() / np.abs(x1).max()
    assert 1e-9 < err <= 2e-5, err
    _, _, om = sip(8, 1, n_levels=3, smoother="schwarz", s_pre=1, s_post=1, precision="mixed_ir")
    om.solve(b)
    assert om.last_report["rel_res_true"] <= 1.0001e-10


def test_restart_after_m_max_directions():
    """Option m_max (bounded direction storage, reading 9): when a level holds
    m_max directions, the next RM restarts from x0 = x, r0 = r with W = Z = {}.
    First cycle of Algorithm 2 on 2 levels with s = 1 and m_max = 2: z1, z2 are
    combined by least squares from b, then z3 = omega D^-1 r2 alone from r2
    (dense); without the restart x spans all three directions (differs).
    Solves with restarts still reach 1e-10 with a monotone residual, and an
    m_max above the number of directions equals no restart bit for bit."""
    prob, nu, o = sip(4, 1, n_levels=2, max_iter=1, s_pre=1, s_post=1, m_max=2)
    b = synth.rhs(prob.n_dofs, 11)
    x = o.solve(b, check=False)
    A, Dinv, P, Ac = _dense_parts(o, prob)
    z1 = 0.7 * Dinv @ b
    _, r1 = _lsq_update(A, [z1], b)
    z2 = P @ np.linalg.solve(Ac, P.T @ r1)
    xa, r2 = _lsq_update(A, [z1, z2], b)
    z3 = 0.7 * Dinv @ r2
    xb, _ = _lsq_update(A, [z3], r2)
    assert np.linalg.norm(x - (xa + xb)) <= 1e-9 * np.linalg.norm(xa + xb)
    xr, _ = _lsq_update(A, [z1, z2, z3], b)
    assert np.linalg.norm(x - xr) > 1e-6 * np.linalg.norm(xr)
    prob, nu, o = sip(8, 1, n_levels=3, m_max=8)
    b = synth.rhs(prob.n_dofs, 0)
    o.solve(b)
    assert o.last_report["rel_res_true"] <= 1.0001e-10
    rn = o.trace()[:, 1]
    assert np.all(rn[1:] <= rn[:-1] * (1 + 1e-14))
    _, _, o1 = sip(8, 1, n_levels=3)
    _, _, o2 = sip(8, 1, n_levels=3, m_max=100000)
    assert np.array_equal(o1.solve(b), o2.solve(b))


def test_level_criteria_counts():
    """Sec. 4.2: level 1 stops at 0.1 r0 or 20 iterations, level 2 at 0.5 r0
    or 2 iterations, deeper levels after one iteration."""
    prob, nu, o = sip(16, 1, n_levels=4)
    b = synth.rhs(prob.n_dofs, 0)
    o.solve(b)
    v = o.visits()
    assert set(v[v[:, 0] == 3][:, 1]) <= {0}  # coarsest level: direct solve, no visits logged
    assert np.all(v[v[:, 0] == 2][:, 1] <= 2) and np.all(v[v[:, 0] == 2][:, 1] >= 1)
    assert np.all(v[v[:, 0] == 1][:, 1] <= 20) and np.all(v[v[:, 0] == 1][:, 1] >= 1)


def test_omega_cancels_with_one_sweep():
    """With one block-Jacobi iteration per smoother call, RM's normalisation
    removes omega: omega = 0.7 and omega = 1 give the same solution."""
    prob, nu, o1 = sip(4, 1, n_levels=2, omega=0.7)
    _, _, o2 = sip(4, 1, n_levels=2, omega=1.0)
    b = synth.rhs(prob.n_dofs, 0)
    x1 = o1.solve(b)
    x2 = o2.solve(b)
    assert np.linalg.norm(x1 - x2) <= 1e-11 * np.linalg.norm(x1)


def test_one_level_is_cholesky():
    prob, nu, o = sip(4, 1, n_levels=1)
    b = synth.rhs(prob.n_dofs, 0)
    x = o.solve(b)
    A = o.scipy_matrix().toarray()
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-9, atol=1e-12 * np.abs(x).max())


def test_single_cell_block_jacobi_is_exact():
    prob, nu, o = sip(2, 1, n_levels=2, omega=1.0)
    A = o.scipy_matrix(1).toarray()  # 1 coarse cell
    # on a one-cell level, one omega=1 block-Jacobi iteration is the exact solve
    _, _, o1 = sip(2, 1, n_levels=2, omega=1.0)
    r = np.random.default_rng(0).standard_normal(prob.n_dofs)
    A0 = o1.scipy_matrix(0).toarray()
    bs = prob.bs
    D = np.zeros_like(A0)
    for c in range(prob.n_cells):
        sl = slice(c * bs, (c + 1) * bs)
        D[sl, sl] = A0[sl, sl]
    assert np.allclose(o1.smoother(r, 1), np.linalg.solve(D, r), rtol=1e-12)
    assert A.shape == (bs, bs)


def test_nu_scaling():
    """A is 1-homogeneous in nu: nu -> c nu gives x -> x / c."""
    prob = synth.make_problem(4, 1, n_levels=2)
    nu = synth.nu_sphere(4, 4, 4, prob.h)
    b = synth.rhs(prob.n_dofs, 0)
    x1 = oracle.Oracle.from_sip(prob, nu).solve(b, tol=1e-12)
    x2 = oracle.Oracle.from_sip(prob, 8.0 * nu).solve(b, tol=1e-12)
    assert np.linalg.norm(8.0 * x2 - x1) <= 1e-10 * np.linalg.norm(x1)


def test_zero_rhs_and_errors():
    prob, nu, o = sip(4, 1, n_levels=2)
    x = o.solve(np.zeros(prob.n_dofs))
    assert np.all(x == 0)
    bad = synth.rhs(prob.n_dofs, 0)
    bad[5] = np.nan
    with pytest.raises(oracle.OracleError) as e:
        o.solve(bad)
    assert e.value.status == oracle.EINVAL
    _, _, o1 = sip(4, 1, n_levels=2, max_iter=1)
    with pytest.raises(oracle.OracleError) as e:
        o1.solve(synth.rhs(prob.n_dofs, 0))
    assert e.value.status == oracle.ENOCONV
    # non-SPD operator: negative penalty
    with pytest.raises(oracle.OracleError) as e:
        oracle.Oracle.from_sip(synth.Problem(4, 4, 4, 1, 2, 0.25, penalty_c=-4.0), nu)
    assert e.value.status == oracle.ENOTSPD
    # malformed BSR: unsorted columns
    rp, ci, v = o.matrix(0)
    ci2 = ci.copy()
    ci2[[0, 1]] = ci2[[1, 0]]
    with pytest.raises(oracle.OracleError) as e:
        oracle.Oracle.from_bsr(rp, ci2, v, 4, 4, 4, 1, 2)
    assert e.value.status == oracle.EINVAL


def test_generic_bsr_input():
    """Setup from a random SPD block matrix (not the SIP operator) solves it."""
    rp, ci, v = synth.random_spd_bsr(4, 4, 4, 4, seed=1)
    o = oracle.Oracle.from_bsr(rp, ci, v, 4, 4, 4, 1, 2)
    b = synth.rhs(64 * 4, 1)
    x = o.solve(b, tol=1e-12)
    A = sp.bsr_matrix((v, ci, rp), shape=(256, 256)).toarray()
    assert np.linalg.norm(b - A @ x) <= 1.0001e-12 * np.linalg.norm(b)


# --------------------------------------------------------------------------
# Mixed precision (FP32 inner, FP64 outer)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("mode", ["mixed_ir", "mixed_flex"])
def test_mixed_precision_reaches_fp64_residual(mode):
    prob, nu, o = sip(8, 1, n_levels=2, precision=mode)
    b = synth.rhs(prob.n_dofs, 0)
    x = o.solve(b, tol=1e-10)
    A = o.scipy_matrix()
    assert np.linalg.norm(b - A @ x) <= 1.0001e-10 * np.linalg.norm(b)


# --------------------------------------------------------------------------
# Gradient (adjoint solve + per-cell dA/dnu contraction)
# --------------------------------------------------------------------------
def test_gradient_identities_and_fd():
    n, p = 4, 1
    prob = synth.make_problem(n, p, n_levels=2)
    nu = synth.nu_sphere(n, n, n, prob.h, nu_out=10.0)
    f = synth.rhs(prob.n_dofs, 0)
    ut = synth.rhs(prob.n_dofs, 1)
    o = oracle.Oracle.from_sip(prob, nu)
    u = o.solve(f, tol=1e-14, check=False)
    g_f, g_nu = o.grad(u, u - ut, tol=1e-14) if False else _grad_loose(o, u, u - ut)
    g_lognu = nu * g_nu
    # Euler: sum_K nu_K dA/dnu_K = A  =>  sum_K dL/dlog nu_K = -lambda^T f = -(u-ut)^T u
    assert abs(g_lognu.sum() + (u - ut) @ u) <= 1e-8 * abs((u - ut) @ u)
    assert abs(g_lognu.sum() + g_f @ f) <= 1e-8 * abs(g_f @ f)

    def loss(lognu):
        oo = oracle.Oracle.from_sip(prob, np.exp(lognu))
        A = oo.scipy_matrix().toarray()
        uu = np.linalg.solve(A, f)
        return 0.5 * np.sum((uu - ut) ** 2)

    lognu = np.log(nu)
    rng = np.random.default_rng(3)
    # step 1e-4: the loss carries ||u_t||^2 ~ 1e2, so a 1e-6 step would sit on
    # the roundoff floor at this size; the central-difference truncation error
    # at 1e-4 is ~1e-8 relative
    for c in rng.choice(prob.n_cells, size=5, replace=False):
        e = np.zeros_like(lognu)
        e[c] = 1e-4
        fd = (loss(lognu + e) - loss(lognu - e)) / 2e-4
        assert abs(fd - g_lognu[c]) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(g_lognu).max())
    # dL/df = A^-1 (u - ut)
    A = o.scipy_matrix().toarray()
    assert np.allclose(g_f, np.linalg.solve(A, u - ut), rtol=1e-8, atol=1e-10 * np.abs(g_f).max())


def _grad_loose(o, u, gu):
    g_f = np.zeros(o.n)
    g_nu = np.zeros(o.n_cells)
    rep = oracle.Report()
    lib = oracle.lib()
    st = lib.oracle_grad(o._h, oracle._p(np.ascontiguousarray(u)), oracle._p(np.ascontiguousarray(gu)),
                         oracle._p(g_f), oracle._p(g_nu), 1e-13, oracle.ctypes.byref(rep))
    assert st in (oracle.OK, oracle.ENOCONV)
    return g_f, g_nu
