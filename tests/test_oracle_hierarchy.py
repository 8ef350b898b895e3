"""Pins of the oracle with a caller-supplied agglomeration hierarchy (the R
and P of Algorithm 2 given as parent/slot maps and the eight embedding
blocks): the 2x2x2 maps reproduce the built-in hierarchy bit for bit, a
renumbering of the cells on every level gives the same solution, and a grid
whose sides are not powers of two (coarse cells with fewer than eight
children) gives Galerkin operators equal to the sparse triple product and
a solve that meets the dense solution's bound."""
import numpy as np
import scipy.sparse as sp

import oracle
import synth


def cartesian_maps(nx, ny, nz, n_levels):
    """parent/slot of the 2x2x2 agglomeration; a side of odd length puts its
    last cell alone in a coarse cell (slot of the left child)."""
    dims = [(nx, ny, nz)]
    for _ in range(n_levels - 1):
        a, b, c = dims[-1]
        dims.append(((a + 1) // 2, (b + 1) // 2, (c + 1) // 2))
    parents, slots = [], []
    for l in range(n_levels - 1):
        a, b, c = dims[l]
        ca, cb, _ = dims[l + 1]
        idx = np.arange(a * b * c)
        i, j, k = idx % a, (idx // a) % b, idx // (a * b)
        parents.append((i // 2 + ca * (j // 2 + cb * (k // 2))).astype(np.int32))
        slots.append(((i & 1) + 2 * (j & 1) + 4 * (k & 1)).astype(np.uint8))
    return [d[0] * d[1] * d[2] for d in dims], parents, slots


def P_of(parent, slot, E, nc):
    bs = E.shape[1]
    rows, cols, vals = [], [], []
    rr, cc = np.meshgrid(np.arange(bs), np.arange(bs), indexing="ij")
    for K, (I, s) in enumerate(zip(parent, slot)):
        rows.append((K * bs + rr).ravel()); cols.append((I * bs + cc).ravel()); vals.append(E[s].ravel())
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(len(parent) * bs, nc * bs))


def fine_operator(n, p, nx=None):
    """SIP operator of an n^3 (or nx*n*n) grid from the oracle's assembly."""
    prob = synth.Problem(nx=nx or n, ny=n, nz=n, p=p, n_levels=1, h=1.0 / n)
    nu = synth.nu_sphere(prob.nx, n, n, prob.h)
    o = oracle.Oracle.from_sip(prob, nu)
    return prob, o.matrix(0)


def test_cartesian_maps_reproduce_builtin_hierarchy():
    prob = synth.make_problem(8, 1, n_levels=3)
    nu = synth.nu_sphere(8, 8, 8, prob.h)
    ob = oracle.Oracle.from_sip(prob, nu)
    rp, ci, v = ob.matrix(0)
    nc, par, sl = cartesian_maps(8, 8, 8, 3)
    oh = oracle.Oracle.from_bsr_hierarchy(rp, ci, v, nc, par, sl, oracle.embedding(1))
    for l in range(3):
        a, b = ob.matrix(l), oh.matrix(l)
        assert all(np.array_equal(x, y) for x, y in zip(a, b))
    bvec = synth.rhs(prob.n_dofs, 0)
    assert np.array_equal(ob.solve(bvec), oh.solve(bvec))
    assert np.array_equal(ob.visits(), oh.visits())


def test_renumbered_cells_give_the_same_solve():
    """Permute the cells of every level (operator rows/columns, maps and right
    hand side alike): the visit log is the same and the solution is the
    permuted one to rounding."""
    prob = synth.make_problem(8, 1, n_levels=3)
    nu = synth.nu_sphere(8, 8, 8, prob.h)
    ob = oracle.Oracle.from_sip(prob, nu)
    A = ob.scipy_matrix(0)
    bs = prob.bs
    nc, par, sl = cartesian_maps(8, 8, 8, 3)
    rng = np.random.default_rng(21)
    perms = [rng.permutation(n) for n in nc]          # new index of old cell
    inv = [np.argsort(p) for p in perms]              # old cell of new index
    dof = np.concatenate([inv[0][:, None] * bs + np.arange(bs)]).reshape(-1)  # old dof of new dof
    Ap = sp.bsr_matrix(A[dof][:, dof], blocksize=(bs, bs))
    Ap.sort_indices()
    par_p = [perms[l + 1][par[l][inv[l]]].astype(np.int32) for l in range(2)]
    sl_p = [sl[l][inv[l]] for l in range(2)]
    op = oracle.Oracle.from_bsr_hierarchy(Ap.indptr, Ap.indices, Ap.data, nc, par_p, sl_p, oracle.embedding(1))
    b = synth.rhs(prob.n_dofs, 0)
    x = ob.solve(b)
    xp = op.solve(b[dof])
    assert np.array_equal(ob.visits(), op.visits())
    assert np.linalg.norm(xp - x[dof]) <= 1e-9 * np.linalg.norm(x)


def test_partial_coarse_cells():
    """6x6x6 P1 -> 3x3x3 -> 2x2x2: the 3 -> 2 step has coarse cells with one,
    two, four or eight children. P^T A P equals the sparse triple product and
    is SPD; the solve reaches 1e-10 and the dense solution's bound."""
    n, p = 6, 1
    prob, (rp, ci, v) = fine_operator(n, p)
    nc, par, sl = cartesian_maps(6, 6, 6, 3)
    assert nc == [216, 27, 8]
    E = oracle.embedding(p)
    o = oracle.Oracle.from_bsr_hierarchy(rp, ci, v, nc, par, sl, E, s_pre=1, s_post=1)
    A = o.scipy_matrix(0)
    for l in range(2):
        P = P_of(par[l], sl[l], E, nc[l + 1])
        G = (P.T @ o.scipy_matrix(l) @ P).toarray()
        Ac = o.scipy_matrix(l + 1).toarray()
        assert np.abs(G - Ac).max() <= 1e-13 * np.abs(G).max()
        assert np.linalg.eigvalsh(Ac)[0] > 0
    counts = np.bincount(par[1], minlength=8)
    assert sorted(set(counts.tolist())) == [1, 2, 4, 8]
    b = synth.rhs(A.shape[0], 0)
    x = o.solve(b, tol=1e-10)
    Ad = A.toarray()
    xs = np.linalg.solve(Ad, b)
    rr = np.linalg.norm(b - Ad @ x) / np.linalg.norm(b)
    assert rr <= 1.0001e-10
    ev = np.linalg.eigvalsh(Ad)
    assert np.linalg.norm(x - xs) <= (ev[-1] / ev[0]) * rr * np.linalg.norm(xs) * 1.01
