"""Pins of the oracle's single-precision emulation (the FP32 inner work of
the mixed forms; the paper's precedent is single-precision local solves with
double-precision residuals, Sec. 3.2): each FP32 level operation equals its
exact result with the operator rounded to float within the float rounding
bound of its sums, and differs from the FP64 operation by the rounding of
the operator (so the float path is really taken)."""
import numpy as np
import pytest

import oracle
import synth

EPS32 = np.finfo(np.float32).eps


@pytest.fixture(scope="module")
def setup():
    prob = synth.make_problem(8, 2, n_levels=3)
    nu = synth.nu_sphere(8, 8, 8, prob.h)
    o = oracle.Oracle.from_sip(prob, nu, s_pre=2, s_post=2)
    return prob, o


def _bound(absA, absx, terms):
    """Float rounding bound of a sum of `terms` products plus the rounding
    of its inputs: (terms + 2) eps |A| |x| (Higham, Sec. 3.1)."""
    return (terms + 2) * EPS32 * (absA @ absx)


def test_spmv32_within_float_bound(setup):
    prob, o = setup
    rng = np.random.default_rng(11)
    for l in range(2):
        A = o.scipy_matrix(l)
        A32 = A.astype(np.float32).astype(np.float64)      # operator rounded to float
        x = rng.standard_normal(A.shape[0])
        x32 = x.astype(np.float32).astype(np.float64)
        b = rng.standard_normal(A.shape[0])
        exact = b.astype(np.float32).astype(np.float64) - A32 @ x32   # exact in FP64
        y = o.spmv(x, l=l, b=b, fp32=True)
        terms = 7 * prob.bs
        bnd = _bound(abs(A32), np.abs(x32), terms) + EPS32 * np.abs(exact)
        assert np.all(np.abs(y - exact) <= bnd)
        # float results: every entry is a float, and differs from the FP64 SpMV
        assert np.array_equal(y, y.astype(np.float32).astype(np.float64))
        y64 = o.spmv(x, l=l, b=b)
        assert np.abs(y - y64).max() > 1e-3 * EPS32 * np.abs(abs(A) @ np.abs(x)).max()


def test_transfers32_within_float_bound(setup):
    prob, o = setup
    E32 = o.embedding().astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(12)
    n, bs = 8, prob.bs
    # P with rounded blocks, built from the 2x2x2 geometry
    rows, cols, vals = [], [], []
    for c in range(n ** 3):
        i, j, k = c % n, (c // n) % n, c // (n * n)
        I = i // 2 + (n // 2) * (j // 2 + (n // 2) * (k // 2))
        s = (i % 2) + 2 * (j % 2) + 4 * (k % 2)
        rr, cc = np.meshgrid(np.arange(bs), np.arange(bs), indexing="ij")
        rows.append((c * bs + rr).ravel()); cols.append((I * bs + cc).ravel()); vals.append(E32[s].ravel())
    import scipy.sparse as sp
    P = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n ** 3 * bs, (n // 2) ** 3 * bs))
    r = rng.standard_normal(P.shape[0])
    r32 = r.astype(np.float32).astype(np.float64)
    rc = o.restrict(r, fp32=True)
    ex = P.T @ r32
    assert np.all(np.abs(rc - ex) <= _bound(abs(P.T), np.abs(r32), 8 * bs + 8))
    assert np.abs(rc - o.restrict(r)).max() > 0
    zc = rng.standard_normal(P.shape[1])
    zc32 = zc.astype(np.float32).astype(np.float64)
    z = o.prolong(zc, fp32=True)
    ex = P @ zc32
    assert np.all(np.abs(z - ex) <= _bound(abs(P), np.abs(zc32), bs))
    assert np.array_equal(z, z.astype(np.float32).astype(np.float64))


def test_block_jacobi32_within_float_bound(setup):
    """One and two single-precision block-Jacobi iterations from zero
    (Algorithm 4) against the same iterations in FP64 on the float-rounded
    operator and inverses: agreement to a small multiple of float rounding."""
    prob, o = setup
    A = o.scipy_matrix(0)
    A32 = A.astype(np.float32).astype(np.float64).toarray()
    bs = prob.bs
    D = o.dinv(0).astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(13)
    r = rng.standard_normal(A.shape[0])
    r32 = r.astype(np.float32).astype(np.float64)
    om = np.float64(np.float32(0.7))

    def dapply(v, M=D):
        return np.einsum("cij,cj->ci", M, v.reshape(-1, bs)).reshape(-1)

    absD = np.abs(D)

    x1 = om * dapply(r32)
    y1 = o.smoother(r, 1, fp32=True)
    scale = dapply(np.abs(r32), absD)
    assert np.all(np.abs(y1 - x1) <= (bs + 4) * EPS32 * scale + 1e-30)
    x2 = x1 + om * dapply(r32 - A32 @ x1)
    y2 = o.smoother(r, 2, fp32=True)
    scale2 = scale + dapply(np.abs(r32) + np.abs(A32) @ np.abs(x1), absD)
    assert np.all(np.abs(y2 - x2) <= (7 * bs + bs + 8) * EPS32 * scale2 * 4)
    y64 = o.smoother(r, 2)
    assert np.abs(y2 - y64).max() > 1e-3 * EPS32 * np.abs(y64).max()
