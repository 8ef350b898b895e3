"""The single-precision level kernels of the mixed forms (SpMV, block-Jacobi,
restriction, prolongation: operator, inverses and embedding rounded to
float, float arithmetic) against the oracle's FP32 emulation, element by
element: both lie within the float rounding bound of the exact result on the
rounded data, so they differ by at most twice that bound. The paper's
precedent is single-precision local solves under double-precision
residuals (Sec. 3.2); the measured errors are printed."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
EPS32 = float(np.finfo(np.float32).eps)


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


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def check_fp32_kernels(prob, o, g, rng, levels):
    bs = prob.bs
    E = o.embedding()
    worst = {}
    for l in levels:
        A = o.scipy_matrix(l)
        absA = abs(A.astype(np.float32).astype(np.float64))
        N = A.shape[0]
        x, b = rng.standard_normal(N), rng.standard_normal(N)
        width = np.diff(A.indptr).max() // bs
        terms = width * bs + 2
        bnd = 2 * terms * EPS32 * (absA @ np.abs(f32(x)) + np.abs(f32(b)))
        yo = o.spmv(x, l, b, fp32=True)
        yg = host(g.level_spmv(l, cuda(x), cuda(b), fp32=True))
        assert np.all(np.abs(yg - yo) <= bnd), l
        worst[f"spmv{l}"] = np.abs(yg - yo).max() / np.abs(yo).max()
        for s in (1, 2):
            so = o.smoother(b, s, l, fp32=True)
            sg = host(g.level_smoother(l, cuda(b), s, fp32=True))
            err = np.abs(sg - so).max() / np.abs(so).max()
            worst[f"bj{l}x{s}"] = err
            assert err <= 2e-5, (l, s, err)
        if l + 1 < prob.n_levels:
            ro = o.restrict(x, l, fp32=True)
            rg = host(g.level_restrict(l, cuda(x), fp32=True))
            nc = len(ro) // bs
            # bound: 8 children x bs products each, |E| |x|
            absE = np.abs(f32(E)).max()
            bnd_r = 2 * (8 * bs + 2) * EPS32 * absE * np.abs(x).max() * 8 * bs
            assert np.abs(rg - ro).max() <= bnd_r, l
            worst[f"restrict{l}"] = np.abs(rg - ro).max() / np.abs(ro).max()
            zc = rng.standard_normal(nc * bs)
            po = o.prolong(zc, l, fp32=True)
            pg = host(g.level_prolong(l, cuda(zc), fp32=True))
            bnd_p = 2 * (bs + 2) * EPS32 * absE * np.abs(zc).max() * bs
            assert np.abs(pg - po).max() <= bnd_p, l
            worst[f"prolong{l}"] = np.abs(pg - po).max() / np.abs(po).max()
    print(" ".join(f"{k} {v:.1e}" for k, v in worst.items()))


@pytest.mark.parametrize("n,p,lv", [(8, 1, 2), (16, 2, 2), (16, 1, 4), (8, 2, 3), (4, 3, 2)])
def test_fp32_level_kernels(n, p, lv):
    prob = synth.make_problem(n, p, n_levels=lv)
    nu = synth.nu_sphere(n, n, n, prob.h)
    o = oracle.Oracle.from_sip(prob, nu)
    g = omg().Solver.from_sip(omg().Solver.make_grid(n, n, n, p, lv, prob.h), cuda(nu))
    check_fp32_kernels(prob, o, g, np.random.default_rng(17), range(lv - 1))
