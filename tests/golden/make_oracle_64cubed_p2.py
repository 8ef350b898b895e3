"""Write the oracle's reference solve of the 64^3 P2 workload.

Runs the FP64 CPU oracle (and nothing else: the seeded inputs come from
``synth``) on the plain-method workload -- 64^3 cells, P2 (2,621,440 DOFs),
coefficient 1 inside the sphere of radius 0.3 about the cube centre and 1000
outside, four agglomeration levels, Algorithm 2 with 2 pre- and 2
post-smoothing block-Jacobi sweeps (omega 0.7), the level tests of Sec. 4.2,
b ~ N(0,1) from seed 0, tolerance 1e-10 -- and stores what a replayed GPU
solve is compared with:

* ``visits``: the (level, iterations) log in completion order;
* ``vnorm``: the per-visit residual log (level, iterations, ||r0||, ||r||
  after each iteration);
* ``idx`` / ``x_idx``: the solution at 65,536 entries drawn by
  ``default_rng(7)``;
* ``x_norm``, ``x_dot_b``, ``x_dot_u``: ||x||, x.b and x.u with
  u ~ N(0,1) from seed 8 (functionals of the whole vector);
* ``report``: iterations, stored directions, recursive and true residuals.

With --perturb the right-hand side is b (1 + 1e-15 xi), xi ~ N(0,1) from
seed 5, and the output goes to oracle_64cubed_p2_perturbed.npz: the same
solve after a perturbation at rounding level, which measures how far two
correct runs of the method (different rounding) can end apart.

The full solve takes about 90 minutes on seven cores and ~33 GB of memory
(the finest level stores ~770 direction pairs of 21 MB each).

    OMP_NUM_THREADS=8 python tests/golden/make_oracle_64cubed_p2.py [--perturb]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

PERTURB = "--perturb" in sys.argv
OUT = os.path.join(HERE, "oracle_64cubed_p2_perturbed.npz" if PERTURB else "oracle_64cubed_p2.npz")


def main():
    prob = synth.make_problem(64, 2)
    assert prob.n_levels == 4
    nu = synth.nu_sphere(64, 64, 64, prob.h)
    b = synth.rhs(prob.n_dofs, 0)
    if PERTURB:
        b = b * (1 + 1e-15 * np.random.default_rng(5).standard_normal(prob.n_dofs))
    t0 = time.time()
    o = oracle.Oracle.from_sip(prob, nu, s_pre=2, s_post=2)
    print(f"setup {time.time() - t0:.1f} s, {oracle.num_threads()} threads", flush=True)
    t0 = time.time()
    x = o.solve(b, tol=1e-10)
    t_solve = time.time() - t0
    rep = o.last_report
    print(f"solve {t_solve:.1f} s: {rep}", flush=True)
    idx = np.sort(np.random.default_rng(7).choice(prob.n_dofs, 65536, replace=False))
    u = synth.rhs(prob.n_dofs, 8)
    vn = o.visit_norms()
    flat = []
    for l, it, r0, rns in vn:
        flat += [l, it, r0, *rns.tolist()]
    np.savez_compressed(
        OUT,
        visits=o.visits().astype(np.int32),
        vnorm=np.array(flat),
        idx=idx.astype(np.int64),
        x_idx=x[idx],
        x_norm=np.linalg.norm(x),
        x_dot_b=float(x @ b),
        x_dot_u=float(x @ u),
        report=json.dumps({**rep, "t_solve_s": t_solve, "threads": oracle.num_threads()}),
    )
    print(f"wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()
