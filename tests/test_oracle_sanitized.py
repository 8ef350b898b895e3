"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU): the source is built with -fsanitize=address,undefined into a
temporary library, and a child interpreter (with the sanitizer runtime
preloaded, as the interpreter itself is not instrumented) runs small solves
through every code path the tests use: setup from the SIP grid and from a
BSR operator with a caller hierarchy (partial coarse cells), the four Table 1
configurations, additive Schwarz, single-precision inner work, m_max
restarts with forced breakdowns, replayed schedules, the visit and norm
logs, level operations and the gradient. Any sanitizer report fails it."""
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r'''
import numpy as np
import oracle, synth
from tests.test_oracle_hierarchy import cartesian_maps, fine_operator
prob = synth.make_problem(8, 1, n_levels=3)
nu = synth.nu_sphere(8, 8, 8, prob.h)
b = synth.rhs(prob.n_dofs, 0)
for opts in (dict(), dict(variant="overlap"), dict(variant="hybrid"), dict(variant="add_sync"),
             dict(smoother="schwarz", omega=0.1), dict(precision="mixed_ir"), dict(precision="mixed_flex"),
             dict(m_max=4, breakdown=0.5)):
    o = oracle.Oracle.from_sip(prob, nu, s_pre=2, s_post=2, **opts)
    o.solve(b, tol=1e-8)
    o.visits(); o.visit_norms()
o = oracle.Oracle.from_sip(prob, nu, variant="overlap")
o.set_step_schedule([3, 2, 4])
o.solve(b, tol=1e-8)
o = oracle.Oracle.from_sip(prob, nu)
x0 = o.solve(b)
o.solve(b, x0=0.5 * x0)
v = np.random.default_rng(1).standard_normal(prob.n_dofs)
for f32 in (False, True):
    o.spmv(v, 0, b, fp32=f32); o.smoother(v, 2, 0, fp32=f32)
    rc = o.restrict(v, 0, fp32=f32); o.prolong(rc, 0, fp32=f32)
o.grad(x0, x0 - b)
_, (rp, ci, val) = fine_operator(6, 1)
nc, par, sl = cartesian_maps(6, 6, 6, 3)
oh = oracle.Oracle.from_bsr_hierarchy(rp, ci, val, nc, par, sl, oracle.embedding(1))
oh.solve(synth.rhs(nc[0] * 4, 0), tol=1e-10)
print("child ok")
'''


def test_oracle_under_address_and_ub_sanitizers():
    if not shutil.which("gcc"):
        pytest.skip("no gcc")
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    ubsan = subprocess.run(["gcc", "-print-file-name=libubsan.so"], capture_output=True, text=True).stdout.strip()
    if not (os.path.isabs(asan) and os.path.exists(asan) and os.path.isabs(ubsan) and os.path.exists(ubsan)):
        pytest.skip("sanitizer runtimes not installed")
    with tempfile.TemporaryDirectory() as d:
        lib = os.path.join(d, "liboracle_san.so")
        subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                               "-fno-sanitize-recover=undefined", "-fopenmp", "-fPIC", "-shared",
                               os.path.join(ROOT, "oracle", "omg_oracle.c"), "-o", lib, "-lm"])
        env = dict(os.environ)
        env.update({"LD_PRELOAD": f"{asan} {ubsan}", "OMG_ORACLE_LIB": lib, "OMP_NUM_THREADS": "2",
                    "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
                    "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1",
                    "PYTHONPATH": ROOT + os.pathsep + env.get("PYTHONPATH", "")})
        r = subprocess.run([sys.executable, "-c", CHILD], env=env, capture_output=True, text=True, timeout=900,
                           cwd=ROOT)
    report = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0 and "child ok" in r.stdout, report
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, report
