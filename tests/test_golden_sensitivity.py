"""How far two correct runs of the method end apart at 64^3 P2 (CPU).

tests/golden/make_oracle_64cubed_p2.py solves the 64^3 P2 plain-method
workload with the FP64 oracle twice: with b, and with b (1 + 1e-15 xi)
(--perturb). Algorithm 2 with the Sec. 4.2 level tests amplifies such a
rounding-level difference: the two solves take the same visit sequence
until the perturbed one stops, but their per-visit residual ratios drift
apart by up to O(1) and their solutions differ by ~1e-8. These facts set
the bar of the GPU's full-size replay test (same visits, then the
perturbed oracle's divergence envelope); at 24^3 and 32^3 the same
perturbation leaves the solutions within 2e-12 and 5e-11."""
import json
import os

import numpy as np
import pytest

import oracle

HERE = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def goldens():
    a = os.path.join(HERE, "oracle_64cubed_p2.npz")
    b = os.path.join(HERE, "oracle_64cubed_p2_perturbed.npz")
    if not (os.path.exists(a) and os.path.exists(b)):
        pytest.skip("golden files not generated")
    return np.load(a, allow_pickle=False), np.load(b, allow_pickle=False)


def test_perturbed_solve_follows_the_same_visits(goldens):
    a, b = goldens
    va, vb = a["visits"], b["visits"]
    ra, rb = json.loads(str(a["report"])), json.loads(str(b["report"]))
    # both reach the tolerance; the perturbed solve stops earlier, on the
    # same sequence of (level, iterations) up to its end
    assert ra["rel_res_rec"] <= 1e-10 and rb["rel_res_rec"] <= 1e-10
    assert rb["iters_fine"] < ra["iters_fine"]
    assert len(vb) < len(va)
    assert np.array_equal(va[:len(vb) - 1], vb[:len(vb) - 1])


def test_perturbed_solve_diverges_beyond_1e9(goldens):
    a, b = goldens
    la, lb = oracle.parse_visit_norms(a["vnorm"]), oracle.parse_visit_norms(b["vnorm"])
    dq = []
    for (l1, i1, r01, rs1), (l2, i2, r02, rs2) in zip(la, lb):
        if (l1, i1) != (l2, i2):
            break
        dq.append(max(abs(r01 / r02 - 1) if l1 == 0 else 0.0, np.abs(rs1 / r01 - rs2 / r02).max(initial=0.0)))
    dq = np.array(dq)
    # the first visits agree to rounding; the drift grows through the solve
    assert dq[:60].max() <= 1e-12
    assert 100 < np.argmax(dq > 1e-9) < 1000
    assert dq.max() > 0.1
    xs, ys = a["x_idx"], b["x_idx"]
    e = np.linalg.norm(xs - ys) / np.linalg.norm(xs)
    assert 1e-9 < e < 1e-7
