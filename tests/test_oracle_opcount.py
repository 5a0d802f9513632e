"""The oracle's operation-counting scalar, which prices the work of a rollout
step for the roofline: its counting rules pinned on a 3x3 product, and the
rollout counts' structure (raw counts grow by the same amount with every
control step of a smooth rollout; non-trivial counts never exceed raw ones)."""
import numpy as np
import pytest

import oracle as O
from paper_2511_19204_amd import synth


def test_counting_rules_on_a_matrix_vector_product():
    """y = A x with 3 terms per row, accumulated from 0: 9 products and 9 sums
    (the first sum adds to 0).  General A: the 9 products and the 6 sums of two
    nonzero terms are non-trivial.  Identity A: every product has a factor 0 or
    1 and every sum a zero operand, so nothing is non-trivial."""
    g, i = O.count_selftest()
    assert g["mul"] == 9 and g["add"] == 9 and g["div"] == 0
    assert g["nt_mul"] == 9 and g["nt_add"] == 6
    assert i["mul"] == 9 and i["add"] == 9
    assert i["nt_mul"] == 0 and i["nt_add"] == 0


def test_raw_counts_grow_linearly_with_the_horizon():
    """The unperturbed sample of the arm (no joint saturates, so every step takes
    the same branches) costs the same raw arithmetic at every control step."""
    m, p, s = synth.config("chain")
    kn = synth.nominal_knots(m, p["n_knots"])
    tot = {}
    for H in (10, 20, 30):
        q = dict(p, horizon=H)
        r = O.count_ops(m, q, m["x0"], kn, s, 0)["rollout"]
        tot[H] = np.array([r[k] for k in ("add", "mul", "div", "sqrt", "trans")])
    assert np.array_equal(tot[30] - tot[20], tot[20] - tot[10])
    assert np.sum(tot[20] - tot[10]) > 0


@pytest.mark.parametrize("name", ["chain", "quadruped_tp", "humanoid"])
def test_non_trivial_counts_are_within_the_raw_counts(name):
    m, p, s = synth.config(name)
    p = dict(p, horizon=20)
    r = O.count_ops(m, p, m["x0"], synth.nominal_knots(m, p["n_knots"]), s, 1)["rollout"]
    for k in ("add", "mul", "div"):
        assert 0 < r["nt_" + k] <= r[k]


def test_stored_counts_are_the_oracles():
    """profiles/flops_per_rollout_step.txt (which prices the roofline) holds what
    oracle/count_flops.py computes from the current oracle."""
    import os
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, os.path.join(root, "oracle"))
    import count_flops
    stored = {}
    for line in open(os.path.join(root, "profiles", "flops_per_rollout_step.txt")):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            if k.endswith("_per_step"):
                stored[k.strip()] = float(v)
    now = count_flops.counts()
    for name, d in now.items():
        for kind in ("raw_per_step", "nontrivial_per_step"):
            assert abs(stored[f"{name}.{kind}"] - d[kind]) <= 0.05 + 1e-9 * d[kind], (name, kind)
