"""Arithmetic per rollout step of the simulate step of Alg. 1, counted by the
oracle's operation-counting scalar (test infrastructure; writes the summary that
prices the roofline of the rollout kernel):

    python oracle/count_flops.py > profiles/flops_per_rollout_step.txt

For each workload model one rollout is counted (sample 1 of iteration 0 around
the nominal knots, H control steps from x0, terminal cost, its sampling); the
per-step figures divide by H.  "raw" counts every operation of the oracle's
dense formulation; "nontrivial" leaves out products with an exact 0 or +-1 and
sums with an exact 0 (see oracle/opcount.hpp).  Flops: add/sub, mul, div,
sqrt and transcendental calls count one each (no fused operations exist in the
oracle); comparisons are not flops.
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2511_19204_amd import synth  # noqa: E402

WORKLOADS = ("chain", "quadruped", "quadruped_tp", "humanoid")


def counts():
    out = {}
    for name in WORKLOADS:
        m, p, seed = synth.config(name)
        c = O.count_ops(m, p, m["x0"], synth.nominal_knots(m, p["n_knots"]), seed, 1)
        r, H = c["rollout"], p["horizon"]
        raw = r["add"] + r["mul"] + r["div"] + r["sqrt"] + r["trans"]
        nt = r["nt_add"] + r["nt_mul"] + r["nt_div"] + r["sqrt"] + r["trans"]
        out[name] = {"horizon": H, "raw_per_step": raw / H, "nontrivial_per_step": nt / H,
                     **{k: float(v) for k, v in r.items()}}
    return out


def main():
    print("# arithmetic per rollout step of the simulate step (oracle op-counting scalar)")
    print("# command: python oracle/count_flops.py > profiles/flops_per_rollout_step.txt")
    for name, d in counts().items():
        print(f"{name}.raw_per_step: {d['raw_per_step']:.1f}")
        print(f"{name}.nontrivial_per_step: {d['nontrivial_per_step']:.1f}")
        print(f"{name}.rollout_counts: " + " ".join(f"{k}={int(d[k])}" for k in O.OP_KINDS) + f" H={d['horizon']}")


if __name__ == "__main__":
    main()
