"""Algorithmic FP32 operation count of one rollout step of the HIP path.

Counted from the formulas the rollout kernel evaluates, with a fused
multiply-add as 2 operations, every other add / mul / div / sqrt and every
elementary function call (sincos, exp, atan2) as 1.  Contacts are counted in
their inactive form (point kinematics, the penalty test, the force transform);
the implicit-damping terms of an active contact (~270 more) are left out, so
the count is a lower bound and the derived throughput a conservative one.

Per physics step, per lane:
  joint lane  Hermite reference 47, PD law and implicit gain 9, sincos 2,
              forward kinematics 171, rigid-body inertia 119, bias force 96,
              backward sweep 313 (+27 per child gathered), forward sweep 38,
              integration 4                                   -> 799 (+27/child)
  base lane   rotation of the quaternion 20, bias force 96, 6x6 Cholesky solve
              180, gravity shift 6, base integration 105      -> 407 (+27/child)
  contact     inactive point kinematics, test and force transform  110
Per control step (running cost): 6 per joint, 10 per contact, 15 for the base.
"""

JOINT = 799
PER_CHILD = 27
BASE = 407
CONTACT = 110
COST_JOINT, COST_CONTACT, COST_BASE = 6, 10, 15


def flops_per_physics_step(model):
    parent = list(model["parent"])
    fb = bool(model["floating_base"])
    nb = len(parent)
    nj = nb - (1 if fb else 0)
    n_child_edges = sum(1 for p in parent if p >= 0)
    f = nj * JOINT + n_child_edges * PER_CHILD + len(model["contact_body"]) * CONTACT
    if fb:
        f += BASE
    return f


def flops_per_rollout_step(model):
    """Operations per control step of one rollout (n_substeps physics steps + cost)."""
    nsub = int(model.get("n_substeps", 1))
    nj = len(model["parent"]) - (1 if model["floating_base"] else 0)
    cost = nj * COST_JOINT + len(model["contact_body"]) * COST_CONTACT + (COST_BASE if model["floating_base"] else 0)
    return nsub * flops_per_physics_step(model) + cost


def bytes_per_rollout(model, n_knots, n_iters=1):
    """HBM bytes one rollout needs per iteration: its state read (shared, counted once
    per rollout as an upper bound), nominal knots read, its sample knots written,
    its cost written."""
    E = 2 * n_knots * model["n_u"]
    nx = model["n_q"] + model["n_v"]
    return 4 * (nx + E + E + 1)
