"""The mixed form with FP64 position differences takes v_j - v_i in FP32
against each cluster's reference velocity (the mass-weighted mean velocity
of a strided sample of the cluster).  Its error scales with |v - v_ref|, so
the reference must sit near the bulk velocity whatever the particle order:
these cases put a particle moving at about 70 times the velocity dispersion
first, and give a whole cluster a bulk velocity hundreds of times its
dispersion, and hold the caller-array evaluation (nbody_forces) and the
initial state evaluation to the 1e-6 acceleration and jerk gates against
the oracle."""
import numpy as np
import pytest

import oracle
from paper_0909_0879_amd import binding, ics
from tests.gpu_util import check_parity, require_gpu, to_np

pytestmark = pytest.mark.gpu

N = 4096
EPS = 1e-3


def _case(name):
    m, x, v = ics.plummer(N, 17)
    if name == "fast_first":
        v = v.copy()
        v[0] += np.array([50.0, -20.0, 10.0])
    elif name == "bulk_motion":
        v = v + np.array([300.0, -200.0, 100.0])
    return m, x, v


@pytest.mark.parametrize("name", ["fast_first", "bulk_motion"])
def test_reference_velocity_robust(name):
    require_gpu()
    print(f"relv {name}", flush=True)
    m, x, v = _case(name)
    a_ref, j_ref = oracle.forces(x, v, m, EPS)
    g = binding.NBody(m, x, v, eps=EPS, precision=binding.MIXED, tuning="auto")
    # the caller-array path (reference from the arrays passed in)
    acc, jerk = g.forces(x, v, m)
    g.sync()
    check_parity(to_np(acc), to_np(jerk), a_ref, j_ref, True, f"{name} forces")
    # the initial state evaluation (reference from the state)
    st = g.get_state()
    check_parity(to_np(st["a"]), to_np(st["j"]), a_ref, j_ref, True, f"{name} initial state")
    g.close()


def test_reference_velocity_per_cluster():
    # Clusters of one ensemble moving at different bulk velocities, each
    # hundreds of times its dispersion: every cluster's differences are taken
    # against its own reference, so all stay within the gates.  No block step
    # is routed to the FP64 kernel, so the mixed kernels evaluate every
    # cluster.
    require_gpu()
    sizes = [700, 2048, 1500]
    bulk = np.array([[300.0, -200.0, 100.0], [-250.0, 150.0, 0.0], [0.0, 0.0, 400.0]])
    eps = [1e-3, 2e-3, 1e-3]
    m, x, v, off = ics.ensemble(3, sizes=sizes, seed=7100)
    v = v.copy()
    for c in range(3):
        v[off[c]:off[c + 1]] += bulk[c]
    print("relv per-cluster ensemble", sizes, flush=True)
    g = binding.NBody(m, x, v, eps=eps, cluster_offsets=off, precision=binding.MIXED,
                      tuning={"small_log2": -1})
    acc, jerk = g.forces(x, v, m)
    g.sync()
    acc, jerk = to_np(acc), to_np(jerk)
    st = g.get_state()
    sa, sj = to_np(st["a"]), to_np(st["j"])
    for c in range(3):
        sl = slice(off[c], off[c + 1])
        a_ref, j_ref = oracle.forces(x[sl], v[sl], m[sl], eps[c])
        check_parity(acc[sl], jerk[sl], a_ref, j_ref, True, f"cluster {c} forces")
        check_parity(sa[sl], sj[sl], a_ref, j_ref, True, f"cluster {c} initial state")
    g.close()
