"""sedimi_step replayed from captured HIP graphs against the same steps
enqueued kernel by kernel (sedimi_set_step_graphs(ctx, 0)): particle state,
accelerations, tangential histories, both mesh fields and the counters are
bit-identical after every call.  Between the calls both contexts do other
work and synchronise (reads of fields and particles, a force evaluation, a
translation), the call shapes change (new captures, alternating buffer
parities), the particles are replaced once (the captured graphs no longer
match and are captured again), and the velocities are high enough that the
neighbour lists are rebuilt inside replays."""
import numpy as np
import pytest

from gpu_helpers import dense_bed, gpu_context

pytestmark = pytest.mark.gpu


def _same(a, b, tag):
    pa, pb = a.get_particles(), b.get_particles()
    for k in pa:
        assert np.array_equal(pa[k], pb[k]), (tag, k)
    for f in (0, 1):
        assert np.array_equal(a.get_field(f), b.get_field(f)), (tag, f)
    ha, hb = a.get_history(), b.get_history()
    assert np.array_equal(ha, hb), tag
    sa, sb = a.stats(), b.stats()
    for k in ("steps", "rebuilds", "max_neighbors", "flags", "solve_iters"):
        assert sa[k] == sb[k], (tag, k, sa[k], sb[k])
    assert sa["solve_residual"] == sb["solve_residual"], tag


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_replayed_steps_match_kernel_by_kernel(precision):
    case = dense_bed(3000, 41)
    case["v"] = case["v"] * 5.0  # with a small skin: lists rebuilt every few steps
    a = gpu_context(case, precision=precision, skin_frac=0.02)
    b = gpu_context(case, precision=precision, skin_frac=0.02)
    b.set_step_graphs(False)
    for g in (a, b):
        g.average()
        g.compute_forces(update_history=False)
    shapes = [(10, 10), (10, 10), (10, 10), (7, 5), (7, 5), (7, 5), (3, 0), (3, 0), (10, 10),
              (10, 10)]
    rebuilds0 = a.stats()["rebuilds"]
    for it, (ns, ae) in enumerate(shapes):
        for g in (a, b):
            g.step(ns, average_every=ae)
        _same(a, b, it)
        if it == 4:
            # new particles: every captured graph is stale
            p = a.get_particles()
            for g in (a, b):
                g.set_particles(p["x"], p["v"], case["d"], case["rho"], omega=p["omega"])
                g.average()
                g.compute_forces(update_history=False)
        if it == 6:
            for g in (a, b):
                g.translate(1e-4, -2e-4)
                g.compute_forces(update_history=False)
        _same(a, b, f"{it} after")
    st = a.stats()
    print(f"{precision}: {st['graph_steps']} graph calls of {len(shapes)}, "
          f"{st['rebuilds'] - rebuilds0} rebuilds")
    assert st["graph_steps"] == len(shapes)
    assert b.stats()["graph_steps"] == 0
    assert st["rebuilds"] - rebuilds0 >= 3


def test_steps_with_a_readback_are_not_captured():
    """The iterative solve reads its residual back inside the call: those
    calls run kernel by kernel, and calls without an averaging are still
    replayed."""
    case = dense_bed(3000, 41)
    a = gpu_context(case, solver="iterative")
    b = gpu_context(case, solver="iterative")
    b.set_step_graphs(False)
    for g in (a, b):
        g.average()
    for ns in (5, 4, 4):
        for g in (a, b):
            g.step(ns, average_every=5)
        _same(a, b, f"iterative {ns}")
    assert a.stats()["graph_steps"] == 1  # only the middle call has no averaging


def test_network_averaging_is_not_captured():
    """With the network answering the averaging (surrogate mode), a call
    whose steps include an averaging runs kernel by kernel and a call
    without one is replayed; both match a context without replay bit for
    bit."""
    import paper_1601_03801_amd as sm
    case = dense_bed(3000, 41)
    dmax = float(case["d"].max())

    def ctx():
        g = sm.Sedimi(dict(case["params"]), len(case["d"]), precision="mixed", d_max=dmax,
                      skin=0.1 * dmax, max_neighbors=24, nn=True, nn_alpha=1.0)
        g.set_fluid(case["U"], case["gradp"], case["dudt"])
        g.set_particles(case["x"], case["v"], case["d"], case["rho"], omega=case["w"])
        g.nn_set_groups(4)
        g.nn_init(3)
        g.average()
        g.set_avg_mode(sm.AVG_SURROGATE)
        return g

    a, b = ctx(), ctx()
    b.set_step_graphs(False)
    for ns in (5, 4, 1, 4):
        for g in (a, b):
            g.step(ns, average_every=5)
        _same(a, b, f"surrogate {ns}")
    # steps 6-9 and 11-14 have no averaging; 1-5 and 10 end in one
    assert a.stats()["graph_steps"] == 2
    assert a.stats()["nn_calls"] == b.stats()["nn_calls"] == 2
