"""Parity of the HIP path with the oracle on the paths the ordinary meshes do
not reach, and on the calls above the single phases:
  - high-degree starts (a centre vertex joined to a ring of 48 or 96), where
    members have rows past the lane groups and commit rows have more than 32
    candidates (the staging path);
  - adjacency pools and staging that run out mid-round (the rows are rebuilt
    from the element list and the round goes on), and the smallest slack;
  - round caps;
  - Algorithm 1 (pm_adapt) and checkpoint / resume of its loop state;
  - the quality functional as a torch.autograd.Function.
"""
import numpy as np
import pytest

from paper_1505_04694_amd import inputs, pmesh
from oracle.orc import OracleMesh
from tests import checker, fdcheck
from tests.parity import both, compare_mesh, compare_quality, compare_stats, run_sweeps

pytestmark = pytest.mark.gpu

FANS = [
    ("hubs48", lambda: inputs.fan(48, hubs=2, layers=-1), 1),
    ("fan48", lambda: inputs.fan(48), 1),
    ("fan96", lambda: inputs.fan(96, radius=0.3), 2),
]


@pytest.mark.parametrize("name,make,seed", FANS)
def test_high_degree_starts(name, make, seed):
    om, gm = both(make(), seed)
    compare_mesh(om, gm, "create")
    run_sweeps(om, gm, 2, smooth_kinds=(0, 1))
    checker.check_mesh(gm.export(), exact=False, rows=gm.rows())
    compare_quality(om, gm, "end")


def test_refinement_at_scale_pass_by_pass():
    """A refinement-dominated start (512 triangles growing past 1e5): parity
    after every refinement pass, then after a swap, smoothing and coarsening."""
    om, gm = both(inputs.refine_start(), 5)
    passes = 0
    while True:
        so, sg = om.refine(max_passes=1), gm.refine(max_passes=1)
        compare_stats(so, sg, f"pass {passes}")
        compare_mesh(om, gm, f"pass {passes}")
        if so["converged"]:
            break
        passes += 1
    assert passes >= 6 and gm.sizes()[1] > 100000
    for name, fo, fg in (("swap", lambda: om.swap(0), lambda: gm.swap(0)),
                         ("smooth", lambda: om.smooth(0, 1, 1), lambda: gm.smooth(0, 1, 1)),
                         ("coarsen", lambda: om.coarsen(1), lambda: gm.coarsen(1))):
        compare_stats(fo(), fg(), name)
        compare_mesh(om, gm, name)
    compare_quality(om, gm, "end")


@pytest.mark.parametrize("name,make,seed", FANS[:1] + [("cfg2_65", lambda: inputs.config2(65), 1),
                                                       ("grid129", lambda: inputs.make_mesh(129, layers=2), 4)])
def test_pools_that_run_out_are_rebuilt_and_the_round_goes_on(name, make, seed):
    mi = make()
    om = OracleMesh.from_input(mi, seed=seed)
    gm = pmesh.Mesh.from_input(mi, seed=seed, slack=1.0, pool_headroom=1.0)
    rebuilds = 0
    for s in range(2):
        for name in ("coarsen", "refine", "swap", "smooth"):
            kw = {} if name == "refine" else {"sweep": s}
            so, sg = getattr(om, name)(**kw), getattr(gm, name)(**kw)
            compare_stats(so, sg, f"sweep {s} {name}")
            compare_mesh(om, gm, f"sweep {s} {name}")
            rebuilds += sg["room_rebuilds"]
    compare_quality(om, gm, "end")
    # the rebuild path really ran
    assert rebuilds > 0, "no round ran out of room"


def test_smallest_slack_equals_the_default():
    mi = inputs.config2(129)
    om, g1 = both(mi, 1)
    g2 = pmesh.Mesh.from_input(mi, seed=1, slack=1.0)
    for s in range(2):
        for name in ("coarsen", "refine", "swap", "smooth"):
            so = getattr(om, name)(**({} if name == "refine" else {"sweep": s}))
            s1 = getattr(g1, name)(**({} if name == "refine" else {"sweep": s}))
            s2 = getattr(g2, name)(**({} if name == "refine" else {"sweep": s}))
            compare_stats(so, s1, name)
            compare_stats(so, s2, name)
            e1, e2 = g1.export(), g2.export()
            for k in ("xy", "tri", "metric", "tags", "valive", "talive"):
                assert np.array_equal(e1[k], e2[k]), f"sweep {s} {name}: {k}"
            for a, b in zip(g1.rows(), g2.rows()):
                assert np.array_equal(a, b)
    compare_mesh(om, g2, "end")


def test_round_caps_stop_the_phase_with_a_valid_mesh():
    mi = inputs.config2(65)
    om, gm = both(mi, 1)
    so, sg = om.coarsen(max_rounds=2), gm.coarsen(max_rounds=2)
    compare_stats(so, sg, "coarsen capped")
    assert sg["converged"] == 0 and sg["status"] == "PM_W_NOT_CONVERGED"
    compare_mesh(om, gm, "coarsen capped")
    so, sg = om.refine(max_passes=1), gm.refine(max_passes=1)
    compare_stats(so, sg, "refine capped")
    so, sg = om.swap(max_rounds=1), gm.swap(max_rounds=1)
    compare_stats(so, sg, "swap capped")
    assert sg["status"] == "PM_W_NOT_CONVERGED"
    compare_mesh(om, gm, "swap capped")
    checker.check_mesh(gm.export(), exact=False, rows=gm.rows())


ADAPT = [
    ("cfg0", inputs.config0, 0),
    ("cfg2_65", lambda: inputs.config2(65), 1),
    ("fan48", lambda: inputs.fan(48), 1),
]


@pytest.mark.parametrize("name,make,seed", ADAPT)
def test_algorithm1_matches_the_oracle(name, make, seed):
    om, gm = both(make(), seed)
    so, fo = om.adapt(max_iterations=4, smooth_kind=1)
    sg, fg = gm.adapt(max_iterations=4, smooth_kind=1)
    assert fo and fg
    compare_stats(so, sg, "adapt")
    compare_mesh(om, gm, "adapt")
    compare_quality(om, gm, "adapt")
    assert gm.get_context()["phase"] == pmesh.PM_PHASE_DONE


@pytest.mark.parametrize("pause", [3, 5, 7])
def test_checkpoint_and_resume_is_bit_identical(pause):
    """Export plus context at a resume point, a new handle from them, and the
    rest of the procedure: the same mesh as an uninterrupted run (and as the
    oracle's)."""
    mi = inputs.config2(65)
    whole = pmesh.Mesh.from_input(mi, seed=1)
    whole.adapt(max_iterations=4)
    first = pmesh.Mesh.from_input(mi, seed=1)
    st, done = first.adapt(max_iterations=4, max_phases=pause)
    assert not done and st["status"] == "PM_W_PAUSED"
    ctx = first.get_context()
    e = first.export()
    assert e["valive"].all() and e["talive"].all()
    first.close()
    resumed = pmesh.Mesh(e["xy"], e["tri"], e["metric"], e["tags"], seed=ctx["seed"])
    resumed.set_context(ctx)
    _, done = resumed.adapt(max_iterations=4)
    assert done
    a, b = whole.export(), resumed.export()
    for k in ("xy", "tri", "metric", "tags", "valive", "talive"):
        assert np.array_equal(a[k], b[k]), k
    for x, y in zip(whole.rows(), resumed.rows()):
        assert np.array_equal(x, y)
    om = OracleMesh.from_input(mi, seed=1)
    om.adapt(max_iterations=4)
    compare_mesh(om, resumed, "resumed")


def test_quality_autograd_function():
    import torch
    mi = inputs.config2(65)
    om, gm = both(mi, 1)
    xy = torch.tensor(mi.xy, device="cuda", requires_grad=True)
    met = torch.tensor(mi.metric, device="cuda", requires_grad=True)
    Q = pmesh.QualityFn.apply(xy, met, gm)
    Q.backward()
    Qo, _, gxo, gmo = om.quality(grad=True)
    assert abs(float(Q.detach()) - Qo) <= 1e-12 * abs(Qo)
    for nm, o, g in (("dQ/dx", gxo, xy.grad.cpu().numpy()), ("dQ/dM", gmo, met.grad.cpu().numpy())):
        floor = 1e-12 * np.abs(o).max(axis=1, keepdims=True)
        assert not (np.abs(o - g) > 1e-12 * np.abs(o) + floor).any(), nm
    # central differences of the patch-local functional at the protocol vertices
    for v in fdcheck.protocol_vertices(mi.V):
        v = int(v)
        fx, fm, Qv, hx, hm = fdcheck.central_differences(om, v, mi.xy[v], mi.metric[v])
        fdcheck.check_entries(fx, xy.grad[v].cpu().numpy(), Qv, hx, f"dQ/dx at {v}")
        fdcheck.check_entries(fm, met.grad[v].cpu().numpy(), Qv, hm, f"dQ/dM at {v}")
    # an upstream gradient scales the adjoint
    xy.grad = None
    (3.0 * pmesh.QualityFn.apply(xy, met, gm)).backward()
    assert torch.equal(xy.grad, 3.0 * torch.tensor(gxo, device="cuda"))


def test_quality_gradient_ascent_with_torch():
    """Gradient-based optimisation of Q through the autograd function: steps
    along dQ/dx on the interior vertices (an optimizer of the caller's
    choosing) raise Q and keep every element valid."""
    import torch
    mi = inputs.config2(65)
    gm = pmesh.Mesh.from_input(mi, seed=1)
    inner = torch.tensor(mi.tags == 0, device="cuda")[:, None]
    xy = torch.tensor(mi.xy, device="cuda", requires_grad=True)
    met = torch.tensor(mi.metric, device="cuda")
    opt = torch.optim.SGD([xy], lr=2e-8, maximize=True)
    Q0 = None
    for _ in range(5):
        opt.zero_grad()
        Q = pmesh.QualityFn.apply(xy, met, gm)
        Q0 = float(Q.detach()) if Q0 is None else Q0
        Q.backward()
        xy.grad.mul_(inner)
        opt.step()
    Q1 = float(pmesh.QualityFn.apply(xy, met, gm).detach())
    assert Q1 > Q0
    checker.check_mesh(gm.export(), exact=False, rows=gm.rows())


def test_update_rejects_inverted_coordinates_and_keeps_the_old_ones():
    mi = inputs.config2(33)
    gm = pmesh.Mesh.from_input(mi, seed=1)
    bad = mi.xy.copy()
    v = int(np.nonzero(mi.tags == 0)[0][0])
    bad[v] += 0.5  # far outside its patch: elements turn over
    with pytest.raises(pmesh.PMError) as e:
        gm.update(xy=bad)
    assert e.value.status == pmesh.PM_E_MESH
    assert np.array_equal(gm.export()["xy"], mi.xy)


def test_psi_benchmark_time_steps():
    """The paper's synthetic benchmark at a reduced size: an isotropic 51 x 51
    start, the Hessian metric of the time-varying psi for about 2e4 elements;
    Algorithm 1 at t = 0, then three time steps, each with the metric of the
    next phase evaluated at the current vertices (on the host, the same array
    for both sides) and Algorithm 1 again. Parity after every step."""
    import math
    mi = inputs.psi_start(51, target=2e4, steps=50)
    eps = mi.info["eps"]
    om, gm = both(mi, 0)
    for step in range(4):
        if step > 0:
            d = om.export()
            assert np.array_equal(d["xy"], gm.export()["xy"])
            met = inputs.psi_metric(d["xy"], 2 * math.pi * step / 50, eps)
            for v in range(met.shape[0]):
                om.set_metric(v, *met[v])
            gm.update(metric=met)
            om.set_context(0, 1, 0)
            gm.set_context(dict(seed=0, iteration=0, phase=pmesh.PM_PHASE_COARSEN, changed=0))
        so, _ = om.adapt(max_iterations=2)
        sg, _ = gm.adapt(max_iterations=2)
        compare_stats(so, sg, f"step {step}")
        compare_mesh(om, gm, f"step {step}")
    assert gm.sizes()[1] > 2 * mi.T
    compare_quality(om, gm, "end")


def test_psi_benchmark_full_size_matches_the_oracle():
    """The psi benchmark at its full size, in the launch configuration that
    bench.py times: the 201 x 201 isotropic start (80,000 triangles) adapted
    to the metric for about 550,000 elements (Algorithm 1, four iterations),
    then two time steps of Algorithm 1 with two iterations each. The metric of
    each step is evaluated once on the host from the oracle's coordinates
    (already checked equal to the device's) and handed to both sides."""
    import math
    mi = inputs.psi_start(201, target=550e3)
    eps = mi.info["eps"]
    om, gm = both(mi, 0)
    compare_stats(om.adapt(max_iterations=4)[0], gm.adapt(max_iterations=4)[0], "start")
    compare_mesh(om, gm, "start")
    assert gm.sizes()[1] > 6 * mi.T
    for step in (1, 2):
        met = inputs.psi_metric(om.export()["xy"], 2 * math.pi * step / 50, eps)
        for v in range(met.shape[0]):
            om.set_metric(v, *met[v])
        gm.update(metric=met)
        om.set_context(0, 1, 0)
        gm.set_context(dict(seed=0, iteration=0, phase=pmesh.PM_PHASE_COARSEN, changed=0))
        compare_stats(om.adapt(max_iterations=2)[0], gm.adapt(max_iterations=2)[0], f"time step {step}")
        compare_mesh(om, gm, f"time step {step}")
    compare_quality(om, gm, "end")


def test_torch_allocator_owns_the_handle_memory():
    """A handle created with torch's caching allocator as its device memory
    provider gives the same mesh as one on the library's own cache; its blocks
    show in torch's statistics while it lives and all go back when it closes."""
    import torch
    mi = inputs.config2(129)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    gm = pmesh.Mesh.from_input(mi, seed=1, allocator="torch")
    ref = pmesh.Mesh.from_input(mi, seed=1)
    assert torch.cuda.memory_allocated() > base
    cur, _ = gm.memory()
    # torch rounds each block up to a multiple of 512 bytes
    assert cur <= torch.cuda.memory_allocated() - base <= cur + 512 * 256
    for m in (gm, ref):
        m.sweep(0, smooth_kind=1)
        m.sweep(1, smooth_kind=2)
    a, b = gm.export(), ref.export()
    for k in ("xy", "tri", "tags", "metric"):
        assert np.array_equal(a[k], b[k]), k
    assert gm.quality() == ref.quality()
    gm.close()
    ref.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base


def test_torch_allocator_on_a_batch():
    import torch
    mis = [inputs.make_mesh(n, amp=0.15, width=0.04, ht=0.08) for n in (17, 33, 20)]
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    gb = pmesh.Batch.from_inputs(mis, seed=2, allocator="torch")
    rb = pmesh.Batch.from_inputs(mis, seed=2)
    for b in (gb, rb):
        b.sweep(0, smooth_kind=0)
    for i in range(3):
        a, c = gb.export_mesh(i), rb.export_mesh(i)
        assert np.array_equal(a["tri"], c["tri"]) and np.array_equal(a["xy"], c["xy"]), i
    gb.close()
    rb.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base
