"""Property tests of the oracle on small seeded meshes.

After every independent set: the mesh is a conforming, positively oriented
triangulation of the unit square with exact total area 1 and V - E + F = 1,
and the adjacency rows equal a rebuild from the elements. Before every set the
members are pairwise non-adjacent (brute force). Results do not depend on the
order in which a set's members are applied (Sec. 3.3: any thread may run any
member). After each phase its stopping condition holds.
"""
import math

import numpy as np
import pytest

from oracle.orc import OracleMesh, PH_COARSEN, PH_SWAP, PH_SMOOTH
from paper_1505_04694_amd import inputs
from tests import checker, fdcheck

CASES = [
    ("grid9", lambda: inputs.make_mesh(9, ht=0.3), 0),
    ("jit17", lambda: inputs.make_mesh(17, layers=2, jitter_seed=5), 5),
    ("cfg0", inputs.config0, 0),
]


def with_hook(om, exact=True, smooth_check=True):
    state = {"classes": 0, "pre": None}

    def hook(phase, rnd, cls, stage):
        d = om.export()
        if stage == 0:
            mem = om.class_members()
            tri = d["tri"][d["talive"]]
            checker.assert_independent(mem, tri)
            if phase == PH_SMOOTH and smooth_check:
                state["pre"] = (mem.copy(), patch_min(d, mem))
            return
        state["classes"] += 1
        checker.check_mesh(d, exact=exact, rows=om.rows())
        if phase == PH_SMOOTH and smooth_check:
            mem, before = state["pre"]
            after = patch_min(d, mem)
            assert (after >= before * (1 - 1e-12)).all(), "smoothing lowered a patch minimum"

    om.set_hook(hook)
    return state


def patch_min(d, members):
    tri = d["tri"][d["talive"]]
    q = checker.mean_ratio(d["xy"], d["metric"], tri)
    out = np.full(len(members), np.inf)
    pos = {int(v): i for i, v in enumerate(members)}
    for t, (a, b, c) in enumerate(tri.tolist()):
        for v in (a, b, c):
            i = pos.get(v)
            if i is not None:
                out[i] = min(out[i], q[t])
    return out


@pytest.mark.parametrize("name,make,seed", CASES)
def test_sweep_invariants_every_class(name, make, seed):
    mi = make()
    om = OracleMesh.from_input(mi, seed=seed)
    st = with_hook(om)
    for s in range(2):
        om.sweep(s)
        checker.check_mesh(om.export(), exact=True, rows=om.rows())
    assert st["classes"] > 0


@pytest.mark.parametrize("name,make,seed", CASES)
@pytest.mark.parametrize("kind", [0, 1])
def test_order_independence(name, make, seed, kind):
    mi = make()
    outs = []
    for order in (0, 1, 99):
        om = OracleMesh.from_input(mi, seed=seed)
        om.set_order_seed(order)
        stats = [om.sweep(s, smooth_kind=kind) for s in range(2)]
        d = om.export()
        outs.append((d, stats))
    for d, stats in outs[1:]:
        assert stats == outs[0][1]
        for k in ("xy", "tri", "metric", "tags"):
            assert np.array_equal(d[k], outs[0][0][k]), k


def collapse_ok(d, v, u, qmin):
    """Would collapsing v onto u keep every re-pointed element valid? (matrix form)"""
    tri = d["tri"][d["talive"]]
    rows = tri[(tri == v).any(1) & ~(tri == u).any(1)].copy()
    rows[rows == v] = u
    if len(rows) == 0:
        return True
    D = checker.doubled_areas(d["xy"], rows)
    if (D <= 0).any():
        return False
    return bool((checker.mean_ratio(d["xy"], d["metric"], rows) >= qmin).all())


@pytest.mark.parametrize("name,make,seed", CASES)
def test_coarsen_fixpoint_every_short_edge_blocked(name, make, seed):
    mi = make()
    om = OracleMesh.from_input(mi, seed=seed)
    st = om.coarsen()
    assert st["converged"] == 1
    d = om.export()
    tri = d["tri"]
    pairs = checker.adjacency_pairs(tri)
    tags = d["tags"]
    a = np.array([p[0] for p in pairs]); b = np.array([p[1] for p in pairs])
    L2 = checker.metric_len2(d["xy"], d["metric"], a, b)
    short = 0
    for i in np.nonzero(L2 < 0.5 * (1 - 1e-12))[0]:
        for v, u in ((a[i], b[i]), (b[i], a[i])):
            if tags[v] & ~tags[u]:
                continue
            short += 1
            # blocked, up to a rounding margin at the quality threshold
            assert not collapse_ok(d, v, u, 0.1 * (1 + 1e-9)), f"collapse {v}->{u} still possible"
    assert short >= 0


@pytest.mark.parametrize("name,make,seed", CASES)
def test_refine_fixpoint_no_long_edge(name, make, seed):
    mi = make()
    om = OracleMesh.from_input(mi, seed=seed)
    om.coarsen()
    V0, _ = om.sizes()
    before = om.export()
    st = om.refine()
    assert st["converged"] == 1
    d = om.export()
    pairs = checker.adjacency_pairs(d["tri"])
    a = np.array([p[0] for p in pairs]); b = np.array([p[1] for p in pairs])
    assert checker.metric_len2(d["xy"], d["metric"], a, b).max() <= 2.0 * (1 + 1e-12)
    checker.check_mesh(d, exact=True, rows=om.rows())
    # old vertices unchanged; every new vertex is the mid-point of two vertices
    assert np.array_equal(d["xy"][:V0], before["xy"])
    assert st["new_vertices"] == d["xy"].shape[0] - V0


@pytest.mark.parametrize("name,make,seed", CASES)
def test_swap_fixpoint_no_improving_flip(name, make, seed):
    mi = make()
    om = OracleMesh.from_input(mi, seed=seed)
    om.coarsen(); om.refine()
    st = om.swap()
    assert st["converged"] == 1
    d = om.export()
    tri = d["tri"]
    xy, met = d["xy"], d["metric"]
    q = checker.mean_ratio(xy, met, tri)
    owner = {}
    for t, (x, y, z) in enumerate(tri.tolist()):
        for p, r, o in ((x, y, z), (y, z, x), (z, x, y)):
            owner[(p, r)] = (t, o)
    for (p, r), (t1, a) in owner.items():
        if (r, p) not in owner or p > r:
            continue
        t2, b = owner[(r, p)]
        new = np.array([[p, b, a], [r, a, b]])
        if (checker.doubled_areas(xy, new) <= 0).any():
            continue
        qn = checker.mean_ratio(xy, met, new).min()
        assert qn <= min(q[t1], q[t2]) * (1 + 1e-9), f"flip of ({p},{r}) still improves"


def test_smoothing_gradient_increases_local_functional():
    mi = inputs.make_mesh(17, layers=2, jitter_seed=2)
    om = OracleMesh.from_input(mi, seed=2)
    d0 = om.export()
    Qv0 = {v: om.patch_quality(v) for v in range(mi.V) if mi.tags[v] == 0}
    moved = 0

    def hook(phase, rnd, cls, stage):
        nonlocal moved
        if stage == 0:
            hook.before = {int(v): om.patch_quality(int(v)) for v in om.class_members()}
            hook.xy = om.export()["xy"].copy()
        else:
            xy = om.export()["xy"]
            for v, q0 in hook.before.items():
                if not np.array_equal(xy[v], hook.xy[v]):
                    moved += 1
                    assert om.patch_quality(v) > q0

    om.set_hook(hook)
    st = om.smooth(kind=1, sweeps=2)
    assert moved == st["committed"] > 0
    assert om.quality()[0] > sum(checker.mean_ratio(d0["xy"], d0["metric"], d0["tri"]))


# ---- adjoint of the quality functional ----------------------------------------------

def test_protocol_priorities_match_the_oracle():
    from oracle.orc import prio
    p = fdcheck.priorities(1, 0, 5000)
    assert all(int(p[i]) == prio(1, 0, i) for i in range(0, 5000, 97))


@pytest.mark.parametrize("n", [17, 65, 2049])
def test_adjoint_matches_central_differences(n):
    """The config-2 protocol: at the 64 largest-key vertices, central
    differences of the patch-local Q_v (x step 1e-7, metric step 1e-7 of the
    tensor's size) against the oracle's dQ/dx and dQ/dM, entry by entry."""
    mi = inputs.config2(n)
    om = OracleMesh.from_input(mi, seed=1)
    Q, qmin, gx, gm = om.quality(grad=True)
    worst = 0.0
    for v in fdcheck.protocol_vertices(mi.V):
        v = int(v)
        fx, fm, Qv, hx, hm = fdcheck.central_differences(om, v, mi.xy[v], mi.metric[v])
        worst = max(worst, fdcheck.check_entries(fx, gx[v], Qv, hx, f"dQ/dx at {v}"))
        worst = max(worst, fdcheck.check_entries(fm, gm[v], Qv, hm, f"dQ/dM at {v}"))
    assert worst <= 1e-6


def test_adjoint_euler_identities():
    # q is invariant under translation and scaling of x and under M -> cM
    mi = inputs.config2(33)
    om = OracleMesh.from_input(mi, seed=1)
    Q, _, gx, gm = om.quality(grad=True)
    xy, met = mi.xy, mi.metric
    scale = np.abs(gx).sum()
    assert abs(gx[:, 0].sum()) <= 1e-10 * scale
    assert abs(gx[:, 1].sum()) <= 1e-10 * scale
    assert abs((xy * gx).sum()) <= 1e-10 * np.abs(xy * gx).sum()
    hom = met * gm
    assert abs(hom.sum()) <= 1e-10 * np.abs(hom).sum()


def test_fan_start_reaches_rows_past_the_register_paths():
    """The high-degree start used by the GPU parity tests: a member with more
    than 16 neighbours (past the lane groups) and a commit row with more than
    32 candidate elements (past the register paths: the target's old row plus
    the rows of the members collapsed onto it) both occur in its first
    coarsening."""
    mi = inputs.fan(48, hubs=2, layers=-1)
    om = OracleMesh.from_input(mi, seed=1)
    seen = dict(deg=0, cand=0)
    snap = {}

    def hook(phase, rnd, cls, stage):
        if phase != PH_COARSEN:
            return
        d = om.export()
        if stage == 0:
            nn_off, _, ne_off, ne = om.rows()
            snap["d"], snap["ne_off"], snap["ne"] = d, ne_off, ne
            for v in om.class_members():
                seen["deg"] = max(seen["deg"], int(nn_off[v + 1] - nn_off[v]))
            return
        b, ne_off, ne = snap["d"], snap["ne_off"], snap["ne"]
        cand = {}
        for w in np.nonzero(b["valive"] & ~d["valive"])[0]:
            rows = ne[ne_off[w]:ne_off[w + 1]]
            for t in rows:
                if d["talive"][t]:
                    u = int((set(d["tri"][t].tolist()) - set(b["tri"][t].tolist())).pop())
                    cand[u] = cand.get(u, int(ne_off[u + 1] - ne_off[u])) + len(rows)
                    break
        if cand:
            seen["cand"] = max(seen["cand"], max(cand.values()))

    om.set_hook(hook)
    om.coarsen()
    assert seen["deg"] > 16 and seen["cand"] > 32, seen


@pytest.mark.parametrize("pause", [1, 3, 5])
def test_oracle_algorithm1_resume_from_an_export(pause):
    """Algorithm 1 stopped at a resume point, exported, and continued on a new
    mesh built from the export with the saved loop state gives the same mesh
    as an uninterrupted run (the export is the whole state besides the loop
    state: slots are live and in id order at every resume point)."""
    mi = inputs.config2(33)
    whole = OracleMesh.from_input(mi, seed=1)
    st_whole, done = whole.adapt(max_iterations=3)
    assert done
    first = OracleMesh.from_input(mi, seed=1)
    _, done = first.adapt(max_iterations=3, max_phases=pause)
    assert not done
    ctx = first.get_context()
    e = first.export()
    assert e["valive"].all() and e["talive"].all()
    resumed = OracleMesh(e["xy"], e["tri"], e["metric"], e["tags"], seed=1)
    resumed.set_context(**ctx)
    _, done = resumed.adapt(max_iterations=3)
    assert done
    a, b = whole.export(), resumed.export()
    for k in ("xy", "tri", "metric", "tags"):
        assert np.array_equal(a[k], b[k]), k


def test_oracle_algorithm1_runs_coarsen_swap_refine_then_smooths_once():
    mi = inputs.config0()
    om = OracleMesh.from_input(mi, seed=0)
    phases = []
    om.set_hook(lambda ph, r, c, stage: phases.append(ph) if stage == 0 and (not phases or phases[-1] != ph) else None)
    st, done = om.adapt(max_iterations=2)
    assert done and st["rounds"] == 2
    # two iterations of coarsen, swap (refinement has no classes), then one smoothing
    assert phases == [PH_COARSEN, PH_SWAP, PH_COARSEN, PH_SWAP, PH_SMOOTH]
    checker.check_mesh(om.export(), exact=False, rows=om.rows())
