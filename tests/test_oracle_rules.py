"""Pins of the oracle's per-member rules against an independent re-derivation.

Each test runs an oracle phase with a per-class hook and checks every class
member's result against what the rule, read from the paper, gives when it is
computed independently (tests/independent.py: numpy matrix forms, torch CPU
autograd in float64). Hand cases with exact arithmetic pin the strictness of
every comparison and every tie rule:
  - Laplacian smoothing in the metric and its acceptance (Sec. 2.4.4);
  - gradient smoothing: direction, step schedule and acceptance (Sec. 2.4.4);
  - flip choice: best new minimum, ties to the smaller far vertex, strict
    improvement (Sec. 2.4.3);
  - re-validation of a colour class against the current graph (Sec. 3.2);
  - the collapse quality bound is inclusive (Sec. 2.4.1);
  - the two-split refinement template's diagonal tie rule (Sec. 2.4.2).
"""
import numpy as np
import pytest

from oracle.orc import OracleMesh, PH_COARSEN, PH_SMOOTH, PH_SWAP, ctx_of, prio
from paper_1505_04694_amd import inputs
from tests import independent as ind

MARGIN = 1e-9     # decisions closer than this (relative) to their threshold are skipped
POS_ATOL = 1e-13  # position agreement between the oracle and the independent solve

JITTERED = [
    ("jit17", lambda: inputs.make_mesh(17, layers=2, jitter_seed=5), 5),
    ("cfg2_33", lambda: inputs.config2(33), 1),
]


def on_classes(om, phase, check):
    """Call check(before, after, members, whole, round) after every class of `phase`."""
    snap = {}

    def hook(ph, rnd, cls, stage):
        if ph != phase:
            return
        if stage == 0:
            snap["d"] = om.export()
            snap["mem"] = om.class_members().copy()
            snap["whole"] = om.class_whole().copy()
        else:
            check(snap["d"], om.export(), snap["mem"], snap["whole"], rnd)

    om.set_hook(hook)


# ---- smoothing ---------------------------------------------------------------------

@pytest.mark.parametrize("name,make,seed", JITTERED)
def test_laplace_moves_to_the_metric_weighted_target(name, make, seed):
    """Every accepted move lands on x_v + G^-1 r with G the sum of edge-mean
    tensors (a 2x2 solve, not Cramer's rule), every rejected vertex stays."""
    om = OracleMesh.from_input(make(), seed=seed)
    tally = dict(moved=0, kept=0, skipped=0)

    def check(before, after, mem, whole, rnd):
        P = ind.Patches(before)
        for v in mem.tolist():
            ok, p, margin = ind.laplace_decision(P, v)
            if margin < MARGIN:
                tally["skipped"] += 1
                continue
            if ok:
                np.testing.assert_allclose(after["xy"][v], p, rtol=0, atol=POS_ATOL, err_msg=f"vertex {v}")
                tally["moved"] += 1
            else:
                assert np.array_equal(after["xy"][v], before["xy"][v]), f"vertex {v} moved but should not"
                tally["kept"] += 1

    on_classes(om, PH_SMOOTH, check)
    st = om.smooth(kind=0, sweeps=2)
    print(tally)
    assert tally["moved"] > 50 and tally["kept"] > 0, tally
    assert tally["moved"] + tally["kept"] + tally["skipped"] == st["evaluated"]
    assert st["committed"] >= tally["moved"]


def test_laplace_accepts_an_equal_minimum():
    """With a constant metric every interior vertex of the criss-cross grid is
    exactly at its target, so the new patch minimum equals the old one; the
    acceptance rule is 'not lower', so every evaluated vertex counts as moved."""
    xy, tri = inputs.grid(17)
    om = OracleMesh(xy, tri, np.tile([40.0, 3.0, 90.0], (len(xy), 1)))
    st = om.smooth(kind=0, sweeps=2)
    assert st["evaluated"] == 2 * 15 * 15
    assert st["committed"] == st["evaluated"]
    assert np.array_equal(om.export()["xy"], xy)


@pytest.mark.parametrize("name,make,seed", JITTERED)
def test_gradient_moves_follow_the_step_schedule(name, make, seed):
    """Direction g/|g|_inf of the patch sum's gradient (torch autograd), trial
    steps h/2 ... h/16 with h the smallest max-norm distance to a neighbour,
    the first trial that keeps areas positive, does not lower the patch
    minimum and raises the patch sum is taken; otherwise the vertex stays."""
    om = OracleMesh.from_input(make(), seed=seed)
    tally = dict(moved=0, kept=0, skipped=0, ks=set())

    def check(before, after, mem, whole, rnd):
        P = ind.Patches(before)
        for v in mem.tolist():
            ok, p, margin, k = ind.gradient_decision(P, v)
            if margin < MARGIN:
                tally["skipped"] += 1
                continue
            if ok:
                np.testing.assert_allclose(after["xy"][v], p, rtol=0, atol=POS_ATOL, err_msg=f"vertex {v}")
                tally["moved"] += 1
                tally["ks"].add(k)
            else:
                assert np.array_equal(after["xy"][v], before["xy"][v]), f"vertex {v} moved but should not"
                tally["kept"] += 1

    on_classes(om, PH_SMOOTH, check)
    st = om.smooth(kind=1, sweeps=2)
    print(tally)
    assert tally["moved"] > 50 and tally["kept"] > 0, tally
    # the schedule is exercised: the first step and a later one were both taken
    assert 1 in tally["ks"] and len(tally["ks"]) >= 2, tally["ks"]
    assert tally["moved"] + tally["kept"] + tally["skipped"] == st["evaluated"]


# ---- swapping ----------------------------------------------------------------------

def apply_flip(tri_rows, d_tid, v, w, a, b, t1, t2):
    lo, hi = sorted((int(d_tid[t1]), int(d_tid[t2])))
    tri_rows[lo] = ind_canon((v, b, a))
    tri_rows[hi] = ind_canon((w, a, b))


def ind_canon(t):
    k = int(np.argmin(t))
    return [t[k], t[(k + 1) % 3], t[(k + 2) % 3]]


@pytest.mark.parametrize("name,make,seed", JITTERED)
def test_flips_match_the_independent_choice(name, make, seed):
    """Every class's element list after the flips equals the one the rule
    gives: per member, the valid flip with the largest new minimum quality,
    kept only if it beats the old minimum strictly (ties to the smaller w)."""
    om = OracleMesh.from_input(make(), seed=seed)
    om.coarsen()
    om.refine()
    tally = dict(flips=0, none=0, multi=0, skipped=0)

    def check(before, after, mem, whole, rnd):
        P = ind.Patches(before)
        exp = before["tri"].copy()
        for v in mem.tolist():
            dec, margin = ind.flip_decision(P, v)
            if margin < MARGIN:
                tally["skipped"] += 1
                for k in P.elems[v]:
                    exp[P.tid[k]] = after["tri"][P.tid[k]]
                continue
            if dec is None:
                tally["none"] += 1
                continue
            w, a, b, t1, t2, _ = dec
            apply_flip(exp, P.tid, v, w, a, b, t1, t2)
            tally["flips"] += 1
        assert np.array_equal(exp, after["tri"]), "flips differ from the independent choice"

    on_classes(om, PH_SWAP, check)
    st = om.swap()
    assert tally["flips"] > 5 and tally["flips"] <= st["committed"], (tally, st)


FAN_BEST = [[-0.5625, 0.5], [-0.4375, -0.375], [-0.25, -0.3125], [-0.3125, -0.75], [0.6875, -0.0625], [0.5, 0.0]]
FAN_TIE = [[0.0, 0.5625], [-0.6875, 0.25], [-0.5, 0.125], [0.0, -0.5625], [0.6875, -0.25], [0.5, -0.125]]


def fan_mesh(ring, seed):
    """Vertex 0 at the origin, ring vertices 1..k in angle order, the fan of
    triangles (0, i, i+1); every vertex untagged, unit metric."""
    xy = np.vstack([[0.0, 0.0], np.asarray(ring, float)])
    k = len(ring)
    tri = np.array([[0, 1 + i, 1 + (i + 1) % k] for i in range(k)], np.int32)
    return OracleMesh(xy, tri, np.tile([1.0, 0.0, 1.0], (k + 1, 1)), np.zeros(k + 1, np.uint8), seed=seed)


def first_class_flip(om):
    """The flip made by the first class of the first swap round: seed 3 gives
    vertex 0 the largest key in that round, so it is alone in class 0."""
    assert max(range(7), key=lambda i: prio(3, ctx_of(0, PH_SWAP, 0), i)) == 0
    out = {}

    def hook(ph, rnd, cls, stage):
        if ph == PH_SWAP and rnd == 0 and cls == 0:
            if stage == 0:
                out["mem"] = om.class_members().tolist()
                out["before"] = om.export()["tri"].copy()
            else:
                out["after"] = om.export()["tri"].copy()

    om.set_hook(hook)
    om.swap(max_rounds=1)
    assert out["mem"] == [0]
    changed = np.nonzero((out["before"] != out["after"]).any(1))[0]
    return out["after"], changed


def test_flip_takes_the_best_not_the_first():
    # vertex 0 has improving flips with ring vertices 2 (new min 0.3773),
    # 4 (0.5059) and 5 (0.2425): the largest new minimum, w = 4, is taken;
    # its elements (0,4,5) [id 3] and (0,3,4) [id 2] become (0,3,5) at the
    # smaller id and (3,4,5) at the larger
    om = fan_mesh(FAN_BEST, seed=3)
    P = ind.Patches(om.export())
    dec, margin = ind.flip_decision(P, 0)
    assert dec[0] == 4 and margin > 1e-2
    after, changed = first_class_flip(om)
    assert changed.tolist() == [2, 3]
    assert after[2].tolist() == [0, 3, 5] and after[3].tolist() == [3, 4, 5]


def test_flip_tie_goes_to_the_smaller_far_vertex():
    # the ring is symmetric under a half turn about vertex 0, which maps
    # vertex i to i+3; the flips of (0,2) and (0,5) give congruent element
    # pairs, so their new minima are equal to the last bit (every coordinate
    # is a multiple of 1/16), and the smaller far vertex, 2, wins
    om = fan_mesh(FAN_TIE, seed=3)
    P = ind.Patches(om.export())
    dec, _ = ind.flip_decision(P, 0)
    assert dec[0] == 2
    after, changed = first_class_flip(om)
    # elements (0,2,3) [id 1] and (0,1,2) [id 0] become (0,1,3) and (1,2,3)
    assert changed.tolist() == [0, 1]
    assert after[0].tolist() == [0, 1, 3] and after[1].tolist() == [1, 2, 3]


def test_flip_needs_a_strict_gain():
    # the unit square split along either diagonal gives two congruent right
    # isosceles triangles: the flip leaves the minimum exactly equal, so none
    xy = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], float)
    om = OracleMesh(xy, np.array([[0, 1, 2], [0, 2, 3]], np.int32), np.tile([1.0, 0, 1.0], (4, 1)),
                    np.zeros(4, np.uint8))
    st = om.swap()
    assert st["committed"] == 0 and st["converged"] == 1


# ---- re-validation -----------------------------------------------------------------

@pytest.mark.parametrize("phase", [PH_COARSEN, PH_SWAP])
@pytest.mark.parametrize("name,make,seed", JITTERED)
def test_revalidation_defers_exactly_the_beaten_members(name, make, seed, phase):
    """A member waits for the next round exactly when a member of its class is
    adjacent to it in the current graph and has a larger key (priority, id)."""
    om = OracleMesh.from_input(make(), seed=seed)
    if phase == PH_SWAP:
        om.coarsen()
        om.refine()
    tally = dict(deferred=0, classes=0)

    def check(before, after, mem, whole, rnd):
        pass

    snap = {}

    def hook(ph, rnd, cls, stage):
        if ph != phase or stage != 0:
            return
        whole = om.class_whole()
        mem = om.class_members()
        P = ind.Patches(om.export())
        ctx = ctx_of(0, phase, rnd)
        deferred = ind.deferred_set(P, whole, lambda v: (prio(seed, ctx, v), v))
        assert sorted(mem.tolist()) == sorted(set(whole.tolist()) - deferred), f"round {rnd} class {cls}"
        tally["deferred"] += len(deferred)
        tally["classes"] += 1

    om.set_hook(hook)
    st = om.coarsen() if phase == PH_COARSEN else om.swap()
    assert tally["deferred"] == st["deferred"] > 0, (tally, st)


# ---- thresholds with exact arithmetic ------------------------------------------------

def test_collapse_quality_bound_is_inclusive():
    # metric diag(0.75, 0.25): the centre's edges have L^2 = 0.25 and tie, so
    # corner 0 is tried first; the two re-pointed elements (0,1,2), (0,2,3)
    # have q^2 = 12 det D^2 / S^2 = 12 * (3/16) / 4 = 0.5625 exactly, which is
    # q_min^2 for q_min = 0.75: allowed (q >= q_min)
    xy = np.array([[0, 0], [1, 0], [1, 1], [0, 1], [0.5, 0.5]], float)
    tri = np.array([[0, 1, 4], [1, 2, 4], [2, 3, 4], [3, 0, 4]], np.int32)
    om = OracleMesh(xy, tri, np.tile([0.75, 0.0, 0.25], (5, 1)))
    st = om.coarsen(q_min=0.75)
    assert st["committed"] == 1
    assert om.export()["tri"].tolist() == [[0, 1, 2], [0, 2, 3]]
    om = OracleMesh(xy, tri, np.tile([0.75, 0.0, 0.25], (5, 1)))
    assert om.coarsen(q_min=0.75 + 2 ** -40)["committed"] == 0


def test_refine_two_splits_tie_cuts_through_the_unsplit_edges_first_vertex():
    # P=(0,0), Q=(1,0), R=(1/2,1), metric diag(1, 8): P-Q has L^2 = 1 (kept),
    # Q-R and R-P have 0.25 + 8 (split). New ids: 3 on (0,2), 4 on (1,2).
    # The diagonals P-4 and Q-3 are mirror images: both L^2 = 0.5625 + 2, a
    # tie, so the quad is cut along the diagonal through P
    om = OracleMesh(np.array([[0, 0], [1, 0], [0.5, 1]], float), np.array([[0, 1, 2]], np.int32),
                    np.tile([1.0, 0.0, 8.0], (3, 1)), np.zeros(3, np.uint8))
    om.refine(max_passes=1)
    d = om.export()
    assert d["xy"][3:].tolist() == [[0.25, 0.5], [0.75, 0.5]]
    assert d["tri"].tolist() == [[2, 3, 4], [0, 1, 4], [0, 4, 3]]


# ---- propagation of the active set between rounds ------------------------------------

def round_log(om, phase):
    """Per round: the active set (the union of its classes), the deferred
    members, and every vertex of an element a class changed."""
    rounds = {}

    def hook(ph, rnd, cls, stage):
        if ph != phase:
            return
        r = rounds.setdefault(rnd, dict(active=set(), deferred=set(), touched=set(), before=None, first=None))
        if stage == 0:
            whole = set(om.class_whole().tolist())
            r["active"] |= whole
            r["deferred"] |= whole - set(om.class_members().tolist())
            r["before"] = om.export()
            if r["first"] is None:
                r["first"] = r["before"]
        else:
            b, a = r["before"], om.export()
            changed = np.nonzero((b["tri"] != a["tri"]).any(1) | (b["talive"] != a["talive"]))[0]
            for t in changed:
                r["touched"] |= set(b["tri"][t].tolist()) | set(a["tri"][t].tolist())

    om.set_hook(hook)
    return rounds


@pytest.mark.parametrize("name,make,seed", JITTERED)
def test_swap_next_round_is_deferred_plus_every_flipped_quad(name, make, seed):
    om = OracleMesh.from_input(make(), seed=seed)
    om.coarsen()
    om.refine()
    rounds = round_log(om, PH_SWAP)
    st = om.swap()
    assert st["rounds"] >= 3
    for r in range(st["rounds"] - 1):
        exp = rounds[r]["deferred"] | rounds[r]["touched"]
        assert rounds[r + 1]["active"] == exp, f"round {r + 1}"
    assert rounds[0]["active"] == set(range(om.sizes()[0]))


@pytest.mark.parametrize("name,make,seed", JITTERED)
def test_coarsen_next_round_is_deferred_plus_changed_rows_with_a_short_edge(name, make, seed):
    """Round r+1 holds the deferred members and every vertex whose adjacency
    changed (the neighbours of a collapsed vertex), kept when it still has a
    short edge it may collapse along (its tags a subset of the neighbour's)."""
    from tests import checker
    om = OracleMesh.from_input(make(), seed=seed)
    rounds = round_log(om, PH_COARSEN)
    st = om.coarsen()
    assert st["rounds"] >= 3
    for r in range(st["rounds"] - 1):
        d = rounds[r + 1]["first"]   # the mesh at the start of round r+1
        P = ind.Patches(d)
        cand = (rounds[r]["deferred"] | rounds[r]["touched"])
        exp = set()
        for v in cand:
            if not d["valive"][v] or not P.nbrs[v]:
                continue
            nb = np.array(P.nbrs[v])
            ok = (d["tags"][v] & ~d["tags"][nb]) == 0
            L2 = checker.metric_len2(d["xy"], d["metric"], np.full(nb.size, v), nb)
            if (ok & (L2 < 0.5)).any():
                exp.add(v)
        assert rounds[r + 1]["active"] == exp, f"round {r + 1}"


def test_quality_constant_is_the_double_nearest_4_sqrt_3():
    # right isosceles triangle with legs 1 and M = I: sqrt(det) = 1, A = 1/2,
    # S = 4, so q = K / 8 with exact scaling; K must be 4 sqrt(3) rounded to
    # the nearest double (computed here with 50 significant digits)
    from decimal import Decimal, getcontext
    getcontext().prec = 50
    k_exact = 4 * Decimal(3).sqrt()
    k = float(k_exact)   # correctly rounded conversion
    om = OracleMesh(np.array([[0, 0], [1, 0], [0, 1]], float), np.array([[0, 1, 2]], np.int32),
                    np.tile([1.0, 0.0, 1.0], (3, 1)), np.zeros(3, np.uint8))
    assert om.element_quality()[0] * 8.0 == k


@pytest.mark.parametrize("name,make,seed", JITTERED)
def test_minmax_moves_follow_the_ascent_on_the_worst_element(name, make, seed):
    """Min-max smoothing: every accepted move is the independent rule's (worst
    element's gradient, or the segment point for two near-equal worst
    elements; halving steps; strict rise of the patch minimum), every rejected
    vertex stays, and the patch minimum rises on every move."""
    om = OracleMesh.from_input(make(), seed=seed)
    tally = dict(moved=0, kept=0, skipped=0)

    def check(before, after, mem, whole, rnd):
        P = ind.Patches(before)
        for v in mem.tolist():
            ok, p, margin = ind.minmax_decision(P, v)
            if margin < 1e-6:
                tally["skipped"] += 1
                continue
            if ok:
                np.testing.assert_allclose(after["xy"][v], p, rtol=0, atol=POS_ATOL, err_msg=f"vertex {v}")
                tally["moved"] += 1
            else:
                assert np.array_equal(after["xy"][v], before["xy"][v]), f"vertex {v} moved but should not"
                tally["kept"] += 1

    on_classes(om, PH_SMOOTH, check)
    q0 = om.quality()[1]
    st = om.smooth(kind=2, sweeps=2)
    assert tally["moved"] > 50 and tally["kept"] > 0, tally
    assert tally["moved"] + tally["kept"] + tally["skipped"] == st["evaluated"]
    assert om.quality()[1] > q0
