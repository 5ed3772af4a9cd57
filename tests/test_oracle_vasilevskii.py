"""Pins of the oracle's second element functional, Vasilevskii's with its size
factor (Sec. 2.2), and of every rule that uses it.

  - closed forms: 1 for the equilateral triangle with unit metric edges in any
    metric; for the equilateral triangle of side h in the unit metric, only the
    size factor is left: 27/64 at h = 1/2 and h = 2, 125/729 at h = 1/3 and 3;
  - an independent evaluation from the three metric edge lengths alone
    (Heron's formula for the metric area), with vertex metrics that differ;
  - invariances: joint scaling (M -> c^2 M, x -> x / c), affine maps, and the
    bound Q <= 1;
  - the adjoint against central differences of the patch-local functional;
  - the decisions that read the functional (collapse bound, both smoothers'
    acceptance and direction, min-max, flip choice) re-derived independently.
"""
import math

import numpy as np
import pytest

from oracle.orc import OracleMesh, PH_SMOOTH, PH_SWAP, QUALITY_VASILEVSKII as VAS
from paper_1505_04694_amd import inputs
from tests import checker, fdcheck
from tests import independent as ind
from tests.test_oracle_rules import JITTERED, MARGIN, POS_ATOL, apply_flip, on_classes

EQ = np.array([[0.0, 0.0], [1.0, 0.0], [0.5, math.sqrt(3.0) / 2.0]])


def one_tri(xy, met):
    met = np.asarray(met, float)
    if met.ndim == 1:
        met = np.tile(met, (len(xy), 1))
    return OracleMesh(np.asarray(xy, float), np.array([[0, 1, 2]], np.int32), met,
                      np.zeros(len(xy), np.uint8), quality=VAS)


def q_of(xy, met):
    return one_tri(xy, met).element_quality()[0]


def ccw(xy):
    if checker.doubled_areas(xy, np.array([[0, 1, 2]]))[0] < 0:
        xy = xy[[0, 2, 1]]
    return xy


def test_unit_equilateral_is_one():
    assert q_of(EQ, [1.0, 0.0, 1.0]) == pytest.approx(1.0, abs=2e-16)


@pytest.mark.parametrize("h,expected", [(0.5, 27 / 64), (2.0, 27 / 64), (1 / 3, 125 / 729), (3.0, 125 / 729)])
def test_equilateral_of_side_h_keeps_only_the_size_factor(h, expected):
    # shape part 1; x = P / 3 = h; m = min(h, 1/h); F = (m (2 - m))^3:
    # m = 1/2 gives (3/4)^3, m = 1/3 gives (5/9)^3, on both sides of x = 1
    assert q_of(EQ * h, [1.0, 0.0, 1.0]) == pytest.approx(expected, rel=1e-14)


@pytest.mark.parametrize("seed", range(5))
def test_unit_equilateral_in_metric_space_is_one(seed):
    rng = np.random.default_rng(seed)
    F = rng.normal(size=(2, 2))
    if np.linalg.det(F) < 0:
        F[:, 0] *= -1
    M = F.T @ F
    xy = np.linalg.solve(F, EQ.T).T
    assert q_of(xy, [M[0, 0], M[0, 1], M[1, 1]]) == pytest.approx(1.0, rel=1e-12)


@pytest.mark.parametrize("seed", range(8))
def test_matches_heron_from_metric_lengths(seed):
    rng = np.random.default_rng(300 + seed)
    xy = ccw(rng.uniform(0, 1, (3, 2)))
    met = []
    for _ in range(3):
        F = rng.normal(size=(2, 2))
        M = F.T @ F * rng.uniform(0.5, 20.0) + 0.1 * np.eye(2)
        met.append([M[0, 0], M[0, 1], M[1, 1]])
    met = np.array(met)
    ref = checker.vasilevskii(xy, met, np.array([[0, 1, 2]]))[0]
    assert q_of(xy, met) == pytest.approx(ref, rel=1e-10)


@pytest.mark.parametrize("seed", range(5))
def test_invariances_and_bound(seed):
    rng = np.random.default_rng(400 + seed)
    xy = ccw(rng.uniform(0, 1, (3, 2)))
    F = rng.normal(size=(2, 2))
    M = F.T @ F * 4.0 + 0.1 * np.eye(2)
    m = np.array([M[0, 0], M[0, 1], M[1, 1]])
    q = q_of(xy, m)
    assert 0 < q <= 1.0
    c = 3.0
    assert q_of(xy / c, m * c * c) == pytest.approx(q, rel=1e-12)      # metric lengths unchanged
    assert q_of(xy * 0.5 + 0.2, m * 4.0) == pytest.approx(q, rel=1e-12)
    L = np.linalg.cholesky(M).T                                        # M = L^T L
    assert q_of((L @ xy.T).T, [1.0, 0.0, 1.0]) == pytest.approx(q, rel=1e-12)
    # unlike the mean ratio, it is not invariant under M -> c M alone
    assert abs(q_of(xy, m * 7.0) - q) > 1e-3 * q


@pytest.mark.parametrize("n", [17, 65])
def test_adjoint_matches_central_differences(n):
    mi = inputs.config2(n)
    om = OracleMesh.from_input(mi, seed=1, quality=VAS)
    Q, qmin, gx, gm = om.quality(grad=True)
    worst = 0.0
    for v in fdcheck.protocol_vertices(mi.V):
        v = int(v)
        fx, fm, Qv, hx, hm = fdcheck.central_differences(om, v, mi.xy[v], mi.metric[v])
        worst = max(worst, fdcheck.check_entries(fx, gx[v], Qv, hx, f"dQ/dx at {v}"))
        worst = max(worst, fdcheck.check_entries(fm, gm[v], Qv, hm, f"dQ/dM at {v}"))
    assert worst <= 1e-6
    # translation invariance holds; scaling does not (the size factor)
    scale = np.abs(gx).sum()
    assert abs(gx[:, 0].sum()) <= 1e-10 * scale and abs(gx[:, 1].sum()) <= 1e-10 * scale


def test_element_quality_is_the_independent_value_on_a_mesh():
    mi = inputs.config2(33)
    om = OracleMesh.from_input(mi, seed=1, quality=VAS)
    d = om.export()
    np.testing.assert_allclose(om.element_quality(), checker.vasilevskii(d["xy"], d["metric"], d["tri"]),
                               rtol=1e-10)


def test_collapse_bound_reads_the_functional():
    # the centre of the square collapses onto corner 0 and leaves two elements
    # whose metric edges are sqrt(3/4), 1/2 and 1; the collapse is allowed
    # exactly when their functional (computed independently) is >= q_min
    xy = np.array([[0, 0], [1, 0], [1, 1], [0, 1], [0.5, 0.5]], float)
    tri = np.array([[0, 1, 4], [1, 2, 4], [2, 3, 4], [3, 0, 4]], np.int32)
    met = np.tile([0.75, 0.0, 0.25], (5, 1))
    qexp = checker.vasilevskii(xy[:4], met[:4], np.array([[0, 1, 2]]))[0]
    assert abs(qexp - 0.75) > 0.01      # the mean ratio of these elements is 0.75
    om = OracleMesh(xy, tri, met, quality=VAS)
    assert om.coarsen(q_min=qexp * (1 - 1e-9))["committed"] == 1
    assert om.export()["tri"].tolist() == [[0, 1, 2], [0, 2, 3]]
    om = OracleMesh(xy, tri, met, quality=VAS)
    assert om.coarsen(q_min=qexp * (1 + 1e-9))["committed"] == 0


def _smoothing_check(kind_smooth, decide):
    name, make, seed = JITTERED[1]
    om = OracleMesh.from_input(make(), seed=seed, quality=VAS)
    tally = dict(moved=0, kept=0, skipped=0)

    def check(before, after, mem, whole, rnd):
        P = ind.Patches(before, kind=VAS)
        for v in mem.tolist():
            ok, p, margin = decide(P, v)[:3]
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
    st = om.smooth(kind=kind_smooth, sweeps=2)
    assert tally["moved"] > 50 and tally["kept"] > 0, tally
    assert tally["moved"] + tally["kept"] + tally["skipped"] == st["evaluated"]


def test_laplace_acceptance_reads_the_functional():
    _smoothing_check(0, ind.laplace_decision)


def test_gradient_smoothing_reads_the_functional():
    _smoothing_check(1, ind.gradient_decision)


def test_minmax_smoothing_reads_the_functional():
    _smoothing_check(2, ind.minmax_decision)


def test_flips_read_the_functional():
    name, make, seed = JITTERED[1]
    om = OracleMesh.from_input(make(), seed=seed, quality=VAS)
    om.coarsen()
    om.refine()
    tally = dict(flips=0)

    def check(before, after, mem, whole, rnd):
        P = ind.Patches(before, kind=VAS)
        exp = before["tri"].copy()
        for v in mem.tolist():
            dec, margin = ind.flip_decision(P, v)
            if margin < MARGIN:
                for k in P.elems[v]:
                    exp[P.tid[k]] = after["tri"][P.tid[k]]
                continue
            if dec is None:
                continue
            w, a, b, t1, t2, _ = dec
            apply_flip(exp, P.tid, v, w, a, b, t1, t2)
            tally["flips"] += 1
        assert np.array_equal(exp, after["tri"]), "flips differ from the independent choice"

    on_classes(om, PH_SWAP, check)
    st = om.swap()
    assert tally["flips"] > 5 and tally["flips"] <= st["committed"], (tally, st)


def test_unknown_functional_is_rejected():
    with pytest.raises(ValueError):
        OracleMesh(EQ, np.array([[0, 1, 2]], np.int32), np.tile([1.0, 0, 1.0], (3, 1)), quality=7)
