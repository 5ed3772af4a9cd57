"""The autotuner of the kernel shapes: every candidate it times gives the same
meshes (it raises otherwise), the choice it keeps matches the oracle, and its
JSON cache answers the second call."""
import numpy as np
import pytest

from paper_1505_04694_amd import autotune, inputs, pmesh
from tests.parity import both, compare_mesh, compare_stats

pytestmark = pytest.mark.gpu


def test_autotuner_on_one_mesh(tmp_path, monkeypatch):
    monkeypatch.setenv(autotune.CACHE_ENV, str(tmp_path / "tune.json"))
    mi = inputs.config2(129)
    tune, rep = autotune.autotune([(mi.xy, mi.tri, mi.metric, mi.tags)], seed=1, repeats=1)
    n_cand = 1 + sum(len(v) - 1 for v in autotune.SPACE.values())
    assert len(rep["tried"]) == n_cand and not rep["cached"]
    om, gm = both(mi, 1)
    gm.tune = tune
    for name in ("coarsen", "refine", "swap", "smooth"):
        kw = {} if name == "refine" else {"sweep": 0}
        compare_stats(getattr(om, name)(**kw), getattr(gm, name)(**kw), name)
    compare_mesh(om, gm, "tuned sweep")
    tune2, rep2 = autotune.autotune([(mi.xy, mi.tri, mi.metric, mi.tags)], seed=1, repeats=1)
    assert rep2["cached"] and tune2 == tune


def test_autotuner_on_a_batch(tmp_path, monkeypatch):
    monkeypatch.setenv(autotune.CACHE_ENV, str(tmp_path / "tune.json"))
    mis = inputs.config3(6, seed=2)
    meshes = [(mi.xy, mi.tri, mi.metric, mi.tags) for mi in mis]
    tune, rep = autotune.autotune(meshes, seed=2, repeats=1)
    assert not rep["cached"] and set(tune) == set(autotune.SPACE)
