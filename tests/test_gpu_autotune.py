"""The autotuner: it returns a valid choice, caches it, and the knobs it picks
leave every result unchanged (the same per-op results, image and counters as
the library's defaults)."""
from __future__ import annotations

import json

import numpy as np
import pytest

from gpu_util import assert_same_image, assert_same_ops, assert_same_stats, gpu_insert, \
    gpu_lookup, gpu_table, keys_for

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("scheme,B", [("sorted", 8), ("queue", 4)])
def test_tune_choice_is_result_neutral(tmp_path, monkeypatch, scheme, B):
    from paper_1605_05236_amd import autotune
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "tune.json"))
    n = 1 << 14
    print(f"autotune {scheme} B={B}", flush=True)
    choice = autotune.tune(n, B, 2, scheme, load=0.95, sample_bins_log2=14,
                           wgs_choices=(1, 4, 16), force=True)
    assert choice["evict_wgs_per_cu"] in (1, 4, 16)
    assert choice["lanes_per_probe"] in (1, B)
    assert set(choice["measured"]["fill"]) == {f"{1 << 20}:{w}" for w in (1, 4, 16)}
    assert all(v > 0 for v in choice["measured"]["fill"].values())
    cached = json.load(open(tmp_path / "tune.json"))
    assert list(cached.values())[0]["evict_wgs_per_cu"] == choice["evict_wgs_per_cu"]
    # a second call is served from the cache
    assert autotune.tune(n, B, 2, scheme, load=0.95, sample_bins_log2=14,
                         wgs_choices=(1, 4, 16)) == cached[list(cached)[0]]

    keys, vals = keys_for(n, B, 0.97, seed=21)
    kw = dict(max_search=500, batch_ops=1 << 12)
    tuned = gpu_table(n, B, 2, scheme, seed=21, evict_wgs_per_cu=choice["evict_wgs_per_cu"],
                      **kw)
    plain = gpu_table(n, B, 2, scheme, seed=21, **kw)
    rt = gpu_insert(tuned, keys, vals)
    assert_same_ops(rt, gpu_insert(plain, keys, vals), "tuned")
    assert_same_image(tuned.export(), plain.export(), "tuned")
    # the arena's size follows the planner grid; every counter of the method matches
    st, sp = tuned.stats(), plain.stats()
    st.pop("arena_moves"), sp.pop("arena_moves")
    assert_same_stats(st, sp, "tuned")
    vt, ft = gpu_lookup(tuned, keys, lpp=choice["lanes_per_probe"])
    vp, fp = gpu_lookup(plain, keys)
    assert np.array_equal(ft, fp) and np.array_equal(vt, vp)
    assert np.array_equal(ft.astype(bool), rt["status"] == 1)
