"""GPU test of the autotuner's search (tune.py): it times every valid (tile,
workgroup) pair on the GPU, caches the fastest, and best() then returns that
choice."""
from __future__ import annotations

import json

import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind,dtype,n", [("heat", "f64", 64), ("euler", "f32", 64)])
def test_search_caches_the_fastest_measured_candidate(tmp_path, monkeypatch, kind, dtype, n):
    from paper_2105_10332_amd import tune

    cache = tmp_path / "tune.json"
    monkeypatch.setenv("SWEPT_TUNE_CACHE", str(cache))
    b, wg, results = tune.tune(kind, dtype, n, steps=16, reps=2, save=True)
    cands = tune.candidates(kind, dtype, n)
    assert sorted((rb, rw) for _, rb, rw in results) == sorted(cands), "every candidate is timed once"
    fastest = min(results)
    assert (b, wg) == (fastest[1], fastest[2])
    entry = json.loads(cache.read_text())[tune._key(kind, dtype, n)]
    assert (entry["tile"], entry["wg"]) == (b, wg) and entry["ms"] == fastest[0]
    assert tune.best(kind, dtype, n) == (b, wg)
    print(f"tune {kind} {dtype} {n}: {len(results)} candidates, fastest tile {b} wg {wg} ({fastest[0]:.3f} ms)")
