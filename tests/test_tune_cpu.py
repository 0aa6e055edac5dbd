"""Host logic of the autotuner: size buckets, cache keys, the candidate lists
per precision, the cache round trip, and the shipped cache (every stored shape
is a valid configuration that passed its accuracy gate).  No GPU here."""
from __future__ import annotations

import json

import pytest

from paper_1907_10514_amd import lion as L
from paper_1907_10514_amd import tune

ALLOWED = {
    "i_per_lane": {1, 2, 4},
    "j_split": set(range(1, 65)),
    "chunk_steps": set(range(1, 1001)),
    "flush_len": {4, 8, 16},
    "batch_block": {256, 512, 1024},
    "use_graph": {1, 2},
    "lds_sources": {1, 2},
    "symmetric": {1, 2},
    "sym_variant": set(range(1, 10)),
    "update_waves": {4, 8, 16},
    "small_trap": {1, 2},
    "batch_tpt": {1, 2, 4},
    "step_launches": {1, 2},
}


@pytest.mark.parametrize("n,bucket", [(1, 1), (8, 8), (1000, 1024), (12000, 16384),
                                      (16384, 16384), (23000, 16384), (24000, 32768),
                                      (65536, 65536), (130408, 131072)])
def test_size_bucket(n, bucket):
    assert tune.size_bucket(n) == bucket


def test_cache_key_fields():
    k = tune.cache_key("gfx950:sramecc+:xnack-", 16000, L.LION_MIXED_F64ACC, False, rocm="7.0")
    assert k == "gfx950|rocm7.0|n16384|p1|single"
    k = tune.cache_key("gfx950", 130408, L.LION_FP64, True, 512, rocm="7.0")
    assert k == "gfx950|rocm7.0|n131072|p0|batch512"


@pytest.mark.parametrize("prec", [L.LION_FP64, L.LION_MIXED_F64ACC, L.LION_MIXED_KAHAN])
def test_candidates_cover_both_kernel_families(prec):
    """Every precision offers all-pairs shapes (symmetric=1, explicit) and,
    while the tile count allows (N <= 131072), the pair-once kernels."""
    for n, sym_ok in ((4096, True), (131072, True), (131073, False)):
        cands = list(tune.single_candidates(n, prec))
        assert all(c.get("symmetric") in (1, 2) for c in cands)
        for c in cands:
            for k, v in c.items():
                assert v in ALLOWED[k], (k, v)
        allp = [c for c in cands if c["symmetric"] == 1]
        once = [c for c in cands if c["symmetric"] == 2]
        assert len(allp) >= 30
        assert bool(once) == sym_ok
        assert len({json.dumps(c, sort_keys=True) for c in cands}) == len(cands)
        if prec == L.LION_MIXED_F64ACC:
            assert {c["flush_len"] for c in allp} == {8, 16}


def test_cache_round_trip(tmp_path, monkeypatch):
    path = tmp_path / "cache.json"
    monkeypatch.setenv(tune.CACHE_ENV, str(path))
    assert tune.load_cache() == {}
    entry = {"best": {"config": {"symmetric": 2, "sym_variant": 7}, "pair_ms": 0.075,
                      "m1_vs_fp64": 1.4e-7, "ok": True}}
    key = tune.cache_key("gfx950", 16384, L.LION_MIXED_F64ACC, False)
    tune.store(key, entry)
    assert tune.lookup("gfx950", 16000, L.LION_MIXED_F64ACC, False) == \
        {"symmetric": 2, "sym_variant": 7}
    assert tune.lookup("gfx950", 16000, L.LION_FP64, False) is None
    path.write_text("{not json")
    assert tune.load_cache() == {}


def test_shipped_cache_is_valid():
    data = tune.load_cache(tune.DEFAULT_CACHE)
    assert data, "no shipped tune cache"
    for key, ent in data.items():
        arch, rocm, nb, prec, shape = key.split("|")
        p = int(prec[1:])
        assert p in (L.LION_FP64, L.LION_MIXED_F64ACC, L.LION_MIXED_KAHAN), key
        for k, v in ent["config"].items():
            assert v in ALLOWED[k], (key, k, v)
        meas = ent["measured"]
        assert all(ent["config"].get(k) == v for k, v in meas["config"].items()), key
        # every stored shape passed its accuracy gate against the FP64 path
        assert meas["ok"] and meas["m1_vs_fp64"] <= 0.5 * tune.BAR[p], key
        if shape == "single":
            if ent["config"].get("symmetric") == 2:
                assert (int(nb[1:]) + 255) // 256 <= 512, key


def test_batch_candidates():
    """Workgroup sizes x targets per thread, with no 4 targets at 1024 threads
    (their register budget); every candidate a valid configuration."""
    cands = list(tune.batch_candidates())
    assert len(cands) == 8
    assert {(c["batch_block"], c["batch_tpt"]) for c in cands} == \
        {(b, t) for b in (256, 512, 1024) for t in (1, 2, 4)} - {(1024, 4)}
    for c in cands:
        for k, v in c.items():
            assert v in ALLOWED[k], (k, v)


def test_batch_scale_is_per_trap():
    """The batch accuracy gate's scale counts sources of the ion's own trap only."""
    import numpy as np

    x = np.array([0.0, 1.0, 10.0, 11.0])
    z0 = np.zeros(4)
    s = tune._batch_scale([2, 2], x, z0, z0)
    assert np.allclose(s, [1.0, 1.0, 1.0, 1.0])
