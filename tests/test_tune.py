"""Tile autotuner host logic on the CPU: the candidate set is legal, buckets
separate what should be tuned apart, the cache round-trips and rejects stale or
illegal entries, and the choice is by median with ties to the default."""

import json

import pytest

import problems
from paper_2110_10191_amd import tune


@pytest.mark.parametrize("cls,maxt", [("sweep", 512), ("update", 256)])
def test_candidates_are_legal_and_cover_the_default(cls, maxt):
    c = tune.candidates(cls)
    assert tune.DEFAULT[cls] in c
    assert len(c) == len(set(c))
    for tx, ty in c:
        assert tx & (tx - 1) == 0 and 16 <= tx <= 256
        assert (tx * ty) % 64 == 0 and tx * ty <= maxt
    assert {(256, 1), (128, 2), (64, 1), (32, 8)} <= set(c)
    assert ((64, 8) in c) == (cls == "sweep")


def test_bucket_separates_recon_precision_and_size():
    a, _ = problems.linear_modes(n=32)
    b, _ = problems.linear_modes(n=32, recon=problems.RECON_WENO5)
    c, _ = problems.linear_modes(n=32, precision=problems.MIXED)
    d, _ = problems.linear_modes(n=64)
    e, _ = problems.linear_modes(n=30)
    keys = {tune.bucket(p) for p in (a, b, c, d)}
    assert len(keys) == 4
    assert tune.bucket(a) == tune.bucket(e)           # same power-of-two bucket
    assert tune.bucket(a) == "mc/fp64/n1<=32/zones<=32768"


def test_cache_roundtrip_and_scoping(tmp_path):
    path = str(tmp_path / "sub" / "tiles.json")
    c1 = tune.TileCache(path, device="devA", lib_hash="h1")
    assert c1.get("k") is None
    c1.put("k", {"sweep": (128, 2), "update": (64, 1)}, {"sweep": 1.5, "update": 2.0})
    assert c1.get("k") == {"sweep": (128, 2), "update": (64, 1)}
    # another library build or device does not see it
    assert tune.TileCache(path, device="devA", lib_hash="h2").get("k") is None
    assert tune.TileCache(path, device="devB", lib_hash="h1").get("k") is None
    with open(path) as f:
        data = json.load(f)
    assert data["devA|h1"]["k"]["ms_per_step"] == {"sweep": 1.5, "update": 2.0}


def test_cache_ignores_illegal_or_corrupt_entries(tmp_path):
    path = tmp_path / "tiles.json"
    path.write_text(json.dumps({"d|h": {"k": {"sweep": [48, 4], "update": [64, 4]}}}))
    assert tune.TileCache(str(path), device="d", lib_hash="h").get("k") is None
    path.write_text(json.dumps({"d|h": {"k": {"sweep": [64, 8], "update": [64, 8]}}}))   # 512 > update bound
    assert tune.TileCache(str(path), device="d", lib_hash="h").get("k") is None
    path.write_text("{not json")
    c = tune.TileCache(str(path), device="d", lib_hash="h")
    assert c.get("k") is None
    c.put("k", {"sweep": (64, 4), "update": (256, 1)})
    assert c.get("k") == {"sweep": (64, 4), "update": (256, 1)}


def test_pick_uses_median_and_keeps_the_first_on_ties():
    times = {(64, 4): [3.0, 1.0, 2.0], (128, 2): [2.0, 2.0, 9.0], (256, 1): [5.0, 0.1, 5.0]}
    assert tune.pick(times) == ((64, 4), 2.0)
    times = {(64, 4): [2.0], (128, 2): [1.9, 1.9, 50.0]}
    assert tune.pick(times)[0] == (128, 2)


def test_library_hash_is_content_based(tmp_path):
    f = tmp_path / "a.so"
    f.write_bytes(b"abc")
    h1 = tune.library_hash(str(f))
    f.write_bytes(b"abd")
    assert tune.library_hash(str(f)) != h1
    assert len(h1) == 16


@pytest.mark.gpu
def test_tuning_returns_a_candidate_and_caches_it(lib, tmp_path):
    prm, P0 = problems.fm_torus(n1=64, n2=32, n3=16)
    cache = tune.TileCache(str(tmp_path / "tiles.json"))
    tiles = tune.tune_problem(prm, P0, cache=cache, steps=1, repeats=1)
    assert tiles["sweep"] in tune.candidates("sweep") and tiles["update"] in tune.candidates("update")
    assert cache.get(tune.bucket(prm)) == tiles
    sim = lib.Sim(prm)
    assert tune.apply(sim, cache) == tiles
    assert sim.get_tiles("sweep") == tiles["sweep"]
    assert sim.get_tiles("update") == tiles["update"]
    sim.close()


def test_search_finds_the_separable_minimum():
    # cost = f(sweep tile) + g(update tile) with distinct minima
    fs = {(128, 2): 1.0}
    gs = {(32, 8): 0.5}
    calls = []

    def measure(t):
        calls.append(t)
        return fs.get(t["sweep"], 3.0) + gs.get(t["update"], 2.0)

    tiles, best = tune.search(measure, repeats=2)
    assert tiles == {"sweep": (128, 2), "update": (32, 8)}
    assert best == {"sweep": 3.0, "update": 1.5}
    assert len(calls) == 2 * (len(tune.candidates("sweep")) + len(tune.candidates("update")))
    # the defaults are tried first
    assert calls[0] == {"sweep": (64, 8), "update": (64, 1)}
