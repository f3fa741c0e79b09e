"""Autotuner logic on the host: candidate space, signature buckets, choice of
the fastest candidate, and the JSON cache."""
import json

from paper_2406_01579_amd import tune


def test_candidate_space_covers_tiles_waves_and_chunks():
    c = tune.candidates()
    assert (8, 8, 4, 64, 32) in c and (8, 8, 4, 32, 16) in c and (8, 8, 1, 0, 0) in c
    assert (16, 16, 1, 0, 0) in c and (32, 8, 1, 0, 0) in c
    # 8x8: one wave, or 2/4/8 waves x forward chunk {32, 64} x backward chunk {16, 32}; four larger tiles
    assert len(c) == len(set(c)) == 1 + 3 * 2 * 2 + 4
    assert len({tune.label(x) for x in c}) == len(c)


def test_signature_buckets():
    a = tune.signature(1572864, 123810, [(512, 512)] * 4, 4, 320.0)
    b = tune.signature(1572864, 120000, [(512, 512)] * 4, 4, 330.0)   # same buckets
    c = tune.signature(1572864, 123810, [(1024, 1024)] * 4, 4, 320.0)
    assert a == b and a != c
    assert json.loads(a)["sizes"] == [[512, 512]]


def test_tune_picks_fastest_and_caches(tmp_path):
    path = str(tmp_path / "tune.json")
    calls = []

    def measure(p):
        k = (p.tile_w, p.tile_h, p.waves, p.chunk_fwd, p.chunk_bwd)
        calls.append(k)
        return {(8, 8, 4, 32, 16): 1.0}.get(k, 2.0)

    t = tune.Autotuner(path)
    best = t.tune("k", measure)
    assert (best.tile_w, best.tile_h, best.waves, best.chunk_fwd, best.chunk_bwd) == (8, 8, 4, 32, 16)
    assert len(calls) == len(tune.candidates())
    # a second tuner reads the cache and measures nothing
    t2 = tune.Autotuner(path)
    calls.clear()
    best2 = t2.tune("k", measure)
    assert (best2.tile_w, best2.tile_h, best2.waves, best2.chunk_bwd) == (8, 8, 4, 16) and not calls
    assert json.load(open(path))["k"]["best"] == [8, 8, 4, 32, 16]
