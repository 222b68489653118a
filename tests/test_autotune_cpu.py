"""Host logic of the launch autotuner (no GPU): candidate set, bucket keys, choice of the
fastest candidate, JSON cache reuse and invalidation when the library changes."""
import json

from paper_2602_22625_amd import autotune


def test_candidates_cover_tiles_and_schedules():
    c = autotune.candidates()
    assert {t for t, _, _, _ in c} == {8, 16, 32}
    assert {s for _, s, _, _ in c} == {0, 1, 2}
    assert {w for _, s, w, _ in c if s == 2} == {2, 4, 8}
    assert {g for _, s, _, g in c if s == 2} == {0, 1, 16}
    assert len(c) == len(set(c)) == 33
    assert len({autotune.cfg_name(x) for x in c}) == 33


def test_bucket_key_rounds_sizes_and_counts():
    assert autotune.bucket_key([(512, 512, 4096)]) == autotune.bucket_key([(530, 500, 5000)])
    assert autotune.bucket_key([(512, 512, 4096)]) != autotune.bucket_key([(512, 512, 8192)])
    a = autotune.bucket_key([(256, 256, 600), (1024, 768, 9000)])
    b = autotune.bucket_key([(1024, 768, 9000), (256, 256, 600)])
    assert a == b  # order of the images in a batch does not matter
    big = autotune.bucket_key([(256 + 128 * (i % 7), 256, 512 << (i % 5)) for i in range(64)])
    assert big.startswith("n64|sha1:") and len(big) < 80


def test_tune_picks_fastest_and_caches(tmp_path):
    path = str(tmp_path / "tune.json")
    calls = []

    def measure(cfg):
        calls.append(cfg)
        t, s, w, g = cfg
        return 1.0 + abs(t - 16) * 0.1 + (0.0 if s == 2 and w == 4 and g == 0 else 0.05)

    tu = autotune.Autotuner(path, version="v1")
    best = tu.tune("k", measure)
    assert best == (16, 2, 4, 0)
    assert len(calls) == 33
    db = json.load(open(path))
    assert db["k"]["tile"] == 16 and db["k"]["schedule"] == 2 and len(db["k"]["all"]) == 33
    # a second tuner on the same file reuses the entry without measuring
    calls.clear()
    assert autotune.Autotuner(path, version="v1").tune("k", measure) == (16, 2, 4, 0)
    assert calls == []
    # a different library version measures again
    assert autotune.Autotuner(path, version="v2").tune("k", measure) == (16, 2, 4, 0)
    assert len(calls) == 33


def test_tune_with_subset_and_force(tmp_path):
    path = str(tmp_path / "t.json")
    tu = autotune.Autotuner(path, version="x")
    a, b = (8, 0, 4, 1), (32, 1, 4, 1)
    assert tu.tune("a", lambda c: {a: 2.0, b: 1.0}[c], [a, b]) == b
    assert tu.tune("a", lambda c: {a: 0.5, b: 1.0}[c], [a, b], force=True) == a
