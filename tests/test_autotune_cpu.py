"""Host logic of the scan autotuner (CPU): candidate lists, problem classes
and the JSON cache; the timing itself runs on the GPU (tests/test_gpu_batch.py)."""

from paper_2411_00991_amd import autotune


def test_candidates_cover_the_allowed_scans():
    c = autotune.candidates(31)
    assert c[0] == 0                                   # pixel-chromatic
    assert -30 in c and -31 in c                       # block-series at s - 1 and s
    assert all(b in c for b in (30, 31, 32, 46, 62))   # block-phase from s - 1 to 2 s
    assert -1015 in c and -1031 in c                   # nine phases at (s - 1)/2 and s
    assert autotune.candidates(31, allow_chromatic=False)[0] != 0
    assert all(b >= 0 for b in autotune.candidates(31, allow_series=False))
    assert all(b > -1000 for b in autotune.candidates(31, allow_nine=False))
    assert all(b >= 0 for b in autotune.candidates(33))     # no series beyond a 31 x 31 PSF


def test_candidate_codes_decode_to_scans():
    from paper_2411_00991_amd import (BDC_SCHED_BLOCK, BDC_SCHED_BLOCK9_SERIES, BDC_SCHED_BLOCK_SERIES,
                                      BDC_SCHED_CHROMATIC)
    assert autotune.decode(0) == (BDC_SCHED_CHROMATIC, 0)
    assert autotune.decode(-30) == (BDC_SCHED_BLOCK_SERIES, 30)
    assert autotune.decode(-1015) == (BDC_SCHED_BLOCK9_SERIES, 15)
    assert autotune.decode(46) == (BDC_SCHED_BLOCK, 46)


def test_problem_classes_keep_allowed_scans_apart():
    keys = {autotune.problem_class(11, 100, 120, 2, ch, se, ni) for ch in (False, True) for se in (False, True)
            for ni in (False, True)}
    assert len(keys) == 6                              # the nine-phase scan only alongside the series scan
    assert autotune.problem_class(11, 100, 120, 2, True) == autotune.problem_class(11, 128, 65, 2, True)
    assert autotune.problem_class(11, 100, 120, 2, True) != autotune.problem_class(11, 129, 65, 2, True)


def test_cache_round_trip(tmp_path, monkeypatch):
    monkeypatch.setenv("BDC_AUTOTUNE_CACHE", str(tmp_path / "sub" / "tune.json"))
    assert autotune.load_cache() == {}
    data = {"dev": {"s11_side128_c2_block": {"block": -11}}}
    autotune.save_cache(data)
    assert autotune.load_cache() == data
    (tmp_path / "sub" / "tune.json").write_text("{not json")
    assert autotune.load_cache() == {}
