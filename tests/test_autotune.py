"""The autotuner's host logic (CPU only): shape classes and the choice among timed candidates."""
from paper_2605_19388_amd import autotune


def test_choose_fastest_then_larger_tile():
    assert autotune.choose({16: 3.0, 32: 2.0, 64: 2.5, 128: 4.0}) == 32
    assert autotune.choose({16: 2.0, 32: 2.0, 64: 2.0, 128: 3.0}) == 64


def test_shape_classes_bin_the_recording_length():
    a = autotune.shape_key(513, 260, (4, 4), 3, 16)
    b = autotune.shape_key(513, 499, (4, 4), 3, 16)
    c = autotune.shape_key(513, 500, (4, 4), 3, 16)
    assert a == b and a != c
    assert autotune.shape_key(513, 260, (4, 4), 3, 16, fp32=False) != a
    assert autotune.shape_key(513, 260, (4, 4, 4), 3, 16) != a


def test_cache_file_is_read(tmp_path):
    path = tmp_path / "tiles.json"
    key = repr(autotune.shape_key(33, 100, (2, 2), 2, 4))
    path.write_text('{"%s": 64}' % key.replace('"', '\\"'))
    autotune._cache.pop(key, None)
    best, timings = autotune.tune(33, 100, (2, 2), 2, 4, cache_path=str(path))   # no GPU touched
    assert best == 64 and timings == {}
