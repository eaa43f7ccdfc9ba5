"""The launch-shape tuner's table and cache file (host logic only: nothing
here launches a kernel)."""

import pytest

HEADER = "# sambaten launch-shape cache v1\n"


@pytest.fixture
def clean(lib):
    lib.autotune_clear()
    yield lib
    lib.autotune_clear()
    lib.autotune_set(lib.SBT_TUNE_ON)


def rows_of(path):
    return sorted(ln for ln in path.read_text().splitlines() if ln and not ln.startswith("#"))


def test_cache_file_round_trip(clean, tmp_path):
    lib = clean
    rows = ["gfx950 1 20 9000 3 1 2 3", "gfx950 2 20 9000 3 1 1 3", "gfx942 0 1 9000 3 0 0 3"]
    src = tmp_path / "in.txt"
    src.write_text(HEADER + "# a comment\n\n" + "\n".join(rows) + "\n")
    lib.autotune_load(src)
    assert lib.autotune_count() == (3, 0)
    out = tmp_path / "out.txt"
    lib.autotune_save(out)
    assert out.read_text().startswith(HEADER)
    assert rows_of(out) == sorted(rows)
    # loading again merges: the file's shape wins for a key present in both
    src.write_text(HEADER + "gfx950 1 20 9000 3 1 0 3\ngfx950 1 20 9000 3 2 1 3\n")
    lib.autotune_load(src)
    assert lib.autotune_count() == (4, 0)
    lib.autotune_save(out)
    assert "gfx950 1 20 9000 3 1 0 3" in rows_of(out)
    lib.autotune_clear()
    assert lib.autotune_count() == (0, 0)


@pytest.mark.parametrize("body", [
    "gfx950 1 20 9000 3 1 3 3\n",      # shape beyond the kernel's choices
    "gfx950 7 20 9000 3 1 0 3\n",      # no such kernel
    "gfx950 1 20 9000 3 1 0\n",        # a field missing
    "gfx950 1 20 9000 3 1 -1 3\n",     # negative shape
])
def test_malformed_files_change_nothing(clean, tmp_path, body):
    lib = clean
    good = tmp_path / "good.txt"
    good.write_text(HEADER + "gfx950 0 2 100 4 0 1 3\n")
    lib.autotune_load(good)
    bad = tmp_path / "bad.txt"
    bad.write_text(HEADER + "gfx950 1 20 9000 3 2 1 3\n" + body)
    with pytest.raises(lib.SbtError):
        lib.autotune_load(bad)
    assert lib.autotune_count() == (1, 0)


def test_file_without_header_or_missing_is_refused(clean, tmp_path):
    lib = clean
    nohead = tmp_path / "nohead.txt"
    nohead.write_text("gfx950 1 20 9000 3 1 2 3\n")
    with pytest.raises(lib.SbtError):
        lib.autotune_load(nohead)
    with pytest.raises(lib.SbtError):
        lib.autotune_load(tmp_path / "absent.txt")
    with pytest.raises(lib.SbtError):
        lib.autotune_save(tmp_path / "no_such_dir" / "out.txt")
    assert lib.autotune_count() == (0, 0)


def test_modes_are_checked(clean):
    lib = clean
    with pytest.raises(lib.SbtError):
        lib.autotune_set(4)
    with pytest.raises(lib.SbtError):
        lib.autotune_set(-1)
    with pytest.raises(lib.SbtError):
        lib.autotune_set(lib.SBT_TUNE_FIXED, 8)
    for m in (lib.SBT_TUNE_OFF, lib.SBT_TUNE_CACHED, lib.SBT_TUNE_ON):
        lib.autotune_set(m)
    lib.autotune_set(lib.SBT_TUNE_FIXED, 2)
