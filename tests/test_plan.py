"""The autotuner's plan table and its file format (host logic, no device
work): storage and lookup, validation of entries, a save/load round trip,
rejection of corrupted files as a whole (the table is left unchanged), and
the TOPROP_PLAN_CACHE file read on first use (a corrupted cache ignored)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture
def capi():
    from paper_2411_18591_amd import _capi
    _capi.plan_clear()
    yield _capi
    _capi.plan_clear()


def test_set_get_clear(capi):
    assert capi.plan_get(2048, 2048, capi.TO_C64) is None
    capi.plan_set(2048, 2048, capi.TO_C64, 2, 64, 12.5)
    capi.plan_set(2048, 2048, capi.TO_C128, 0, 256)
    assert capi.plan_get(2048, 2048, capi.TO_C64) == {"col_variant": 2, "chunk_mb": 64, "row_fpb": 0, "us": 12.5}
    assert capi.plan_get(2048, 2048, capi.TO_C128)["col_variant"] == 0
    assert capi.plan_get(2048, 1024, capi.TO_C64) is None
    capi.plan_set(2048, 2048, capi.TO_C64, 1, 128)  # replaces
    assert capi.plan_get(2048, 2048, capi.TO_C64)["col_variant"] == 1
    capi.plan_clear()
    assert capi.plan_get(2048, 2048, capi.TO_C64) is None


@pytest.mark.parametrize("py,px,variant,chunk,us,fpb", [
    (2048, 2047, 1, 128, 0.0, 0), (4, 2048, 1, 128, 0.0, 0), (16384, 16, 1, 128, 0.0, 0),
    (2048, 2048, 5, 128, 0.0, 0), (2048, 2048, -1, 128, 0.0, 0), (2048, 2048, 1, 0, 0.0, 0),
    (2048, 2048, 1, 65537, 0.0, 0), (2048, 2048, 1, 64, -1.0, 0), (2048, 2048, 1, 64, float("nan"), 0),
    (2048, 2048, 1, 64, 1.0, -1), (2048, 2048, 1, 64, 1.0, 9),
])
def test_set_rejects_invalid_entries(capi, py, px, variant, chunk, us, fpb):
    with pytest.raises(capi.ToError) as e:
        capi.plan_set(py, px, capi.TO_C64, variant, chunk, us, fpb)
    assert e.value.status == capi.TO_E_INVAL
    assert capi.plan_get(2048, 2048, capi.TO_C64) is None


def test_save_load_round_trip(capi, tmp_path):
    entries = [(8, 8, capi.TO_C64, 0, 1, 0.5, 0), (8192, 16, capi.TO_C128, 2, 65536, 1e6, 8),
               (2048, 2048, capi.TO_C64, 1, 128, 144.667, 2)]
    for py, px, dt, v, c, us, fpb in entries:
        capi.plan_set(py, px, dt, v, c, us, fpb)
    path = str(tmp_path / "plans.txt")
    capi.plan_save(path)
    text = open(path).read().splitlines()
    assert text[0] == "toprop-plan 2"
    assert not os.path.exists(path + ".tmp")
    capi.plan_clear()
    capi.plan_load(path)
    for py, px, dt, v, c, us, fpb in entries:
        p = capi.plan_get(py, px, dt)
        assert (p["col_variant"], p["chunk_mb"], p["row_fpb"]) == (v, c, fpb)
        assert abs(p["us"] - us) <= 1e-3


def test_version_1_files_still_load(capi, tmp_path):
    """A file of the first format (no row_fpb field) loads with row_fpb 0."""
    path = tmp_path / "v1.txt"
    path.write_text("toprop-plan 1\nc64 2048 2048 1 128 144.5\n")
    capi.plan_load(str(path))
    assert capi.plan_get(2048, 2048, capi.TO_C64) == {"col_variant": 1, "chunk_mb": 128, "row_fpb": 0, "us": 144.5}


GOOD = "toprop-plan 2\n# comment\nc64 2048 2048 1 128 0 144.5\n"
CORRUPT = {
    "empty": "",
    "bad header": "toprop-plan 3\nc64 2048 2048 1 128 0 1\n",
    "no header": "c64 2048 2048 1 128 0 1\n",
    "bad dtype": "toprop-plan 2\nc32 2048 2048 1 128 0 1\n",
    "short line": "toprop-plan 2\nc64 2048 2048 1 128 1\n",
    "long line": "toprop-plan 2\nc64 2048 2048 1 128 0 1 7\n",
    "v1 long line": "toprop-plan 1\nc64 2048 2048 1 128 0 1\n",
    "non-integer": "toprop-plan 2\nc64 2048 2048 1.5 128 0 1\n",
    "trailing junk": "toprop-plan 2\nc64 2048 2048x 1 128 0 1\n",
    "not pow2": "toprop-plan 2\nc64 2048 3000 1 128 0 1\n",
    "variant range": "toprop-plan 2\nc64 2048 2048 7 128 0 1\n",
    "chunk range": "toprop-plan 2\nc64 2048 2048 1 0 0 1\n",
    "row range": "toprop-plan 2\nc64 2048 2048 1 128 9 1\n",
    "negative time": "toprop-plan 2\nc64 2048 2048 1 128 0 -3\n",
    "inf time": "toprop-plan 2\nc64 2048 2048 1 128 0 inf\n",
    "duplicate": "toprop-plan 2\nc64 2048 2048 1 128 0 1\nc64 2048 2048 2 64 0 1\n",
    "binary": "toprop-plan 2\n\x00\x01\x02\n",
}


@pytest.mark.parametrize("name", sorted(CORRUPT))
def test_corrupted_file_rejected_whole(capi, tmp_path, name):
    capi.plan_set(1024, 1024, capi.TO_C64, 2, 32, 9.0)
    path = tmp_path / "bad.txt"
    # a valid record first, so a partial merge would be visible
    text = CORRUPT[name]
    for head, rec in (("toprop-plan 2\n", "c128 512 512 0 64 0 3\n"), ("toprop-plan 1\n", "c128 512 512 0 64 3\n")):
        if text.startswith(head):
            text = head + rec + text[len(head):]
    path.write_bytes(text.encode("latin-1"))
    with pytest.raises(capi.ToError) as e:
        capi.plan_load(str(path))
    assert e.value.status == capi.TO_E_INVAL
    assert capi.plan_get(512, 512, capi.TO_C128) is None
    assert capi.plan_get(1024, 1024, capi.TO_C64) == {"col_variant": 2, "chunk_mb": 32, "row_fpb": 0, "us": 9.0}


def test_missing_file_rejected(capi, tmp_path):
    with pytest.raises(capi.ToError):
        capi.plan_load(str(tmp_path / "absent.txt"))


def _cache_probe(cache_path: str) -> str:
    code = ("from paper_2411_18591_amd import _capi as c; "
            "p = c.plan_get(2048, 2048, c.TO_C64); print(p and p['col_variant'])")
    env = dict(os.environ, TOPROP_PLAN_CACHE=cache_path)
    return subprocess.check_output([sys.executable, "-c", code], cwd=ROOT, env=env, text=True).strip()


def test_env_cache_loaded_on_first_use(tmp_path):
    path = tmp_path / "cache.txt"
    path.write_text(GOOD)
    assert _cache_probe(str(path)) == "1"


def test_env_cache_corrupted_is_ignored(tmp_path):
    path = tmp_path / "cache.txt"
    path.write_text(GOOD + "c64 4096 4096 9 1 1\n")
    assert _cache_probe(str(path)) == "None"
    assert _cache_probe(str(tmp_path / "missing.txt")) == "None"
