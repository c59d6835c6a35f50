"""CPU checks of the launch-shape tuner's table and cache file (host logic
only: no sketch is created, so nothing is timed)."""
import os

import pytest

from paper_1501_06561_amd import fdsketch as F


@pytest.fixture
def table(tmp_path):
    """An empty table on a cache file of its own; restores mode and path."""
    old_path, old_mode = F.tune_path(), F.tune_mode()
    path = str(tmp_path / "sub" / "tune.tsv")
    F.tune_path(path)
    F.tune_clear()
    yield path
    F.tune_clear()
    F.tune_path(old_path)
    F.tune_mode(old_mode)


def test_modes_round_trip(table):
    for m in ("off", "refresh", "on"):
        assert F.tune_mode(m) == m
    with pytest.raises(KeyError):
        F.tune_mode("sometimes")
    assert F.lib().fdsk_tune_set_mode(7) == -1


def test_set_lookup_and_clear(table):
    assert F.tune_lookup("gfx950/256|gram|p0|m224|d1024") is None
    F.tune_set("gfx950/256|gram|p0|m224|d1024", 4)
    F.tune_set("gfx950/256|rebuild|p3|m512|d4096", 64)
    assert F.tune_lookup("gfx950/256|gram|p0|m224|d1024") == 4
    assert F.tune_table()["gfx950/256|rebuild|p3|m512|d4096"] == (64, "set")
    F.tune_clear()
    assert F.tune_table() == {}


@pytest.mark.parametrize("key", ["", "a\tb", "a\nb"])
def test_bad_keys_are_rejected(table, key):
    with pytest.raises(F.FdskError):
        F.tune_set(key, 1)


def test_save_then_load_restores_the_table(table):
    F.tune_set("dev|bgram|p3|m224|d2048|n128", 1024)
    F.tune_set("dev|brebuild|p0|m64|d256|n16", 32)
    F.tune_save()                      # creates the missing directory
    assert os.path.exists(table)
    text = open(table).read().splitlines()
    assert text[0].startswith("#")
    assert "dev|bgram|p3|m224|d2048|n128\t1024\tset" in text
    F.tune_clear()
    F.tune_load()
    assert F.tune_lookup("dev|bgram|p3|m224|d2048|n128") == 1024
    assert F.tune_lookup("dev|brebuild|p0|m64|d256|n16") == 32


def test_load_skips_comments_and_malformed_lines(table):
    with open(os.path.join(os.path.dirname(os.path.dirname(table)), "hand.tsv"), "w") as f:
        f.write("# comment\n\nk1\t8\t1:10.5 8:4.0\nk2\tnot-a-number\n\tno-key\nk3\n k4\t-3\n")
        hand = f.name
    F.tune_load(hand)
    t = F.tune_table()
    assert t["k1"] == (8, "1:10.5 8:4.0")
    assert t[" k4"] == (-3, "")
    assert "k2" not in t and "k3" not in t and len(t) == 2


def test_load_of_a_missing_file_fails_and_keeps_the_table(table):
    F.tune_set("k", 2)
    with pytest.raises(F.FdskError):
        F.tune_load(table + ".missing")
    assert F.tune_lookup("k") == 2


def test_save_without_a_path_fails(table):
    F.tune_path("")
    with pytest.raises(F.FdskError):
        F.tune_save()


def test_dump_truncates_to_the_buffer(table):
    import ctypes
    F.tune_set("abcdef", 123)
    L = F.lib()
    n = L.fdsk_tune_dump(None, 0)
    assert n == len("abcdef\t123\tset\n")
    buf = ctypes.create_string_buffer(5)
    assert L.fdsk_tune_dump(buf, 5) == n
    assert buf.value == b"abcd"
