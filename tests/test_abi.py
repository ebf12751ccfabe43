"""The C-ABI library loads and exports every entry point its header declares
(no GPU work is launched here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "codag.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(codag_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = _declared()
    for n in ("codag_decompress", "codag_decompress_ex", "codag_get_error",
              "codag_status_string", "codag_shutdown"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2307_03760_amd as codag
    if not os.path.exists(codag.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(codag.LIB_PATH)
    for n in _declared():
        assert hasattr(lib, n), n


def test_status_strings_and_argument_checks():
    """Host-side validation paths that return before touching a device."""
    import paper_2307_03760_amd as codag
    if not os.path.exists(codag.LIB_PATH):
        pytest.skip("library not built")
    lib = codag.lib()
    assert lib.codag_status_string(0) == b"ok"
    assert lib.codag_status_string(-3) == b"corrupt stream"
    assert lib.codag_status_string(12345) == b"unknown status"
    # unknown codec, NULL pointers with chunks: rejected before any HIP call
    assert lib.codag_decompress(7, None, None, None, None, 1, None) == codag.E_INVALID_ARGUMENT
    assert lib.codag_decompress(1, None, None, None, None, 5, None) == codag.E_INVALID_ARGUMENT
    # zero chunks is a no-op even with NULL buffers
    assert lib.codag_decompress(3, None, None, None, None, 0, None) == codag.OK


def test_binding_has_no_cpu_fallback(monkeypatch, tmp_path):
    import paper_2307_03760_amd as codag
    monkeypatch.setattr(codag, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(codag, "_lib", None)
    with pytest.raises(ImportError):
        codag.lib()


def test_autotune_cache_text_round_trip():
    """The autotune cache's text form is checked and merged on the host."""
    import paper_2307_03760_amd as codag
    if not os.path.exists(codag.LIB_PATH):
        pytest.skip("library not built")
    codag.autotune_cache_clear()
    assert codag.autotune_cache_save() == ""
    good = ("gfx950 cus=256 mix=3,3,2,0,0,0 out=2^16 n=2^14 order=0|8|10|2|1|12|0|41.500000\n"
            "gfx950 cus=256 mix=0,0,0,8,0,0 out=2^16 n=2^14 order=2|4|9|1|4|16|2|40.250000\n")
    codag.autotune_cache_load(good)
    assert codag.autotune_cache_save() == good
    # a key already cached is replaced, not duplicated
    codag.autotune_cache_load(good.splitlines(True)[0].replace("|41.500000", "|39.000000"))
    text = codag.autotune_cache_save()
    assert text.count("\n") == 2 and "|39.000000" in text
    bad = [
        "no separators\n",
        "|8|10|2|1|12|0|1.0\n",                       # empty key
        "k|8|10|2|1|12|0\n",                          # a field missing
        "k|8|11|2|1|12|0|1.0\n",                      # table bits the launch rejects
        "k|5|9|2|1|12|0|1.0\n",                       # window size the launch rejects
        "k|8|9|3|1|12|0|1.0\n",                       # waves per workgroup
        "k|8|9|2|1|12|9|1.0\n",                       # unknown order
        "k|8|9|2|1|12|0|1.0 trailing\n",
        "k|8|9|2|1|12|0|1.0",                         # no newline
    ]
    for line in bad:
        before = codag.autotune_cache_save()
        with pytest.raises(codag.CodagError):
            codag.autotune_cache_load(good.splitlines(True)[1] + line)
        assert codag.autotune_cache_save() == before, line
    codag.autotune_cache_clear()
    assert codag.autotune_cache_save() == ""
