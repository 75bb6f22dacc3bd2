"""The C ABI: every symbol include/aeraunfold.h declares is exported by the
built library and bound in Python, and argument validation that needs no
device works on the CPU.  No compute calls."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "aeraunfold.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w]+\s*\*?\s*(au_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_1507_07733_amd import api
    if not os.path.exists(api.LIB_PATH):
        from paper_1507_07733_amd import build
        build.build(verbose=False)
    return api.lib()


def test_header_declares_the_path():
    names = declared()
    for need in ("au_load_pattern_table", "au_unfold_event", "au_unfold_direction_scan",
                 "au_plan_create", "au_plan_run", "au_last_error"):
        assert need in names


def test_every_declared_symbol_is_exported_and_bound(lib):
    from paper_1507_07733_amd import api
    names = declared()
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(api.declared_symbols()) == names


def test_validation_without_device(lib):
    from paper_1507_07733_amd import api
    ev = api.make_event(10, 2048)
    assert api.band_bins(ev) == (308, 512)
    assert api.band_bins(api.make_event(3, 4096)) == (615, 1024)
    n = C.c_uint64()
    assert lib.au_workspace_bytes(None, C.byref(ev), 1, C.byref(n)) == api.AU_EINVAL
    assert b"table" in lib.au_last_error()
    assert lib.au_plan_create(None, None, None) == api.AU_EINVAL
    assert lib.au_unfold_event(None, C.byref(ev), None, 0.0, 0.0, None, None, 0, None, None) == api.AU_EINVAL
    assert lib.au_reconstruct_workspace_bytes(None, C.byref(ev), 4, C.byref(n)) == api.AU_EINVAL
    assert lib.au_reconstruct(None, C.byref(ev), None, None, 4, None, None, None, None, None, None, None, 0,
                              None) == api.AU_EINVAL
    assert lib.au_direction_fit_workspace_bytes(None, C.byref(ev), 4, 1, 3, C.byref(n)) == api.AU_EINVAL
    assert lib.au_direction_fit(None, C.byref(ev), None, None, 4, None, 1, 3, 1.0, 1.0, None, None, None, None,
                                None, None, 0, None) == api.AU_EINVAL
    assert lib.au_pattern_response_quantized(None, C.byref(ev), 1, None, 8, None, None) == api.AU_EINVAL
    assert lib.au_reconstruct_batch(None, C.byref(ev), 0, None, None, None, None, 4, None, None, None, None, None,
                                    0, None) == api.AU_EINVAL
    assert lib.au_free_pattern_table(None) == api.AU_OK


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_1507_07733_amd import api
    monkeypatch.setattr(api, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(api, "_lib", None)
    with pytest.raises(RuntimeError):
        api.lib()
