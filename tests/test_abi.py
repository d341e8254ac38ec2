"""The C-ABI library loads and exports every entry point include/rdos.h
declares, and the Python binding names the same calls (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "rdos.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rdos_[a-z_]+)\s*\(", src)))


def test_header_declares_the_expected_calls():
    names = _declared()
    for must in ["rdos_create", "rdos_set_mesh", "rdos_add_species", "rdos_add_reaction", "rdos_finalize",
                 "rdos_set_counts", "rdos_get_counts", "rdos_step", "rdos_run_until", "rdos_destroy",
                 "rdos_engine_create", "rdos_engine_submit", "rdos_engine_poll", "rdos_engine_drain"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_1512_03126_amd as P

    L = ctypes.CDLL(P.LIB_PATH)
    for name in _declared():
        assert hasattr(L, name), name
    assert sorted(_declared()) == sorted(P.EXPORTED)
    P.lib()  # argtypes for every symbol resolve


def test_library_has_no_host_fallback():
    """Without a usable device the library refuses to create a simulation."""
    import paper_1512_03126_amd as P

    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:
        has_gpu = False
    if has_gpu:
        pytest.skip("a GPU is present")
    with pytest.raises(P.RdosError) as ei:
        P.rdos_create(0, 1, 1)
    assert ei.value.status == -3


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    import paper_1512_03126_amd as P

    monkeypatch.setattr(P, "_lib", None)
    monkeypatch.setattr(P, "LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(ImportError):
        P.lib()


def test_kernels_are_built_for_gfx950_without_fast_math():
    flags = open(os.path.join(ROOT, "paper_1512_03126_amd", "build.py")).read()
    assert "-ffp-contract=off" in flags and "gfx950" in flags and "-packed-fp32-ops" in flags
    assert "ffast-math" not in flags.replace("-fno-fast-math", "")


def test_atomic_probe_rejects_bad_sizes_before_touching_a_device():
    import paper_1512_03126_amd as P

    L = P.lib()
    r = ctypes.c_double(-1.0)
    assert L.rdos_atomic_probe(0, 1 << 20, 0, 1, ctypes.byref(r)) == -1        # no atomics
    assert L.rdos_atomic_probe(0, 1 << 20, 1000, 0, ctypes.byref(r)) == -1     # no timed launch
    assert L.rdos_atomic_probe(0, 2, 1000, 1, ctypes.byref(r)) == -1           # no int32 slot
    assert L.rdos_atomic_probe(0, 16 << 30, 1000, 1, ctypes.byref(r)) == -1    # 2^32 slots
    assert L.rdos_atomic_probe(0, 1 << 20, 1000, 1, None) == -1
    assert r.value == -1.0
