"""The C ABI library loads and exports every function that include/vcheck.h declares;
argument validation that needs no GPU behaves as documented."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vcheck.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(vc_[a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["vc_ctx_create", "vc_ctx_destroy", "vc_last_error", "vc_trace_load", "vc_trace_set_arrays",
                     "vc_translate", "vc_check", "vc_sync", "vc_read_events", "vc_read_event_status",
                     "vc_read_violations", "vc_read_final_status", "vc_trace_free", "vc_batch_check",
                     "vc_server_create", "vc_stream_open", "vc_stream_submit", "vc_poll", "vc_stream_close"]:
        assert required in names, required


def test_library_exports_every_declared_symbol():
    from paper_1910_11110_amd import vcheck as V
    lib = V.lib()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"
    # exported names come from the built object itself
    so = C.CDLL(V.LIB_PATH)
    for n in declared_functions():
        getattr(so, n)


def test_binding_declares_every_signature():
    """Every function of the header has its argument and result types declared in the
    binding (an undeclared one would pass 64-bit arguments as C ints)."""
    from paper_1910_11110_amd import vcheck as V
    lib = V.lib()
    missing = [n for n in declared_functions() if getattr(lib, n).argtypes is None]
    assert not missing, f"no argtypes: {missing}"


def test_null_arguments_rejected_without_gpu():
    from paper_1910_11110_amd import vcheck as V
    L = V.lib()
    out = C.c_void_p()
    assert L.vc_trace_load(None, None, 0, 1, None, 0, C.byref(out)) == V.VC_EINVAL
    assert b"NULL" in L.vc_last_error()
    assert L.vc_check(None) == V.VC_EINVAL
    assert L.vc_sync(None) == V.VC_EINVAL
    assert L.vc_poll(None, None, 0, None) == V.VC_EINVAL


def test_context_on_machine_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_1910_11110_amd import vcheck as V
    with pytest.raises(V.VCError) as ex:
        V.Context(0)
    assert ex.value.code in (V.VC_EDEVICE, V.VC_EINVAL)


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_1910_11110_amd import vcheck as V
    monkeypatch.setattr(V, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(V, "_lib", None)
    with pytest.raises(ImportError):
        V.lib()
