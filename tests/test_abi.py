"""The C-ABI library loads on a machine without a GPU, exports every entry
point that include/nyxrt.h declares, and rejects bad descriptors in its host
code (no compute call is made here)."""
import ctypes as C
import os
import re

import pytest

import paper_2512_12466_amd as nrt

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "nyxrt.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nrt_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    lib = C.CDLL(nrt.LIB_PATH)
    names = _declared()
    assert len(names) >= 15
    missing = [s for s in names if not hasattr(lib, s)]
    assert not missing, missing


def test_binding_covers_every_entry_point():
    nrt.load()
    for s in _declared():
        assert getattr(nrt.load(), s).argtypes is not None or s in ("nrt_status_str",), s


def test_status_strings_and_workspace_plan():
    L = nrt.load()
    assert L.nrt_status_str(0) == b"ok"
    assert L.nrt_status_str(4) == b"queue overflow"
    d = nrt.make_desc(32, 1e20, l_max=7)
    b64 = nrt.workspace_bytes(d, 100, 1 << 16)
    dm = nrt.make_desc(32, 1e20, l_max=7, precision=nrt.MIXED)
    b32 = nrt.workspace_bytes(dm, 100, 1 << 16)
    cells = 32 ** 3
    # both paths hold the absorber as one FP64 array
    assert b32 == b64 > cells * 24
    # queues: levels 1..l_max, 24 bytes per slot; direction table: 24 bytes
    # per pixel of levels 0..min(l_max, 11)
    d2 = nrt.make_desc(32, 1e20, l_max=8)
    assert nrt.workspace_bytes(d2, 100, 1 << 16) - b64 == 24 * (1 << 16) + 24 * 12 * 4 ** 8
    d11, d12 = nrt.make_desc(32, 1e20, l_max=11), nrt.make_desc(32, 1e20, l_max=12)
    assert (nrt.workspace_bytes(d12, 100, 1 << 16) - nrt.workspace_bytes(d11, 100, 1 << 16)
            == 24 * (1 << 16))
    # polychromatic table: node moments (3 x 4097 FP64, padded to 256 B) and
    # 4096 interval records of 64 B (FP64) + 32 B (FP32), padded to 256 B
    dp = nrt.make_desc(32, 1e20, l_max=7, spectrum=nrt.SPEC_BLACKBODY, spec_param=5e4)
    nodes = (3 * 4097 * 8 + 255) // 256 * 256
    assert nrt.workspace_bytes(dp, 100, 1 << 16) - b64 == nodes + 4096 * 96


@pytest.mark.parametrize("field,value", [("n", 0), ("h_cm", -1.0), ("l_max", 15),
                                         ("tau_max", 0.0), ("corr", 9), ("precision", 2),
                                         ("n_min_ray", -1.0), ("periodic", 3),
                                         ("spectrum", 3), ("spec_param", 1e8),
                                         ("spec_param", 0.0)])
def test_bad_descriptor_rejected(field, value):
    d = nrt.make_desc(16, 1e20)
    if field == "spec_param":  # a blackbody out of [1e3, 1e7] K
        d.spectrum = nrt.SPEC_BLACKBODY
    setattr(d, field, value)
    with pytest.raises(nrt.NyxRTError) as e:
        nrt.workspace_bytes(d, 10, 1 << 16)
    assert e.value.status == 1


def test_bad_capacity_rejected():
    d = nrt.make_desc(16, 1e20)
    with pytest.raises(nrt.NyxRTError):
        nrt.workspace_bytes(d, 10, 100)
    with pytest.raises(nrt.NyxRTError):
        nrt.workspace_bytes(d, -1, 1 << 16)


def test_init_rejects_null_and_small_workspace():
    L = nrt.load()
    d = nrt.make_desc(16, 1e20)
    ctx = C.c_void_p()
    st = L.nrt_init_grid(C.byref(ctx), C.byref(d), None, None, 10, 1 << 16, None, 0, None)
    assert st == 1 and not ctx.value
    assert b"NULL" in L.nrt_last_error(None)
    st = L.nrt_init_grid(C.byref(ctx), C.byref(d), 256, 256, 10, 1 << 16, 256, 1024, None)
    assert st == 3 and not ctx.value  # workspace too small: nothing touched


def test_destroy_null_is_noop():
    assert nrt.load().nrt_destroy(None) == 0
