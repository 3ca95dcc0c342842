"""Host-only checks of the C ABI: the library loads, exports every symbol the
headers declare, and rejects bad arguments before anything is launched (every
call below fails validation on the host, so no GPU is touched)."""
import ctypes as ct
import os
import re

import pytest

from paper_1801_04720_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    inc = os.path.join(ROOT, "include")
    for f in sorted(os.listdir(inc)):
        if not f.endswith(".h"):
            continue
        text = open(os.path.join(inc, f)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"\b(sf_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libsf.so is not built (run __graft_entry__.build())")
    return _lib.lib()


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert len(names) >= 8
    for n in names:
        assert hasattr(L, n), n
    # The Python binding declares a signature for each of them.
    missing = [n for n in names if n not in _lib.SIGNATURES]
    assert not missing, missing


def test_abi_version(L):
    assert L.sf_abi_version() == 1


FAKE = ct.c_void_p(0x1000)  # never dereferenced: validation fails first


def expect(status, code, fragment):
    assert status == code, (status, _lib.lib().sf_last_error())
    assert fragment in _lib.lib().sf_last_error().decode()


def test_census_validation(L):
    expect(L.sf_census(None, 4, 4, 4, FAKE, None), 1, "NULL")
    expect(L.sf_census(FAKE, 0, 4, 4, FAKE, None), 1, "positive")
    expect(L.sf_census(FAKE, 4, 4, 3, FAKE, None), 1, "pitch")


def test_cost_validation(L):
    expect(L.sf_cost(FAKE, None, 4, 4, 8, 0, FAKE, None), 1, "NULL")
    expect(L.sf_cost(FAKE, FAKE, 4, 4, 0, 0, FAKE, None), 1, "D must")
    expect(L.sf_cost(FAKE, FAKE, 4, 4, 257, 0, FAKE, None), 1, "D must")


def test_aggregate_validation(L):
    ws = 1 << 20
    expect(L.sf_sgm_aggregate(FAKE, 4, 4, 32, 20, 10, 255, FAKE, FAKE, ws, None), 1, "P1 <= P2")
    expect(L.sf_sgm_aggregate(FAKE, 4, 4, 32, 10, 9000, 255, FAKE, FAKE, ws, None), 1, "8000")
    expect(L.sf_sgm_aggregate(FAKE, 4, 4, 32, 10, 120, 0, FAKE, FAKE, ws, None), 1, "path_mask")
    expect(L.sf_sgm_aggregate(FAKE, 4, 4, 32, 10, 120, 256, FAKE, FAKE, ws, None), 1, "path_mask")
    expect(L.sf_sgm_aggregate(FAKE, 4, 4, 48, 10, 120, 255, FAKE, FAKE, ws, None), 2, "multiple of 32")
    expect(L.sf_sgm_aggregate(FAKE, 4, 4, 32, 10, 120, 255, FAKE, FAKE, 100, None), 4, "workspace")
    expect(L.sf_sgm_aggregate(None, 4, 4, 32, 10, 120, 255, FAKE, FAKE, ws, None), 1, "NULL")
    assert L.sf_sgm_workspace_bytes(375, 1242, 128) == 8 * 375 * 1242 * 128
    assert L.sf_sgm_workspace_bytes(0, 4, 4) == 0


def test_wta_validation(L):
    args = dict(Sl=FAKE, Sr=None, img=None, pitch=4, H=4, W=4, D=32, P2=120, tol=1, wl=FAKE, wr=None,
                disp=FAKE, valid=FAKE, feat=None)

    def call(**kw):
        a = dict(args, **kw)
        return L.sf_wta_lr(a["Sl"], a["Sr"], a["img"], a["pitch"], a["H"], a["W"], a["D"], a["P2"],
                           a["tol"], a["wl"], a["wr"], a["disp"], a["valid"], a["feat"], None)

    expect(call(Sl=None), 1, "NULL")
    expect(call(Sr=FAKE), 1, "wta_right")
    expect(call(feat=FAKE), 1, "img_left")
    expect(call(tol=-1), 1, "lr_tol")
    expect(call(D=0), 1, "D must")


def test_combine_validation(L):
    cam = _lib.SfCamera(721.5, 0.54, 620.5, 187.0)
    expect(L.sf_combine(FAKE, FAKE, FAKE, FAKE, None, 4, 4, None, FAKE, FAKE, None, None, None), 1, "NULL")
    expect(L.sf_combine(FAKE, FAKE, FAKE, FAKE, FAKE, 4, 4, ct.byref(cam), FAKE, FAKE, None, None, None),
           1, "xyz0")
    bad = _lib.SfCamera(0.0, 0.54, 1.0, 1.0)
    expect(L.sf_combine(FAKE, FAKE, FAKE, FAKE, FAKE, 4, 4, ct.byref(bad), FAKE, FAKE, FAKE, FAKE, None),
           1, "focal")


def test_last_error_cleared_by_next_call(L):
    L.sf_census(None, 4, 4, 4, FAKE, None)
    assert L.sf_last_error() != b""
    L.sf_sgm_aggregate(FAKE, 4, 4, 32, 20, 10, 255, FAKE, FAKE, 0, None)
    assert b"P1" in L.sf_last_error()


def test_variant_validation(L):
    expect(L.sf_wta_right_diag(None, 4, 4, 8, FAKE, None), 1, "NULL")
    expect(L.sf_wta_right_diag(FAKE, 4, 4, 0, FAKE, None), 1, "D must")
    expect(L.sf_lr_check(FAKE, FAKE, FAKE, 4, 4, -1, FAKE, FAKE, None), 1, "lr_tol")
    expect(L.sf_lr_check(FAKE, None, FAKE, 4, 4, 1, FAKE, FAKE, None), 1, "NULL")
    expect(L.sf_median3x3(FAKE, None, 4, 4, FAKE, None), 1, "must not be the same")
    expect(L.sf_median3x3(FAKE, None, 0, 4, ct.c_void_p(0x2000), None), 1, "positive")
    plan = ct.c_void_p()
    # Diagonal search and learned mask exclude each other; the diagonal kernel keeps a row in LDS.
    expect(L.sf_frame_plan_create(64, 64, 32, 10, 120, 1, 4 | 2, None, ct.byref(plan)), 1, "exclude")
    expect(L.sf_frame_plan_create(64, 5000, 32, 10, 120, 1, 4, None, ct.byref(plan)), 2, "4096")
    expect(L.sf_frame_plan_create(64, 64, 32, 10, 120, 1, 64, None, ct.byref(plan)), 1, "unknown flags")


def test_aggregate_census_validation(L):
    ws = 1 << 20
    f = L.sf_sgm_aggregate_census
    expect(f(None, FAKE, 4, 4, 32, 0, 10, 120, 255, FAKE, FAKE, ws, None), 1, "NULL census")
    expect(f(FAKE, None, 4, 4, 32, 0, 10, 120, 255, FAKE, FAKE, ws, None), 1, "NULL census")
    expect(f(FAKE, FAKE, 4, 4, 32, 2, 10, 120, 255, FAKE, FAKE, ws, None), 1, "base_is_right")
    expect(f(FAKE, FAKE, 4, 4, 32, 0, 20, 10, 255, FAKE, FAKE, ws, None), 1, "P1 <= P2")
    expect(f(FAKE, FAKE, 4, 4, 32, 1, 10, 120, 0, FAKE, FAKE, ws, None), 1, "path_mask")
    expect(f(FAKE, FAKE, 4, 4, 48, 0, 10, 120, 255, FAKE, FAKE, ws, None), 2, "multiple of 32")
    expect(f(FAKE, FAKE, 4, 4, 32, 0, 10, 120, 255, FAKE, FAKE, 100, None), 4, "workspace")
    expect(f(FAKE, FAKE, 4, 4, 32, 0, 10, 120, 255, None, FAKE, ws, None), 1, "NULL")
    expect(f(FAKE, FAKE, 8192, 1024, 256, 0, 10, 120, 255, FAKE, FAKE, 1 << 40, None), 1, "2^31")


def test_volume_offset_limit(L):
    # H * W * D must stay below 2^31 for the 32-bit volume offsets of the kernels.
    plan = ct.c_void_p()
    expect(L.sf_frame_plan_create(8192, 1024, 256, 10, 120, 1, 0, None, ct.byref(plan)), 1, "2^31")
    expect(L.sf_sgm_aggregate(FAKE, 8192, 1024, 256, 10, 120, 255, FAKE, FAKE, 1 << 40, None), 1, "2^31")
    pair = _lib.SfPair(8192, 1024, 256, 1024, 0x1000, 0x1000, 0x1000, 0x1000, 0x1000)
    arr = (_lib.SfPair * 1)(pair)
    expect(L.sf_batch_plan_create(arr, 1, 10, 120, 1, None, 0, 0, ct.byref(plan)), 1, "2^31")


def test_tuning_packed_flag_validated(L):
    """packed must be 0 or 1; a plan refuses anything else before touching a device."""
    plan = ct.c_void_p()
    t = _lib.SfAggTuning(16, 8, 0, 0, 2)
    expect(L.sf_frame_plan_create(64, 64, 128, 10, 120, 1, 0, ct.byref(t), ct.byref(plan)), 1, "packed")


def test_frame_autotune_validation(L):
    t = _lib.SfAggTuning()
    ms = ct.c_float()
    expect(L.sf_frame_autotune(64, 64, 32, 10, 120, 1, 0, None, None, ct.byref(ms)), 1, "NULL best")
    # Invalid plans are refused before any buffer is allocated.
    expect(L.sf_frame_autotune(64, 64, 32, 10, 120, 1, 4 | 2, None, ct.byref(t), ct.byref(ms)), 1, "exclude")
    expect(L.sf_frame_autotune(8192, 1024, 256, 10, 120, 1, 0, None, ct.byref(t), ct.byref(ms)), 1, "2^31")


def test_network_and_judge_validation(L):
    expect(L.sf_lrnet_backward(FAKE, FAKE, None, 1, 4, 4, FAKE, FAKE, 1 << 30, None), 1, "NULL")
    expect(L.sf_lrnet_backward(FAKE, FAKE, FAKE, 0, 4, 4, FAKE, FAKE, 1 << 30, None), 1, "positive")
    expect(L.sf_lrnet_backward(FAKE, FAKE, FAKE, 1, 4, 4, FAKE, FAKE, 16, None), 4, "workspace")
    expect(L.sf_mask_agreement(FAKE, None, 10, FAKE, None), 1, "NULL")
    expect(L.sf_mask_agreement(FAKE, FAKE, 0, FAKE, None), 1, "positive")
    expect(L.sf_lrnet_forward_noalloc(None, FAKE, 1, 4, 4, FAKE, None), 1, "NULL")
    expect(L.sf_lrnet_forward_noalloc(FAKE, FAKE, 1, 0, 4, FAKE, None), 1, "positive")
    expect(L.sf_lrnet_forward_noalloc(FAKE, FAKE, 70000, 4, 4, FAKE, None), 1, "too large")


def test_checked_build_flags(L):
    import ctypes

    assert L.sf_debug_checked() == 0
    expect(L.sf_debug_check(None, 0), 1, "NULL")
    expect(L.sf_debug_selftest(-1, None), 1, "n must")
    path = os.path.join(ROOT, "paper_1801_04720_amd", "libsf_checked.so")
    if not os.path.exists(path):
        pytest.fail("libsf_checked.so is not built (run __graft_entry__.build())")
    C = ctypes.CDLL(path)
    assert C.sf_debug_checked() == 1
