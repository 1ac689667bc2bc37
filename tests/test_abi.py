"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function declared in include/*.h, and validates sizes on the host."""
import ctypes
import os
import re

import pytest

import paper_2210_11295_amd as bs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    inc = os.path.join(ROOT, "include")
    text = "\n".join(open(os.path.join(inc, f)).read()
                     for f in sorted(os.listdir(inc)) if f.endswith(".h"))
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", text)
    skip = {"defined", "if", "sizeof"}
    return sorted({n for n in names if n not in skip})


def test_header_lists_the_boundary():
    names = _declared_functions()
    for required in ("bsrht_plan", "bsrht_apply", "rsvd", "nystrom"):
        assert required in names
    assert set(names) == set(bs.EXPORTED_SYMBOLS)


def test_library_exports_every_declared_symbol():
    L = bs.lib()
    for name in _declared_functions():
        assert hasattr(L, name), name
    assert L.bsrht_version().decode().startswith("bsrht-gfx950")
    assert L.bsrht_strerror(0) == b"ok"
    assert L.bsrht_strerror(-1) == b"invalid argument"


@pytest.mark.parametrize("n,p,l,ok", [
    (4096, 4, 128, True), (1 << 20, 16, 512, True), (40, 40, 5, True), (64, 1, 64, True),
    (12, 1, 4, True),       # r = 12: partial SRHT, blocks padded to 16
    (300, 3, 20, True),     # r = 100 -> 128
    (16, 3, 4, False),      # p does not divide n
    (16, 2, 17, False),     # l > n
    (16, 2, 0, False),      # l = 0
    (0, 1, 1, False),
    (1 << 31, 1, 4, False),  # n too large for the int32 tables
])
def test_plan_bytes_validation(n, p, l, ok):
    nb = bs.bsrht_plan_bytes(n, p, l)
    if not ok:
        assert nb == 0
        return
    a256 = lambda x: (x + 255) // 256 * 256
    rp = 1 << (n // p - 1).bit_length()
    # R, D bits, Dt bits, then the two gather lane orders (l int32 each)
    expect = a256(a256(a256(4 * l) + 4 * ((p * rp + 31) // 32)) + 4 * p * ((l + 31) // 32))
    expect = a256(a256(expect + 4 * l) + 4 * l)
    assert nb == expect


def test_plan_rejects_bad_arguments_before_touching_the_device():
    L = bs.lib()
    h = ctypes.c_void_p()
    # null table memory, bad mode, without replacement with l > r: all EINVAL
    assert L.bsrht_plan(64, 4, 8, 1, 0, 0, None, 0, None, ctypes.byref(h)) == -1
    assert L.bsrht_plan(64, 4, 8, 1, 7, 0, ctypes.c_void_p(256), 4096, None, ctypes.byref(h)) == -1
    assert L.bsrht_plan(64, 4, 8, 1, 0, 9, ctypes.c_void_p(256), 4096, None, ctypes.byref(h)) == -1
    assert L.bsrht_plan(64, 4, 17, 1, 1, 0, ctypes.c_void_p(256), 4096, None, ctypes.byref(h)) == -1
    # table memory smaller than bsrht_plan_bytes: ENOMEM
    assert L.bsrht_plan(64, 4, 8, 1, 0, 0, ctypes.c_void_p(256), 16, None, ctypes.byref(h)) == -2
    assert L.bsrht_plan(64, 4, 8, 1, 0, 0, None, 0, None, None) == -1


def test_null_plan_is_rejected():
    L = bs.lib()
    assert L.bsrht_apply(None, None, 4, 4, None, 4, None, 0, None) == -1
    assert L.bsrht_apply_workspace(None, 4) == 0
    assert L.bsrht_plan_destroy(None) == 0
    assert L.bsrht_plan_info(None, None, None, None, None, None) == -1


def test_task_calls_reject_bad_arguments_on_the_host():
    """rsvd_start / nystrom_start / rsvd_single_view_start and the task calls check their arguments
    before any HIP call (no GPU needed): NULL plans and tasks are refused and
    the task handle is cleared."""
    L = bs.lib()
    h = ctypes.c_void_p(1)
    null = ctypes.c_void_p()
    assert L.rsvd_start(None, None, 1, 1, 1, None, None, None, None, None, 0, None,
                        ctypes.byref(h)) == -1
    assert h.value is None
    h = ctypes.c_void_p(1)
    assert L.nystrom_start(None, None, 1, 1, None, None, None, None, 0, None,
                           ctypes.byref(h)) == -1
    assert h.value is None
    assert L.nystrom_shifted_start(None, None, 1, 1, None, None, None, None, 0, None,
                                   None) == -1
    h = ctypes.c_void_p(1)
    assert L.rsvd_single_view_start(None, None, None, None, None, 1, 1, None, None, None, None,
                                    None, 0, None, ctypes.byref(h)) == -1
    assert h.value is None
    st = ctypes.c_int(7)
    assert L.bsrht_task_poll(null, ctypes.byref(st)) == -1 and st.value == 7
    assert L.bsrht_task_wait(null) == -1
    assert L.bsrht_task_destroy(null) == -1

