"""Host logic of the serving scheduler (serve_core.h) against a fake executor.

Compiled with g++ at test time from the library's own scheduler header; no
GPU is involved.  Covers admission by byte budget in arrival order, tile
accounting, mixed-frame launches, queue-full and oversize errors, and launch
failures that fail exactly the requests whose tiles they carried."""
import ctypes
import os
import subprocess
import time

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "serve_harness.cpp")
INC = os.path.join(ROOT, "paper_2405_19056_amd", "csrc")
S_OK, S_INVAL, S_DEVICE, S_AGAIN, S_BUSY = 0, -1, -3, -5, -6


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    out = tmp_path_factory.mktemp("serve") / "libserve_harness.so"
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-shared", "-fPIC", "-pthread",
                    "-fsanitize=undefined", f"-I{INC}", SRC, "-o", str(out)], check=True)
    L = ctypes.CDLL(str(out))
    L.h_create.restype = ctypes.c_void_p
    L.h_create.argtypes = [ctypes.c_ulonglong, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                           ctypes.c_int, ctypes.c_int]
    for n in ("h_submit", "h_poll", "h_drain", "h_forget", "h_tiles"):
        getattr(L, n).restype = ctypes.c_int
    L.h_submit.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                           ctypes.POINTER(ctypes.c_ulonglong)]
    L.h_poll.argtypes = [ctypes.c_void_p, ctypes.c_ulonglong, ctypes.POINTER(ctypes.c_int),
                         ctypes.POINTER(ctypes.c_double)]
    L.h_drain.argtypes = [ctypes.c_void_p]
    L.h_forget.argtypes = [ctypes.c_void_p, ctypes.c_ulonglong]
    L.h_hold.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.h_fail.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
    L.h_max_inflight_bytes.restype = ctypes.c_ulonglong
    L.h_max_inflight_bytes.argtypes = [ctypes.c_void_p]
    L.h_launches.restype = ctypes.c_longlong
    L.h_launches.argtypes = [ctypes.c_void_p]
    L.h_mixed.restype = ctypes.c_longlong
    L.h_mixed.argtypes = [ctypes.c_void_p]
    L.h_frame_bytes.restype = ctypes.c_ulonglong
    L.h_frame_bytes.argtypes = [ctypes.c_int, ctypes.c_int]
    L.h_tiles.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.c_int]
    L.h_destroy.argtypes = [ctypes.c_void_p]
    return L


def submit(L, h, hw, k, n=1):
    t = ctypes.c_ulonglong()
    rc = L.h_submit(h, hw, k, n, ctypes.byref(t))
    return rc, t.value


def poll(L, h, t):
    d = ctypes.c_int()
    tm = (ctypes.c_double * 4)()
    rc = L.h_poll(h, t, ctypes.byref(d), tm)
    return rc, d.value, list(tm)


def tiles(L, h):
    buf = (ctypes.c_int * 200000)()
    n = L.h_tiles(h, buf, 100000)
    return [(buf[2 * i], buf[2 * i + 1]) for i in range(min(n, 100000))]


def test_every_tile_of_every_frame_runs_once(lib):
    h = lib.h_create(1 << 40, 1000, 64, 2, 8192, 0)
    sizes = [(256 * 256, 4), (360 * 640, 2), (37 * 53, 8), (1, 0), (512 * 512, 8)]
    tickets = [submit(lib, h, hw, k)[1] for hw, k in sizes]
    assert lib.h_drain(h) == S_OK
    for t in tickets:
        rc, done, tm = poll(lib, h, t)
        assert rc == S_OK and done == 1
        assert tm[0] <= tm[1] <= tm[2] <= tm[3]
    seen = tiles(lib, h)
    for hw, k in sizes:
        q0s = sorted(q for fhw, q in seen if fhw == hw)
        assert q0s == list(range(0, hw, 256))
    lib.h_destroy(h)


def test_budget_admits_in_arrival_order_and_is_never_exceeded(lib):
    fb = lib.h_frame_bytes(512 * 512, 8)
    h = lib.h_create(int(fb * 1.5), 1000, 128, 2, 8192, 0)   # room for one frame at a time
    ts = [submit(lib, h, 512 * 512, 8)[1] for _ in range(6)]
    assert lib.h_drain(h) == S_OK
    admits = [poll(lib, h, t)[2][1] for t in ts]
    dones = [poll(lib, h, t)[2][3] for t in ts]
    assert admits == sorted(admits)
    for i in range(1, len(ts)):              # next admitted only after the previous finished
        assert admits[i] >= dones[i - 1]
    assert lib.h_max_inflight_bytes(h) <= fb * 1.5
    lib.h_destroy(h)


def test_small_frames_share_launches(lib):
    h = lib.h_create(1 << 40, 1000, 1024, 2, 8192, 1)         # hold: nothing completes
    ts = [submit(lib, h, 64 * 64, 2)[1] for _ in range(40)]
    time.sleep(0.05)
    lib.h_hold(h, 0)
    assert lib.h_drain(h) == S_OK
    assert lib.h_mixed(h) >= 1
    assert all(poll(lib, h, t)[1] == 1 for t in ts)
    lib.h_destroy(h)


def test_oversize_frame_and_full_queue(lib):
    fb = lib.h_frame_bytes(256 * 256, 4)
    h = lib.h_create(fb, 3, 64, 1, 8192, 1)                   # hold keeps work in flight
    rc, _ = submit(lib, h, 512 * 512, 8)
    assert rc == S_INVAL                                      # larger than the whole budget
    rcs = [submit(lib, h, 256 * 256, 4)[0] for _ in range(8)]
    assert rcs[0] == S_OK and S_BUSY in rcs
    lib.h_hold(h, 0)
    assert lib.h_drain(h) == S_OK
    lib.h_destroy(h)


def test_a_failed_launch_fails_only_its_requests(lib):
    h = lib.h_create(1 << 40, 1000, 256, 1, 8192, 1)
    lib.h_fail(h, 0, 1)                                       # first completion reports failure
    t_bad = submit(lib, h, 256 * 256, 4)[1]                   # 256 tiles = one launch
    t_ok = [submit(lib, h, 128 * 128, 2)[1] for _ in range(3)]
    time.sleep(0.02)
    lib.h_hold(h, 0)
    assert lib.h_drain(h) == S_DEVICE
    rc, done, _ = poll(lib, h, t_bad)
    assert rc == S_DEVICE and done == 1
    for t in t_ok:
        assert poll(lib, h, t)[:2] == (S_OK, 1)
    assert lib.h_drain(h) == S_OK                             # failure reported once
    lib.h_destroy(h)


def test_launch_error_and_ticket_bookkeeping(lib):
    h = lib.h_create(1 << 40, 1000, 64, 2, 8192, 0)
    lib.h_fail(h, 1, 0)                                       # first launch cannot be issued
    t1 = submit(lib, h, 64 * 64, 1)[1]
    lib.h_drain(h)
    assert poll(lib, h, t1)[0] == S_DEVICE
    t2 = submit(lib, h, 64 * 64, 1)[1]
    assert lib.h_drain(h) == S_OK
    assert poll(lib, h, t2)[:2] == (S_OK, 1)
    assert lib.h_forget(h, t2) == S_OK
    assert poll(lib, h, t2)[0] == S_INVAL
    assert lib.h_forget(h, 123456) == S_INVAL
    lib.h_destroy(h)


def test_multi_frame_request(lib):
    h = lib.h_create(1 << 40, 1000, 100, 2, 8192, 0)
    rc, t = submit(lib, h, 300, 3, n=5)
    assert rc == S_OK
    assert lib.h_drain(h) == S_OK
    assert poll(lib, h, t)[:2] == (S_OK, 1)
    seen = tiles(lib, h)
    assert len([1 for hw, q in seen if hw == 300]) == 5 * 2
    lib.h_destroy(h)
