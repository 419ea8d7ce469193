"""CPU tests of the serving core (admission under the memory cap, FIFO order,
continuous batching over several slots, queue limits, failure propagation,
ticket lifetime) with a fake executor, plus a ThreadSanitizer stress run of
the same core with concurrent clients."""
import ctypes as C
import os
import subprocess
import time

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = [os.path.join(ROOT, "tests", "serve_core_shim.cpp"),
       os.path.join(ROOT, "paper_1402_2020_amd", "csrc", "bsm_serve_core.cpp")]
OK, EAGAIN, ETOOBIG, ENOTFOUND = 0, -4, -5, -6


@pytest.fixture(scope="module")
def shim(tmp_path_factory):
    out = tmp_path_factory.mktemp("shim") / "libshim.so"
    subprocess.run(["g++", "-std=c++17", "-O2", "-fPIC", "-shared", "-pthread", *SRC, "-o",
                    str(out)], check=True)
    lib = C.CDLL(str(out))
    vp, sz, u64p = C.c_void_p, C.c_size_t, C.POINTER(C.c_uint64)
    lib.shim_create.argtypes = [sz, C.c_int, C.c_int, C.c_double, C.c_int]
    lib.shim_create.restype = vp
    lib.shim_destroy.argtypes = [vp]
    lib.shim_configure.argtypes = [vp, sz, C.c_int, C.c_int]
    lib.shim_submit.argtypes = [vp, vp, vp, C.c_int, C.c_int, C.c_int, vp, sz, u64p]
    lib.shim_poll.argtypes = [vp, C.c_uint64, C.POINTER(C.c_int32), C.POINTER(C.c_double)]
    lib.shim_drain.argtypes = [vp]
    lib.shim_fail.argtypes = [vp, C.c_int, C.c_int]
    lib.shim_stats.argtypes = [vp, u64p]
    lib.shim_now.restype = C.c_double
    return lib


class Client:
    def __init__(self, lib, cap, queue, slots, work_ms, max_group=1 << 20):
        self.lib = lib
        self.h = lib.shim_create(cap, queue, slots, work_ms, max_group)
        self.keep = {}

    def submit(self, bytes_, W=4, H=3, dmax=2, seed=0):
        L = np.full((H, W, 3), seed % 200, np.uint8)
        R = np.full((H, W, 3), (seed * 7) % 50, np.uint8)
        D = np.full((H, W), -1, np.int32)
        t = C.c_uint64()
        st = self.lib.shim_submit(self.h, L.ctypes.data, R.ctypes.data, W, H, dmax,
                                  D.ctypes.data, bytes_, C.byref(t))
        if st == OK:
            self.keep[t.value] = (L, R, D, dmax)
        return st, t.value

    def poll(self, ticket):
        s = C.c_int32()
        times = (C.c_double * 4)()
        st = self.lib.shim_poll(self.h, ticket, C.byref(s), times)
        return st, s.value, list(times)

    def wait(self, ticket, timeout=10.0):
        t0 = time.time()
        while time.time() - t0 < timeout:
            st, s, times = self.poll(ticket)
            if st != OK or s != 0:
                return st, s, times
            time.sleep(0.0005)
        raise TimeoutError(ticket)

    def stats(self):
        a = (C.c_uint64 * 7)()
        self.lib.shim_stats(self.h, a)
        return dict(zip(["submitted", "completed", "failed", "groups", "max_bytes",
                         "max_group", "max_slots"], list(a)))

    def close(self):
        self.lib.shim_destroy(self.h)


def test_too_big_and_queue_full(shim):
    c = Client(shim, 1000, 3, 1, 50.0)
    assert c.submit(1001)[0] == ETOOBIG
    got = [c.submit(600, seed=i)[0] for i in range(8)]
    # one admitted (running), then at most 3 waiting; the rest bounce
    assert got[0] == OK and EAGAIN in got
    shim.shim_drain(c.h)
    c.close()


def test_fifo_admission_and_results(shim):
    c = Client(shim, 1000, 100, 2, 2.0)
    tickets = [c.submit(700, seed=i)[1] for i in range(10)]  # one fits at a time
    admits = []
    for i, t in enumerate(tickets):
        st, s, times = c.wait(t)
        assert st == OK and s == 1
        L, R, D, dmax = c.keep[t]
        assert np.all(D == int(L[0, 0, 0]) + int(R[0, 0, 0]) + dmax)
        assert times[0] <= times[1] <= times[2] <= times[3]
        admits.append(times[1])
    assert admits == sorted(admits)
    st = c.stats()
    assert st["max_bytes"] <= 1000 and st["max_group"] == 1 and st["completed"] == 10
    c.close()


def test_continuous_batching_overlaps_slots(shim):
    c = Client(shim, 10_000, 1000, 3, 5.0)
    tickets = [c.submit(100, seed=i)[1] for i in range(60)]
    shim.shim_drain(c.h)
    for t in tickets:
        assert c.poll(t)[1] == 1
    st = c.stats()
    assert st["completed"] == 60
    assert st["max_group"] > 1          # later arrivals joined a group
    assert st["max_slots"] > 1          # groups overlapped
    assert st["max_bytes"] <= 10_000
    c.close()


def test_group_size_limit(shim):
    c = Client(shim, 10_000, 1000, 2, 5.0, max_group=4)
    tickets = [c.submit(100, seed=i)[1] for i in range(40)]
    shim.shim_drain(c.h)
    assert all(c.poll(t)[1] == 1 for t in tickets)
    st = c.stats()
    assert st["completed"] == 40 and 1 < st["max_group"] <= 4
    c.close()


def test_cap_limits_bytes_in_flight(shim):
    c = Client(shim, 1000, 1000, 3, 1.0)
    for i in range(40):
        c.submit(300 + (i % 5) * 50, seed=i)
    shim.shim_drain(c.h)
    st = c.stats()
    assert st["completed"] == 40 and st["max_bytes"] <= 1000
    c.close()


def test_failures_propagate_and_slots_recover(shim):
    c = Client(shim, 10_000, 100, 1, 1.0)
    shim.shim_fail(c.h, 1, 1)   # first group fails at start, the next at completion
    t1 = c.submit(100)[1]
    assert c.wait(t1)[1] == -1
    t2 = c.submit(100)[1]
    assert c.wait(t2)[1] == -1
    t3 = c.submit(100, seed=5)[1]
    assert c.wait(t3)[1] == 1
    assert c.stats()["failed"] == 2
    c.close()


def test_ticket_reported_once_and_unknown(shim):
    c = Client(shim, 10_000, 100, 2, 0.5)
    t = c.submit(10)[1]
    assert c.wait(t)[1] == 1
    assert c.poll(t)[0] == ENOTFOUND
    assert c.poll(123456)[0] == ENOTFOUND
    c.close()


def test_lowering_cap_fails_waiting_requests_that_no_longer_fit(shim):
    c = Client(shim, 1000, 100, 1, 20.0)
    t1 = c.submit(900)[1]
    t2 = c.submit(900)[1]           # waits behind t1
    t0 = time.time()
    while c.poll(t1)[2][1] == 0.0:  # until t1 is admitted
        assert time.time() - t0 < 5
        time.sleep(0.0005)
    shim.shim_configure(c.h, 500, 100, 1 << 20)
    assert c.wait(t1)[1] == 1       # already admitted
    assert c.wait(t2)[1] == -1      # can never fit any more
    c.close()


def test_destroy_with_requests_in_flight(shim):
    c = Client(shim, 10_000, 100, 2, 5.0)
    for i in range(20):
        c.submit(100, seed=i)
    c.close()                       # finishes the work, then stops


def test_thread_sanitizer_stress(tmp_path):
    exe = tmp_path / "stress"
    r = subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-pthread",
                        "-DSHIM_STRESS_MAIN", "-DBSM_TSAN_SYSTEM_CLOCK_WAITS", *SRC, "-o",
                        str(exe)], capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("ThreadSanitizer build unavailable: " + r.stderr[-300:])
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300,
                         env={**os.environ, "TSAN_OPTIONS": "halt_on_error=1"})
    assert "ThreadSanitizer" not in run.stderr, run.stderr[-3000:]
    assert run.returncode == 0, run.stdout + run.stderr[-2000:]
