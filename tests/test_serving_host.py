"""Scheduling logic of the serving loop on the host-only executor (no GPU):
admission by footprint against the HBM budget, first fit in arrival order,
retire/admit at quantum boundaries, cancel, rejection of jobs that can never
fit, a full queue, and the statistics."""
import time

import pytest

from paper_2403_04714_amd import fibersim as F
from paper_2403_04714_amd import netgen as g


@pytest.fixture(scope="module")
def design():
    return F.Design(None, g.gen_tiny(0), pack=F.PACK_SINGLE)


def footprint(design, n):
    import ctypes as C
    fp = C.c_size_t()
    F._check(F.lib().fsim_sim_footprint(design._h, n, C.byref(fp)), "footprint")
    return fp.value


def test_all_jobs_complete(design):
    srv = F.Server(None, 1 << 34, quantum_cycles=100)
    ids = [srv.submit(design, 1 + k, 250 + 10 * k, k) for k in range(10)]
    for j in ids:
        srv.wait(j, 10)
    for j, k in zip(ids, range(10)):
        st = srv.poll(j)
        assert st["state"] == F.JOB_DONE and st["cycles_done"] == 250 + 10 * k
        assert st["t_submit"] <= st["t_start"] <= st["t_done"]
    s = srv.stats()
    assert s["completed"] == 10 and s["submitted"] == 10
    assert s["instance_cycles"] == sum((1 + k) * (250 + 10 * k) for k in range(10))
    assert s["hbm_used"] == 0
    srv.close()


def test_admission_respects_budget(design):
    fp = footprint(design, 64)
    srv = F.Server(None, 2 * fp, quantum_cycles=100)      # room for two jobs at a time
    ids = [srv.submit(design, 64, 20_000, k) for k in range(5)]
    seen_max = 0
    deadline = time.time() + 20
    while time.time() < deadline:
        s = srv.stats()
        seen_max = max(seen_max, s["running"])
        assert s["hbm_used"] <= 2 * fp
        if s["completed"] == 5:
            break
    assert srv.stats()["completed"] == 5
    assert seen_max <= 2
    # later jobs started only after earlier ones finished
    st = [srv.poll(j) for j in ids]
    assert st[2]["t_start"] >= min(st[0]["t_done"], st[1]["t_done"])
    srv.close()


def test_never_fits_is_rejected(design):
    srv = F.Server(None, footprint(design, 1) - 1)
    with pytest.raises(F.FsimError) as e:
        srv.submit(design, 1, 10, 0)
    assert e.value.code == F.E_CAPACITY
    assert srv.stats()["rejected"] == 1
    srv.close()


def test_queue_full(design):
    fp = footprint(design, 8)
    srv = F.Server(None, fp, quantum_cycles=1, max_queue=2)
    a = srv.submit(design, 8, 10**9, 0)                   # occupies the budget
    time.sleep(0.05)
    srv.submit(design, 8, 10, 1)
    srv.submit(design, 8, 10, 2)
    with pytest.raises(F.FsimError) as e:
        srv.submit(design, 8, 10, 3)
    assert e.value.code == F.E_BUSY
    srv.cancel(a)
    srv.close()


def test_cancel_queued_and_running(design):
    fp = footprint(design, 4)
    srv = F.Server(None, fp, quantum_cycles=1)
    run = srv.submit(design, 4, 10**12, 0)
    queued = srv.submit(design, 4, 10, 1)
    time.sleep(0.05)
    assert srv.poll(run)["state"] == F.JOB_RUNNING
    assert srv.poll(queued)["state"] == F.JOB_QUEUED
    srv.cancel(queued)
    assert srv.poll(queued)["state"] == F.JOB_CANCELLED
    srv.cancel(run)
    srv.wait(run, 10)
    assert srv.poll(run)["state"] == F.JOB_CANCELLED
    s = srv.stats()
    assert s["cancelled"] == 2 and s["hbm_used"] == 0
    srv.release(run)
    with pytest.raises(F.FsimError):
        srv.poll(run)
    srv.close()


def test_first_fit_lets_small_jobs_pass(design):
    small, big = footprint(design, 1), footprint(design, 4096)
    srv = F.Server(None, big, quantum_cycles=1000)
    hog = srv.submit(design, 64, 10**7, 0)     # takes part of the budget
    time.sleep(0.05)
    b = srv.submit(design, 4096, 10, 1)        # does not fit next to the hog
    s = srv.submit(design, 1, 10, 2)           # fits: overtakes the big job
    srv.wait(s, 10)
    assert srv.poll(b)["state"] == F.JOB_QUEUED
    srv.cancel(hog)
    srv.wait(b, 20)
    assert srv.poll(b)["state"] == F.JOB_DONE
    srv.close()


def test_results_unavailable_on_host_executor(design):
    srv = F.Server(None, 1 << 30)
    j = srv.submit(design, 2, 5, 0)
    srv.wait(j, 10)
    with pytest.raises(F.FsimError) as e:
        srv.result(j, 0, design)
    assert e.value.code == F.E_STATE
    srv.close()
