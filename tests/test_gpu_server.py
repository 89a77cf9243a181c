"""Serving (continuous batching) on the GPU: every job's result is the same
alone and in the mix, and equals the oracle's run of that job."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1706_01094_amd.mclg import E_INVAL, MclgError, Server

pytestmark = pytest.mark.gpu

SEED = 5
JOBS = [  # job_id, L, steps, rho, u0
    (3, 5000, 40, 20.0, 0.0),
    (8, 1000, 7, 60.0, 0.1),
    (1, 12345, 25, 10.0, -0.1),
    (40, 300, 33, 5.0, 0.0),
    (17, 4096, 18, 90.0, 0.0),
    (2, 700, 1, 30.0, 0.2),
]


def say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


def run(jobs, arena_bytes=1 << 24, max_slots=4, k=5):
    srv = Server(arena_bytes, max_slots, SEED)
    for j in jobs:
        srv.submit(*j)
    res = {}
    for _ in range(10000):
        srv.tick(k)
        for jid, m in srv.poll():
            res[jid] = m
        q, r, _ = srv.stats()
        if q == 0 and r == 0:
            break
    srv.close()
    return res


def oracle_moments(job):
    jid, L, steps, rho, u0 = job
    o = O.OracleSim([L], SEED, C=10, replica_id=[jid])
    o.init_poisson(0, rho, u0)
    o.step(steps)
    return o.moments(0)


KEYS = ("t", "sum_n", "sum_n2", "sum_nn", "sum_N", "sum_J", "sum_N2", "n0_odd", "max_N")


def test_jobs_alone_equal_jobs_in_mix_equal_oracle():
    say("mix of", len(JOBS))
    mix = run(JOBS)
    assert sorted(mix) == sorted(j[0] for j in JOBS)
    for job in JOBS:
        say("alone", job)
        alone = run([job])[job[0]]
        want = oracle_moments(job)
        for k in KEYS:
            assert mix[job[0]][k] == alone[k] == want[k], (job, k)


def test_admission_waits_for_arena_space():
    """An arena that holds about two of the jobs at a time: the rest wait in
    the queue and still produce the same results."""
    jobs = [(100 + i, 20000, 6 + i, 15.0 + i, 0.0) for i in range(5)]
    res = run(jobs, arena_bytes=2 * 3 * 20096 * 2 + 512, max_slots=8, k=3)
    for job in jobs:
        want = oracle_moments(job)
        for k in KEYS:
            assert res[job[0]][k] == want[k], (job, k)


def test_job_larger_than_arena_is_rejected():
    srv = Server(1 << 16, 2, SEED)
    with pytest.raises(MclgError) as e:
        srv.submit(1, 1 << 20, 10, 10.0, 0.0)
    assert e.value.code == E_INVAL
    srv.close()
