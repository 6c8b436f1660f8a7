"""Serving scheduler logic on a virtual clock (modelled device, no GPU).

The scheduler is the one the device server runs; here its executor models a
device that runs launches one after another, each taking
launch_us + per_vector_us * vectors, with forced failures and slow jobs.
"""
import math

import numpy as np
import pytest

import paper_2409_14355_amd as mp

DONE, REJ, DROP, FAIL = mp.MPNL_JOB_DONE, mp.MPNL_JOB_REJECTED, mp.MPNL_JOB_DROPPED, mp.MPNL_JOB_FAILED


def _check_invariants(jobs, comp):
    assert len(comp) == len(jobs)
    for i, c in enumerate(comp):
        assert c["id"] == i
        assert c["arrival_us"] == pytest.approx(jobs[i]["arrival_us"])
        assert c["done_us"] >= c["start_us"] >= c["arrival_us"] - 1e-9


def test_single_job_latency_is_the_launch():
    cfg = mp.server_config(max_batch_jobs=4, max_inflight=1)
    jobs = [dict(arrival_us=10.0, bytes=100, vectors=1000)]
    comp, nl = mp.mpnl_sched_simulate(cfg, jobs, launch_us=5.0, per_vector_us=0.01)
    _check_invariants(jobs, comp)
    assert nl == 1 and comp[0]["status"] == DONE
    assert comp[0]["start_us"] == pytest.approx(10.0)
    assert comp[0]["done_us"] == pytest.approx(10.0 + 5.0 + 10.0)


def test_continuous_batching_merges_jobs_that_wait():
    """Jobs that arrive while the only launch slot is busy go together into
    the next launch."""
    cfg = mp.server_config(max_batch_jobs=16, max_inflight=1)
    jobs = [dict(arrival_us=0.0, bytes=1, vectors=100)] + \
           [dict(arrival_us=1.0 + i, bytes=1, vectors=100) for i in range(5)]
    comp, nl = mp.mpnl_sched_simulate(cfg, jobs, launch_us=50.0, per_vector_us=0.0)
    _check_invariants(jobs, comp)
    assert nl == 2
    assert all(c["status"] == DONE for c in comp)
    assert comp[0]["done_us"] == pytest.approx(50.0)
    # the five late arrivals start together when the first launch ends
    assert {round(c["start_us"], 6) for c in comp[1:]} == {50.0}
    assert all(c["done_us"] == pytest.approx(100.0) for c in comp[1:])


def test_batch_size_limit():
    cfg = mp.server_config(max_batch_jobs=3, max_inflight=1)
    jobs = [dict(arrival_us=0.0, bytes=1, vectors=10) for _ in range(10)]
    comp, nl = mp.mpnl_sched_simulate(cfg, jobs, launch_us=1.0)
    _check_invariants(jobs, comp)
    assert nl == math.ceil(10 / 3)
    starts = sorted({c["start_us"] for c in comp})
    assert len(starts) == nl


def test_several_launches_in_flight_overlap_in_the_queue():
    """With two launch slots a second launch is enqueued while the first runs
    (the modelled device still runs them one after the other)."""
    cfg = mp.server_config(max_batch_jobs=1, max_inflight=2)
    jobs = [dict(arrival_us=0.0, bytes=1, vectors=0), dict(arrival_us=1.0, bytes=1, vectors=0),
            dict(arrival_us=2.0, bytes=1, vectors=0)]
    comp, nl = mp.mpnl_sched_simulate(cfg, jobs, launch_us=10.0)
    _check_invariants(jobs, comp)
    assert comp[1]["start_us"] == pytest.approx(1.0)       # enqueued at once
    assert comp[1]["done_us"] == pytest.approx(20.0)       # runs after the first
    assert comp[2]["start_us"] == pytest.approx(10.0)      # waits for a free slot
    assert comp[2]["done_us"] == pytest.approx(30.0)


def test_budget_admission_serialises_and_rejects_oversize():
    cfg = mp.server_config(hbm_budget=1000, max_batch_jobs=8, max_inflight=4)
    jobs = [dict(arrival_us=0.0, bytes=600, vectors=10) for _ in range(4)] + \
           [dict(arrival_us=1.0, bytes=5000, vectors=10)]
    comp, nl = mp.mpnl_sched_simulate(cfg, jobs, launch_us=10.0)
    _check_invariants(jobs, comp)
    assert comp[4]["status"] == REJ
    done = [c for c in comp[:4]]
    assert all(c["status"] == DONE for c in done)
    # 600 + 600 > 1000: never two of them admitted together
    spans = sorted((c["start_us"], c["done_us"]) for c in done)
    for (s0, d0), (s1, d1) in zip(spans, spans[1:]):
        assert s1 >= d0 - 1e-9
    assert nl == 4


def test_budget_fits_two_jobs_per_launch():
    cfg = mp.server_config(hbm_budget=1000, max_batch_jobs=8, max_inflight=1)
    jobs = [dict(arrival_us=0.0, bytes=500, vectors=10) for _ in range(6)]
    comp, nl = mp.mpnl_sched_simulate(cfg, jobs, launch_us=10.0)
    assert nl == 3 and all(c["status"] == DONE for c in comp)


def test_queue_limit_rejects_a_burst():
    cfg = mp.server_config(max_batch_jobs=1, max_inflight=1, max_queue=5)
    jobs = [dict(arrival_us=0.0, bytes=1, vectors=0) for _ in range(20)]
    comp, nl = mp.mpnl_sched_simulate(cfg, jobs, launch_us=10.0)
    _check_invariants(jobs, comp)
    st = np.array([c["status"] for c in comp])
    # all arrive before the first admission: five wait, the rest are rejected
    assert (st == REJ).sum() == 15 and (st == DONE).sum() == 5


def test_drop_late_keeps_admitted_jobs_within_deadline():
    cfg = mp.server_config(max_batch_jobs=1, max_inflight=1, deadline_us=100.0, drop_late=True)
    rng = np.random.default_rng(7)
    t = np.cumsum(rng.exponential(10.0, size=200))  # 100 k jobs/s offered
    jobs = [dict(arrival_us=float(x), bytes=1, vectors=1000) for x in t]
    comp, nl = mp.mpnl_sched_simulate(cfg, jobs, launch_us=20.0, per_vector_us=0.02)  # 40 us per job
    _check_invariants(jobs, comp)
    st = np.array([c["status"] for c in comp])
    assert (st == DROP).sum() > 0 and (st == DONE).sum() > 0
    for c in comp:
        if c["status"] == DONE:
            assert c["start_us"] - c["arrival_us"] <= 100.0 + 1e-9
        if c["status"] == DROP:
            assert c["start_us"] - c["arrival_us"] > 100.0


def test_without_drop_every_job_runs_in_arrival_order():
    cfg = mp.server_config(max_batch_jobs=2, max_inflight=1, deadline_us=1.0)
    rng = np.random.default_rng(8)
    t = np.cumsum(rng.exponential(5.0, size=100))
    jobs = [dict(arrival_us=float(x), bytes=1, vectors=100) for x in t]
    comp, nl = mp.mpnl_sched_simulate(cfg, jobs, launch_us=3.0, per_vector_us=0.05)
    _check_invariants(jobs, comp)
    assert all(c["status"] == DONE for c in comp)
    starts = [c["start_us"] for c in comp]
    assert starts == sorted(starts)  # FIFO


def test_failed_launch_fails_only_its_jobs():
    cfg = mp.server_config(max_batch_jobs=2, max_inflight=1)
    jobs = [dict(arrival_us=float(i), bytes=1, vectors=10) for i in range(6)]
    comp, nl = mp.mpnl_sched_simulate(cfg, jobs, launch_us=10.0, fail_launch=1)
    _check_invariants(jobs, comp)
    failed = [c for c in comp if c["status"] == FAIL]
    assert 1 <= len(failed) <= 2
    assert all(c["error"] == mp.MPNL_E_HIP for c in failed)
    assert all(c["status"] == DONE for c in comp if c not in failed)


def test_slow_job_delays_the_jobs_behind_it():
    cfg = mp.server_config(max_batch_jobs=1, max_inflight=1)
    jobs = [dict(arrival_us=float(i), bytes=1, vectors=0) for i in range(4)]
    fast, _ = mp.mpnl_sched_simulate(cfg, jobs, launch_us=10.0)
    slow, _ = mp.mpnl_sched_simulate(cfg, jobs, launch_us=10.0, slow_job=1, slow_extra_us=500.0)
    assert slow[0]["done_us"] == pytest.approx(fast[0]["done_us"])
    for i in (1, 2, 3):
        assert slow[i]["done_us"] == pytest.approx(fast[i]["done_us"] + 500.0)


def test_bad_configs_are_refused():
    for cfg in (mp.server_config(max_batch_jobs=0), mp.server_config(max_inflight=0),
                mp.server_config(max_inflight=9), mp.server_config(max_queue=-1)):
        with pytest.raises(mp.MpnlError) as ei:
            mp.mpnl_sched_simulate(cfg, [dict(arrival_us=0.0)])
        assert ei.value.code == mp.MPNL_E_INVAL
    with pytest.raises(mp.MpnlError):  # arrivals out of order
        mp.mpnl_sched_simulate(mp.server_config(), [dict(arrival_us=5.0), dict(arrival_us=1.0)])


def test_job_bytes_grows_with_the_job_and_rejects_bad_shapes():
    a = mp.mpnl_job_bytes(100, 14, 16, 16, 4, 64)
    b = mp.mpnl_job_bytes(200, 14, 16, 16, 4, 64)
    c = mp.mpnl_job_bytes(100, 14, 16, 16, 4, 256)
    assert 0 < a < b and a < c
    assert mp.mpnl_job_bytes(100, 14, 4, 8, 4, 64) == 0   # N > M
    assert mp.mpnl_job_bytes(0, 14, 4, 4, 4, 64) == 0


def test_antenna_search_takes_the_first_count_meeting_the_target():
    import bench
    calls = []

    def ber(M):
        calls.append(M)
        return 1.0 / M
    M, trace = bench.antenna_search(ber, 2, 40, 0.1)
    assert M == 10 and calls == list(range(2, 11)) and trace[-1] == (10, 0.1)
    M, trace = bench.antenna_search(lambda m: 1.0, 3, 6, 0.5)
    assert M is None and [m for m, _ in trace] == [3, 4, 5, 6]


# ---- pieces of split jobs and the slack policy ----------------------------
SLACK = mp.MPNL_SCHED_SLACK


def test_split_job_completes_with_its_last_piece():
    cfg = mp.server_config(max_batch_jobs=1, max_inflight=1, split_vectors=2500)
    jobs = [dict(arrival_us=0.0, bytes=4000, vectors=10000)]
    comp, nl = mp.mpnl_sched_simulate(cfg, jobs, launch_us=10.0, per_vector_us=0.01)
    _check_invariants(jobs, comp)
    assert nl == 4  # four pieces of 2500 vectors, one launch each
    assert comp[0]["status"] == DONE
    assert comp[0]["start_us"] == pytest.approx(0.0)
    assert comp[0]["done_us"] == pytest.approx(4 * (10.0 + 25.0))


def test_uneven_split_covers_every_vector():
    cfg = mp.server_config(max_batch_jobs=8, max_inflight=1, split_vectors=3000)
    jobs = [dict(arrival_us=0.0, bytes=100, vectors=10001)]
    comp, nl = mp.mpnl_sched_simulate(cfg, jobs, launch_us=0.0, per_vector_us=1.0)
    assert nl == 1  # four pieces, all in one launch
    assert comp[0]["done_us"] == pytest.approx(10001.0)


@pytest.mark.parametrize("policy", [mp.MPNL_SCHED_FIFO, SLACK])
def test_small_job_between_pieces_of_a_large_one(policy):
    """A large job split into eight pieces arrives first, a small job right
    after.  Under the slack policy the small job (which can still meet the
    deadline) runs after the first piece; in arrival order it waits for all
    eight."""
    cfg = mp.server_config(max_batch_jobs=1, max_inflight=1, split_vectors=5000, policy=policy,
                           est_fixed_us=10.0, est_us_per_gflop=1.0)
    jobs = [dict(arrival_us=0.0, bytes=1, vectors=40000, gflop=4000.0),
            dict(arrival_us=1.0, bytes=1, vectors=1000, gflop=10.0)]
    comp, nl = mp.mpnl_sched_simulate(cfg, jobs, launch_us=10.0, per_vector_us=0.01)
    _check_invariants(jobs, comp)
    assert nl == 9
    piece = 10.0 + 50.0
    if policy == SLACK:
        assert comp[1]["start_us"] == pytest.approx(piece)
        assert comp[1]["done_us"] == pytest.approx(piece + 20.0)
        assert comp[0]["done_us"] == pytest.approx(8 * piece + 20.0)
    else:
        assert comp[1]["start_us"] == pytest.approx(8 * piece)
        assert comp[0]["done_us"] == pytest.approx(8 * piece)


def test_slack_takes_the_most_urgent_feasible_job_first():
    """While the device is busy, B (little work) and then A (much work)
    arrive; when it frees up A has less slack and goes first, although it
    arrived later."""
    cfg = mp.server_config(max_batch_jobs=1, max_inflight=1, policy=SLACK, deadline_us=500.0,
                           est_fixed_us=10.0, est_us_per_gflop=1.0)
    jobs = [dict(arrival_us=0.0, vectors=9000, gflop=90.0),     # X: occupies the device until 100
            dict(arrival_us=10.0, vectors=4000, gflop=40.0),    # B: slack at 100 is 360
            dict(arrival_us=20.0, vectors=39000, gflop=390.0)]  # A: slack at 100 is 20
    comp, nl = mp.mpnl_sched_simulate(cfg, jobs, launch_us=10.0, per_vector_us=0.01)
    _check_invariants(jobs, comp)
    assert comp[2]["start_us"] == pytest.approx(100.0)
    assert comp[2]["done_us"] == pytest.approx(500.0)
    assert comp[1]["start_us"] == pytest.approx(500.0)
    cfg.policy = mp.MPNL_SCHED_FIFO
    comp, _ = mp.mpnl_sched_simulate(cfg, jobs, launch_us=10.0, per_vector_us=0.01)
    assert comp[1]["start_us"] == pytest.approx(100.0)


def test_jobs_that_cannot_meet_the_deadline_go_last():
    cfg = mp.server_config(max_batch_jobs=1, max_inflight=1, policy=SLACK, deadline_us=500.0,
                           est_fixed_us=10.0, est_us_per_gflop=1.0)
    jobs = [dict(arrival_us=0.0, vectors=100, gflop=0.0),        # occupies the device until 11
            dict(arrival_us=1.0, vectors=100000, gflop=990.0),   # C: estimated 1000 us, infeasible
            dict(arrival_us=2.0, vectors=1000, gflop=10.0),      # D: feasible
            dict(arrival_us=3.0, vectors=100000, gflop=990.0)]   # E: infeasible, after C
    comp, _ = mp.mpnl_sched_simulate(cfg, jobs, launch_us=10.0, per_vector_us=0.01)
    _check_invariants(jobs, comp)
    assert comp[2]["start_us"] < comp[1]["start_us"] < comp[3]["start_us"]
    assert all(c["status"] == DONE for c in comp)


def test_drop_late_spares_a_job_whose_pieces_have_started():
    cfg = mp.server_config(max_batch_jobs=1, max_inflight=1, split_vectors=1000, drop_late=True,
                           deadline_us=100.0)
    jobs = [dict(arrival_us=0.0, vectors=4000),   # four pieces of 80 us: runs past the deadline
            dict(arrival_us=1.0, vectors=100)]    # waits 320 us: dropped
    comp, _ = mp.mpnl_sched_simulate(cfg, jobs, launch_us=0.0, per_vector_us=0.08)
    _check_invariants(jobs, comp)
    assert comp[0]["status"] == DONE and comp[0]["done_us"] == pytest.approx(320.0)
    assert comp[1]["status"] == DROP


def test_budget_counts_pieces():
    """Pieces are admitted against the budget one by one: a job twice the
    budget runs when split into pieces that fit."""
    cfg = mp.server_config(hbm_budget=1000, max_batch_jobs=8, max_inflight=4, split_vectors=500)
    jobs = [dict(arrival_us=0.0, bytes=2000, vectors=2000)]
    comp, nl = mp.mpnl_sched_simulate(cfg, jobs, launch_us=1.0, per_vector_us=0.0)
    assert comp[0]["status"] == DONE and nl >= 2
    cfg.split_vectors = 0
    comp, _ = mp.mpnl_sched_simulate(cfg, jobs, launch_us=1.0, per_vector_us=0.0)
    assert comp[0]["status"] == REJ


def test_bad_policy_config_is_rejected():
    for cfg in (mp.server_config(policy=7), mp.server_config(split_vectors=-1)):
        with pytest.raises(mp.MpnlError):
            mp.mpnl_sched_simulate(cfg, [dict(arrival_us=0.0, vectors=1)])
