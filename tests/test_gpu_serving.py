"""The serving loop on the GPU: jobs of different shapes arrive, are merged
into overlapping launches, and each result equals the job detected alone."""
import numpy as np
import pytest

import oracle
import synth
from parity_util import check

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def mp():
    import paper_2409_14355_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(mp):
    c = mp.Context(0)
    yield c
    c.close()


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def _pool(n, seed, s_max=600, with_slots=False):
    cells = synth.draw_cells(n, seed=(seed,), s_min=40, s_max=s_max)
    jobs, slots = [], []
    for i, c in enumerate(cells):
        sl = synth.make_slot(S=c.S, T=14, M=c.M, N=c.N, bits=c.bits, snr_db=18, seed=(seed, 1, i),
                             channel="kron", rho_rx=0.5, rho_tx=0.3)
        slots.append(sl)
        jobs.append(dict(H=_dev(sl.H), y=_dev(sl.y), mod=c.bits, n_paths=c.n_paths,
                         out=torch.full((14, c.S, c.N), -1, dtype=torch.int32, device="cuda:0")))
    return (jobs, slots) if with_slots else jobs


def _oracle_sample(sl, got, K, label, rng, n_sub=6):
    """Sampled subcarriers of a served job against the FP64 oracle."""
    sub = np.sort(rng.choice(sl.H.shape[0], size=min(n_sub, sl.H.shape[0]), replace=False))
    H, y = sl.H[sub], np.ascontiguousarray(sl.y[:, sub])
    ref, diag = oracle.detect_slot("mpnl", H, y, sl.bits, n_paths=K, want_diag=True, nthreads=8)
    return check(H, y, got[:, sub], ref, diag, sl.bits, label=label)


@pytest.mark.parametrize("prec,split", [(0, 0), (1, 0), (0, 1)], ids=["fp32", "fp16", "fp32-split-slack"])
def test_results_in_the_mix_equal_alone(ctx, mp, prec, split):
    """split: jobs above 2000 vectors run as pieces of whole subcarriers
    under the slack policy (pieces of one job in different launches)."""
    _say("serving mix vs alone, precision", prec, "split", split)
    jobs, slots = _pool(24, 400 + prec + 10 * split, with_slots=True)
    ctx.set_precision(prec)
    try:
        cfg = mp.server_config(max_batch_jobs=5, max_inflight=3)
        if split:
            cfg = mp.server_config(max_batch_jobs=3, max_inflight=3, split_vectors=2000,
                                   policy=mp.MPNL_SCHED_SLACK)
            assert sum(j["H"].shape[0] * 14 > 2000 for j in jobs) >= 10
        srv = mp.Server(ctx, cfg)
        try:
            got = []
            for i, j in enumerate(jobs):
                srv.submit(j, i)
                got += srv.poll()
            got += srv.drain()
        finally:
            srv.close()
        torch.cuda.synchronize()
        assert sorted(c["id"] for c in got) == list(range(len(jobs)))
        assert all(c["status"] == mp.MPNL_JOB_DONE for c in got)
        assert all(c["done_us"] >= c["start_us"] >= c["arrival_us"] - 1.0 for c in got)
        for j in jobs:
            alone = ctx.detect(j["H"], j["y"], j["mod"], j["n_paths"])
            torch.cuda.synchronize()
            assert torch.equal(alone, j["out"])
        if prec == 0:
            # every served FP32 result against the FP64 oracle on sampled
            # subcarriers (the parity protocol: near-ties only)
            rng = np.random.default_rng(403)
            for i, (j, sl) in enumerate(zip(jobs, slots)):
                _oracle_sample(sl, j["out"].cpu().numpy(), j["n_paths"], f"served job {i}", rng)
        else:
            # reduced precision: close to the FP64 oracle (few decisions differ)
            n_bad = n_vec = 0
            for j, sl in zip(jobs, slots):
                got = j["out"].cpu().numpy()[:, :4]
                ref = oracle.detect_slot("mpnl", sl.H[:4], np.ascontiguousarray(sl.y[:, :4]), sl.bits,
                                         n_paths=j["n_paths"], nthreads=8)
                n_bad += int(np.any(got != ref, axis=-1).sum())
                n_vec += ref.shape[0] * ref.shape[1]
            print(f"served FP16 jobs: {n_bad} of {n_vec} sampled vectors differ from the FP64 oracle",
                  flush=True)
            assert n_bad <= max(2, 0.01 * n_vec)
    finally:
        ctx.set_precision(0)


def test_budget_admission_on_the_device(ctx, mp):
    """A budget that holds about one job at a time: every job still
    completes, the jobs that run together never exceed the budget, and
    results are unchanged."""
    _say("serving budget")
    jobs = _pool(6, 410, s_max=300)
    need = [mp.mpnl_job_bytes(j["H"].shape[0], 14, j["H"].shape[1], j["H"].shape[2], j["mod"], j["n_paths"])
            for j in jobs]
    budget = max(need) + max(need) // 2
    srv = mp.Server(ctx, mp.server_config(hbm_budget=budget, max_batch_jobs=4, max_inflight=3))
    try:
        for i, j in enumerate(jobs):
            srv.submit(j, i)
        got = sorted(srv.drain(), key=lambda c: c["id"])
    finally:
        srv.close()
    torch.cuda.synchronize()
    assert [c["id"] for c in got] == list(range(len(jobs)))
    assert all(c["status"] == mp.MPNL_JOB_DONE for c in got)
    # a job is admitted only after the host saw the completions that freed
    # its memory; event times may differ from the host clock by a few us
    for c in got:
        together = [o for o in got if o["start_us"] < c["done_us"] - 50.0 and o["done_us"] > c["start_us"] + 50.0]
        assert sum(need[o["id"]] for o in together) <= budget
    for j in jobs:
        alone = ctx.detect(j["H"], j["y"], j["mod"], j["n_paths"])
        torch.cuda.synchronize()
        assert torch.equal(alone, j["out"])


def test_poisson_run_completes_every_job(ctx, mp):
    _say("serving poisson")
    pool = _pool(8, 420, s_max=400)
    srv = mp.Server(ctx, mp.server_config(max_batch_jobs=8, max_inflight=2, max_queue=64, deadline_us=500.0))
    try:
        comp = srv.run_poisson(pool, 300, 5000.0, 421)
    finally:
        srv.close()
    torch.cuda.synchronize()
    st = np.array([c["status"] for c in comp])
    assert set(st.tolist()) <= {mp.MPNL_JOB_DONE, mp.MPNL_JOB_REJECTED}
    assert (st == mp.MPNL_JOB_DONE).sum() > 0
    lat = np.array([c["done_us"] - c["arrival_us"] for c in comp if c["status"] == mp.MPNL_JOB_DONE])
    assert (lat > 0).all()
    arr = np.array([c["arrival_us"] for c in comp])
    assert (np.diff(arr) >= 0).all()
    assert all(0 <= c["entry"] < len(pool) for c in comp)
