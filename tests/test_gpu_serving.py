"""GPU tests of the served form: jobs of uneven n, d, eps and MinPts run
together in the persistent loop; each result equals the same job run alone
(dbscan_fit) and the CPU oracle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1506_02226_amd as pkg
from oracle import c_oracle, dbscan_oracle as orc
from paper_1506_02226_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda:0")


def _host(out):
    lab, core, cnt = (t.cpu().numpy() for t in out)
    return lab, core.astype(bool), cnt


def _mixed_jobs(count, seed, n_max=6000):
    rng = np.random.default_rng(seed)
    jobs = []
    for j in range(count):
        n = int(np.exp(rng.uniform(np.log(200), np.log(n_max))))
        d = int(rng.choice([2, 3, 16, 64]))
        k = int(rng.integers(3, 12))
        minpts = int(rng.choice([5, 10, 20]))
        if d <= 3:
            pts = wl.isotropic_blobs(rng, n, d, k, 40.0, 0.05, 0.2, 1.0)
        else:
            pts = wl.mixture_blobs(rng, n, d, k, 0.05)
        eps = wl.core_distance_quantile(pts, minpts, 0.3, 128, rng)
        jobs.append((pts, eps, minpts))
    return jobs


def test_served_mix_equals_alone_and_oracle():
    jobs = _mixed_jobs(24, seed=5)
    xs = [_gpu(p) for p, _, _ in jobs]
    with pkg.Server(max_slots=64) as srv:
        ids = [srv.submit(x, eps, mp) for x, (_, eps, mp) in zip(xs, jobs)]
        sts = [srv.wait(i, timeout=120) for i in ids]
        stats = srv.stats()
        torch.cuda.synchronize()
        mixed = [_host(srv.outputs(i)) for i in ids]
    assert all(s is not None and s["state"] == pkg._lib.JOB_DONE and s["error"] == 0 for s in sts)
    assert stats["jobs_done"] == len(jobs) and stats["epochs"] >= 1
    assert any(s["fallback"] == 0 for s in sts)
    for (pts, eps, mp), x, got, st in zip(jobs, xs, mixed, sts):
        alone = pkg.fit(x, eps, mp)
        torch.cuda.synchronize()
        alone = _host(alone)
        for a, b in zip(got, alone):
            np.testing.assert_array_equal(a, b)
        ref = c_oracle.dbscan(pts, eps, mp)
        np.testing.assert_array_equal(got[2], ref[2])
        np.testing.assert_array_equal(got[1], ref[1])
        np.testing.assert_array_equal(got[0], ref[0])
        assert st["t_submit_ns"] <= st["t_admit_ns"] <= st["t_done_ns"]


def test_served_admission_by_footprint():
    """A budget that holds about two jobs at a time: every job still runs,
    and the arena never holds more than the budget."""
    jobs = _mixed_jobs(10, seed=9, n_max=3000)
    budget = 48 << 20
    with pkg.Server(hbm_budget=budget, max_slots=8) as srv:
        ids = [srv.submit(_gpu(p), eps, mp) for p, eps, mp in jobs]
        sts = [srv.wait(i, timeout=120) for i in ids]
        stats = srv.stats()
        outs = [_host(srv.outputs(i)) for i in ids]
    assert all(s["state"] == pkg._lib.JOB_DONE for s in sts)
    assert stats["peak_bytes"] <= budget
    assert max(s["footprint"] for s in sts) <= budget
    for (pts, eps, mp), got in zip(jobs, outs):
        ref = orc.dbscan(pts, eps, mp)
        np.testing.assert_array_equal(got[0], ref[0])


def test_served_rejects_and_fallbacks():
    rng = np.random.default_rng(3)
    with pkg.Server(hbm_budget=8 << 20, max_slots=4) as srv:
        # a job whose footprint exceeds the whole arena
        big = _gpu(rng.uniform(0, 1, size=(200_000, 2)))
        with pytest.raises(pkg.DbscanError) as ei:
            srv.submit(big, 0.01, 5)
        assert ei.value.code == pkg._lib.DBSCAN_E_NOMEM
        # d = 8 is not in the persistent loop: it runs through dbscan_fit
        p8 = rng.uniform(0, 3, size=(700, 8)).astype(np.float32)
        j8 = srv.submit(_gpu(p8), 1.0, 4)
        # eps above the diameter: n^2/2 pairs overflow the pair list -> refit
        pd = rng.uniform(0, 1, size=(500, 3)).astype(np.float32)
        jd = srv.submit(_gpu(pd), 5.0, 3)
        # non-finite input
        pn = rng.uniform(0, 1, size=(300, 2)).astype(np.float32)
        pn[7, 0] = np.inf
        jn = srv.submit(_gpu(pn), 0.1, 3)
        # coordinates beyond the half-precision range: the filter gives up
        pw = rng.uniform(0, 40000, size=(400, 16)).astype(np.float32)
        pw[:200] = pw[0] + rng.normal(0, 1, size=(200, 16)).astype(np.float32)
        jw = srv.submit(_gpu(pw), 4.0, 5)
        s8, sd, sn, sw = srv.wait(j8), srv.wait(jd), srv.wait(jn), srv.wait(jw)
        o8, od, on, ow = (_host(srv.outputs(j)) for j in (j8, jd, jn, jw))
    assert s8["fallback"] == 1 and sd["fallback"] == 1 and sw["fallback"] == 1
    assert sw["state"] == pkg._lib.JOB_DONE and sw["error"] == 0
    for (p, eps, mp), got in (((p8, 1.0, 4), o8), ((pd, 5.0, 3), od), ((pw, 4.0, 5), ow)):
        ref = orc.dbscan(p, eps, mp)
        for a, b in zip(got, ref):
            np.testing.assert_array_equal(a, np.asarray(b).astype(a.dtype))
    assert sn["error"] == pkg._lib.DBSCAN_E_NONFINITE and (on[0] == -2).all()


def test_served_jobs_arriving_while_others_run():
    """Submit a large job, then small ones while it is in flight: the large
    one runs on a worker stream, the small ones are admitted into the
    persistent loop beside it, and every output equals the same job alone
    (and the oracle).  When the small ones are admitted and which finishes
    first is up to the device's scheduling: the large job's kernels can hold
    every CU until they drain, and the loop's epoch boundaries wait for them
    (the timings are printed).  Every input and output is allocated before the
    large job is submitted: an allocation in between may wait for the device,
    and so for the large job."""
    # 200,000 points at d = 64 in float32 (no matrix cores, no pruning):
    # tens of milliseconds on a worker
    big = wl.mix64d_300k(0, n=200_000, eps_rule="q50")
    big_eps, big_minpts = big.eps, big.minpts
    small = _mixed_jobs(6, seed=12, n_max=2000)
    xb = _gpu(big.points)
    xs = [_gpu(p) for p, _, _ in small]
    outs_dev = [(torch.empty(len(p), dtype=torch.int32, device="cuda:0"),
                 torch.empty(len(p), dtype=torch.uint8, device="cuda:0"),
                 torch.empty(len(p), dtype=torch.int32, device="cuda:0")) for p, _, _ in small]
    torch.cuda.synchronize()
    with pkg.Server(max_slots=16) as srv:
        jb = srv.submit(xb, big_eps, big_minpts, precision="fp32")
        ids = [srv.submit(x, eps, mp, out=o)
               for x, (_, eps, mp), o in zip(xs, small, outs_dev)]
        sts = [srv.wait(i, timeout=120) for i in ids]
        sb = srv.wait(jb, timeout=120)
        outs = [_host(srv.outputs(i)) for i in ids]
        ob = _host(srv.outputs(jb))
    states = [(s["state"], s["error"]) for s in sts + [sb]]
    assert all(st == (pkg._lib.JOB_DONE, 0) for st in states), states
    assert sb["fallback"] == 1  # a worker runs it, beside the loop
    assert all(s["fallback"] == 0 for s in sts)
    for s in sts:  # submitted while the large job was in flight
        assert sb["t_submit_ns"] < s["t_submit_ns"] < sb["t_done_ns"], (s, sb)
    t0 = sb["t_submit_ns"]
    print("large: admit %.2f ms done %.2f ms; small: done %s ms" % (
        (sb["t_admit_ns"] - t0) / 1e6, (sb["t_done_ns"] - t0) / 1e6,
        [round((s["t_done_ns"] - t0) / 1e6, 2) for s in sts]))
    for (pts, eps, mp), got in zip(small, outs):
        np.testing.assert_array_equal(got[0], orc.dbscan(pts, eps, mp)[0])
    alone = _host(pkg.fit(_gpu(big.points), big_eps, big_minpts, precision="fp32"))
    for a, b in zip(ob, alone):
        np.testing.assert_array_equal(a, b)


def test_served_full_recipe_jobs():
    """Jobs 0-31 of the served workload itself (its recipe at full size, n up
    to 1.6e5) in one server: every output equals the oracle's element by
    element (digests written by the C oracle)."""
    from helpers import assert_golden, golden_job
    loop = [1, 10, 18, 21, 23]  # n <= 9,275, d = 2, 64, 3, 16, 64: the persistent loop
    workers = [3, 9]            # n = 147,911 (d = 64), 158,412 (d = 3): a worker
    jobs = {j: wl.served_job(j) for j in range(32)}
    with pkg.Server(max_slots=32) as srv:
        ids = {j: srv.submit(_gpu(w.points), w.eps, w.minpts) for j, w in jobs.items()}
        sts = {j: srv.wait(i, timeout=300) for j, i in ids.items()}
        outs = {j: _host(srv.outputs(i)) for j, i in ids.items()}
    for j, st in sts.items():
        assert st["state"] == pkg._lib.JOB_DONE and st["error"] == 0, (j, st)
    for j in loop:
        assert sts[j]["fallback"] == 0, j
    for j in workers:
        assert sts[j]["fallback"] == 1, j
    for j, w in jobs.items():
        assert_golden(golden_job(j), w.points, outs[j], f"served job {j}")


@pytest.mark.parametrize("prec", ["auto", "fp32", "fp16", "bf16"])
def test_served_precision(prec):
    """dbscan_job.precision: every precision gives the oracle's outputs; the
    loop runs float32 (d <= 4) and FP16 (16 <= d <= 76) jobs, the workers
    the rest (BF16, float32 at d >= 16)."""
    jobs = _mixed_jobs(12, seed=31, n_max=5000)
    if prec in ("fp16", "bf16"):
        jobs = [j for j in jobs if j[0].shape[1] >= 16]
    with pkg.Server(max_slots=16) as srv:
        ids = [srv.submit(_gpu(p), eps, mp, precision=prec) for p, eps, mp in jobs]
        sts = [srv.wait(i, timeout=120) for i in ids]
        outs = [_host(srv.outputs(i)) for i in ids]
    for (pts, eps, mp), got, st in zip(jobs, outs, sts):
        assert st["state"] == pkg._lib.JOB_DONE and st["error"] == 0
        d = pts.shape[1]
        in_loop = (d <= 4 and prec in ("auto", "fp32")) or (d >= 16 and prec in ("auto", "fp16"))
        if not in_loop:
            assert st["fallback"] == 1, (d, prec, st)
        ref = orc.dbscan(pts, eps, mp)
        for a, b in zip(got, ref):
            np.testing.assert_array_equal(a, np.asarray(b).astype(a.dtype), err_msg=f"{prec} d={d}")


def test_served_precision_rejected_for_wide_d():
    with pkg.Server(max_slots=4) as srv:
        with pytest.raises(pkg.DbscanError) as ei:
            srv.submit(_gpu(np.zeros((100, 100), np.float32)), 1.0, 3, precision="fp16")
        assert ei.value.code == pkg._lib.DBSCAN_E_UNSUPPORTED


def test_served_overflow_moves_to_a_worker():
    """A small job whose pair list overflows in the persistent loop moves to
    a worker (the loop thread never runs it itself), beside a large job on
    another worker; the small jobs submitted after them run in the loop, and
    every output equals the oracle's."""
    big = wl.mix64d_300k(0, n=100_000, eps_rule="q50")
    rng = np.random.default_rng(4)
    dense = rng.uniform(0, 1, size=(8000, 3)).astype(np.float32)  # eps 5: pair list overflows
    small = _mixed_jobs(16, seed=41, n_max=3000)
    with pkg.Server(max_slots=32) as srv:
        jb = srv.submit(_gpu(big.points), big.eps, big.minpts, precision="fp32")
        jd = srv.submit(_gpu(dense), 5.0, 3)
        ids = [srv.submit(_gpu(p), eps, mp) for p, eps, mp in small]
        sts = [srv.wait(i, timeout=120) for i in ids]
        sb, sd = srv.wait(jb, timeout=120), srv.wait(jd, timeout=120)
        outs = [_host(srv.outputs(i)) for i in ids]
        od = _host(srv.outputs(jd))
        ob = _host(srv.outputs(jb))
    assert sb["fallback"] == 1 and sd["fallback"] == 1
    assert sd["state"] == pkg._lib.JOB_DONE and sd["error"] == 0
    assert all(s["fallback"] == 0 and s["state"] == pkg._lib.JOB_DONE for s in sts)
    for (pts, eps, mp), got in zip(small, outs):
        np.testing.assert_array_equal(got[0], orc.dbscan(pts, eps, mp)[0])
    assert (od[0] == 0).all() and (od[2] == 8000).all()
    ref = c_oracle.dbscan(big.points, big.eps, big.minpts)
    for a, b in zip(ob, ref):
        np.testing.assert_array_equal(a, np.asarray(b).astype(a.dtype))


def test_finished_status_is_returned_once():
    pts = np.random.default_rng(1).uniform(0, 1, size=(500, 2)).astype(np.float32)
    with pkg.Server(max_slots=4) as srv:
        j = srv.submit(_gpu(pts), 0.05, 3)
        st = srv.wait(j, timeout=60)
        assert st["state"] == pkg._lib.JOB_DONE
        with pytest.raises(pkg.DbscanError) as ei:
            srv.poll(j)
        assert ei.value.code == pkg._lib.DBSCAN_E_INVAL
