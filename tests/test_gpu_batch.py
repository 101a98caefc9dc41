"""Batched filter over independent problems of uneven size, captured into a
HIP graph (pawfe_batch_*): every replay against the oracle's filter of each
problem, replays against each other with eager work and synchronization in
between, explicit and autotuned schedules, in place."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def problems():
    from oracle import chfsi
    from oracle.paw import PAWOperator
    from paper_2604_26037_amd import Operator
    from workloads.configs import batch_systems
    out = []
    for i, s in enumerate(batch_systems(4, small=True)):
        ref = PAWOperator(s)
        op = Operator(s)
        X = s.trial(s.nstates)
        Psi, lam, _ = chfsi.rayleigh_ritz(ref, X)
        t0, t1, beta = chfsi.lanczos_bounds(ref, k=20)
        bU = 1.02 * max(t1 + abs(beta), float(lam[-1])) + 1.0
        m = 5 + 2 * i                                   # uneven degrees
        b0, bW = float(lam[0]), float(lam[-1])
        want = chfsi.rchfsi_filter(ref, Psi, lam, m, b0, bW, bU, block=s.nstates)
        out.append(dict(s=s, ref=ref, op=op, Psi=Psi, lam=lam, m=m, b0=b0, bW=bW, bU=bU, want=want))
    return out


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _jobs(problems, block=None, inplace=False):
    jobs, keep = [], []
    for p in problems:
        X = _dev(p["Psi"])
        out = X if inplace else torch.empty_like(X)
        lam = _dev(p["lam"])
        j = dict(op=p["op"], X=X, out=out, lam=lam, degree=p["m"], b0=p["b0"], bW=p["bW"], bU=p["bU"])
        if block is not None:
            j["block"] = block
        jobs.append(j)
        keep.append((X, out, lam))
    return jobs, keep


def test_batch_graph_autotuned_vs_oracle_and_replays(problems):
    from paper_2604_26037_amd import Batch
    jobs, keep = _jobs(problems)
    b = Batch(jobs)                                     # block sizes and streams autotuned
    ns, blocks, sof = b.schedule()
    assert ns in (1, 2, 4)
    for j, p in enumerate(problems):
        n = p["s"].nstates
        assert 1 <= blocks[j] <= n and 0 <= sof[j] < ns
    b.run()
    torch.cuda.synchronize()
    first = [j["out"].cpu().numpy() for j in jobs]
    for got, p in zip(first, problems):
        assert _rel(got, p["want"]) < 1e-9
    for rep in range(3):
        # eager work and a synchronization between replays
        p0 = problems[0]
        p0["op"].apply_H(_dev(p0["Psi"]))
        torch.cuda.synchronize()
        for j in jobs:
            j["out"].zero_()
        b.run()
        torch.cuda.synchronize()
        for got, j in zip(first, jobs):
            np.testing.assert_array_equal(j["out"].cpu().numpy(), got)
    b.close()


def test_batch_graph_fixed_schedule_fp32(problems):
    from paper_2604_26037_amd import FP32, Batch
    jobs, keep = _jobs(problems, block=5)             # ragged blocks
    b = Batch(jobs, prec=FP32, nstreams=2)
    ns, blocks, _ = b.schedule()
    assert ns == 2 and all(int(x) == 5 for x in blocks)
    b.run()
    torch.cuda.synchronize()
    for j, p in zip(jobs, problems):
        assert _rel(j["out"].cpu().numpy(), p["want"]) < 1e-4
    b.close()


def test_batch_graph_in_place(problems):
    from paper_2604_26037_amd import Batch
    jobs, keep = _jobs(problems, inplace=True)
    b = Batch(jobs, nstreams=1)
    for j, p in zip(jobs, problems):                   # tuning runs never touch the jobs' buffers
        np.testing.assert_array_equal(j["X"].cpu().numpy(), p["Psi"])
    b.run()
    torch.cuda.synchronize()
    for j, p in zip(jobs, problems):
        assert _rel(j["X"].cpu().numpy(), p["want"]) < 1e-9
    b.close()


def test_batch_one_graph_per_job(problems):
    """A launch budget below any one job's filter puts every job into a graph
    of its own; the replay (graphs in order) equals the oracle's filters and
    replays are bit-identical."""
    from paper_2604_26037_amd import Batch
    jobs, keep = _jobs(problems)
    b = Batch(jobs, nstreams=2, max_graph_launches=1)
    assert b.ngraphs == len(jobs)
    b.run()
    torch.cuda.synchronize()
    first = [j["out"].cpu().numpy() for j in jobs]
    for got, p in zip(first, problems):
        assert _rel(got, p["want"]) < 1e-9
    for j in jobs:
        j["out"].zero_()
    b.run()
    torch.cuda.synchronize()
    for got, j in zip(first, jobs):
        np.testing.assert_array_equal(j["out"].cpu().numpy(), got)
    b.close()


def test_batch_default_budget_one_graph(problems):
    """Small batches stay within the default launch budget: one graph."""
    from paper_2604_26037_amd import Batch
    jobs, keep = _jobs(problems)
    b = Batch(jobs, nstreams=1)
    assert b.ngraphs == 1
    b.close()


@pytest.fixture(scope="module")
def wide_problems():
    """Jobs of 64, 128 and 192 states, so the autotuner times several block
    sizes per job (64, 128, then the job's own width)."""
    from oracle import chfsi
    from oracle.paw import PAWOperator
    from paper_2604_26037_amd import Operator
    from workloads.configs import custom_system
    specs = [((3, 3, 3), 3, 64, [(1.1, 2.0, 0.7)]), ((3, 3, 3), 4, 128, [(2.0, 1.0, 2.6)]),
             ((4, 3, 3), 4, 192, [(1.0, 1.2, 1.3), (3.9, 2.6, 2.4)])]
    out = []
    for i, (n, p, nst, pos) in enumerate(specs):
        box = tuple(1.25 * v for v in n)
        s = custom_system(n, box, p, p + 2, pos=pos, rcut=1.0, channels="spd8",
                          wells=[(0.5, 0.5, 0.5), (2.0, 2.5, 1.0)], s_H=0.5, s_S=0.4, seed=40 + i,
                          nstates=nst)
        ref = PAWOperator(s)
        op = Operator(s)
        X = s.trial(nst)
        Psi, lam, _ = chfsi.rayleigh_ritz(ref, X)
        t0, t1, beta = chfsi.lanczos_bounds(ref, k=20)
        bU = 1.02 * max(t1 + abs(beta), float(lam[-1])) + 1.0
        m = 4 + i
        b0, bW = float(lam[0]), float(lam[-1])
        want = chfsi.rchfsi_filter(ref, Psi, lam, m, b0, bW, bU, block=nst)
        out.append(dict(s=s, ref=ref, op=op, Psi=Psi, lam=lam, m=m, b0=b0, bW=bW, bU=bU, want=want))
    return out


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_autotuned_several_block_candidates(wide_problems, prec):
    """Jobs with 64 or more states: the autotuner times several block sizes on
    one job workspace, and each filter of the batch gets one block state of its
    own block size, so it keeps all blocks on the job's stream.  Every job's
    result matches the oracle's filter (FP64 1e-9, FP32 1e-4) on the first
    replay and bit-identically on the next."""
    from paper_2604_26037_amd import FP32, FP64, Batch
    jobs, keep = _jobs(wide_problems)
    b = Batch(jobs, prec=FP64 if prec == "fp64" else FP32)
    ns, blocks, sof = b.schedule()
    for j, p in enumerate(wide_problems):
        n = p["s"].nstates
        assert int(blocks[j]) in {c for c in (64, 128, 256) if c <= n} | {n}
    tol = 1e-9 if prec == "fp64" else 1e-4
    for rep in range(2):
        for j in jobs:
            j["out"].zero_()
        b.run()
        torch.cuda.synchronize()
        got = [j["out"].cpu().numpy() for j in jobs]
        if rep == 0:
            first = got
            for g, p in zip(got, wide_problems):
                assert _rel(g, p["want"]) < tol
        else:
            for g, f in zip(got, first):
                np.testing.assert_array_equal(g, f)
    b.close()


def test_batch_tuning_cache_round_trip(wide_problems, tmp_path):
    """A batch tuned once, its decisions saved to a file, the table cleared
    and loaded again: the second batch times nothing, keeps the schedule and
    matches the oracle's filters."""
    from paper_2604_26037_amd import FP64, Batch, tune_cache_clear, tune_cache_load, tune_cache_save
    tune_cache_clear()
    jobs, keep = _jobs(wide_problems)
    b1 = Batch(jobs, prec=FP64)
    assert b1.tuning_runs > 0
    s1 = b1.schedule()
    b1.close()
    path = str(tmp_path / "tune.cache")
    tune_cache_save(path)
    tune_cache_clear()
    tune_cache_load(path)
    jobs2, keep2 = _jobs(wide_problems)
    b2 = Batch(jobs2, prec=FP64)
    assert b2.tuning_runs == 0
    s2 = b2.schedule()
    assert s1[0] == s2[0]
    np.testing.assert_array_equal(s1[1], s2[1])
    np.testing.assert_array_equal(s1[2], s2[2])
    b2.run()
    torch.cuda.synchronize()
    for j, p in zip(jobs2, wide_problems):
        assert _rel(j["out"].cpu().numpy(), p["want"]) < 1e-9
    b2.close()
    tune_cache_clear()
