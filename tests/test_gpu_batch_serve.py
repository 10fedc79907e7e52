"""GPU parity of the batched and served forms: every lattice, swept in shared
launches (graph-replayed chunks) or as a job among others in the server, must
follow exactly the trajectory the oracle computes for it alone."""
import sys

import numpy as np
import pytest

import oracle

sw = pytest.importorskip("paper_1403_7560_amd")
pytestmark = pytest.mark.gpu

from test_gpu_parity import compare_lattice, compare_records  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


MIX = [
    dict(model=0, dim=2, L=70, q=2, beta=0.44, seed=11, replica=0),
    dict(model=1, dim=3, L=20, q=4, beta=0.6, seed=12, replica=1),
    dict(model=2, dim=2, L=40, q=0, beta=1.1, seed=13, replica=2),
    dict(model=0, dim=3, L=17, q=2, beta=0.22, seed=14, replica=0),
    dict(model=1, dim=2, L=130, q=3, beta=1.0, seed=15, replica=0),
    dict(model=2, dim=3, L=9, q=0, beta=0.45, seed=16, replica=5),
    dict(model=0, dim=2, L=64, q=2, beta=0.44, seed=11, replica=1),
]


def oracle_run(j, n):
    s0 = oracle.init_state(j["model"], j["dim"], j["L"], j["q"], j["seed"], j["replica"])
    return oracle.sweeps(j["model"], j["dim"], j["L"], j["q"], j["beta"], j["seed"], j["replica"],
                         0, n, s0)


@pytest.mark.parametrize("chunk", [1, 4, 16])
def test_batch_matches_oracle(chunk):
    say(f"[batch] chunk={chunk}")
    b = sw.Batch(MIX)
    b.set_chunk(chunk)
    b.sweep(3)
    b.sweep(4)
    for j, m in zip(MIX, b.members):
        ref = oracle_run(j, 7)
        compare_lattice(j["model"], m.get_state(), m.get_labels(), m.get_bonds(), ref)
        compare_records(j["model"], j["dim"], j["L"], j["q"], m.series(), ref["records"])
        assert m.sweep_index() == 7
    b.close()


def test_batch_uneven_counts():
    say("[batch] uneven counts")
    b = sw.Batch(MIX)
    b.set_chunk(4)
    counts = [0, 1, 9, 3, 5, 6, 2]
    b.sweep_counts(counts)
    for j, m, n in zip(MIX, b.members, counts):
        if n == 0:
            assert m.sweep_index() == 0
            continue
        ref = oracle_run(j, n)
        compare_lattice(j["model"], m.get_state(), m.get_labels(), m.get_bonds(), ref)
    b.close()


def test_server_jobs_match_oracle():
    say("[serve] 10 jobs under a small budget")
    jobs = []
    for k in range(10):
        j = dict(MIX[k % len(MIX)])
        j["seed"] = 100 + k
        j["sweeps"] = 3 + (k * 5) % 11
        jobs.append(j)
    # budget for about three of the larger jobs at once
    budget = 3 * max(sw.footprint(j["model"], j["dim"], j["L"], j["q"]) for j in jobs)
    srv = sw.Server(budget, max_active=4, chunk=4)
    ids = [srv.submit(j["model"], j["dim"], j["L"], j["q"], j["beta"], j["seed"], j["replica"],
                      j["sweeps"]) for j in jobs]
    left = len(jobs)
    steps = 0
    while left > 0:
        left = srv.step()
        steps += 1
        assert steps < 200
    for i, j in zip(ids, jobs):
        r = srv.poll(i, j["model"], j["L"] ** j["dim"])
        assert r is not None and r["status"] == 0 and r["sweeps"] == j["sweeps"]
        ref = oracle_run(j, j["sweeps"])
        st = r["state"]
        if j["model"] == 2:
            d = np.abs(st.astype(np.float64) - ref["state"])
            assert np.minimum(d, 2 * np.pi - d).max() < 1e-5
        else:
            np.testing.assert_array_equal(st, ref["state"])
        N = j["L"] ** j["dim"]
        rec = ref["records"]
        m2 = (rec["mx"] / N) ** 2 if j["model"] == 0 else (
            rec["mx"] / N ** 2 if j["model"] == 1 else (rec["mx"] ** 2 + rec["my"] ** 2) / N ** 2)
        assert r["m2"] == pytest.approx(m2.mean(), rel=1e-9)
        assert r["energy"] == pytest.approx(rec["energy"].mean() / N, rel=1e-9, abs=1e-12)
        assert r["finish_s"] >= r["start_s"] >= r["submit_s"]
    with pytest.raises(sw.SWError):
        srv.submit(0, 2, 4096, 2, 0.4, 1, 0, 10)  # larger than the whole budget
    srv.close()


def test_streams_do_not_change_results():
    """A batch on one stream or three, a server on one stream or three: the
    same trajectories as the oracle."""
    say("[streams] batch of the mix on 1 and 3 streams")
    for ns in (1, 3):
        b = sw.Batch(MIX)
        b.set_streams(ns)
        b.sweep(4)
        for j, m in zip(MIX, b.members):
            compare_lattice(j["model"], m.get_state(), m.get_labels(), m.get_bonds(), oracle_run(j, 4))
        b.close()
    say("[streams] server of 8 jobs on 1 and 3 streams")
    jobs = []
    for k in range(8):
        j = dict(MIX[k % len(MIX)])
        j["seed"] = 300 + k
        j["sweeps"] = 2 + k % 5
        jobs.append(j)
    for ns in (1, 3):
        srv = sw.Server(1 << 34, max_active=5, chunk=3)
        srv.set_streams(ns)
        ids = [srv.submit(j["model"], j["dim"], j["L"], j["q"], j["beta"], j["seed"], j["replica"], j["sweeps"])
               for j in jobs]
        steps = 0
        while srv.step() > 0:
            steps += 1
            assert steps < 100
        for i, j in zip(ids, jobs):
            r = srv.poll(i, j["model"], j["L"] ** j["dim"])
            assert r["status"] == 0 and r["sweeps"] == j["sweeps"]
            ref = oracle_run(j, j["sweeps"])
            if j["model"] == 2:
                d = np.abs(r["state"].astype(np.float64) - ref["state"])
                assert np.minimum(d, 2 * np.pi - d).max() < 1e-5
            else:
                np.testing.assert_array_equal(r["state"], ref["state"])
        with pytest.raises(sw.SWError):
            srv.set_streams(9)
        srv.close()


def test_server_cancel():
    """A job cancelled while it runs keeps the sweeps it ran (state and
    averages as the oracle's after them); one cancelled in the queue never
    runs; the others finish as if alone."""
    say("[serve] cancel a running and a queued job")
    jobs = []
    for k in range(4):
        j = dict(MIX[k])
        j["seed"] = 500 + k
        j["sweeps"] = 10
        jobs.append(j)
    srv = sw.Server(1 << 34, max_active=2, chunk=3)
    ids = [srv.submit(j["model"], j["dim"], j["L"], j["q"], j["beta"], j["seed"], j["replica"], j["sweeps"])
           for j in jobs]
    srv.step()  # admits jobs 0 and 1
    srv.step()  # runs their first 3 sweeps
    assert srv.cancel(ids[0]) is True
    assert srv.cancel(ids[3]) is True
    assert srv.cancel(ids[0]) is False
    with pytest.raises(sw.SWError) as e:
        srv.cancel(12345)
    assert e.value.code == -6
    j0 = jobs[0]
    r = srv.poll(ids[0], j0["model"], j0["L"] ** j0["dim"])
    assert r["status"] == -7 and r["sweeps"] == 3
    ref = oracle_run(j0, 3)
    np.testing.assert_array_equal(r["state"], ref["state"])
    N = j0["L"] ** j0["dim"]
    assert r["m2"] == pytest.approx(np.mean((ref["records"]["mx"] / N) ** 2), rel=1e-9)
    r3 = srv.poll(ids[3])
    assert r3["status"] == -7 and r3["sweeps"] == 0
    steps = 0
    while srv.step() > 0:
        steps += 1
        assert steps < 100
    for i in (1, 2):
        j = jobs[i]
        r = srv.poll(ids[i], j["model"], j["L"] ** j["dim"])
        assert r["status"] == 0 and r["sweeps"] == 10
        ref = oracle_run(j, 10)
        if j["model"] == 2:
            d = np.abs(r["state"].astype(np.float64) - ref["state"])
            assert np.minimum(d, 2 * np.pi - d).max() < 1e-5
        else:
            np.testing.assert_array_equal(r["state"], ref["state"])
    srv.close()
