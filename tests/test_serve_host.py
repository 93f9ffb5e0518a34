"""Scheduler logic of the request loop, on the CPU (dry-run executor: no device work)."""
import time

import numpy as np
import pytest

from paper_2406_10765_amd import pw, synth


def wait_all(srv, tickets, nb, timeout=20.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t not in out:
                r = srv.poll(t, nb)
                if r is not None:
                    out[t] = r
        assert time.time() - t0 < timeout
        time.sleep(0.002)
    return out


def small_cell(i):
    return synth.silicon_cell((1, 1, 1), 10.0, disp_seed=100 + i)


def footprint(cell):
    info = pw.plan(cell, pw.PW_MIXED)
    ld = (info.npw + 15) // 16 * 16
    return ((info.footprint_bytes + 255) // 256 * 256) + ((cell.nbands * ld * 8 + 255) // 256 * 256)


def test_all_requests_complete_fcfs_and_slots():
    srv = pw.Server(1 << 34, max_slots=2, dry_run=True)
    cells = [small_cell(i) for i in range(8)]
    tickets = [srv.submit(c, seed=i) for i, c in enumerate(cells)]
    res = wait_all(srv, tickets, cells[0].nbands)
    admits = [res[t]["t_admit"] for t in tickets]
    assert admits == sorted(admits)  # first come, first served
    iv = [(res[t]["t_admit"], res[t]["t_done"]) for t in tickets]
    for a, _ in iv:  # never more than two running at once
        assert sum(1 for s, e in iv if s <= a < e) <= 2
    assert all(res[t]["status"] == pw.PW_OK for t in tickets)
    srv.close()


def test_admission_by_footprint_serialises_requests():
    cell = small_cell(0)
    need = footprint(cell)
    srv = pw.Server(int(need * 1.5), max_slots=4, dry_run=True)  # room for one request at a time
    tickets = [srv.submit(small_cell(i), seed=i) for i in range(4)]
    res = wait_all(srv, tickets, cell.nbands)
    iv = sorted((res[t]["t_admit"], res[t]["t_done"]) for t in tickets)
    for (s0, e0), (s1, e1) in zip(iv, iv[1:]):
        assert s1 >= e0
    srv.close()


def test_request_larger_than_arena_is_rejected():
    srv = pw.Server(1 << 20, max_slots=1, dry_run=True)
    with pytest.raises(pw.PWError) as ei:
        srv.submit(small_cell(0))
    assert ei.value.status == pw.PW_ENOMEM
    srv.close()


def test_bad_requests_and_poll_semantics():
    srv = pw.Server(1 << 34, max_slots=1, dry_run=True)
    with pytest.raises(pw.PWError):
        srv.submit(small_cell(0), tol=-1.0)
    bad = synth.Cell(L=(10.26,) * 3, tau=np.zeros((1, 3)), ecut=10.0, nbands=4,
                     modes=synth.Modes(np.array([[1, 0, 0]]), np.array([np.nan]), np.array([0.0])))
    with pytest.raises(pw.PWError) as ei:
        srv.submit(bad)
    assert ei.value.status == pw.PW_EINVAL
    t = srv.submit(small_cell(1), t_arrive=0.0)
    r = wait_all(srv, [t], small_cell(1).nbands)[t]
    assert r["t_arrive"] == 0.0 and r["t_admit"] >= 0.0 and r["t_done"] >= r["t_admit"]
    with pytest.raises(pw.PWError):  # a result is handed out once
        srv.poll(t, 4)
    srv.close()


def test_serving_mix_recipe():
    mix = synth.serving_mix(40, 20.0)
    assert len(mix) == 40
    t = np.array([m["t_arrive"] for m in mix])
    assert np.all(np.diff(t) > 0)
    assert {m["name"] for m in mix} <= set(synth.SERVING_CELLS)
    for m in mix:
        assert m["cell"].nbands == 2 * m["cell"].natoms + 8
        assert m["cell"].ecut in (10.0, 15.0, 20.0)


def _need(cell):
    return footprint(cell)


def test_concurrent_submitters_respect_slots_and_arena():
    """Six client threads submit 30 requests of two sizes at once into an arena that holds only a
    few: at every instant the admitted requests fit the arena and the slots, and all complete."""
    import threading

    small = [synth.silicon_cell((1, 1, 1), 10.0, disp_seed=300 + i) for i in range(15)]
    large = [synth.silicon_cell((1, 1, 1), 20.0, disp_seed=400 + i) for i in range(15)]
    cells = [c for pair in zip(small, large) for c in pair]
    arena = int(2.5 * _need(large[0]))
    srv = pw.Server(arena, max_slots=4, dry_run=True)
    tickets = [None] * len(cells)

    def client(k):
        for i in range(k, len(cells), 6):
            tickets[i] = srv.submit(cells[i], seed=i)

    th = [threading.Thread(target=client, args=(k,)) for k in range(6)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    out = {}
    t0 = time.time()
    while len(out) < len(cells):
        for i, t in enumerate(tickets):
            if i not in out:
                r = srv.poll(t, cells[i].nbands)
                if r is not None:
                    out[i] = r
        assert time.time() - t0 < 30
        time.sleep(0.002)
    srv.close()
    assert all(r["status"] == pw.PW_OK and r["message"] == "" and r["retried"] == 0 for r in out.values())
    iv = [(out[i]["t_admit"], out[i]["t_done"], _need(cells[i])) for i in range(len(cells))]
    for a, _, _ in iv:
        running = [(s, e, n) for s, e, n in iv if s <= a < e]
        assert len(running) <= 4
        assert sum(n for _, _, n in running) <= arena


def test_small_requests_pass_a_large_head_a_bounded_number_of_times():
    """A request that does not fit yet is passed by later, smaller ones, but only 16 times."""
    big = synth.silicon_cell((1, 1, 2), 20.0, disp_seed=7)
    small = [synth.silicon_cell((1, 1, 1), 10.0, disp_seed=500 + i) for i in range(40)]
    nb_big, ns = _need(big), _need(small[0])
    assert nb_big > 2 * ns
    arena = nb_big + ns // 2  # the big one fits only when nothing else runs
    srv = pw.Server(arena, max_slots=2, dry_run=True)
    first = [srv.submit(small[i], seed=i) for i in range(2)]
    tb = srv.submit(big, seed=99)
    rest = [srv.submit(small[i], seed=i) for i in range(2, 40)]
    res = wait_all(srv, first + [tb] + rest, big.nbands, timeout=60)
    srv.close()
    t_big = res[tb]["t_admit"]
    passed = [t for t in rest if res[t]["t_admit"] < t_big]
    assert res[tb]["status"] == pw.PW_OK
    assert 1 <= len(passed) <= 16
    # the ones behind it that did not pass were admitted after it
    assert all(res[t]["t_admit"] >= t_big for t in rest if t not in passed)
