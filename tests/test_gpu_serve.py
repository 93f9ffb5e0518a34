"""Request loop on the device: results are identical alone and in a concurrent mix, converge
to the oracle's dense eigenvalues, and a failing request fails alone."""
import sys
import time

import numpy as np
import pytest

from oracle import pw_oracle as O
from paper_2406_10765_amd import pw, synth

pytestmark = pytest.mark.gpu
FLAGS = pw.PW_FLAG_BF16_ALL


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def requests():
    out = []
    # Si8 and Si16 at each cutoff, then a Si64 and a Si216 cell (the latter on the 81-point grid)
    for i, (nc, ec) in enumerate([((1, 1, 1), 10.0), ((1, 1, 2), 10.0), ((1, 1, 1), 15.0), ((1, 1, 1), 20.0),
                                  ((1, 1, 2), 15.0), ((1, 1, 1), 10.0), ((2, 2, 2), 10.0), ((3, 3, 3), 15.0)]):
        out.append((synth.silicon_cell(nc, ec, disp_seed=synth.SEED_REQUEST + i), synth.SEED_REQUEST + i))
    return out


def run(srv, reqs, **kw):
    tickets = [srv.submit(c, pw.PW_MIXED, FLAGS, seed=s, tol=1e-4, nconv=c.nocc, **kw) for c, s in reqs]
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t, (c, _) in zip(tickets, reqs):
            if t not in out:
                r = srv.poll(t, c.nbands)
                if r is not None:
                    out[t] = r
        assert time.time() - t0 < 240
        time.sleep(0.005)
    return [out[t] for t in tickets]


def test_alone_equals_mix_and_dense():
    import torch
    assert torch.cuda.is_available()
    reqs = requests()
    say("cells", [(c.natoms, c.ecut, c.nbands) for c, _ in reqs])
    srv = pw.Server(8 << 30, max_slots=4)
    mix = run(srv, reqs)
    srv.close()
    say("mix steps", [r["steps"] for r in mix], "status", [r["status"] for r in mix])
    srv1 = pw.Server(8 << 30, max_slots=1)
    alone = []
    for q in reqs:
        alone += run(srv1, [q])
    srv1.close()
    say("alone steps", [r["steps"] for r in alone])
    for a, b in zip(mix, alone):
        assert a["status"] == pw.PW_OK and b["status"] == pw.PW_OK
        assert np.array_equal(a["eig"], b["eig"])
        assert a["steps"] == b["steps"]
    # the two Si8 E_cut = 10 requests against the dense oracle
    for k in (0, 5):
        cell = reqs[k][0]
        lam = np.linalg.eigvalsh(O.dense_h(O.model_from_cell(cell)))
        d = np.abs(mix[k]["eig"][: cell.nocc] - lam[: cell.nocc]).max()
        say("request", k, "max |de| vs dense", d)
        assert d < 1e-5


def test_non_converging_request_fails_alone():
    reqs = requests()[:3]
    srv = pw.Server(8 << 30, max_slots=3)
    c0, s0 = reqs[0]
    t_bad = srv.submit(c0, pw.PW_MIXED, FLAGS, seed=s0, tol=1e-12, max_steps=2, nconv=c0.nocc)
    good = run(srv, reqs[1:])
    while True:
        r = srv.poll(t_bad, c0.nbands)
        if r is not None:
            break
        time.sleep(0.005)
    srv.close()
    assert r["status"] == pw.PW_ENOTCONV and r["steps"] == 2
    assert all(g["status"] == pw.PW_OK for g in good)
