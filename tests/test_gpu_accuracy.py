"""Accuracy of the mixed-precision solve at convergence, per cluster of (nearly) degenerate
eigenvalues: principal angles against exact (dense) or FP64 eigenvectors stay within the
Davis-Kahan bound of the computed Ritz pairs, eigenvalues within 1e-5 Ha; after the FP64 polish
(FP64 steps started from the mixed block) eigenvalues agree to 1e-8 Ha and angles to 1e-6.
"""
import sys

import numpy as np
import pytest

from oracle import pw_oracle as O
from paper_2406_10765_amd import accuracy as acc
from paper_2406_10765_amd import pw, synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible device"
    pw.lib()
    return torch


def converge_pair(cell, flags, seed):
    """Mixed solve, the FP64 Rayleigh-Ritz on its span, and the FP64 polish from it."""
    import torch
    nb, nocc = cell.nbands, cell.nocc
    hm = pw.Handle(cell, pw.PW_MIXED, flags=flags)
    h64 = pw.Handle(cell, pw.PW_FP64)
    assert np.array_equal(hm.gvectors(), h64.gvectors())
    X0 = hm.random_block(nb, seed)
    Xm = X0.clone()
    em, rm, sm, cm = hm.solve(Xm, nocc, 5e-5, 10, 200)
    assert cm, "mixed solve did not converge"
    Y = Xm.to(torch.complex128)
    erep, rrep, _ = h64.eig_step(Y, 0, b=1.0)
    Xp = Y.clone()
    ep, rp, sp, cp = h64.solve(Xp, nocc, 1e-10, 10, 400)
    assert cp, "FP64 polish did not converge"
    return h64, X0, em, (h64.to_host(Y), erep, rrep), (h64.to_host(Xp), ep, rp, sp)


@pytest.mark.parametrize("flags", [pw.PW_FLAG_BF16_ALL, 0])
def test_si8_mixed_vs_dense_eigenvectors(flags):
    cell = synth.make_cell("si8")
    model = O.model_from_cell(cell)
    lam, V = np.linalg.eigh(O.dense_h(model))
    h64, _, em, (Am, erep, rrep), (Ap, ep, rp, sp) = converge_pair(cell, flags, 4242)
    p = pw.permutation_to(model.miller, h64.gvectors())
    Vg = V[p][:, : cell.nbands]
    nocc = cell.nocc
    zeros = np.zeros(cell.nbands)
    rows = acc.cluster_report(Am, erep, rrep, Vg, lam, zeros, nocc)
    rows_p = acc.cluster_report(Ap, ep, rp, Vg, lam, zeros, nocc)
    de = np.abs(em[:nocc] - lam[:nocc]).max()
    say("si8 flags", flags, "mixed |de|", de, "max angle", max(r[2] for r in rows), "max bound", max(r[3] for r in rows),
        "polish steps", sp, "|de|", np.abs(ep[:nocc] - lam[:nocc]).max(), "angle", max(r[2] for r in rows_p))
    assert de < 1e-5
    for lo, hi, ang, bound in rows:
        assert np.sin(ang) <= bound * (1 + 1e-6) + 1e-13, (lo, hi, ang, bound)
    assert np.abs(ep[:nocc] - lam[:nocc]).max() < 1e-8
    assert max(r[2] for r in rows_p) < 1e-6


def test_si64_mixed_vs_fp64_at_convergence():
    import torch
    cell = synth.make_cell("si64")
    nb, nocc = cell.nbands, cell.nocc
    h64, X0, em, (Am, erep, rrep), (Ap, ep, rp, sp) = converge_pair(cell, pw.PW_FLAG_BF16_ALL, 4343)
    X64 = X0.to(torch.complex128)
    e64, r64, s64, c64 = h64.solve(X64, nocc, 1e-10, 10, 400)
    assert c64
    A64 = h64.to_host(X64)
    rows = acc.cluster_report(Am, erep, rrep, A64, e64, r64, nocc)
    rows_p = acc.cluster_report(Ap, ep, rp, A64, e64, r64, nocc)
    de = np.abs(em[:nocc] - e64[:nocc]).max()
    say("si64 mixed |de|", de, "max angle", max(r[2] for r in rows), "max bound", max(r[3] for r in rows),
        "polish steps", sp, "of", s64, "|de|", np.abs(ep[:nocc] - e64[:nocc]).max(), "angle", max(r[2] for r in rows_p))
    assert de < 1e-5
    for lo, hi, ang, bound in rows:
        assert np.sin(ang) <= bound * (1 + 1e-6) + 1e-13, (lo, hi, ang, bound)
    assert np.abs(ep[:nocc] - e64[:nocc]).max() < 1e-8
    assert max(r[2] for r in rows_p) < 1e-6
    assert sp < s64  # the polish starts from a converged span
