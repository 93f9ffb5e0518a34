"""Parity of the HIP path against the oracle at every compiled FFT size and at the sizes the
product runs: H X on grids forced to 32 ... 192 (the stick and plane kernels compiled per size,
their LDS swizzles, the pencil form of 192^2 planes that do not fit in LDS, in FP64 and FP32),
a band-blocked step with uneven blocks on Si216, and the Rayleigh-Ritz step of the full Si512
block (the wide projection and Gram tiles) against the oracle's step.

Tolerances as in test_gpu_parity: H X 1e-12 relative (FP64), 2e-5 (FP32), 5e-5 (bf16-split
projector products); steps: eigenvalues 1e-10 Ha (FP64), 1e-5 Ha (mixed), residual norms 1e-9.
"""
import sys

import numpy as np
import pytest

from oracle import pw_oracle as O
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


# --- H X at every compiled FFT size (Si8 with the grid forced) --------------------------------
SIZES = [32, 48, 54, 81, 96, 128, 192]
CASES = []
for n in SIZES:
    CASES.append((n, pw.PW_FP64, 0, 1e-12))
    CASES.append((n, pw.PW_MIXED, 0, 2e-5))
for n in (81, 96, 192):
    CASES.append((n, pw.PW_MIXED, pw.PW_FLAG_BF16_KB, 5e-5))
for n in (81, 96):
    CASES.append((n, pw.PW_FP64, pw.PW_FLAG_PENCIL_FFT, 1e-12))
    CASES.append((n, pw.PW_MIXED, pw.PW_FLAG_PENCIL_FFT, 2e-5))


@pytest.mark.parametrize("n,prec,flags,tol", CASES)
def test_apply_h_forced_grid(n, prec, flags, tol):
    cell = synth.make_cell("si8", modes=True)
    nb = 3
    model = O.model_from_cell(cell, grid=(n, n, n))
    h = pw.Handle(cell, prec, nbands=nb, fft_n=(n, n, n), flags=flags)
    assert tuple(h.info.fft_n) == (n, n, n)
    say("apply_h grid", n, "prec", prec, "flags", flags, "fused planes", h.info.fused_planes)
    if flags & pw.PW_FLAG_PENCIL_FFT or n == 192:
        assert h.info.fused_planes == 0
    p = pw.permutation_to(model.miller, h.gvectors())
    X = synth.random_block(model.npw, nb, 1000 + n)
    if prec == pw.PW_MIXED:
        X = X.astype(np.complex64).astype(np.complex128)
    ref = O.apply_h(model, X)
    out = h.to_host(h.apply_h(h.to_device(X[p])))
    err = float(np.abs(out - ref[p]).max() / np.abs(ref).max())
    say("  rel err", err)
    assert err < tol
    h.close()


# --- band-blocked step with uneven blocks (Si216: 440 bands in blocks of 128, 128, 128, 56) ---
@pytest.fixture(scope="module")
def si216():
    cell = synth.silicon_cell((3, 3, 3), 10.0, disp_seed=synth.SEED_REQUEST + 3,
                              modes_seed=synth.SEED_MODES + 7)
    model = O.model_from_cell(cell)
    hop = lambda X: O.apply_h(model, X)
    X0 = synth.initial_block(model.miller, cell.L, cell.nbands, synth.SEED_X0 + 5)
    X0 = X0.astype(np.complex64).astype(np.complex128)  # the same input for both precisions
    b = 1.01 * O.lanczos_max(hop, model.npw, 20, seed=5)
    say("si216 oracle steps: npw", model.npw, "bands", cell.nbands)
    s1 = O.eig_step(hop, X0, 0, 0.0, 0.0, b)
    s2 = O.eig_step(hop, s1.X, 10, s1.a_lo, s1.a, b)
    return cell, model, X0, b, s1, s2


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec,flags,etol", [(pw.PW_FP64, 0, 1e-10), (pw.PW_MIXED, pw.PW_FLAG_BF16_ALL, 1e-5)])
def test_blocked_step_uneven_blocks_si216(si216, prec, flags, etol):
    cell, model, X0, b, s1, s2 = si216
    h = pw.Handle(cell, prec, flags=flags, filter_block=128)
    assert h.info.filter_block == 128 and cell.nbands == 440
    p = pw.permutation_to(model.miller, h.gvectors())
    inv = np.argsort(p)
    Xd = h.to_device(X0[p])
    e1, r1, _ = h.eig_step(Xd, 0, b=b)
    # the second step starts from the oracle's first iterate, so it tests one step alone
    Xd = h.to_device(s1.X[p].astype(np.complex64).astype(np.complex128) if prec == pw.PW_MIXED else s1.X[p])
    if prec == pw.PW_MIXED:
        t1 = O.eig_step(lambda X: O.apply_h(model, X), s1.X.astype(np.complex64).astype(np.complex128), 10,
                        s1.a_lo, s1.a, b)
    else:
        t1 = s2
    e2, r2, _ = h.eig_step(Xd, 10, s1.a_lo, s1.a, b)
    nocc = cell.nocc
    d1 = np.abs(e1 - s1.eig)[:nocc].max()
    d2 = np.abs(e2 - t1.eig)[:nocc].max()
    say("si216 blocked", prec, flags, "m=0", d1, "m=10", d2, "resid", np.abs(r2 - t1.resid).max())
    assert d1 < etol and d2 < etol
    if prec == pw.PW_FP64:
        assert np.abs(r1 - s1.resid).max() < 1e-9
        assert np.abs(r2 - t1.resid).max() < 1e-9
        Xg = h.to_host(Xd)[inv]
        for lo, hi in O.clusters(t1.eig):
            if hi >= cell.nbands:
                break
            assert O.subspace_sin(t1.X[:, lo:hi], Xg[:, lo:hi]) < 1e-8
    h.close()


# --- the full Si512 block: Rayleigh-Ritz step (wide projection / Gram tiles) vs the oracle -------
@pytest.fixture(scope="module")
def si512_rr():
    cell = synth.make_cell("si512")
    model = O.model_from_cell(cell, with_projectors=False)  # projectors applied atom by atom
    local = O.model_from_cell(cell, d0=0.0, d1=0.0)  # kinetic and local parts only
    X0 = synth.initial_block(model.miller, cell.L, cell.nbands, synth.SEED_X0 + 2)
    X0 = X0.astype(np.complex64).astype(np.complex128)
    # H X0 = (kinetic + local) X0, in column groups, + the nonlocal part, each atom's projectors
    # generated once for all columns
    W = O.apply_nonlocal_atomwise(model, X0, progress=lambda n: say("si512 oracle: nonlocal part,", n, "atoms"))
    say("si512 oracle: nonlocal part of H X0 done")
    for c0 in range(0, cell.nbands, 136):
        W[:, c0:c0 + 136] += O.apply_h(local, X0[:, c0:c0 + 136])
        say("si512 oracle: H X0 columns", c0, "to", min(cell.nbands, c0 + 136), "done")
    lam, C = O.rayleigh_ritz(X0, W)
    Xn = X0 @ C
    Wn = W @ C
    del W
    resid = np.sqrt((np.abs(Wn - Xn * lam[None, :]) ** 2).sum(axis=0))
    del Wn
    return cell, model, X0, lam, Xn, resid


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("prec,flags,etol", [(pw.PW_FP64, 0, 1e-10), (pw.PW_MIXED, pw.PW_FLAG_BF16_ALL, 1e-5),
                                             (pw.PW_MIXED, 0, 1e-5)])
def test_si512_rayleigh_ritz_step_vs_oracle(si512_rr, prec, flags, etol):
    cell, model, X0, lam, Xn, resid = si512_rr
    h = pw.Handle(cell, prec, flags=flags)
    p = pw.permutation_to(model.miller, h.gvectors())
    inv = np.argsort(p)
    Xd = h.to_device(X0[p])
    e, r, _ = h.eig_step(Xd, 0, b=1.0)
    nocc = cell.nocc
    d = np.abs(e - lam)[:nocc].max()
    dr = np.abs(r - resid).max() / resid.max()
    say("si512 RR step", prec, flags, "max |de| occ", d, "rel resid diff", dr)
    assert d < etol
    if prec == pw.PW_FP64:
        assert np.abs(r - resid).max() < 1e-9
        Xg = h.to_host(Xd)[inv]
        worst = 0.0
        for lo, hi in O.clusters(lam[: nocc + 1]):
            if hi > nocc:
                break
            worst = max(worst, O.subspace_sin(Xn[:, lo:hi], Xg[:, lo:hi]))
        say("  largest per-cluster sin angle", worst)
        assert worst < 1e-8
    h.close()


# --- the fused density on 128 x 128 FP32 planes (band groups summed in order) --------------------
@pytest.mark.parametrize("name,nb", [("si8", 1), ("si8", 37), ("si8", 80), ("si64", 144)])
def test_density_forced_grid_128(name, nb):
    """Grid forced to 128^3 in mixed precision: the fused density kernel against the oracle, 1e-5 of
    max rho.  Si8: one band group per plane written straight into rho (the work buffer cannot hold
    group sums), one or several batches; Si64: two band groups per plane summed in order, in more
    than one batch."""
    cell = synth.make_cell(name, modes=True)
    n = 128
    model = O.model_from_cell(cell, grid=(n, n, n), with_projectors=False)
    h = pw.Handle(cell, pw.PW_MIXED, nbands=max(nb, cell.nbands), fft_n=(n, n, n))
    assert h.info.fused_planes == 1
    p = pw.permutation_to(model.miller, h.gvectors())
    X = synth.random_block(model.npw, nb, 1300 + nb).astype(np.complex64).astype(np.complex128)
    occ = np.where(np.arange(nb) % 5 == 4, 0.0, 2.0) - 0.01 * np.arange(nb)
    ref = O.density(X, occ, model.miller, model.grid).transpose(2, 1, 0)
    rho = h.density(h.to_device(X[p]), occ).cpu().numpy()
    err = float(np.abs(rho - ref).max() / np.abs(ref).max())
    say("density 128^3 nb", nb, "rel err", err)
    assert err < 1e-5
