"""Parity of the HIP path (through the C ABI) against the CPU FP64 oracle.

Tolerances:
  FP64 H application: 1e-12 relative to max|HX| (double rounding of an FFT of length
    <= 192 and of K <= 1e4-term sums stays below 1e-14 relative; 100x margin).
  Mixed H application: 2e-5 relative to max|HX| (fp32 unit roundoff 6e-8 times the
    log2 N FFT depth and the sqrt(K) growth of the projector sums; the oracle gets
    the same fp32-rounded input).
  FP64 step: eigenvalues 1e-10 Ha, residual norms 1e-9; mixed step: eigenvalues 1e-5 Ha.
"""
import math
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


@pytest.fixture(scope="module")
def si8_dense():
    cell = synth.make_cell("si8")
    model = O.model_from_cell(cell)
    lam, V = np.linalg.eigh(O.dense_h(model))
    return cell, model, lam, V


def to_gpu_order(h, model):
    """p with model.miller[p] == gpu miller (oracle row p[i] is GPU row i)."""
    return pw.permutation_to(model.miller, h.gvectors())


def apply_case(cell, prec, nb, seed, flags=0):
    model = O.model_from_cell(cell)
    h = pw.Handle(cell, prec, nbands=max(nb, 1), flags=flags)
    p = to_gpu_order(h, model)
    X = synth.random_block(model.npw, nb, seed)
    if prec == pw.PW_MIXED:
        X = X.astype(np.complex64).astype(np.complex128)
    ref = O.apply_h(model, X)
    out = h.to_host(h.apply_h(h.to_device(X[p])))
    err = float(np.abs(out - ref[p]).max() / np.abs(ref).max())
    return err, h


@pytest.mark.parametrize("name,modes,nb", [("si8", False, 20), ("si8", True, 5), ("si64", True, 7)])
def test_apply_h_fp64(name, modes, nb):
    say("apply_h fp64", name, modes, nb)
    err, h = apply_case(synth.make_cell(name, modes=modes), pw.PW_FP64, nb, 100 + nb)
    say("  rel err", err)
    assert err < 1e-12


@pytest.mark.parametrize("name,modes,nb", [("si8", True, 20), ("si64", True, 9)])
def test_apply_h_mixed(name, modes, nb):
    say("apply_h mixed", name, modes, nb)
    err, h = apply_case(synth.make_cell(name, modes=modes), pw.PW_MIXED, nb, 200 + nb)
    say("  rel err", err)
    assert err < 2e-5


@pytest.mark.parametrize("prec,tol", [(pw.PW_FP64, 1e-12), (pw.PW_MIXED, 2e-5)])
def test_apply_h_pencil_fft(prec, tol):
    say("apply_h pencil", prec)
    err, h = apply_case(synth.make_cell("si8", modes=True), prec, 3, 300, flags=pw.PW_FLAG_PENCIL_FFT)
    assert h.info.fused_planes == 0
    say("  rel err", err)
    assert err < tol


def test_apply_h_radix3_grid():
    # E_cut = 15 Ha on one cubic cell gives a 27^3 grid (radix 3 only); 1 x 1 x 2 cells a 27 x 27 x 54 grid
    for cell in (synth.silicon_cell((1, 1, 1), 15.0, nbands=6, disp_seed=5),
                 synth.silicon_cell((1, 1, 2), 15.0, nbands=6, disp_seed=6)):
        say("apply_h radix-3", cell.L, cell.ecut)
        err, h = apply_case(cell, pw.PW_FP64, 6, 400)
        assert tuple(h.info.fft_n)[0] == 27
        say("  rel err", err)
        assert err < 1e-12


def test_apply_h_hermitian(gpu):
    cell = synth.make_cell("si8", modes=True)
    h = pw.Handle(cell, pw.PW_FP64, nbands=2)
    X = synth.random_block(h.npw, 2, 7)
    HX = h.to_host(h.apply_h(h.to_device(X)))
    lhs = np.vdot(X[:, 0], HX[:, 1])
    rhs = np.conj(np.vdot(X[:, 1], HX[:, 0]))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_step_parity_fp64_si8(si8_dense):
    cell, model, lam, V = si8_dense
    h = pw.Handle(cell, pw.PW_FP64)
    p = to_gpu_order(h, model)
    inv = np.argsort(p)
    hop = lambda X: O.apply_h(model, X)
    X0g = synth.initial_block(h.gvectors(), cell.L, cell.nbands, synth.SEED_X0)
    X0o = X0g[inv]
    b = 1.01 * lam[-1]
    Xd = h.to_device(X0g)
    e1, r1, bnd1 = h.eig_step(Xd, 0, b=b)
    s1 = O.eig_step(hop, X0o, 0, 0.0, 0.0, b)
    say("step m=0 max |de|", np.abs(e1 - s1.eig).max(), "max |dr|", np.abs(r1 - s1.resid).max())
    assert np.abs(e1 - s1.eig).max() < 1e-10
    assert np.abs(r1 - s1.resid).max() < 1e-9
    e2, r2, bnd2 = h.eig_step(Xd, 10, s1.a_lo, s1.a, b)
    s2 = O.eig_step(hop, s1.X, 10, s1.a_lo, s1.a, b)
    say("step m=10 max |de|", np.abs(e2 - s2.eig).max(), "max |dr|", np.abs(r2 - s2.resid).max())
    assert np.abs(e2 - s2.eig).max() < 1e-10
    assert np.abs(r2 - s2.resid).max() < 1e-9
    Xg = h.to_host(Xd)[inv]
    assert np.abs(Xg.conj().T @ Xg - np.eye(cell.nbands)).max() < 1e-12
    for lo, hi in O.clusters(s2.eig):
        if hi >= cell.nbands:
            break  # the top cluster may be cut by the block edge
        assert O.subspace_sin(s2.X[:, lo:hi], Xg[:, lo:hi]) < 1e-8
    assert bnd2[0] == e2[0] and bnd2[1] == e2[-1] and bnd2[2] == b


@pytest.mark.parametrize("prec", [pw.PW_FP64, pw.PW_MIXED])
def test_lanczos_bound_across_chunks(si8_dense, prec):
    """The Lanczos recurrence keeps its coefficients on the device and the host reads them once per
    chunk of 64 steps: runs that end inside, at and across chunk boundaries (up to the largest step
    count the call accepts) bound the top of the dense spectrum and repeat exactly."""
    cell, model, lam, V = si8_dense
    h = pw.Handle(cell, prec)
    for steps in (63, 64, 65, 130, 1000):
        b = h.spectrum_bound(steps, 1)
        say("lanczos steps", steps, "bound", b, "lam max", lam[-1])
        assert b >= lam[-1]
        assert h.spectrum_bound(steps, 1) == b


@pytest.mark.parametrize("prec,tol,etol", [(pw.PW_FP64, 1e-7, 1e-8), (pw.PW_MIXED, 1e-4, 1e-5)])
def test_solve_si8_matches_dense(si8_dense, prec, tol, etol):
    cell, model, lam, V = si8_dense
    h = pw.Handle(cell, prec)
    Xd = h.to_device(synth.initial_block(h.gvectors(), cell.L, cell.nbands, synth.SEED_X0))
    b = h.spectrum_bound(20, 1)
    say("lanczos bound", b, "lam max", lam[-1])
    assert b >= lam[-1]
    eig, res, steps, conv = h.solve(Xd, cell.nocc, tol, degree=10, b=b)
    say("solve prec", prec, "steps", steps, "max |de| occ", np.abs(eig[: cell.nocc] - lam[: cell.nocc]).max())
    assert conv
    assert np.abs(eig[: cell.nocc] - lam[: cell.nocc]).max() < etol


def test_empty_lattice_gpu():
    cell0 = synth.make_cell("si8")
    cell = synth.Cell(L=cell0.L, tau=cell0.tau, ecut=cell0.ecut, nbands=33,
                      pseudo=synth.Pseudo(zval=0.0, gauss_c=0.0, d0=0.0, d1=0.0))
    h = pw.Handle(cell, pw.PW_FP64)
    assert h.info.nproj == 0
    Xd = h.to_device(synth.initial_block(h.gvectors(), cell.L, 33, 11))
    kin = 0.5 * ((2 * np.pi * h.gvectors() / np.asarray(cell.L)) ** 2).sum(axis=1)
    eig, res, steps, conv = h.solve(Xd, 27, 1e-9, degree=10, b=1.01 * kin.max())
    unit = 0.5 * (2 * np.pi / cell.L[0]) ** 2
    expect = unit * np.array([0] + [1] * 6 + [2] * 12 + [3] * 8, float)
    assert conv
    assert np.abs(eig[:27] - expect).max() < 1e-12


def test_step_parity_si64():
    cell = synth.make_cell("si64")
    model = O.model_from_cell(cell)
    hop = lambda X: O.apply_h(model, X)
    for prec, etol in ((pw.PW_FP64, 1e-10), (pw.PW_MIXED, 1e-5)):
        h = pw.Handle(cell, prec)
        p = to_gpu_order(h, model)
        inv = np.argsort(p)
        X0g = synth.initial_block(h.gvectors(), cell.L, cell.nbands, synth.SEED_X0 + 1)
        if prec == pw.PW_FP64:
            b = 1.01 * O.lanczos_max(hop, model.npw, 20, seed=3)
            s1 = O.eig_step(hop, X0g[inv], 0, 0.0, 0.0, b)
            s2 = O.eig_step(hop, s1.X, 10, s1.a_lo, s1.a, b)
        Xd = h.to_device(X0g)
        e1, r1, _ = h.eig_step(Xd, 0, b=b)
        e2, r2, _ = h.eig_step(Xd, 10, s1.a_lo, s1.a, b)
        d1 = np.abs(e1 - s1.eig)[: cell.nocc].max()
        d2 = np.abs(e2 - s2.eig)[: cell.nocc].max()
        say("si64 prec", prec, "m=0", d1, "m=10", d2, "resid", np.abs(r2 - s2.resid).max())
        assert d1 < etol and d2 < etol
        if prec == pw.PW_FP64:
            assert np.abs(r2 - s2.resid).max() < 1e-9
        h.close()


def test_rank_deficient_block_reports_enotpd():
    cell = synth.make_cell("si8")
    h = pw.Handle(cell, pw.PW_FP64)
    X = synth.initial_block(h.gvectors(), cell.L, cell.nbands, 3)
    X[:, 5] = 0.0
    with pytest.raises(pw.PWError) as ei:
        h.eig_step(h.to_device(X), 0, b=10.0)
    assert ei.value.status == pw.PW_ENOTPD


def test_bad_block_arguments():
    cell = synth.make_cell("si8")
    h = pw.Handle(cell, pw.PW_FP64, nbands=4)
    X = h.empty_block(5)
    with pytest.raises(pw.PWError) as ei:
        h.apply_h(X)
    assert ei.value.status == pw.PW_EINVAL
    X = h.empty_block(4)
    with pytest.raises(pw.PWError):
        h.eig_step(X, 3, 1.0, 0.5, 2.0)  # a_lo > a


# --- split-bf16 products (mixed precision only) -----------------------------------------

@pytest.mark.parametrize("name,nb", [("si8", 20), ("si64", 9)])
def test_apply_h_bf16_projectors(name, nb):
    say("apply_h bf16x3 projectors", name, nb)
    err, h = apply_case(synth.make_cell(name, modes=True), pw.PW_MIXED, nb, 500 + nb, flags=pw.PW_FLAG_BF16_KB)
    say("  rel err", err)
    assert err < 5e-5


def test_bf16_flags_need_mixed():
    with pytest.raises(pw.PWError) as ei:
        pw.Handle(synth.make_cell("si8"), pw.PW_FP64, flags=pw.PW_FLAG_BF16_GRAM)
    assert ei.value.status == pw.PW_EINVAL


@pytest.mark.parametrize("flags", [pw.PW_FLAG_BF16_GRAM, pw.PW_FLAG_BF16_KB | pw.PW_FLAG_BF16_ROT,
                                   pw.PW_FLAG_BF16_ALL])
def test_step_parity_si64_bf16(flags):
    cell = synth.make_cell("si64")
    model = O.model_from_cell(cell)
    hop = lambda X: O.apply_h(model, X)
    h = pw.Handle(cell, pw.PW_MIXED, flags=flags)
    p = to_gpu_order(h, model)
    inv = np.argsort(p)
    X0g = synth.initial_block(h.gvectors(), cell.L, cell.nbands, synth.SEED_X0 + 1)
    b = 1.01 * O.lanczos_max(hop, model.npw, 20, seed=3)
    s1 = O.eig_step(hop, X0g[inv], 0, 0.0, 0.0, b)
    s2 = O.eig_step(hop, s1.X, 10, s1.a_lo, s1.a, b)
    Xd = h.to_device(X0g)
    e1, r1, _ = h.eig_step(Xd, 0, b=b)
    e2, r2, _ = h.eig_step(Xd, 10, s1.a_lo, s1.a, b)
    d1 = np.abs(e1 - s1.eig)[: cell.nocc].max()
    d2 = np.abs(e2 - s2.eig)[: cell.nocc].max()
    say("si64 bf16 flags", flags, "m=0", d1, "m=10", d2)
    assert d1 < 1e-5 and d2 < 1e-5


def test_solve_si8_bf16_matches_dense(si8_dense):
    cell, model, lam, V = si8_dense
    h = pw.Handle(cell, pw.PW_MIXED, flags=pw.PW_FLAG_BF16_ALL)
    Xd = h.to_device(synth.initial_block(h.gvectors(), cell.L, cell.nbands, synth.SEED_X0))
    eig, res, steps, conv = h.solve(Xd, cell.nocc, 1e-4, degree=10, b=1.01 * lam[-1])
    say("solve bf16 steps", steps, "max |de| occ", np.abs(eig[: cell.nocc] - lam[: cell.nocc]).max())
    assert conv
    assert np.abs(eig[: cell.nocc] - lam[: cell.nocc]).max() < 1e-5



# --- band-blocked step (the memory plan of the largest cells), forced at small sizes ---------

@pytest.mark.parametrize("prec,flags,etol", [(pw.PW_FP64, 0, 1e-10), (pw.PW_MIXED, 0, 1e-5),
                                             (pw.PW_MIXED, pw.PW_FLAG_BF16_ALL, 1e-5)])
def test_blocked_step_parity_si64(prec, flags, etol):
    cell = synth.make_cell("si64")
    model = O.model_from_cell(cell)
    hop = lambda X: O.apply_h(model, X)
    h = pw.Handle(cell, prec, flags=flags, filter_block=64)  # blocks of 64, 64, 16 bands
    assert h.info.filter_block == 64
    p = to_gpu_order(h, model)
    inv = np.argsort(p)
    X0g = synth.initial_block(h.gvectors(), cell.L, cell.nbands, synth.SEED_X0 + 1)
    b = 1.01 * O.lanczos_max(hop, model.npw, 20, seed=3)
    s1 = O.eig_step(hop, X0g[inv], 0, 0.0, 0.0, b)
    s2 = O.eig_step(hop, s1.X, 10, s1.a_lo, s1.a, b)
    Xd = h.to_device(X0g)
    HX = h.empty_block(cell.nbands)
    e1, r1, _ = h.eig_step(Xd, 0, b=b)
    e2, r2, _ = h.eig_step(Xd, 10, s1.a_lo, s1.a, b, HX=HX)
    d1 = np.abs(e1 - s1.eig)[: cell.nocc].max()
    d2 = np.abs(e2 - s2.eig)[: cell.nocc].max()
    say("blocked si64", prec, flags, "m=0", d1, "m=10", d2, "resid", np.abs(r2 - s2.resid).max())
    assert d1 < etol and d2 < etol
    if prec == pw.PW_FP64:
        assert np.abs(r2 - s2.resid).max() < 1e-9
        # H X' returned for the rotated block
        Xn, HXn = h.to_host(Xd)[inv], h.to_host(HX)[inv]
        assert np.abs(HXn - hop(Xn)).max() < 1e-10 * np.abs(HXn).max()
    h.close()


def test_blocked_apply_h_and_solve_si8():
    cell = synth.make_cell("si8", modes=True)
    err, h = apply_case(cell, pw.PW_FP64, 20, 600, flags=0)
    model = O.model_from_cell(cell)
    hb = pw.Handle(cell, pw.PW_FP64, filter_block=8)
    p = to_gpu_order(hb, model)
    X = synth.random_block(model.npw, 20, 601)
    out = hb.to_host(hb.apply_h(hb.to_device(X[p])))
    ref = O.apply_h(model, X)[p]
    assert np.abs(out - ref).max() < 1e-12 * np.abs(ref).max()
    lam = np.linalg.eigvalsh(O.dense_h(model))
    Xd = hb.to_device(synth.initial_block(hb.gvectors(), cell.L, cell.nbands, synth.SEED_X0))
    eig, res, steps, conv = hb.solve(Xd, cell.nocc, 1e-7, degree=10, b=1.01 * lam[-1])
    say("blocked solve steps", steps, "max |de|", np.abs(eig[: cell.nocc] - lam[: cell.nocc]).max())
    assert conv and np.abs(eig[: cell.nocc] - lam[: cell.nocc]).max() < 1e-8


# --- projectors generated inside the GEMMs (no table) ------------------------------------------

@pytest.mark.parametrize("name,prec,nb,tol", [("si8", pw.PW_FP64, 20, 1e-12), ("si64", pw.PW_FP64, 7, 1e-12),
                                               ("si64", pw.PW_MIXED, 9, 2e-5)])
def test_apply_h_generated_projectors(name, prec, nb, tol):
    say("apply_h generated projectors", name, prec, nb)
    err, h = apply_case(synth.make_cell(name, modes=True), prec, nb, 700 + nb, flags=pw.PW_FLAG_BETA_OTF)
    say("  rel err", err)
    assert err < tol


@pytest.mark.parametrize("prec,etol", [(pw.PW_FP64, 1e-10), (pw.PW_MIXED, 1e-5)])
def test_blocked_step_generated_projectors_si64(prec, etol):
    """The memory plan of Si4096 in FP64 (band blocks + generated projectors), forced at Si64,
    against the oracle's step from the same block and bounds."""
    cell = synth.make_cell("si64")
    model = O.model_from_cell(cell)
    hop = lambda X: O.apply_h(model, X)
    h = pw.Handle(cell, prec, flags=pw.PW_FLAG_BETA_OTF, filter_block=64)
    assert h.info.filter_block == 64
    p = to_gpu_order(h, model)
    inv = np.argsort(p)
    X0g = synth.initial_block(h.gvectors(), cell.L, cell.nbands, synth.SEED_X0 + 1)
    b = 1.01 * O.lanczos_max(hop, model.npw, 20, seed=3)
    s1 = O.eig_step(hop, X0g[inv], 0, 0.0, 0.0, b)
    s2 = O.eig_step(hop, s1.X, 10, s1.a_lo, s1.a, b)
    Xd = h.to_device(X0g)
    e1, r1, _ = h.eig_step(Xd, 0, b=b)
    e2, r2, _ = h.eig_step(Xd, 10, s1.a_lo, s1.a, b)
    d1 = np.abs(e1 - s1.eig)[: cell.nocc].max()
    d2 = np.abs(e2 - s2.eig)[: cell.nocc].max()
    say("generated projectors si64", prec, "m=0", d1, "m=10", d2)
    assert d1 < etol and d2 < etol
    if prec == pw.PW_FP64:
        assert np.abs(r2 - s2.resid).max() < 1e-9
    h.close()


# --- charge density (pw_density) --------------------------------------------------------------
# Tolerances relative to max rho: FP64 1e-12 (double FFTs of length <= 128, sums over <= 40
# bands); mixed 1e-5 (fp32 transforms: unit roundoff times the log2 N depth, squared magnitude).
@pytest.mark.parametrize("name,prec,flags,nb,tol", [
    ("si8", pw.PW_FP64, 0, 20, 1e-12),
    ("si8", pw.PW_MIXED, 0, 20, 1e-5),
    ("si8", pw.PW_MIXED, pw.PW_FLAG_PENCIL_FFT, 9, 1e-5),
    ("si64", pw.PW_FP64, pw.PW_FLAG_PENCIL_FFT, 13, 1e-12),
    ("si64", pw.PW_MIXED, 0, 37, 1e-5),
])
def test_density_matches_oracle(name, prec, flags, nb, tol):
    cell = synth.make_cell(name, modes=True)
    model = O.model_from_cell(cell)
    h = pw.Handle(cell, prec, nbands=max(nb, cell.nbands), flags=flags)
    p = to_gpu_order(h, model)
    X = synth.random_block(model.npw, nb, 700 + nb)
    if prec == pw.PW_MIXED:
        X = X.astype(np.complex64).astype(np.complex128)
    occ = np.where(np.arange(nb) % 5 == 4, 0.0, 2.0) - 0.01 * np.arange(nb)
    say("density", name, prec, flags, nb, "grid", tuple(h.info.fft_n))
    ref = O.density(X, occ, model.miller, model.grid).transpose(2, 1, 0)
    rho = h.density(h.to_device(X[p]), occ).cpu().numpy()
    err = float(np.abs(rho - ref).max() / np.abs(ref).max())
    say("  rel err", err)
    assert err < tol
    # bands enter in index order and one at a time: a single band alone is its own density
    one = h.density(h.to_device(X[p][:, :1]), occ[:1]).cpu().numpy()
    ref1 = O.density(X[:, :1], occ[:1], model.miller, model.grid).transpose(2, 1, 0)
    assert float(np.abs(one - ref1).max() / np.abs(ref1).max()) < tol


def test_density_argument_errors():
    cell = synth.make_cell("si8")
    h = pw.Handle(cell, pw.PW_MIXED)
    X = h.to_device(synth.random_block(h.npw, 4, 3))
    with pytest.raises(Exception):
        h.density(X, np.array([1.0, 1.0, 1.0]))  # one weight short
    with pytest.raises(Exception):
        h.density(X, np.array([1.0, np.nan, 1.0, 1.0]))


# --- LOBPCG step (pw_lobpcg_step) -------------------------------------------------------------
@pytest.mark.parametrize("name,prec,flags,nb,etol", [
    ("si8", pw.PW_FP64, 0, 12, 1e-10),
    ("si8", pw.PW_MIXED, 0, 12, 1e-5),
    ("si64", pw.PW_MIXED, pw.PW_FLAG_BF16_ALL, 24, 1e-5),
])
def test_lobpcg_steps_match_oracle(name, prec, flags, nb, etol):
    """Two steps (without, then with search directions) from the same orthonormal block."""
    cell = synth.make_cell(name, modes=True)
    model = O.model_from_cell(cell)
    hop = lambda Y: O.apply_h(model, Y)
    h = pw.Handle(cell, prec, nbands=nb, flags=flags | pw.PW_FLAG_LOBPCG)
    p = to_gpu_order(h, model)
    inv = np.argsort(p)
    X0 = synth.random_block(model.npw, nb, 900 + nb)
    X0, _ = np.linalg.qr(X0)
    if prec == pw.PW_MIXED:
        X0 = X0.astype(np.complex64).astype(np.complex128)
    r1 = O.lobpcg_step(hop, X0, None, model.kin)
    r2 = O.lobpcg_step(hop, r1.X, r1.P, model.kin)
    Xd = h.to_device(X0[p])
    Pd = h.empty_block(nb)
    Pd.zero_()
    e1, s1 = h.lobpcg_step(Xd, Pd, False)
    e2, s2 = h.lobpcg_step(Xd, Pd, True)
    say("lobpcg", name, prec, flags, "eig", np.abs(e1 - r1.eig).max(), np.abs(e2 - r2.eig).max(),
        "resid", np.abs(s1 - r1.resid).max() / r1.resid.max(), np.abs(s2 - r2.resid).max() / r2.resid.max())
    assert np.abs(e1 - r1.eig).max() < etol and np.abs(e2 - r2.eig).max() < etol
    # residual norms: of the same input block at step 1; at step 2 of each side's own first
    # iterate, which differ to first order in the compute precision
    rtol1, rtol2 = (1e-9, 1e-9) if prec == pw.PW_FP64 else (1e-3, 1e-2)
    assert np.abs(s1 - r1.resid).max() < rtol1 * r1.resid.max()
    assert np.abs(s2 - r2.resid).max() < rtol2 * r2.resid.max()
    if prec == pw.PW_FP64:
        # the new block spans the oracle's (principal angles per eigenvalue cluster)
        Xg = h.to_host(Xd)[inv]
        for a, b in O.clusters(r2.eig):
            if b == nb:
                continue  # the top cluster may continue past the block
            assert O.subspace_sin(r2.X[:, a:b], Xg[:, a:b]) < 1e-7


def test_lobpcg_converges_to_dense_gpu(si8_dense):
    cell, model, lam, V = si8_dense
    nb = cell.nbands  # 20 bands for the 16 occupied ones
    h = pw.Handle(cell, pw.PW_FP64, nbands=nb, flags=pw.PW_FLAG_LOBPCG)
    X0, _ = np.linalg.qr(synth.random_block(model.npw, nb, 77))
    p = to_gpu_order(h, model)
    Xd = h.to_device(X0[p])
    Pd = h.empty_block(nb)
    have_p = False
    for it in range(80):
        eig, res = h.lobpcg_step(Xd, Pd, have_p)
        have_p = True
        if res[: cell.nocc].max() < 1e-8:
            break
    say("lobpcg gpu steps", it + 1, "max |de| occ", np.abs(eig[: cell.nocc] - lam[: cell.nocc]).max())
    assert np.abs(eig[: cell.nocc] - lam[: cell.nocc]).max() < 1e-8


def test_lobpcg_needs_its_plan():
    cell = synth.make_cell("si8")
    h = pw.Handle(cell, pw.PW_FP64)
    X = h.to_device(np.linalg.qr(synth.random_block(h.npw, 4, 1))[0])
    P = h.empty_block(4)
    with pytest.raises(Exception):
        h.lobpcg_step(X, P, False)
