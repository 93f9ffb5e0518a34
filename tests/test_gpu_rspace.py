"""Parity of the real-space projector route (PW_FLAG_RSPACE_KB) and of the localized projector
family in reciprocal space, against the oracle.

* H X with the real-space passes against the oracle's real-space route at the same radius (the
  plain definition: grid sums over the balls), on Si8 and Si64 with 128^3 grids and on sampled
  columns of the full Si512 block in the launch configuration the bench times: FP32 tolerance
  2e-5 relative, as for every mixed H X.
* The same against the untruncated reciprocal-space route of the localized family: the radius
  adds at most the chi-distribution tail bound of the oracle's pins (below 1e-7 here).
* The reciprocal-space GEMM route with the localized family (FP64 table, FP32 table, bf16 planes)
  against the oracle: 1e-12 / 2e-5 / 5e-5.
* Filter steps (degree 0, then 10) with the real-space route against the oracle's steps with
  its real-space route, unblocked and band-blocked: occupied eigenvalues within 1e-5 Ha.
* Grids with 96 and 192 z planes (the second on a 1 x 1 x 2 cell, unequal steps along x, y, z).
* pw_apply_h_noalloc refuses such handles (the argument errors of the flag are host tests).
"""
import sys

import numpy as np
import pytest

from oracle import pw_oracle as O
from paper_2406_10765_amd import pw, synth

pytestmark = pytest.mark.gpu

LOC = pw.PW_PROJ_LOCALIZED
RS = pw.PW_FLAG_RSPACE_KB


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible device"
    pw.lib()
    return torch


def radius_for(cell, nsigma=7.0):
    # nsigma sigma where the cell allows it, else just below half the smallest cell length
    return min(nsigma * cell.pseudo.beta_sigma, 0.49 * float(np.min(cell.L)))


def rs_case(name, nb, seed, grid=(128, 128, 128), flags=0, nsigma=7.0):
    cell = synth.make_cell(name, modes=True)
    R = radius_for(cell, nsigma)
    model = O.model_from_cell(cell, grid=grid, proj_form=O.PROJ_LOCALIZED, rs_radius=R)
    h = pw.Handle(cell, pw.PW_MIXED, nbands=nb, fft_n=grid, flags=RS | flags, proj_form=LOC, rs_radius=R)
    assert tuple(h.info.fft_n) == tuple(grid) and h.info.fused_planes == 1
    p = pw.permutation_to(model.miller, h.gvectors())
    X = synth.random_block(model.npw, nb, seed).astype(np.complex64).astype(np.complex128)
    out = h.to_host(h.apply_h(h.to_device(X[p])))
    return cell, model, h, X, p, R, out


@pytest.mark.parametrize("name,nb,nsigma", [("si8", 20, 7.0), ("si64", 9, 7.0), ("si64", 9, 5.5)])
def test_rspace_apply_h_matches_oracle_realspace(name, nb, nsigma):
    cell, model, h, X, p, R, out = rs_case(name, nb, 500 + nb, nsigma=nsigma)
    ref = O.apply_h(model, X)
    err = float(np.abs(out - ref[p]).max() / np.abs(ref).max())
    say("rspace apply_h", name, "R", R, "rel err vs oracle real-space route", err)
    assert err < 2e-5
    # against the untruncated reciprocal-space route of the same family
    model.rs_radius = 0.0
    ref_g = O.apply_h(model, X)
    err_g = float(np.abs(out - ref_g[p]).max() / np.abs(ref_g).max())
    say("  rel err vs reciprocal-space localized route", err_g)
    assert err_g < 2e-5
    h.close()


@pytest.mark.parametrize("ncells,grid", [((1, 1, 1), (128, 128, 96)), ((1, 1, 2), (128, 128, 192))])
def test_rspace_apply_h_other_z_grids(ncells, grid):
    # z planes other than 128 (and an orthorhombic cell: different steps along x, y and z)
    cell = synth.silicon_cell(ncells, 10.0, nbands=6, disp_seed=synth.SEED_REQUEST + 11,
                              modes_seed=synth.SEED_MODES + 5)
    R = radius_for(cell)
    model = O.model_from_cell(cell, grid=grid, proj_form=O.PROJ_LOCALIZED, rs_radius=R)
    h = pw.Handle(cell, pw.PW_MIXED, nbands=6, fft_n=grid, flags=RS, proj_form=LOC, rs_radius=R)
    assert tuple(h.info.fft_n) == grid
    p = pw.permutation_to(model.miller, h.gvectors())
    X = synth.random_block(model.npw, 6, 733).astype(np.complex64).astype(np.complex128)
    out = h.to_host(h.apply_h(h.to_device(X[p])))
    ref = O.apply_h(model, X)
    err = float(np.abs(out - ref[p]).max() / np.abs(ref).max())
    say("rspace apply_h grid", grid, "L", cell.L, "R", R, "rel err", err)
    assert err < 2e-5
    h.close()


def test_rspace_blocked_step_matches_oracle():
    # band-blocked filter (blocks of 8, 8, 4 bands) with the real-space route
    cell = synth.make_cell("si8", modes=True)
    grid = (128, 128, 128)
    R = radius_for(cell)
    model = O.model_from_cell(cell, grid=grid, proj_form=O.PROJ_LOCALIZED, rs_radius=R)
    hop = lambda X: O.apply_h(model, X)
    h = pw.Handle(cell, pw.PW_MIXED, fft_n=grid, flags=RS, proj_form=LOC, rs_radius=R, filter_block=8)
    assert h.info.filter_block == 8
    p = pw.permutation_to(model.miller, h.gvectors())
    inv = np.argsort(p)
    X0g = synth.initial_block(h.gvectors(), cell.L, cell.nbands, synth.SEED_X0 + 10)
    X0g = X0g.astype(np.complex64).astype(np.complex128)
    b = 1.01 * O.lanczos_max(hop, model.npw, 20, seed=3)
    s1 = O.eig_step(hop, X0g[inv], 0, 0.0, 0.0, b)
    s2 = O.eig_step(hop, s1.X, 10, s1.a_lo, s1.a, b)
    Xd = h.to_device(X0g)
    e1, _, _ = h.eig_step(Xd, 0, b=b)
    e2, _, _ = h.eig_step(Xd, 10, s1.a_lo, s1.a, b)
    d1 = np.abs(e1 - s1.eig)[: cell.nocc].max()
    d2 = np.abs(e2 - s2.eig)[: cell.nocc].max()
    say("rspace blocked steps m=0", d1, "m=10", d2)
    assert d1 < 1e-5 and d2 < 1e-5
    h.close()


def test_rspace_apply_h_several_batches():
    # more bands than one FFT batch holds: the partials and D P are indexed per batch
    cell = synth.make_cell("si8", modes=True)
    R = radius_for(cell)
    import os
    os.environ["PW_FFT_BATCH_MB"] = "1"  # a few bands per FFT batch
    try:
        h = pw.Handle(cell, pw.PW_MIXED, nbands=40, fft_n=(128, 128, 128), flags=RS, proj_form=LOC, rs_radius=R)
    finally:
        del os.environ["PW_FFT_BATCH_MB"]
    model = O.model_from_cell(cell, grid=(128, 128, 128), proj_form=O.PROJ_LOCALIZED, rs_radius=R)
    p = pw.permutation_to(model.miller, h.gvectors())
    X = synth.random_block(model.npw, 40, 611).astype(np.complex64).astype(np.complex128)
    out = h.to_host(h.apply_h(h.to_device(X[p])))
    ref = O.apply_h(model, X)
    err = float(np.abs(out - ref[p]).max() / np.abs(ref).max())
    say("rspace apply_h, 40 bands in batches", err)
    assert err < 2e-5


def test_rspace_apply_h_is_deterministic():
    cell, model, h, X, p, R, out = rs_case("si8", 6, 77)
    again = h.to_host(h.apply_h(h.to_device(X[p])))
    assert np.array_equal(out, again)


@pytest.mark.parametrize("prec,flags,tol", [(pw.PW_FP64, 0, 1e-12), (pw.PW_MIXED, 0, 2e-5),
                                            (pw.PW_MIXED, pw.PW_FLAG_BF16_KB, 5e-5)])
def test_localized_gspace_route_matches_oracle(prec, flags, tol):
    cell = synth.make_cell("si64", modes=True)
    model = O.model_from_cell(cell, proj_form=O.PROJ_LOCALIZED)
    h = pw.Handle(cell, prec, nbands=7, flags=flags, proj_form=LOC)
    p = pw.permutation_to(model.miller, h.gvectors())
    X = synth.random_block(model.npw, 7, 909)
    if prec == pw.PW_MIXED:
        X = X.astype(np.complex64).astype(np.complex128)
    out = h.to_host(h.apply_h(h.to_device(X[p])))
    ref = O.apply_h(model, X)
    err = float(np.abs(out - ref[p]).max() / np.abs(ref).max())
    say("localized reciprocal-space route, prec", prec, "flags", flags, "rel err", err)
    assert err < tol
    h.close()


@pytest.mark.parametrize("flags", [0, pw.PW_FLAG_BF16_GRAM | pw.PW_FLAG_BF16_ROT])
def test_rspace_steps_match_oracle(flags):
    cell = synth.make_cell("si8", modes=True)
    grid = (128, 128, 128)
    R = radius_for(cell)
    model = O.model_from_cell(cell, grid=grid, proj_form=O.PROJ_LOCALIZED, rs_radius=R)
    hop = lambda X: O.apply_h(model, X)
    h = pw.Handle(cell, pw.PW_MIXED, fft_n=grid, flags=RS | flags, proj_form=LOC, rs_radius=R)
    p = pw.permutation_to(model.miller, h.gvectors())
    inv = np.argsort(p)
    X0g = synth.initial_block(h.gvectors(), cell.L, cell.nbands, synth.SEED_X0 + 9)
    X0g = X0g.astype(np.complex64).astype(np.complex128)
    b = 1.01 * O.lanczos_max(hop, model.npw, 20, seed=3)
    s1 = O.eig_step(hop, X0g[inv], 0, 0.0, 0.0, b)
    s2 = O.eig_step(hop, s1.X, 10, s1.a_lo, s1.a, b)
    Xd = h.to_device(X0g)
    e1, r1, _ = h.eig_step(Xd, 0, b=b)
    e2, r2, _ = h.eig_step(Xd, 10, s1.a_lo, s1.a, b)
    d1 = np.abs(e1 - s1.eig)[: cell.nocc].max()
    d2 = np.abs(e2 - s2.eig)[: cell.nocc].max()
    say("rspace steps flags", flags, "m=0", d1, "m=10", d2)
    assert d1 < 1e-5 and d2 < 1e-5
    h.close()


def test_rspace_si512_sampled_columns():
    cols = [0, 1, 543, 1086, 1087]
    cell = synth.make_cell("si512")
    R = radius_for(cell)
    model = O.model_from_cell(cell, with_projectors=False, proj_form=O.PROJ_LOCALIZED, rs_radius=R)
    say("Si512 rspace apply_h full block, R", R)
    h = pw.Handle(cell, pw.PW_MIXED, flags=RS, proj_form=LOC, rs_radius=R)
    p = pw.permutation_to(model.miller, h.gvectors())
    X = synth.initial_block(h.gvectors(), cell.L, cell.nbands, 78).astype(np.complex64).astype(np.complex128)
    HX = h.apply_h(h.to_device(X))
    out = HX[cols].cpu().numpy().astype(np.complex128).T[: h.npw]
    inv = np.argsort(p)
    ref = O.apply_h(model, X[:, cols][inv])[p]
    err = float(np.abs(out - ref).max() / np.abs(ref).max())
    say("  rel err", err)
    assert err < 2e-5
    h.close()


def test_rspace_noalloc_rejects():
    cell = synth.make_cell("si8", modes=True)
    h = pw.Handle(cell, pw.PW_MIXED, nbands=2, fft_n=(128, 128, 128), flags=RS, proj_form=LOC, rs_radius=4.0)
    X = h.to_device(synth.random_block(h.npw, 2, 5).astype(np.complex64))
    HX = X.clone()
    with pytest.raises(pw.PWError) as ei:
        h.apply_h_noalloc(X, HX)
    assert ei.value.status == pw.PW_EINVAL
    h.close()
