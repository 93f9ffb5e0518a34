"""C ABI tests that need no GPU: library load, exported symbols, planner, argument checks."""
import ctypes

import numpy as np
import pytest

from oracle import pw_oracle as O
from paper_2406_10765_amd import pw, synth


def test_library_exports_every_declared_function():
    L = pw.lib()
    names = pw.declared_functions()
    assert "pw_setup" in names and "pw_eig_step" in names and "pw_apply_h" in names
    for n in names:
        assert hasattr(L, n), n


@pytest.mark.parametrize("name,npw,nst,grid", [
    ("si8", 1647, 177, 24), ("si64", 37073, 1353, 64), ("si512", 295667, 5377, 128),
    ("si4096", 835537, 10733, 192)])
def test_plan_sizes(name, npw, nst, grid):
    cell = synth.make_cell(name)
    info = pw.plan(cell)
    assert info.npw == npw
    assert info.nst == nst
    assert tuple(info.fft_n) == (grid,) * 3
    assert info.nproj == 4 * cell.natoms
    assert info.footprint_bytes > 0


def test_plan_gvectors_match_oracle_sphere():
    for cell in (synth.make_cell("si8"), synth.silicon_cell((1, 1, 2), 15.0),
                 synth.silicon_cell((1, 1, 1), 20.0)):
        m = pw.plan_gvectors(cell)
        ref = O.sphere_millers(cell.L, cell.ecut)
        assert m.shape == ref.shape
        # stick order: lexicographic (n1, n2, n3), which is also the oracle's order
        assert np.array_equal(m, ref)
        assert tuple(pw.plan(cell).fft_n) == O.fft_grid(cell.L, cell.ecut)


def test_plan_mixed_uses_fused_planes_at_128():
    cell = synth.make_cell("si512")
    assert pw.plan(cell, pw.PW_MIXED).fused_planes == 1
    # 128^2 complex double does not fit in LDS: pencil form
    assert pw.plan(cell, pw.PW_FP64).fused_planes == 0
    assert pw.plan(synth.make_cell("si64"), pw.PW_FP64).fused_planes == 1


def _desc(cell, **kw):
    d, keep = pw.make_desc(cell)
    for k, v in kw.items():
        if k == "fft_n":
            d.fft_n[:] = v
        elif k == "L":
            d.L[:] = v
        else:
            setattr(d, k, v)
    return d, keep


@pytest.mark.parametrize("change", [
    dict(ecut=-1.0), dict(ecut=float("nan")), dict(nbands=0), dict(nbands=100000), dict(prec=7),
    dict(flags=8), dict(fft_n=[16, 24, 24]), dict(fft_n=[25, 25, 25]), dict(L=[10.0, -1.0, 10.0]),
    dict(natoms=-1), dict(beta_sigma=0.0)])
def test_plan_rejects_bad_descriptions(change):
    cell = synth.make_cell("si8")
    d, keep = _desc(cell, **change)
    info = pw.Info()
    assert pw.lib().pw_plan(ctypes.byref(d), ctypes.byref(info)) == pw.PW_EINVAL
    assert pw.lib().pw_last_error(None)


def test_plan_accepts_larger_smooth_grid():
    cell = synth.make_cell("si8")
    d, keep = _desc(cell, fft_n=[27, 32, 36])
    info = pw.Info()
    assert pw.lib().pw_plan(ctypes.byref(d), ctypes.byref(info)) == pw.PW_OK
    assert tuple(info.fft_n) == (27, 32, 36)


def test_setup_argument_errors_without_device():
    cell = synth.make_cell("si8")
    d, keep = pw.make_desc(cell)
    h = ctypes.c_void_p()
    L = pw.lib()
    assert L.pw_setup(ctypes.byref(d), None, 0, None, ctypes.byref(h)) == pw.PW_EINVAL
    assert L.pw_setup(ctypes.byref(d), ctypes.c_void_p(0x1001), 1 << 30, None, ctypes.byref(h)) == pw.PW_EINVAL
    assert L.pw_apply_h(None, None, None, 1, 1) == pw.PW_EINVAL
    assert L.pw_eig_step(None, None, None, 1, 1, None, None, None, None) == pw.PW_EINVAL
    assert L.pw_density(None, None, 1, 1, None, None) == pw.PW_EINVAL
    assert L.pw_lobpcg_step(None, None, None, 1, 1, 0, None, None, None) == pw.PW_EINVAL
    assert L.pw_destroy(None) == pw.PW_OK


def test_status_strings():
    L = pw.lib()
    for s in (0, 1, -1, -2, -3, -4, -5, -6, -7):
        assert L.pw_status_string(s)


def test_filter_block_planning():
    si512, si4096 = synth.make_cell("si512"), synth.make_cell("si4096")
    assert pw.plan(si512, pw.PW_MIXED).filter_block == si512.nbands  # fits: one block
    info = pw.plan(si4096, pw.PW_MIXED)
    assert 64 <= info.filter_block < si4096.nbands and info.filter_block % 64 == 0
    # the blocked Si4096 mixed plan fits in the 288 GB of one MI355X next to the 55 GB block X
    assert info.footprint_bytes + si4096.nbands * ((info.npw + 15) // 16 * 16) * 8 < 270e9
    assert pw.plan(synth.make_cell("si8"), filter_block=8).filter_block == 8


def test_generated_projector_plan():
    si64, si4096 = synth.make_cell("si64"), synth.make_cell("si4096")
    table = pw.plan(si64, pw.PW_FP64)
    gen = pw.plan(si64, pw.PW_FP64, flags=pw.PW_FLAG_BETA_OTF)
    # the 16-byte table of N_pw x 4 N_atoms entries is replaced by O(N_pw + N_atoms) tables
    ldw = (gen.npw + 15) // 16 * 16
    assert table.footprint_bytes - gen.footprint_bytes >= 16 * ldw * gen.nproj - 40 * ldw
    # Si4096 in FP64 fits one MI355X only with generated projectors: plan + X below 288 GB
    info = pw.plan(si4096, pw.PW_FP64, flags=pw.PW_FLAG_BETA_OTF)
    x_bytes = si4096.nbands * ((info.npw + 15) // 16 * 16) * 16
    assert info.filter_block < si4096.nbands
    assert info.footprint_bytes + x_bytes < 260e9
    assert pw.plan(si4096, pw.PW_FP64).footprint_bytes + x_bytes > 288e9
    # not combinable with the pre-split projector planes
    d, keep = _desc(si64, prec=pw.PW_MIXED, flags=pw.PW_FLAG_BETA_OTF | pw.PW_FLAG_BF16_KB)
    info = pw.Info()
    assert pw.lib().pw_plan(ctypes.byref(d), ctypes.byref(info)) == pw.PW_EINVAL


def test_lobpcg_plan_needs_one_block():
    cell = synth.make_cell("si64")
    ok = pw.plan(cell, pw.PW_MIXED, flags=pw.PW_FLAG_LOBPCG)
    base = pw.plan(cell, pw.PW_MIXED)
    assert ok.footprint_bytes > base.footprint_bytes
    with pytest.raises(Exception):
        pw.plan(cell, pw.PW_MIXED, flags=pw.PW_FLAG_LOBPCG, filter_block=64)


def test_binding_flags_and_statuses_match_the_header():
    """The Python constants mirror include/pw.h (flags and status codes)."""
    import os
    import re
    hdr = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "pw.h")).read()
    for name, val in re.findall(r"#define (PW_FLAG_[A-Z0-9_]+) (\d+)u", hdr):
        assert getattr(pw, name) == int(val), name
    for name, val in re.findall(r"\b(PW_[A-Z]+) = (-?\d+)", hdr):
        if hasattr(pw, name):
            assert getattr(pw, name) == int(val), name


def test_solve_retries_of_a_null_handle():
    assert pw.lib().pw_solve_retries(None, None) == -1
