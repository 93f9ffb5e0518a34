"""Host checks of the real-space projector option (no GPU): the planner's argument errors, and
that the plan of a real-space handle holds no projector table (at Si512 its footprint shrinks by
the table of N_pw x 4 N_atoms complex words; the entry tables and partials are small)."""
import numpy as np
import pytest

from paper_2406_10765_amd import pw, synth

LOC = pw.PW_PROJ_LOCALIZED
RS = pw.PW_FLAG_RSPACE_KB
G128 = (128, 128, 128)


@pytest.mark.parametrize("kw", [
    dict(prec=pw.PW_MIXED, fft_n=G128, flags=RS, proj_form=pw.PW_PROJ_GSPACE, rs_radius=4.0),  # wrong family
    dict(prec=pw.PW_FP64, fft_n=G128, flags=RS, proj_form=LOC, rs_radius=4.0),  # FP64
    dict(prec=pw.PW_MIXED, fft_n=(0, 0, 0), flags=RS, proj_form=LOC, rs_radius=4.0),  # 24^3 grid
    dict(prec=pw.PW_MIXED, fft_n=G128, flags=RS, proj_form=LOC, rs_radius=5.13),  # half the 10.26 bohr cell
    dict(prec=pw.PW_MIXED, fft_n=G128, flags=RS, proj_form=LOC, rs_radius=0.0),
    dict(prec=pw.PW_MIXED, fft_n=G128, flags=RS, proj_form=LOC, rs_radius=float("nan")),
    dict(prec=pw.PW_MIXED, fft_n=G128, flags=RS | pw.PW_FLAG_BF16_KB, proj_form=LOC, rs_radius=4.0),
    dict(prec=pw.PW_MIXED, fft_n=G128, flags=RS | pw.PW_FLAG_PENCIL_FFT, proj_form=LOC, rs_radius=4.0),
    dict(prec=pw.PW_MIXED, fft_n=(0, 0, 0), flags=pw.PW_FLAG_BETA_OTF, proj_form=LOC, rs_radius=0.0),
    dict(prec=pw.PW_MIXED, fft_n=(0, 0, 0), flags=0, proj_form=7, rs_radius=0.0),
])
def test_rspace_plan_argument_errors(kw):
    cell = synth.make_cell("si8", modes=True)
    with pytest.raises(pw.PWError) as ei:
        pw.plan(cell, kw["prec"], None, kw["fft_n"], kw["flags"], 0, kw["proj_form"], kw["rs_radius"])
    assert ei.value.status == pw.PW_EINVAL


def test_rspace_plan_has_no_projector_table():
    # Si512 on its 128^3 grid: the 4.8 GB complex64 table is gone; the per-entry partials of one
    # FFT batch take tens of MB
    cell = synth.make_cell("si512")
    g = pw.plan(cell, pw.PW_MIXED, None, (0, 0, 0), 0, 0, LOC, 0.0)
    r = pw.plan(cell, pw.PW_MIXED, None, (0, 0, 0), RS, 0, LOC, 4.4)
    table = 8 * g.npw * 4 * cell.natoms
    assert tuple(r.fft_n) == G128 and r.fused_planes == 1
    assert g.footprint_bytes - r.footprint_bytes > 0.9 * table


def test_localized_form_plans_without_flag():
    cell = synth.make_cell("si8", modes=True)
    for prec, flags in ((pw.PW_FP64, 0), (pw.PW_MIXED, 0), (pw.PW_MIXED, pw.PW_FLAG_BF16_KB)):
        pw.plan(cell, prec, None, (0, 0, 0), flags, 0, LOC, 0.0)
