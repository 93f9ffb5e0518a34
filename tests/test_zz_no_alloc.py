"""pw_apply_h_noalloc (work buffers in the library's static device array) against pw_apply_h.

Both entry points run the same kernels; the allocation-free one places the FFT intermediates,
the projection partials, D P and the bf16 planes in the static array and processes the bands in
groups that fit it.  Two calls in a row, the second with fewer bands (the array then holds the
first call's data), must each match pw_apply_h to the parity tolerances: 1e-12 relative in FP64,
2e-5 in mixed precision, 5e-5 with bf16-split projector products.
"""
import sys

import numpy as np
import pytest

from paper_2406_10765_amd import pw, synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("name,prec,flags,nbs,tol", [
    ("si8", pw.PW_FP64, 0, (20, 5), 1e-12),
    ("si8", pw.PW_MIXED, pw.PW_FLAG_BF16_ALL, (20, 3), 5e-5),
    ("si64", pw.PW_MIXED, pw.PW_FLAG_BF16_ALL, (144, 37), 5e-5),
    ("si64", pw.PW_FP64, pw.PW_FLAG_PENCIL_FFT, (40, 9), 1e-12),
])
def test_noalloc_matches_apply_h(name, prec, flags, nbs, tol):
    import torch
    assert torch.cuda.is_available()
    cell = synth.make_cell(name, modes=True)
    h = pw.Handle(cell, prec, flags=flags)
    for k, nb in enumerate(nbs):
        say("noalloc", name, prec, flags, "call", k, "nb", nb)
        X = h.to_device(synth.random_block(h.npw, nb, 40 + k))
        ref = h.apply_h(X)
        out = torch.full_like(X, float("nan"))
        h.apply_h_noalloc(X, out)
        torch.cuda.synchronize()
        a = out[:, : h.npw].cpu().numpy()
        b = ref[:, : h.npw].cpu().numpy()
        err = float(np.abs(a - b).max() / np.abs(b).max())
        say("  rel diff", err, "bitwise", bool(np.array_equal(a, b)))
        assert np.isfinite(a).all()
        assert err <= tol
    h.close()


def test_noalloc_rejects_a_band_beyond_the_array():
    """A 192^3 FP64 grid needs about 100 MB of FFT intermediates for one band: PW_ENOMEM."""
    cell = synth.make_cell("si4096", nbands=8)
    h = pw.Handle(cell, pw.PW_FP64, flags=pw.PW_FLAG_BETA_OTF)
    X = h.empty_block(8)
    X.zero_()
    HX = h.empty_block(8)
    with pytest.raises(pw.PWError) as ei:
        h.apply_h_noalloc(X, HX)
    say("  error:", ei.value)
    assert ei.value.status == pw.PW_ENOMEM
    h.close()
