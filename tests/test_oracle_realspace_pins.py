"""Pins of the oracle's localized projectors and of its real-space nonlocal route.

* The real-space functions (a Gaussian and a Gaussian times x, y, z) have unit norm and are
  mutually orthogonal (quadrature on a fine box around the atom).
* The reciprocal-space columns of the localized form are (1/sqrt(Omega)) times the continuum
  Fourier transforms of those functions about an off-centre atom: checked against a direct
  quadrature of integral p(r - tau) exp(-i G.r) d^3r, which shares no arithmetic with the
  closed form (this fixes the normalisation, the -i of l = 1, the axis order and the sign of the
  structure factor).
* The real-space route (grid sums over balls around the atoms) equals B D B^H X of those columns
  within the truncation bound: for a unit-norm projector p and its part p_out outside the ball,
  || (p p^T - p_R p_R^T) psi || <= 2 ||p_out|| ||psi||, summed with |D| over all projectors, where
  ||p_out||^2 is the tail of a chi distribution (3 degrees of freedom for l = 0, 5 for l = 1,
  scale sigma / sqrt 2).  A small radius must give a visible error inside the bound, a radius near
  half the cell an error below 1e-5 of the nonlocal part.
* Each pin is run again with a planted mistake and must then fail.  CPU only.
"""
import math

import numpy as np
import pytest

from oracle import pw_oracle as O

L_ORTHO = np.array([9.0, 10.26, 11.5])
TAU = np.array([[2.3, 7.9, 0.6], [6.1, 2.2, 5.9], [4.4, 5.0, 10.9]])
SIGMA = 0.8
D0, D1 = 1.5, -0.7


def _box(sigma=SIGMA, half=9.0, step=0.1):
    h = sigma * step
    n = int(round(half * sigma / h))
    ax = np.arange(-n, n + 1) * h
    x, y, z = np.meshgrid(ax, ax, ax, indexing="ij")
    return np.stack([x, y, z], axis=-1), h


def _tail_norms(radius, sigma=SIGMA):
    """||p_out|| for l = 0 and l = 1: the chi-3 and chi-5 tails beyond x = radius / sigma."""
    x = radius / sigma
    e = math.exp(-x * x)
    t0 = math.erfc(x) + 2.0 / math.sqrt(math.pi) * x * e
    t1 = math.erfc(x) + 2.0 / math.sqrt(math.pi) * (x + 2.0 * x ** 3 / 3.0) * e
    return math.sqrt(t0), math.sqrt(t1)


def pin_realspace_functions():
    d, h = _box()
    p = O.localized_projector_values(d, SIGMA).reshape(4, -1)
    gram = (p @ p.T) * h ** 3
    return float(np.abs(gram - np.eye(4)).max())


def pin_fourier_columns():
    mil = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [2, -1, 3], [-1, 2, -2], [3, 1, 0]])
    omega = float(np.prod(L_ORTHO))
    B = O.projector_matrix(mil, L_ORTHO, TAU[:1], SIGMA, form=O.PROJ_LOCALIZED) * math.sqrt(omega)
    d, h = _box()
    p = O.localized_projector_values(d, SIGMA).reshape(4, -1)
    r = d.reshape(-1, 3) + TAU[0]
    G = 2.0 * math.pi * mil / L_ORTHO
    worst = 0.0
    for gi in range(mil.shape[0]):
        ph = np.exp(-1j * (r @ G[gi]))
        q = (p * ph[None, :]).sum(axis=1) * h ** 3
        worst = max(worst, float(np.abs(q - B[gi]).max()))
    return worst


def _routes(radius, ecut=10.0, nb=3, seed=7):
    mg = O.build_model(L_ORTHO, TAU, ecut, d0=D0, d1=D1, proj_form=O.PROJ_LOCALIZED)
    mr = O.build_model(L_ORTHO, TAU, ecut, d0=D0, d1=D1, proj_form=O.PROJ_LOCALIZED, rs_radius=radius)
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((mg.npw, nb)) + 1j * rng.standard_normal((mg.npw, nb))
    nl_g = mg.B @ (mg.D[:, None] * (mg.B.conj().T @ X))
    nl_r = O.apply_nonlocal_realspace(mr, X, radius)
    t0, t1 = _tail_norms(radius)
    per_atom = abs(D0) * t0 + 3 * abs(D1) * t1
    bound = 2.0 * TAU.shape[0] * per_atom * np.linalg.norm(X, axis=0)
    err = np.linalg.norm(nl_r - nl_g, axis=0)
    return err, bound, np.linalg.norm(nl_g, axis=0)


def pin_routes_small_radius():
    """(ratio of the error to its bound, error relative to the nonlocal part) at radius 2 bohr."""
    err, bound, ref = _routes(2.0)
    return float((err / bound).max()), float((err / ref).min())


def pin_routes_large_radius():
    err, bound, ref = _routes(0.49 * L_ORTHO.min())
    return float((err / bound).max()), float((err / ref).max())


def test_realspace_functions_orthonormal():
    assert pin_realspace_functions() < 1e-12


def test_localized_columns_are_fourier_transforms():
    assert pin_fourier_columns() < 1e-12


def test_localized_l0_equals_gspace_l0():
    # the two forms share the l = 0 projector exactly
    mil = O.sphere_millers(L_ORTHO, 8.0)
    a = O.projector_matrix(mil, L_ORTHO, TAU, SIGMA, form=O.PROJ_GSPACE)
    b = O.projector_matrix(mil, L_ORTHO, TAU, SIGMA, form=O.PROJ_LOCALIZED)
    assert np.array_equal(a[:, 0::4], b[:, 0::4])


def test_realspace_route_small_radius_within_bound():
    ratio, rel = pin_routes_small_radius()
    assert ratio <= 1.0
    assert rel > 1e-4  # the truncation is really applied


def test_realspace_route_large_radius_matches():
    ratio, rel = pin_routes_large_radius()
    assert ratio <= 1.0
    assert rel < 1e-5  # tail norm of the l = 1 projectors at this radius: 2.9e-6


def test_apply_h_takes_the_realspace_route():
    m = O.build_model(L_ORTHO, TAU, 10.0, d0=D0, d1=D1, proj_form=O.PROJ_LOCALIZED, rs_radius=2.0)
    X = np.random.default_rng(3).standard_normal((m.npw, 2)) + 0j
    full = O.apply_h(m, X)
    m.rs_radius = 0.0
    gsp = O.apply_h(m, X)
    nl = O.apply_nonlocal_realspace(m, X, 2.0)
    nlg = m.B @ (m.D[:, None] * (m.B.conj().T @ X))
    assert np.allclose(full - gsp, nl - nlg, rtol=0, atol=1e-12 * np.abs(full).max())


def test_ball_points_match_brute_force():
    grid = (24, 27, 30)
    for a in range(TAU.shape[0]):
        flat, d = O.ball_points(L_ORTHO, grid, TAU[a], 3.0)
        h = L_ORTHO / np.asarray(grid)
        idx = np.indices(grid).reshape(3, -1).T
        r = idx * h
        dd = r - TAU[a]
        dd -= L_ORTHO * np.round(dd / L_ORTHO)
        inside = np.flatnonzero((dd * dd).sum(axis=1) <= 9.0)
        assert np.array_equal(np.sort(flat), inside)


# ---- planted mistakes (test-only mutants of the oracle) ------------------------------------

_orig_pm = O.projector_matrix
_orig_lpv = O.localized_projector_values


def _pm_mutant(kind):
    def f(miller, L, tau, sigma, sf_sign=-1.0, form=O.PROJ_GSPACE):
        B = _orig_pm(miller, L, tau, sigma, sf_sign, form)
        if form != O.PROJ_LOCALIZED:
            return B
        B = B.copy()
        if kind == "no_minus_i":
            B[:, 1::4] *= 1j
            B[:, 2::4] *= 1j
            B[:, 3::4] *= 1j
        elif kind == "axes_swapped":
            B[:, 1::4], B[:, 2::4] = B[:, 2::4].copy(), B[:, 1::4].copy()
        elif kind == "sf_sign":
            B = _orig_pm(miller, L, tau, sigma, -sf_sign, form)
        return B
    return f


def _lpv_mutant(kind):
    def f(d, sigma):
        if kind == "displacement_sign":
            return _orig_lpv(-d, sigma)
        if kind == "centre_shift":
            return _orig_lpv(d + np.array([0.3, 0.0, 0.0]), sigma)
        if kind == "width":
            return _orig_lpv(d, 1.1 * sigma)
        p = _orig_lpv(d, sigma)
        if kind == "l1_norm":
            p = p.copy()
            p[1:] *= sigma
        return p
    return f


@pytest.mark.parametrize("kind", ["displacement_sign", "centre_shift", "width"])
def test_planted_mistake_in_realspace_functions_fails_fourier_pin(monkeypatch, kind):
    # p -> -p for l = 1 leaves V_NL unchanged (it enters twice), so the sign is fixed by the
    # Fourier pin alone
    monkeypatch.setattr(O, "localized_projector_values", _lpv_mutant(kind))
    assert pin_fourier_columns() > 1e-3


@pytest.mark.parametrize("kind", ["l1_norm", "centre_shift", "width"])
def test_planted_mistake_in_realspace_route_fails(monkeypatch, kind):
    monkeypatch.setattr(O, "localized_projector_values", _lpv_mutant(kind))
    if kind == "l1_norm":
        assert pin_realspace_functions() > 1e-3
    ratio, _ = pin_routes_large_radius()
    assert ratio > 1.0


def test_planted_mistake_dropped_volume_factor_fails(monkeypatch):
    orig = O.apply_nonlocal_realspace

    def mutant(model, X, radius):
        return orig(model, X, radius) / math.sqrt(model.omega)

    monkeypatch.setattr(O, "apply_nonlocal_realspace", mutant)
    ratio, _ = pin_routes_large_radius()
    assert ratio > 1.0
