"""Pins of the oracle's local potential and of the LOBPCG search-direction update.

The local potential of the analytic pseudopotential has three parts, each pinned here against
a form that shares no arithmetic with the oracle's reciprocal-space formula:

* the perturbation modes, against their defining real-space sum of cosines at every grid point;
* the short-range Gaussian term of one atom, against the periodic sum of its real-space Gaussian
  (the continuum Fourier transform of c exp(-G^2 rc^2/4) is c (pi rc^2)^(-3/2) exp(-r^2/rc^2));
* the Coulomb term of one atom, through Poisson's equation: -G^2 v_C(G) / (4 pi) must be the
  Fourier series of a positive Gaussian ion charge Z (pi rc^2)^(-3/2) exp(-r^2/rc^2) with its
  neutralising background (v_C is the attractive potential of that charge).

The cutoff is raised so that the band-limit tail (exp(-G^2 rc^2/4) beyond |G|^2 = 2 E_cut) is
below 1e-11 and the comparison is exact to rounding.  Each pin is run again with a planted
mistake in the oracle (a wrong Gaussian width, a dropped 1/Omega, a flipped Coulomb sign, the full
amplitude on both +G and -G) and must then fail.  CPU only.
"""
import math

import numpy as np
import pytest

from oracle import pw_oracle as O
from paper_2406_10765_amd import synth

# Orthorhombic, so that a permuted axis or a wrong length is seen.
L_ORTHO = (9.0, 10.26, 11.5)
TAU_ONE = np.array([[2.3, 7.9, 0.6]])
ECUT_HIGH = 60.0  # exp(-G^2/4) at |G|^2 = 120 is 9e-14


def _grid_points(L, grid):
    """r_j = (j1 L1/N1, j2 L2/N2, j3 L3/N3) for every grid index, shape (N1, N2, N3, 3)."""
    axes = [np.arange(n) * (L[i] / n) for i, n in enumerate(grid)]
    r = np.meshgrid(*axes, indexing="ij")
    return np.stack(r, axis=-1)


def _periodic_gaussian(L, grid, tau, width):
    """sum over images R of (pi w^2)^(-3/2) exp(-|r - tau - R|^2 / w^2) on the grid (unit weight)."""
    r = _grid_points(L, grid)
    L = np.asarray(L, float)
    out = np.zeros(r.shape[:3])
    norm = (math.pi * width * width) ** -1.5
    for a in range(tau.shape[0]):
        for i in range(-2, 3):
            for j in range(-2, 3):
                for k in range(-2, 3):
                    d = r - (tau[a] + L * np.array([i, j, k]))
                    out += norm * np.exp(-(d * d).sum(axis=-1) / (width * width))
    return out


def modes_error():
    """max |V(r_j) - sum_k amp_k cos(G_k.r_j + phi_k)| for the Si8 cell with only the modes on."""
    cell = synth.make_cell("si8", modes=True)
    model = O.model_from_cell(cell, zval=0.0, gauss_c=0.0, d0=0.0, d1=0.0)
    r = _grid_points(model.L, model.grid)
    want = np.zeros(model.grid)
    G = 2 * math.pi * cell.modes.miller / np.asarray(cell.L, float)
    for k in range(G.shape[0]):
        want += cell.modes.amp[k] * np.cos(r @ G[k] + cell.modes.phase[k])
    assert np.abs(want).max() > 0.3  # 32 modes of 0.05 Ha add up: the check is not vacuous
    return float(np.abs(model.vr - want).max())


def gaussian_term_error():
    """max |V(r_j) - (c sum_R g(r_j - tau - R) - c/Omega)| for one atom, Gaussian term only."""
    c = 2.0
    model = O.build_model(L_ORTHO, TAU_ONE, ECUT_HIGH, zval=0.0, gauss_c=c, rc=1.0, d0=0.0, d1=0.0)
    omega = float(np.prod(L_ORTHO))
    want = c * _periodic_gaussian(L_ORTHO, model.grid, TAU_ONE, 1.0) - c / omega
    return float(np.abs(model.vr - want).max())


def coulomb_charge_error():
    """Poisson's equation: -G^2 V(G) / (4 pi) against a Gaussian ion charge Z minus its average."""
    z, rc = 4.0, 1.0
    grid = O.fft_grid(L_ORTHO, ECUT_HIGH)
    miller = O.sphere_millers(L_ORTHO, ECUT_HIGH)
    vg = O.local_potential_g(miller, np.asarray(L_ORTHO), ECUT_HIGH, TAU_ONE, z, rc, 0.0,
                             np.zeros((0, 3), np.int64), np.zeros(0), np.zeros(0))
    G = 2 * math.pi * miller / np.asarray(L_ORTHO, float)
    q = -(G * G).sum(axis=1) * vg / (4 * math.pi)
    qr = O.to_real_space(q, miller, grid)
    omega = float(np.prod(L_ORTHO))
    want = z * _periodic_gaussian(L_ORTHO, grid, TAU_ONE, rc) - z / omega
    assert float(np.abs(qr.imag).max()) < 1e-12
    return float(np.abs(qr.real - want).max())


PINS = {"modes": modes_error, "gaussian": gaussian_term_error, "coulomb": coulomb_charge_error}


@pytest.mark.parametrize("pin", sorted(PINS))
def test_local_potential_pin(pin):
    assert PINS[pin]() < 1e-9


def _mutant(kind):
    """The oracle's local_potential_g with one plausible mistake planted (test-only)."""
    orig = O.local_potential_g

    def wrapped(miller, L, ecut, tau, zval, rc, gauss_c, mm, ma, mp, sf_sign=-1.0):
        if kind == "width":      # exp(-G^2 rc^2/2) in place of exp(-G^2 rc^2/4)
            return orig(miller, L, ecut, tau, zval, rc * math.sqrt(2.0), gauss_c, mm, ma, mp, sf_sign)
        if kind == "omega":      # 1/Omega dropped
            return orig(miller, L, ecut, tau, zval, rc, gauss_c, mm, ma, mp, sf_sign) * float(np.prod(L))
        if kind == "coulomb":    # Coulomb sign flipped
            return orig(miller, L, ecut, tau, -zval, rc, gauss_c, mm, ma, mp, sf_sign)
        if kind == "amp":        # amp in place of amp/2 on each of +G, -G
            return orig(miller, L, ecut, tau, zval, rc, gauss_c, mm, 2.0 * np.asarray(ma), mp, sf_sign)
        if kind == "phase":      # phase sign flipped
            return orig(miller, L, ecut, tau, zval, rc, gauss_c, mm, ma, -np.asarray(mp), sf_sign)
        raise ValueError(kind)

    return wrapped


# (mistake, the pins that must catch it)
MUTANTS = [
    ("width", ("gaussian", "coulomb")),
    ("omega", ("gaussian", "coulomb")),
    ("coulomb", ("coulomb",)),
    ("amp", ("modes",)),
    ("phase", ("modes",)),
]


@pytest.mark.parametrize("kind,pins", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_fails_its_pin(monkeypatch, kind, pins):
    monkeypatch.setattr(O, "local_potential_g", _mutant(kind))
    for pin in pins:
        assert PINS[pin]() > 1e-4, (kind, pin)


# --- LOBPCG search directions ------------------------------------------------------------------

@pytest.fixture(scope="module")
def si8_dense():
    cell = synth.make_cell("si8")
    model = O.model_from_cell(cell)
    H = O.dense_h(model)
    return model, H, np.linalg.eigvalsh(H)


def test_lobpcg_new_directions_complete_x_within_span_x(si8_dense):
    """X' = Z C_1 = X C_1[X rows] + P' by construction: X' - P' lies in span X.  A P' built from the
    wrong rows of C_1, or from R alone when P is in the basis, leaves a component outside span X."""
    model, H, lam = si8_dense
    hop = lambda Y: H @ Y
    rng = np.random.default_rng(21)
    X, _ = np.linalg.qr(rng.standard_normal((model.npw, 8)) + 1j * rng.standard_normal((model.npw, 8)))
    r1 = O.lobpcg_step(hop, X, None, model.kin)
    r2 = O.lobpcg_step(hop, r1.X, r1.P, model.kin)
    for prev, res in ((X, r1), (r1.X, r2)):
        Q, _ = np.linalg.qr(prev)
        D = res.X - res.P
        out = D - Q @ (Q.conj().T @ D)
        assert np.abs(out).max() < 1e-10
        # and P' is not trivially zero: the step moved X out of its old span
        assert np.linalg.norm(res.P) > 1e-3


def test_lobpcg_directions_accelerate_convergence(si8_dense):
    """With the search directions the iteration is a conjugate-gradient method: it needs clearly
    fewer steps than the same steps on span[X, R] alone (preconditioned steepest descent)."""
    model, H, lam = si8_dense
    hop = lambda Y: H @ Y
    nb, nconv, tol = 10, 8, 1e-8

    def steps(use_p):
        rng = np.random.default_rng(12)
        X, _ = np.linalg.qr(rng.standard_normal((model.npw, nb)) + 1j * rng.standard_normal((model.npw, nb)))
        P = None
        for it in range(1, 400):
            r = O.lobpcg_step(hop, X, P if use_p else None, model.kin)
            X, P = r.X, r.P
            if r.resid[:nconv].max() < tol:
                assert np.abs(r.eig[:nconv] - lam[:nconv]).max() < 1e-9
                return it
        return 400

    with_p, without_p = steps(True), steps(False)
    assert with_p < 400
    assert with_p <= 0.75 * without_p, (with_p, without_p)
