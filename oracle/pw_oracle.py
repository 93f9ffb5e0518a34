"""Plain CPU FP64 oracle for one block-eigensolver step of plane-wave DFT.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the bench may import this module.  It shares no code with
the HIP library: it takes the seeded inputs (atom positions, perturbation
modes, starting blocks) as plain arrays and computes everything else itself,
in float64 / complex128, with numpy and scipy primitives.

What it computes, and where the paper fixes it:

* The problem is the eigenproblem H X = X Lambda of the plane-wave
  Hamiltonian (Section II-A, Eq. 1); X are plane-wave coefficients and the
  wanted output is the lowest part of the spectrum.
* The cutoff E_cut selects the plane waves (Section II-A): a reciprocal
  lattice vector G is kept iff |G|^2 / 2 <= E_cut (Gamma point).
* The inner solver is an iterative block eigensolver (Section II-A) whose
  subspace part forms S = Psi^* (H Psi) and solves a dense Hermitian
  eigenproblem ("Syevd", Sections II-B and III-D).
* The pseudopotential acts atom by atom on every wavefunction
  (Section III-A); here as Kleinman-Bylander projectors B D B^H.  A second
  projector family (PROJ_LOCALIZED: a Gaussian and a Gaussian times x, y, z in
  real space) vanishes a few widths from its atom, so V_NL can also be applied
  on the real-space grid over a ball around each atom
  (apply_nonlocal_realspace), touching only the grid points near the atom.

Where the paper is silent the readings are: a Chebyshev-filtered subspace
step (degree m; m = 0 is plain Rayleigh-Ritz), an alias-free FFT grid, a
potential band-limited to the wavefunction sphere, real spherical harmonics,
structure factors exp(-i G.tau), and the unnormalised inverse FFT
psi(r) = sum_G c_G exp(+i G.r).

Every function below is pinned by tests in tests/test_oracle_pins.py and the
other tests/test_oracle_*_pins.py files (the localized projectors and the
real-space route in tests/test_oracle_realspace_pins.py).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional, Sequence, Tuple

import numpy as np
import scipy.fft
import scipy.linalg

TWO_PI = 2.0 * math.pi

# Worker threads for scipy.fft (-1: all CPUs); the CPU-baseline timing sets it explicitly.
FFT_WORKERS = -1


# ----------------------------------------------------------------------------
# Basis and grid (Section II-A: E_cut fixes the basis and the real-space grid)
# ----------------------------------------------------------------------------

def sphere_millers(L: Sequence[float], ecut: float) -> np.ndarray:
    """All Miller triples n with |G|^2/2 <= ecut, G = 2 pi n / L, sorted n1, n2, n3."""
    L = np.asarray(L, float)
    nmax = [int(math.floor(math.sqrt(2.0 * ecut) * L[i] / TWO_PI)) for i in range(3)]
    r = [np.arange(-nmax[i], nmax[i] + 1) for i in range(3)]
    n1, n2, n3 = np.meshgrid(r[0], r[1], r[2], indexing="ij")
    n = np.stack([n1.ravel(), n2.ravel(), n3.ravel()], axis=1)
    g2 = ((TWO_PI * n / L) ** 2).sum(axis=1)
    return n[0.5 * g2 <= ecut].astype(np.int64)


def gvectors(miller: np.ndarray, L: Sequence[float]) -> np.ndarray:
    """Cartesian G = 2 pi (n1/L1, n2/L2, n3/L3)."""
    return TWO_PI * np.asarray(miller, float) / np.asarray(L, float)


def paper_grid(L: Sequence[float], ecut: float) -> Tuple[int, ...]:
    """The paper's grid rule (Section II-A): N_i = sqrt(2 E_cut) L_i / pi,

    rounded up to the next size whose prime factors are all <= 7 (a common
    FFT size set; the paper does not state its rounding).  Used only to check
    Table I; the oracle itself uses the alias-free grid of fft_grid().
    """
    out = []
    for Li in L:
        x = math.sqrt(2.0 * ecut) * Li / math.pi
        n = int(math.ceil(x - 1e-9))
        while True:
            m = n
            for p in (2, 3, 5, 7):
                while m % p == 0:
                    m //= p
            if m == 1:
                break
            n += 1
        out.append(n)
    return tuple(out)


def fft_grid(L: Sequence[float], ecut: float) -> Tuple[int, int, int]:
    """Alias-free grid: N_i = smallest 2^p 3^q >= 3 floor(n_max,i) + 1.

    A product V(r) psi(r) with both factors band-limited to |n_i| <= n_max
    has components up to 2 n_max; projecting back on the sphere is exact iff
    N_i > 3 n_max.
    """
    out = []
    for Li in L:
        nmax = int(math.floor(math.sqrt(2.0 * ecut) * Li / TWO_PI))
        need = 3 * nmax + 1
        best = None
        p2 = 1
        while p2 < 4 * need:
            p3 = p2
            while p3 < 4 * need:
                if p3 >= need and (best is None or p3 < best):
                    best = p3
                p3 *= 3
            p2 *= 2
        out.append(best)
    return tuple(out)


# ----------------------------------------------------------------------------
# Potential and projectors (analytic synthetic pseudopotential)
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Model:
    """Everything H needs, built once from a cell description."""

    L: np.ndarray
    ecut: float
    tau: np.ndarray
    miller: np.ndarray  # (npw, 3)
    G: np.ndarray  # (npw, 3)
    kin: np.ndarray  # (npw,)   |G|^2/2
    grid: Tuple[int, int, int]
    vr: np.ndarray  # real-space local potential on the grid, indexed [j1, j2, j3]
    B: np.ndarray  # (npw, 4*natoms) projector matrix
    D: np.ndarray  # (4*natoms,) KB energies
    zval: float
    rc: float
    gauss_c: float
    mode_miller: np.ndarray
    mode_amp: np.ndarray
    mode_phase: np.ndarray
    sf_sign: float = -1.0

    @property
    def npw(self) -> int:
        return self.miller.shape[0]

    @property
    def omega(self) -> float:
        return float(np.prod(self.L))


def local_potential_g(miller: np.ndarray, L: np.ndarray, ecut: float, tau: np.ndarray,
                      zval: float, rc: float, gauss_c: float, mode_miller: np.ndarray,
                      mode_amp: np.ndarray, mode_phase: np.ndarray,
                      sf_sign: float = -1.0) -> np.ndarray:
    """V(G) for arbitrary Miller triples.

    V(G) = S(G) v(|G|) + dV(G) for 0 < |G|^2/2 <= ecut, and 0 otherwise, with
      v(G) = (1/Omega) (-4 pi Z exp(-G^2 rc^2/4) / G^2 + c exp(-G^2 rc^2/4)),
      S(G) = sum_a exp(sf_sign * i G.tau_a),
      dV(+-G_k) = (amp_k/2) exp(+-i phase_k)  (from amp cos(G_k.r + phase_k)).
    """
    miller = np.asarray(miller, np.int64)
    G = gvectors(miller, L)
    g2 = (G * G).sum(axis=1)
    omega = float(np.prod(L))
    inside = (g2 > 0) & (0.5 * g2 <= ecut)
    out = np.zeros(miller.shape[0], complex)
    if np.any(inside):
        gi = G[inside]
        g2i = g2[inside]
        gauss = np.exp(-g2i * rc * rc / 4.0)
        v = (-4.0 * math.pi * zval * gauss / g2i + gauss_c * gauss) / omega
        phase = gi @ np.asarray(tau, float).T  # (n, natoms)
        sf = np.exp(sf_sign * 1j * phase).sum(axis=1)
        out[inside] = sf * v
    for k in range(mode_miller.shape[0]):
        mk = mode_miller[k]
        plus = np.all(miller == mk, axis=1) & inside
        minus = np.all(miller == -mk, axis=1) & inside
        out[plus] += 0.5 * mode_amp[k] * np.exp(1j * mode_phase[k])
        out[minus] += 0.5 * mode_amp[k] * np.exp(-1j * mode_phase[k])
    return out


def real_harmonics_l01(G: np.ndarray) -> np.ndarray:
    """Real spherical harmonics Y_00, Y_1x, Y_1y, Y_1z of the direction of G.

    Y_00 = 1/(2 sqrt(pi)); Y_1a = sqrt(3/(4 pi)) G_a/|G|; Y_1a(0) = 0.
    """
    g = np.sqrt((G * G).sum(axis=1))
    out = np.zeros((G.shape[0], 4))
    out[:, 0] = 0.5 / math.sqrt(math.pi)
    nz = g > 0
    c1 = math.sqrt(3.0 / (4.0 * math.pi))
    for a in range(3):
        out[nz, 1 + a] = c1 * G[nz, a] / g[nz]
    return out


PROJ_GSPACE = 0      # projectors exp(-sigma^2 |G|^2/2) Y_lm(G/|G|) (reading A7)
PROJ_LOCALIZED = 1   # projectors that are Gaussians times r^l Y_lm in real space


def projector_matrix(miller: np.ndarray, L: np.ndarray, tau: np.ndarray, sigma: float,
                     sf_sign: float = -1.0, form: int = PROJ_GSPACE) -> np.ndarray:
    """B[G, 4a+m] = (c/sqrt(Omega)) exp(-sigma^2 |G|^2/2) Y_m(G) exp(sf_sign i G.tau_a).

    c = sqrt(32 pi^(5/2) sigma^3) gives unit norm in the continuum limit.
    Projector order per atom: l=0, then l=1 x, y, z.

    form PROJ_LOCALIZED keeps l = 0 and replaces the l = 1 direction factor sqrt(3/(4 pi)) G_m/|G|
    by -i sigma G_m / sqrt(2 pi): the columns are then (1/sqrt(Omega)) times the continuum Fourier
    transforms, integral p(r - tau) exp(-i G.r) d^3r, of the unit-norm real-space functions of
    `localized_projector_values` (a Gaussian and a Gaussian times x, y, z), so that each
    projector vanishes beyond a few sigma of its atom (Section III-A: a projector acts near its
    atom only).
    """
    G = gvectors(miller, L)
    g2 = (G * G).sum(axis=1)
    omega = float(np.prod(L))
    c = math.sqrt(32.0 * math.pi ** 2.5 * sigma ** 3)
    radial = (c / math.sqrt(omega)) * np.exp(-0.5 * sigma * sigma * g2)
    if form == PROJ_LOCALIZED:
        ylm = np.empty((G.shape[0], 4), complex)
        ylm[:, 0] = 0.5 / math.sqrt(math.pi)
        for a in range(3):
            ylm[:, 1 + a] = -1j * sigma * G[:, a] / math.sqrt(2.0 * math.pi)
    else:
        ylm = real_harmonics_l01(G)
    natoms = tau.shape[0]
    B = np.empty((G.shape[0], 4 * natoms), complex)
    for a in range(natoms):
        sf = np.exp(sf_sign * 1j * (G @ tau[a]))
        for m in range(4):
            B[:, 4 * a + m] = radial * ylm[:, m] * sf
    return B


def localized_projector_values(d: np.ndarray, sigma: float) -> np.ndarray:
    """The four real-space projector functions of one atom at displacements d (..., 3) from it,
    shape (4, ...): p_0 = pi^(-3/4) sigma^(-3/2) e^(-|d|^2/(2 sigma^2)) and
    p_m = sqrt(2) pi^(-3/4) sigma^(-5/2) d_m e^(-|d|^2/(2 sigma^2)) (m = x, y, z), each of unit
    norm over all space."""
    g = np.exp(-0.5 * (d * d).sum(axis=-1) / (sigma * sigma))
    c0 = math.pi ** -0.75 * sigma ** -1.5
    c1 = math.sqrt(2.0) * math.pi ** -0.75 * sigma ** -2.5
    return np.stack([c0 * g, c1 * d[..., 0] * g, c1 * d[..., 1] * g, c1 * d[..., 2] * g])


def ball_points(L: np.ndarray, grid: Sequence[int], tau: np.ndarray, radius: float):
    """Grid points within `radius` of tau (nearest periodic image): (flat indices into the
    (N1, N2, N3) grid, displacements r_j - tau of shape (npts, 3)).  Needs 2 radius < min L, so
    that no point is near two images of the atom."""
    L = np.asarray(L, float)
    assert 2.0 * radius < L.min(), "ball radius must stay below half the cell"
    h = L / np.asarray(grid, float)
    rng = []
    for i in range(3):
        lo = int(math.ceil((tau[i] - radius) / h[i]))
        hi = int(math.floor((tau[i] + radius) / h[i]))
        rng.append(np.arange(lo, hi + 1))
    j1, j2, j3 = np.meshgrid(rng[0], rng[1], rng[2], indexing="ij")
    j = np.stack([j1.ravel(), j2.ravel(), j3.ravel()], axis=1)
    d = j * h - tau
    keep = (d * d).sum(axis=1) <= radius * radius
    j, d = j[keep], d[keep]
    N = np.asarray(grid)
    jw = np.mod(j, N)
    flat = (jw[:, 0] * N[1] + jw[:, 1]) * N[2] + jw[:, 2]
    return flat, d


def apply_nonlocal_realspace(model: "Model", X: np.ndarray, radius: float) -> np.ndarray:
    """V_NL X with the localized projectors applied on the real-space grid, each truncated to the
    ball of `radius` around its atom (the one-GPU form of Section III-A's atom-by-atom
    pseudopotential: a projector touches only the grid points near its atom):

        psi_n(r)       = (1/sqrt(Omega)) sum_G X[G, n] e^{i G.r}        (normalised wavefunction)
        P[a, m, n]     = dV sum_{r in ball a} p_m(r - tau_a) psi_n(r)      (dV = Omega / N_r)
        NL_n(r)        = sum_a sum_m p_m(r - tau_a) D_m P[a, m, n]
        (V_NL X)[G, n] = (1/sqrt(Omega)) dV sum_r NL_n(r) e^{-i G.r}

    Without truncation this equals B D B^H X of the PROJ_LOCALIZED columns up to aliasing of the
    projectors beyond the grid's reciprocal box."""
    omega = model.omega
    grid = model.grid
    nr = int(np.prod(grid))
    dv = omega / nr
    X = np.asarray(X, complex)
    psi = to_real_space(X, model.miller, grid).reshape(X.shape[1], nr) / math.sqrt(omega)
    nl = np.zeros_like(psi)
    d = model.D[:4]
    for a in range(model.tau.shape[0]):
        flat, disp = ball_points(model.L, grid, model.tau[a], radius)
        p = localized_projector_values(disp, model.sigma)          # (4, npts)
        Pa = dv * (psi[:, flat] @ p.T)                              # (nb, 4)
        nl[:, flat] += (Pa * d[None, :]) @ p                        # (nb, npts)
    nl = nl.reshape((X.shape[1],) + tuple(grid))
    # to_g_space includes 1/N_r; (1/sqrt(Omega)) dV N_r = sqrt(Omega)
    return math.sqrt(omega) * to_g_space(nl, model.miller)


def scatter_to_grid(x: np.ndarray, miller: np.ndarray, grid: Sequence[int]) -> np.ndarray:
    """Place sphere coefficients on the FFT grid at n mod N.

    x of shape (npw,) gives a grid (N1, N2, N3); x of shape (npw, nb) gives (nb, N1, N2, N3).
    """
    N = tuple(grid)
    idx = tuple(np.mod(miller[:, i], N[i]) for i in range(3))
    if x.ndim == 1:
        out = np.zeros(N, complex)
        out[idx] = x
        return out
    out = np.zeros((x.shape[1],) + N, complex)
    out[(slice(None),) + idx] = x.T
    return out


def gather_from_grid(f: np.ndarray, miller: np.ndarray) -> np.ndarray:
    """Inverse of scatter_to_grid: (N1, N2, N3) -> (npw,), (nb, N1, N2, N3) -> (npw, nb)."""
    N = f.shape[-3:]
    idx = tuple(np.mod(miller[:, i], N[i]) for i in range(3))
    if f.ndim == 3:
        return f[idx]
    return f[(slice(None),) + idx].T


def to_real_space(c: np.ndarray, miller: np.ndarray, grid: Sequence[int]) -> np.ndarray:
    """psi(r_j) = sum_G c_G exp(+i G.r_j): unnormalised inverse DFT (bands first for blocks)."""
    f = scatter_to_grid(c, miller, grid)
    return scipy.fft.ifftn(f, axes=(-3, -2, -1), norm="forward", workers=FFT_WORKERS)


def to_g_space(f: np.ndarray, miller: np.ndarray) -> np.ndarray:
    """c_G = (1/N_r) sum_j f(r_j) exp(-i G.r_j), gathered on the sphere."""
    F = scipy.fft.fftn(f, axes=(-3, -2, -1), norm="forward", workers=FFT_WORKERS)
    return gather_from_grid(F, miller)


def density(X: np.ndarray, occ: np.ndarray, miller: np.ndarray, grid: Sequence[int]) -> np.ndarray:
    """Charge density from the eigenfunctions (Section II-A, the SCF part): the weighted sum of
    |psi_n(r_j)|^2 over the bands, psi_n the unnormalised inverse DFT of column n of X (npw x nb).
    occ holds one weight per band (the paper sums |psi_j|^2 over its occupied index range; here
    the caller states the weights, e.g. 2 for a doubly occupied band).  Grid shape (N1, N2, N3)."""
    rho = np.zeros(tuple(grid))
    for n in range(X.shape[1]):
        if occ[n] != 0.0:
            psi = to_real_space(X[:, n], miller, grid)
            rho += occ[n] * (psi.real ** 2 + psi.imag ** 2)
    return rho


def build_model(L: Sequence[float], tau: np.ndarray, ecut: float, zval: float = 4.0,
                rc: float = 1.0, gauss_c: float = 2.0, sigma: float = 0.8, d0: float = 1.5,
                d1: float = -0.7, mode_miller: Optional[np.ndarray] = None,
                mode_amp: Optional[np.ndarray] = None, mode_phase: Optional[np.ndarray] = None,
                grid: Optional[Sequence[int]] = None, sf_sign: float = -1.0,
                with_projectors: bool = True, proj_form: int = PROJ_GSPACE,
                rs_radius: float = 0.0) -> Model:
    """rs_radius > 0 (PROJ_LOCALIZED only) makes apply_h take the nonlocal part in real space on
    balls of that radius (apply_nonlocal_realspace); B still holds the reciprocal-space columns."""
    L = np.asarray(L, float)
    tau = np.asarray(tau, float)
    mm = np.zeros((0, 3), np.int64) if mode_miller is None else np.asarray(mode_miller, np.int64)
    ma = np.zeros(0) if mode_amp is None else np.asarray(mode_amp, float)
    mp = np.zeros(0) if mode_phase is None else np.asarray(mode_phase, float)
    miller = sphere_millers(L, ecut)
    G = gvectors(miller, L)
    kin = 0.5 * (G * G).sum(axis=1)
    grid = tuple(fft_grid(L, ecut)) if grid is None else tuple(grid)
    vg = local_potential_g(miller, L, ecut, tau, zval, rc, gauss_c, mm, ma, mp, sf_sign)
    vr_c = to_real_space(vg, miller, grid)
    scale = max(1.0, float(np.abs(vr_c).max()))
    assert float(np.abs(vr_c.imag).max()) <= 1e-12 * scale, "V(r) must be real"
    have = (d0 != 0 or d1 != 0) and tau.shape[0] > 0
    B = projector_matrix(miller, L, tau, sigma, sf_sign, proj_form) if (have and with_projectors) else \
        np.zeros((miller.shape[0], 0), complex)
    D = np.tile(np.array([d0, d1, d1, d1]), tau.shape[0]) if have else np.zeros(0)
    m = Model(L=L, ecut=ecut, tau=tau, miller=miller, G=G, kin=kin, grid=grid,
              vr=vr_c.real.copy(), B=B, D=D, zval=zval, rc=rc, gauss_c=gauss_c,
              mode_miller=mm, mode_amp=ma, mode_phase=mp, sf_sign=sf_sign)
    m.sigma = sigma
    m.atomwise = have and not with_projectors
    if rs_radius > 0.0:
        assert proj_form == PROJ_LOCALIZED, "real-space projectors need the localized form"
    m.proj_form = proj_form
    m.rs_radius = rs_radius if have else 0.0
    return m


def model_from_cell(cell, **over) -> Model:
    """Convenience: build from a synth.Cell-like object (duck-typed)."""
    p = cell.pseudo
    kw = dict(zval=p.zval, rc=p.rc, gauss_c=p.gauss_c, sigma=p.beta_sigma, d0=p.d0, d1=p.d1,
              mode_miller=cell.modes.miller, mode_amp=cell.modes.amp,
              mode_phase=cell.modes.phase)
    kw.update(over)
    return build_model(cell.L, cell.tau, cell.ecut, **kw)


# ----------------------------------------------------------------------------
# The Hamiltonian (Section II-A, Eq. 1)
# ----------------------------------------------------------------------------

def dense_h(model: Model) -> np.ndarray:
    """H[G, G'] = delta ½|G|^2 + V(G - G') + sum_p B[G,p] D_p conj(B[G',p]).

    V(G - G') is evaluated from the analytic formula (with the band limit),
    not through an FFT.  Only for tiny cells (npw up to a few thousand).
    """
    m = model.miller
    # Every difference n - n' lies in the box |d_i| <= 2 max|n_i|: tabulate V there.
    span = 2 * np.abs(m).max(axis=0)
    r = [np.arange(-span[i], span[i] + 1) for i in range(3)]
    d1, d2, d3 = np.meshgrid(r[0], r[1], r[2], indexing="ij")
    box = np.stack([d1.ravel(), d2.ravel(), d3.ravel()], axis=1)
    vbox = local_potential_g(box, model.L, model.ecut, model.tau, model.zval, model.rc,
                             model.gauss_c, model.mode_miller, model.mode_amp,
                             model.mode_phase, model.sf_sign)
    vbox = vbox.reshape(d1.shape)
    i1 = m[:, None, 0] - m[None, :, 0] + span[0]
    i2 = m[:, None, 1] - m[None, :, 1] + span[1]
    i3 = m[:, None, 2] - m[None, :, 2] + span[2]
    H = vbox[i1, i2, i3]
    H = H + np.diag(model.kin)
    if model.B.shape[1]:
        H = H + (model.B * model.D) @ model.B.conj().T
    return H


def apply_nonlocal_atomwise(model: Model, X: np.ndarray,
                            progress: Optional[Callable[[int], None]] = None) -> np.ndarray:
    """V_NL X = sum_a B_a D (B_a^H X), one atom at a time (Section III-A: the pseudopotential
    of each atom is applied to every wavefunction).  Never forms the full projector matrix.
    progress, when given, is called with the number of atoms done after every 64 atoms."""
    out = np.zeros_like(X)
    d = model.D[:4]
    for a in range(model.tau.shape[0]):
        Ba = projector_matrix(model.miller, model.L, model.tau[a:a + 1], model.sigma, model.sf_sign,
                               getattr(model, "proj_form", PROJ_GSPACE))
        out += Ba @ (d[:, None] * (Ba.conj().T @ X))
        if progress is not None and (a + 1) % 64 == 0:
            progress(a + 1)
    return out


def apply_h(model: Model, X: np.ndarray) -> np.ndarray:
    """Matrix-free H X: kinetic + FFT local potential + B (D (B^H X))."""
    X = np.asarray(X, complex)
    one = X.ndim == 1
    Xb = X[:, None] if one else X
    out = model.kin[:, None] * Xb
    chunk = 16
    for j in range(0, Xb.shape[1], chunk):
        psi = to_real_space(Xb[:, j:j + chunk], model.miller, model.grid)
        out[:, j:j + chunk] += to_g_space(model.vr[None] * psi, model.miller)
    if getattr(model, "rs_radius", 0.0) > 0.0:
        out = out + apply_nonlocal_realspace(model, Xb, model.rs_radius)
    elif model.B.shape[1]:
        P = model.B.conj().T @ Xb
        out = out + model.B @ (model.D[:, None] * P)
    elif getattr(model, "atomwise", False):
        out = out + apply_nonlocal_atomwise(model, Xb)
    return out[:, 0] if one else out


# ----------------------------------------------------------------------------
# One step of the block eigensolver (Chebyshev-filtered subspace iteration)
# ----------------------------------------------------------------------------

def chebyshev_filter(hop: Callable[[np.ndarray], np.ndarray], X: np.ndarray, m: int,
                     a_lo: float, a: float, b: float) -> np.ndarray:
    """Scaled degree-m Chebyshev filter that damps [a, b] and keeps values near a_lo.

    With e = (b-a)/2, c = (b+a)/2, s_1 = e/(a_lo - c), tau = 2/s_1:
      Y_1 = (s_1/e) (H - c) X,
      s_{k+1} = 1/(tau - s_k),
      Y_{k+1} = (2 s_{k+1}/e) (H - c) Y_k - s_k s_{k+1} Y_{k-1},  Y_0 = X.
    Result: T_m((H - c)/e) X / T_m((a_lo - c)/e).
    """
    if m == 0:
        return X.copy()
    e = 0.5 * (b - a)
    c = 0.5 * (b + a)
    s1 = e / (a_lo - c)
    tau = 2.0 / s1
    y_prev = X
    y = (hop(X) - c * X) * (s1 / e)
    s = s1
    for _ in range(1, m):
        s_new = 1.0 / (tau - s)
        y_new = (2.0 * s_new / e) * (hop(y) - c * y) - (s * s_new) * y_prev
        y_prev, y = y, y_new
        s = s_new
    return y


@dataclasses.dataclass
class StepResult:
    eig: np.ndarray
    X: np.ndarray
    HX: np.ndarray
    resid: np.ndarray
    a_lo: float
    a: float


def rayleigh_ritz(Y: np.ndarray, W: np.ndarray):
    """Generalised Rayleigh-Ritz on span(Y) with W = H Y (Sections II-B, III-D).

    S = Y^H Y, H_s = Y^H W (both symmetrised), S = L L^H, L^-1 H_s L^-H = Q diag(lam) Q^H,
    C = L^-H Q.  Raises numpy.linalg.LinAlgError if S is not positive definite.
    """
    S = Y.conj().T @ Y
    Hs = Y.conj().T @ W
    S = 0.5 * (S + S.conj().T)
    Hs = 0.5 * (Hs + Hs.conj().T)
    Lc = np.linalg.cholesky(S)
    T = scipy.linalg.solve_triangular(Lc, Hs, lower=True)
    Hh = scipy.linalg.solve_triangular(Lc, T.conj().T, lower=True)
    Hh = 0.5 * (Hh + Hh.conj().T)
    lam, Q = np.linalg.eigh(Hh)
    C = scipy.linalg.solve_triangular(Lc.conj().T, Q, lower=False)
    return lam, C


def eig_step(hop: Callable[[np.ndarray], np.ndarray], X: np.ndarray, m: int, a_lo: float,
             a: float, b: float) -> StepResult:
    """One block-eigensolver step: filter, W = H Y, Rayleigh-Ritz, rotate, residuals."""
    Y = chebyshev_filter(hop, X, m, a_lo, a, b)
    W = hop(Y)
    lam, C = rayleigh_ritz(Y, W)
    Xn = Y @ C
    Wn = W @ C
    R = Wn - Xn * lam[None, :]
    resid = np.sqrt((np.abs(R) ** 2).sum(axis=0))
    return StepResult(eig=lam, X=Xn, HX=Wn, resid=resid, a_lo=float(lam[0]), a=float(lam[-1]))


def svqb_rayleigh_ritz(S: np.ndarray, Hs: np.ndarray, drop_tol: float):
    """Rayleigh-Ritz on the span of a basis whose Gram matrix S may be singular (S, Hs Hermitian).

    The basis is scaled to unit columns (D = diag(S)^-1/2; a zero column gets weight 0), the
    scaled Gram matrix is diagonalised, D S D = U diag(sigma) U^H, and the directions with
    sigma <= drop_tol * max(sigma) are dropped: T = D U_kept diag(sigma_kept)^-1/2 spans the kept
    part of the span with T^H S T = I (the SVQB orthonormalisation of Stathopoulos and Wu, here
    with truncation).  Then T^H Hs T = V diag(lam) V^H and C = T V, so that C^H S C = I and
    C^H Hs C = diag(lam).  Returns lam (ascending), C (k x k_kept) and k_kept.
    """
    dS = np.real(np.diag(S)).copy()
    d = np.where(dS > 0.0, 1.0 / np.sqrt(np.where(dS > 0.0, dS, 1.0)), 0.0)
    St = d[:, None] * S * d[None, :]
    St = 0.5 * (St + St.conj().T)
    sig, U = np.linalg.eigh(St)
    keep = sig > drop_tol * sig.max()
    T = d[:, None] * U[:, keep] / np.sqrt(sig[keep])[None, :]
    A = T.conj().T @ Hs @ T
    A = 0.5 * (A + A.conj().T)
    lam, V = np.linalg.eigh(A)
    return lam, T @ V, int(keep.sum())


def numerically_definite(S: np.ndarray, drop_tol: Optional[float]) -> bool:
    """Whether a Gram matrix is safe for the Cholesky-based Rayleigh-Ritz: its Cholesky factor
    exists and every pivot keeps more than drop_tol of its diagonal entry, |L_ii|^2 > drop_tol S_ii
    (the squared sine between column i and the span of the columns before it, for unit columns).
    Without drop_tol a failed factorisation raises numpy.linalg.LinAlgError."""
    try:
        Lc = np.linalg.cholesky(S)
    except np.linalg.LinAlgError:
        if drop_tol is None:
            raise
        return False
    if drop_tol is None:
        return True
    piv = np.abs(np.diag(Lc)) ** 2 / np.real(np.diag(S))
    return bool(piv.min() > drop_tol)


@dataclasses.dataclass
class LobpcgResult:
    X: np.ndarray  # the nb lowest Ritz vectors
    P: np.ndarray  # their components along [R, P] (the next search directions)
    eig: np.ndarray  # the nb lowest Ritz values
    resid: np.ndarray  # ||H x_i - theta_i x_i|| of the input block
    kept: int = 0  # basis directions kept in the Rayleigh-Ritz (all of them unless S was singular)


def lobpcg_step(hop: Callable[[np.ndarray], np.ndarray], X: np.ndarray, P: Optional[np.ndarray],
                kin: np.ndarray, drop_tol: Optional[float] = None) -> LobpcgResult:
    """One step of the locally optimal block preconditioned conjugate gradient method, one of
    the inner eigensolvers of Section II-A (Knyazev's block form).  The Rayleigh quotients of the
    columns of X give the residuals W - X theta; the diagonal preconditioner 1 / (1 + |G|^2/2)
    acts on them; R and P are scaled to unit columns; Rayleigh-Ritz of H on span[X, R, P] (or
    span[X, R] without P) keeps the nb lowest Ritz pairs; the new P is the part of the new X
    along [R, P].  When drop_tol is given and the Gram matrix of [X, R, P] is not numerically
    positive definite (numerically_definite), the Rayleigh-Ritz runs on the kept part of the span
    (svqb_rayleigh_ritz) instead of failing."""
    nb = X.shape[1]
    W = hop(X)
    theta = np.real(np.sum(X.conj() * W, axis=0)) / np.real(np.sum(X.conj() * X, axis=0))
    Rraw = W - X * theta
    resid = np.linalg.norm(Rraw, axis=0)
    R = Rraw / (1.0 + kin)[:, None]
    R = R / np.linalg.norm(R, axis=0)
    blocks = [X, R]
    if P is not None:
        blocks.append(P / np.linalg.norm(P, axis=0))
    Z = np.hstack(blocks)
    HZ = hop(Z)
    S = Z.conj().T @ Z
    Hs = Z.conj().T @ HZ
    S = 0.5 * (S + S.conj().T)
    Hs = 0.5 * (Hs + Hs.conj().T)
    kept = Z.shape[1]
    if numerically_definite(S, drop_tol):
        lam, C = scipy.linalg.eigh(Hs, S)
    else:
        lam, C, kept = svqb_rayleigh_ritz(S, Hs, drop_tol)
    C1 = C[:, :nb]
    return LobpcgResult(X=Z @ C1, P=Z[:, nb:] @ C1[nb:], eig=lam[:nb], resid=resid, kept=kept)


@dataclasses.dataclass
class PpcgResult:
    X: np.ndarray  # the next iterate (columns x_j', not orthonormalised)
    P: np.ndarray  # the next search directions p_j'
    eig: np.ndarray  # Ritz values of the input block
    resid: np.ndarray  # ||H x_j - lam_j x_j|| of the input block's Ritz vectors
    coef: np.ndarray  # nb x 3 coefficients (alpha, beta, gamma) of x_j' on (x_j, w_j, p_j)


def small_lowest_pair(G: np.ndarray, A: np.ndarray, drop_tol: float) -> np.ndarray:
    """The lowest Ritz vector of the pencil (A, G) on a basis of up to three vectors (G their Gram
    matrix, A the matrix of H on them), by svqb_rayleigh_ritz, with its phase fixed so that its
    first component is real and non-negative."""
    _, C, _ = svqb_rayleigh_ritz(G, A, drop_tol)
    c = C[:, 0]
    if abs(c[0]) > 0.0:
        c = c * (abs(c[0]) / c[0])
    return c


def ppcg_step(hop: Callable[[np.ndarray], np.ndarray], X: np.ndarray, P: Optional[np.ndarray],
              kin: np.ndarray, drop_tol: float) -> PpcgResult:
    """One step of the projected preconditioned conjugate gradient method (Vecharynski, Yang and
    Pask), one of the inner eigensolvers of Section II-A, in this order:

    1. Rayleigh-Ritz on span X (X^H X and X^H H X, FP64 generalised eigenproblem): X <- X C are
       the Ritz vectors, lam their Ritz values; the directions follow the columns, P <- P C.
    2. Residuals R = H X - X diag(lam); preconditioned residuals W = K R with the diagonal
       K = 1 / (1 + |G|^2/2); W and P are projected against span X: Y <- Y - X (X^H Y).
    3. For each column j, Rayleigh-Ritz of H on span{x_j, w_j, p_j} (span{x_j, w_j} without P):
       the lowest Ritz vector x_j' = alpha x_j + beta w_j + gamma p_j (alpha real >= 0), and
       p_j' = beta w_j + gamma p_j.  The entry of H for (x_j, x_j) is lam_j.

    The next step's Rayleigh-Ritz orthonormalises X' again, so the output is not orthonormal."""
    nb = X.shape[1]
    HX = hop(X)
    S = X.conj().T @ X
    Hs = X.conj().T @ HX
    lam, C = rayleigh_ritz_gram(0.5 * (S + S.conj().T), 0.5 * (Hs + Hs.conj().T))
    X = X @ C
    HX = HX @ C
    if P is not None:
        P = P @ C
    R = HX - X * lam[None, :]
    resid = np.linalg.norm(R, axis=0)
    W = R / (1.0 + kin)[:, None]
    W = W - X @ (X.conj().T @ W)
    if P is not None:
        P = P - X @ (X.conj().T @ P)
    HW = hop(W)
    HP = hop(P) if P is not None else None
    Xn = np.empty_like(X)
    Pn = np.empty_like(X)
    coef = np.zeros((nb, 3), dtype=complex)
    for j in range(nb):
        basis = [X[:, j], W[:, j]] + ([P[:, j]] if P is not None else [])
        hbasis = [None, HW[:, j]] + ([HP[:, j]] if P is not None else [])
        n = len(basis)
        G = np.array([[np.vdot(basis[a], basis[b]) for b in range(n)] for a in range(n)])
        A = np.zeros((n, n), dtype=complex)
        A[0, 0] = lam[j]
        for a in range(n):
            for b in range(max(a, 1), n):
                A[a, b] = np.vdot(basis[a], hbasis[b])
                A[b, a] = np.conj(A[a, b])
        c = small_lowest_pair(0.5 * (G + G.conj().T), A, drop_tol)
        coef[j, :n] = c
        Xn[:, j] = sum(c[i] * basis[i] for i in range(n))
        Pn[:, j] = sum(c[i] * basis[i] for i in range(1, n))
    return PpcgResult(X=Xn, P=Pn, eig=lam, resid=resid, coef=coef)


def rayleigh_ritz_gram(S: np.ndarray, Hs: np.ndarray):
    """Rayleigh-Ritz from the Gram matrix S and the projected matrix Hs of a basis (the second half
    of rayleigh_ritz): S = L L^H, L^-1 Hs L^-H = Q diag(lam) Q^H, C = L^-H Q."""
    Lc = np.linalg.cholesky(S)
    T = scipy.linalg.solve_triangular(Lc, Hs, lower=True)
    Hh = scipy.linalg.solve_triangular(Lc, T.conj().T, lower=True)
    Hh = 0.5 * (Hh + Hh.conj().T)
    lam, Q = np.linalg.eigh(Hh)
    return lam, scipy.linalg.solve_triangular(Lc.conj().T, Q, lower=False)


def lanczos_max(hop: Callable[[np.ndarray], np.ndarray], npw: int, steps: int = 20,
                seed: int = 7) -> float:
    """Largest Ritz value of a `steps`-step Lanczos run from a seeded random vector."""
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.standard_normal(npw) + 1j * rng.standard_normal(npw)
    v /= np.linalg.norm(v)
    v_prev = np.zeros_like(v)
    alpha, beta = [], []
    bprev = 0.0
    for _ in range(min(steps, npw)):
        w = hop(v) - bprev * v_prev
        al = float(np.vdot(v, w).real)
        w = w - al * v
        bt = float(np.linalg.norm(w))
        alpha.append(al)
        beta.append(bt)
        if bt < 1e-14:
            break
        v_prev, v, bprev = v, w / bt, bt
    k = len(alpha)
    T = np.diag(alpha) + np.diag(beta[: k - 1], 1) + np.diag(beta[: k - 1], -1)
    ev = np.linalg.eigvalsh(T)
    return float(ev[-1] + beta[k - 1])


@dataclasses.dataclass
class SolveResult:
    eig: np.ndarray
    X: np.ndarray
    resid: np.ndarray
    steps: int
    converged: bool


def solve(hop: Callable[[np.ndarray], np.ndarray], X0: np.ndarray, b: float, nocc: int,
          tol: float = 1e-7, m: int = 10, max_steps: int = 200) -> SolveResult:
    """Iterate steps: first m = 0 (bounds), then degree m until max resid over nocc <= tol."""
    st = eig_step(hop, X0, 0, 0.0, 0.0, b)
    steps = 1
    while True:
        if float(st.resid[:nocc].max()) <= tol:
            return SolveResult(st.eig, st.X, st.resid, steps, True)
        if steps >= max_steps:
            return SolveResult(st.eig, st.X, st.resid, steps, False)
        st = eig_step(hop, st.X, m, st.a_lo, st.a, b)
        steps += 1


# ----------------------------------------------------------------------------
# Comparison helpers (degenerate clusters; several answers are correct)
# ----------------------------------------------------------------------------

def clusters(eig: np.ndarray, gap: float = 1e-3):
    """Split sorted eigenvalues into runs whose consecutive gaps are < gap."""
    out = []
    start = 0
    for i in range(1, len(eig) + 1):
        if i == len(eig) or eig[i] - eig[i - 1] >= gap:
            out.append((start, i))
            start = i
    return out


def subspace_sin(Xref: np.ndarray, X: np.ndarray) -> float:
    """sin of the largest principal angle between span(Xref) and span(X)."""
    Qr, _ = np.linalg.qr(Xref)
    Qx, _ = np.linalg.qr(X)
    R = Qx - Qr @ (Qr.conj().T @ Qx)
    return float(np.linalg.norm(R, 2))


def chebyshev_t(m: int, x: np.ndarray) -> np.ndarray:
    """T_m(x) by its trigonometric / hyperbolic closed form."""
    x = np.asarray(x, float)
    out = np.empty_like(x)
    inside = np.abs(x) <= 1
    out[inside] = np.cos(m * np.arccos(x[inside]))
    xo = x[~inside]
    out[~inside] = np.cosh(m * np.arccosh(np.abs(xo))) * np.sign(xo) ** m
    return out
