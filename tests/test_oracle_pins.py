"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test names what it pins; together they are chosen so that a plausible
mistake in the oracle (a dropped term, a wrong sign or index, a transposed
operand, a wrong constant) fails at least one of them.  CPU only.
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg

from oracle import pw_oracle as O
from paper_2406_10765_amd import synth


@pytest.fixture(scope="module")
def si8():
    cell = synth.make_cell("si8")
    model = O.model_from_cell(cell)
    H = O.dense_h(model)
    lam, V = np.linalg.eigh(H)
    return cell, model, H, lam, V


@pytest.fixture(scope="module")
def si8_modes():
    """Si8 with the smooth perturbation switched on (exercises dV)."""
    cell = synth.make_cell("si8", modes=True)
    model = O.model_from_cell(cell)
    return cell, model


def brute_sphere(L, ecut):
    """Independent enumeration with explicit loops (different code from the oracle)."""
    out = []
    n = [int(math.sqrt(2 * ecut) * Li / (2 * math.pi)) + 2 for Li in L]
    for a in range(-n[0], n[0] + 1):
        for b in range(-n[1], n[1] + 1):
            for c in range(-n[2], n[2] + 1):
                e = 0.5 * ((2 * math.pi * a / L[0]) ** 2 + (2 * math.pi * b / L[1]) ** 2
                           + (2 * math.pi * c / L[2]) ** 2)
                if e <= ecut:
                    out.append((a, b, c, e))
    return out


# --- P14: numbers the paper prints -------------------------------------------

def test_paper_table1_grid_si4096():
    # Table I: Si4096 at E_cut = 5 Ha uses an 84 x 84 x 84 grid (592704 points).
    # With the 8x8x8 diamond supercell of a = 10.26 bohr, sqrt(2 Ecut) L / pi = 82.6,
    # rounded up to the next 7-smooth FFT size.
    L = (82.08, 82.08, 82.08)
    g = O.paper_grid(L, 5.0)
    assert g == (84, 84, 84)
    assert g[0] * g[1] * g[2] == 592704


def test_paper_two_wavefunctions_per_atom():
    # Section III-B3: Si4096 has 8192 wavefunctions (two per silicon atom).
    for name, nocc in (("si8", 16), ("si64", 128), ("si512", 1024), ("si4096", 8192)):
        cell = synth.make_cell(name)
        assert cell.nocc == nocc
        assert cell.nbands >= nocc


# --- Basis and grid ----------------------------------------------------------

@pytest.mark.parametrize("name,npw,grid", [("si8", 1647, 24), ("si64", 37073, 64)])
def test_sphere_matches_brute_force(name, npw, grid):
    cell = synth.make_cell(name)
    m = O.sphere_millers(cell.L, cell.ecut)
    bf = brute_sphere(cell.L, cell.ecut)
    assert m.shape[0] == len(bf) == npw
    assert {tuple(r) for r in m.tolist()} == {r[:3] for r in bf}
    # no plane wave sits on the boundary within rounding (a tie would be ambiguous)
    e = np.array([r[3] for r in bf])
    assert np.all(np.abs(e - cell.ecut) > 1e-9)
    assert O.fft_grid(cell.L, cell.ecut) == (grid, grid, grid)


def test_grid_rule_reproduces_stated_grids():
    # The stated workload grids (24^3, 64^3, 128^3, 192^3) and the serving grids.
    for name, g in (("si8", 24), ("si64", 64), ("si512", 128), ("si4096", 192)):
        cell = synth.make_cell(name)
        assert O.fft_grid(cell.L, cell.ecut) == (g, g, g)
    a = synth.A0_BOHR
    assert O.fft_grid((a, a, a), 15.0) == (27, 27, 27)
    assert O.fft_grid((a, a, 2 * a), 20.0) == (32, 32, 64)
    assert O.fft_grid((3 * a,) * 3, 15.0) == (81, 81, 81)


# --- P3: FFT conventions ----------------------------------------------------

def test_fft_plane_wave_and_parseval():
    L = np.array([10.26, 10.26, 20.52])
    miller = O.sphere_millers(L, 6.0)
    grid = O.fft_grid(L, 6.0)
    k = 17
    c = np.zeros(miller.shape[0], complex)
    c[k] = 1.0
    psi = O.to_real_space(c, miller, grid)
    # explicit exp(+i G.r) on the grid points r_j = j_i L_i / N_i
    j = np.meshgrid(*[np.arange(n) for n in grid], indexing="ij")
    G = 2 * np.pi * miller[k] / L
    phase = sum(G[i] * j[i] * L[i] / grid[i] for i in range(3))
    assert np.abs(psi - np.exp(1j * phase)).max() < 1e-13
    back = O.to_g_space(psi, miller)
    expect = np.zeros_like(back)
    expect[k] = 1.0
    assert np.abs(back - expect).max() < 1e-14
    # Parseval: sum_j |psi(r_j)|^2 = N_r sum_G |c_G|^2
    x = synth.random_block(miller.shape[0], 1, 3)[:, 0]
    f = O.to_real_space(x, miller, grid)
    nr = grid[0] * grid[1] * grid[2]
    assert abs((np.abs(f) ** 2).sum() - nr * (np.abs(x) ** 2).sum()) < 1e-12 * nr * (np.abs(x) ** 2).sum()


# --- P1: empty lattice ---------------------------------------------------------

def test_empty_lattice_closed_form():
    cell = synth.make_cell("si8")
    model = O.model_from_cell(cell, zval=0.0, gauss_c=0.0, d0=0.0, d1=0.0)
    H = O.dense_h(model)
    assert np.abs(H - np.diag(np.diag(H))).max() == 0.0
    lam = np.linalg.eigvalsh(H)
    bf = np.sort([r[3] for r in brute_sphere(cell.L, cell.ecut)])
    assert np.abs(lam - bf).max() < 1e-12
    # cubic shells |n|^2 = 0,1,2,3,4,5 have 1,6,12,8,6,24 members
    unit = 0.5 * (2 * np.pi / cell.L[0]) ** 2
    lows = lam[:57]
    shells = np.round(lows / unit).astype(int)
    counts = [int((shells == s).sum()) for s in range(6)]
    assert counts == [1, 6, 12, 8, 6, 24]


def test_empty_lattice_solve_converges():
    cell = synth.make_cell("si8")
    model = O.model_from_cell(cell, zval=0.0, gauss_c=0.0, d0=0.0, d1=0.0)
    hop = lambda X: O.apply_h(model, X)
    X0 = synth.initial_block(model.miller, cell.L, 27 + 6, 11)
    b = model.kin.max() * 1.01
    res = O.solve(hop, X0, b, nocc=27, tol=1e-9, m=10, max_steps=100)
    assert res.converged
    unit = 0.5 * (2 * np.pi / cell.L[0]) ** 2
    expect = unit * np.array([0] + [1] * 6 + [2] * 12 + [3] * 8, float)
    assert np.abs(res.eig[:27] - expect).max() < 1e-12


# --- P2: Hermiticity -----------------------------------------------------------

def test_dense_hermitian(si8):
    _, _, H, _, _ = si8
    assert np.abs(H - H.conj().T).max() <= 1e-15 * np.abs(H).max()


def test_matrix_free_hermitian(si8_modes):
    _, model = si8_modes
    x = synth.random_block(model.npw, 1, 5)[:, 0]
    y = synth.random_block(model.npw, 1, 6)[:, 0]
    lhs = np.vdot(x, O.apply_h(model, y))
    rhs = np.conj(np.vdot(y, O.apply_h(model, x)))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


# --- P4: FFT application equals the dense textbook H (no aliasing) ------------

def test_fft_h_equals_dense_h(si8_modes):
    _, model = si8_modes
    H = O.dense_h(model)
    X = synth.random_block(model.npw, 4, 9)
    HX = H @ X
    err = np.abs(O.apply_h(model, X) - HX).max()
    assert err <= 1e-12 * np.abs(H).max() * np.abs(X).max() * 10
    # negative control: a grid below the alias-free size must disagree
    small = O.build_model(model.L, model.tau, model.ecut, mode_miller=model.mode_miller,
                          mode_amp=model.mode_amp, mode_phase=model.mode_phase, grid=(16, 16, 16))
    err_small = np.abs(O.apply_h(small, X) - HX).max()
    assert err_small > 1e-6


# --- P6 / P11: rigid shift and conjugation symmetry ------------------------------

def test_rigid_shift_invariance(si8):
    cell, model, _, lam, _ = si8
    t = np.array([0.37, -1.1, 2.9])
    moved = O.build_model(cell.L, cell.tau + t, cell.ecut)
    lam2 = np.linalg.eigvalsh(O.dense_h(moved))
    assert np.abs(lam2 - lam).max() < 1e-10


def test_rigid_shift_with_modes():
    cell = synth.make_cell("si8", modes=True)
    m0 = O.model_from_cell(cell)
    lam = np.linalg.eigvalsh(O.dense_h(m0))[:40]
    t = np.array([0.37, -1.1, 2.9])
    G = 2 * np.pi * cell.modes.miller / np.asarray(cell.L)
    shifted_phase = cell.modes.phase - G @ t
    m1 = O.build_model(cell.L, cell.tau + t, cell.ecut, mode_miller=cell.modes.miller,
                       mode_amp=cell.modes.amp, mode_phase=shifted_phase)
    lam1 = np.linalg.eigvalsh(O.dense_h(m1))[:40]
    assert np.abs(lam1 - lam).max() < 1e-10
    # negative control: moving the atoms but not the perturbation changes the spectrum
    m2 = O.build_model(cell.L, cell.tau + t, cell.ecut, mode_miller=cell.modes.miller,
                       mode_amp=cell.modes.amp, mode_phase=cell.modes.phase)
    lam2 = np.linalg.eigvalsh(O.dense_h(m2))[:40]
    assert np.abs(lam2 - lam).max() > 1e-5


def test_structure_factor_sign_symmetry(si8):
    cell, _, _, lam, _ = si8
    flipped = O.build_model(cell.L, cell.tau, cell.ecut, sf_sign=+1.0)
    lam2 = np.linalg.eigvalsh(O.dense_h(flipped))
    assert np.abs(lam2 - lam).max() < 1e-12


# --- P7 / P12: projectors ------------------------------------------------------------

def l1_norm_deficit(L, sigma=0.8):
    """Y_1m(0) := 0 removes the G = 0 reciprocal cell from the l = 1 lattice sum.

    In the continuum that cell holds (c^2/Omega) <Y_1m^2>_sphere = c^2 / (4 pi Omega).
    """
    c2 = 32.0 * math.pi ** 2.5 * sigma ** 3
    return c2 / (4.0 * math.pi * float(np.prod(L)))


def test_projector_continuum_norm(si8):
    cell, model, _, _, _ = si8
    n2 = (np.abs(model.B) ** 2).sum(axis=0)
    # l = 0: unit norm up to the Gaussian tail beyond the cutoff
    assert np.abs(n2[0::4] - 1.0).max() <= 1e-4
    # l = 1: unit norm minus the G = 0 cell
    for m in (1, 2, 3):
        assert np.abs(n2[m::4] - (1.0 - l1_norm_deficit(cell.L))).max() <= 1e-4


def test_single_atom_nonlocal_rank4():
    L = (10.26, 10.26, 10.26)
    tau = np.array([[1.3, 2.2, 0.4]])
    model = O.build_model(L, tau, 10.0, zval=0.0, gauss_c=0.0)
    Hnl = O.dense_h(model) - np.diag(model.kin)
    lam = np.linalg.eigvalsh(Hnl)
    nz = lam[np.abs(lam) > 1e-10]
    assert nz.size == 4
    # projector norms: 1 for l = 0, 1 - c^2/(4 pi Omega) for l = 1 (up to the Gaussian tail)
    d1 = -0.7 * (1.0 - l1_norm_deficit(L))
    assert np.abs(np.sort(nz) - np.array([d1, d1, d1, 1.5])).max() < 2e-4
    # and exactly D_p |beta_p|^2 (the projectors are mutually orthogonal in a cubic cell)
    n2 = (np.abs(model.B) ** 2).sum(axis=0)
    assert np.abs(np.sort(nz) - np.sort(model.D * n2)).max() < 1e-12
    assert np.abs(n2[1:] - n2[1]).max() < 1e-14


# --- P8: Chebyshev closed form -----------------------------------------------------

def test_chebyshev_closed_form(si8):
    _, model, _, lam, V = si8
    hop = lambda X: O.apply_h(model, X)
    k = 24
    X = V[:, :k]
    m = 10
    a_lo, a, b = lam[0], lam[30], lam[-1] * 1.01
    Y = O.chebyshev_filter(hop, X, m, a_lo, a, b)
    e, c = 0.5 * (b - a), 0.5 * (b + a)
    scale = O.chebyshev_t(m, (lam[:k] - c) / e) / O.chebyshev_t(m, np.array([(a_lo - c) / e]))[0]
    ref = X * scale[None, :]
    assert np.abs(Y - ref).max() <= 1e-11 * np.abs(ref).max()
    # closed form of T_m itself against numpy's Chebyshev series
    x = np.linspace(-3, 3, 61)
    cheb = np.polynomial.chebyshev.chebval(x, [0] * m + [1])
    assert np.abs(O.chebyshev_t(m, x) - cheb).max() <= 1e-9 * np.abs(cheb).max()


# --- P9 / P5: Rayleigh-Ritz ------------------------------------------------------

def test_rr_exact_subspace(si8):
    _, model, _, lam, V = si8
    hop = lambda X: O.apply_h(model, X)
    k = 20
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((k, k)) + 1j * rng.standard_normal((k, k)))
    X = V[:, :k] @ Q * 3.0  # a non-orthonormal basis of the invariant subspace
    st = O.eig_step(hop, X, 0, 0.0, 0.0, 1.0)
    assert np.abs(st.eig - lam[:k]).max() < 1e-12
    assert np.abs(st.X.conj().T @ st.X - np.eye(k)).max() < 1e-12
    assert st.resid.max() < 1e-11


def test_rr_matches_generalised_eig(si8):
    _, model, _, _, _ = si8
    hop = lambda X: O.apply_h(model, X)
    Y = synth.random_block(model.npw, 12, 4)
    W = hop(Y)
    lam, C = O.rayleigh_ritz(Y, W)
    import scipy.linalg
    S = Y.conj().T @ Y
    Hs = Y.conj().T @ W
    ref = scipy.linalg.eigh(0.5 * (Hs + Hs.conj().T), 0.5 * (S + S.conj().T), eigvals_only=True)
    assert np.abs(lam - ref).max() < 1e-11 * np.abs(ref).max()
    # C makes the block orthonormal and diagonalises the projected H
    assert np.abs(C.conj().T @ S @ C - np.eye(12)).max() < 1e-11


def test_step_orthonormal_output(si8):
    cell, model, _, lam, _ = si8
    hop = lambda X: O.apply_h(model, X)
    X0 = synth.initial_block(model.miller, cell.L, cell.nbands, 5)
    st = O.eig_step(hop, X0, 0, 0.0, 0.0, 1.0)
    st = O.eig_step(hop, st.X, 10, st.a_lo, st.a, lam[-1] * 1.01)
    assert np.abs(st.X.conj().T @ st.X - np.eye(cell.nbands)).max() < 1e-12
    R = O.apply_h(model, st.X) - st.X * st.eig[None, :]
    assert np.abs(np.linalg.norm(R, axis=0) - st.resid).max() < 1e-12


# --- P10: convergence to dense eigenvalues and to ARPACK ---------------------------

def test_solve_converges_to_dense(si8):
    cell, model, _, lam, V = si8
    hop = lambda X: O.apply_h(model, X)
    X0 = synth.initial_block(model.miller, cell.L, cell.nbands, synth.SEED_X0)
    b = O.lanczos_max(hop, model.npw, 20, seed=1)
    assert b >= lam[-1] * (1 - 1e-3)
    res = O.solve(hop, X0, 1.01 * b, nocc=cell.nocc, tol=1e-7)
    assert res.converged
    nocc = cell.nocc
    assert np.abs(res.eig[:nocc] - lam[:nocc]).max() < 1e-8
    for lo, hi in O.clusters(lam[: nocc + 1]):
        if hi > nocc:
            break
        assert O.subspace_sin(V[:, lo:hi], res.X[:, lo:hi]) < 1e-6


@pytest.mark.slow
def test_solve_matches_arpack_si16():
    cell = synth.silicon_cell((1, 1, 2), 10.0, disp_seed=synth.SEED_REQUEST)
    model = O.model_from_cell(cell)
    hop = lambda X: O.apply_h(model, X)
    n = model.npw
    op = scipy.sparse.linalg.LinearOperator((n, n), matvec=hop, dtype=complex)
    ref = np.sort(scipy.sparse.linalg.eigsh(op, k=cell.nocc, which="SA", tol=1e-12,
                                            return_eigenvectors=False))
    X0 = synth.initial_block(model.miller, cell.L, cell.nbands, 21)
    b = 1.01 * O.lanczos_max(hop, n, 20, seed=2)
    res = O.solve(hop, X0, b, nocc=cell.nocc, tol=1e-7)
    assert res.converged
    assert np.abs(res.eig[: cell.nocc] - ref).max() < 1e-8


def test_atomwise_nonlocal_equals_matrix_form(si8):
    cell, model, _, _, _ = si8
    lite = O.model_from_cell(cell, with_projectors=False)
    assert lite.B.shape[1] == 0 and lite.atomwise
    X = synth.random_block(model.npw, 3, 12)
    a = O.apply_h(model, X)
    b = O.apply_h(lite, X)
    assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max()


# --- charge density -----------------------------------------------------------------------
def _grid_points(L, grid, idx):
    """Cartesian r_j = (j1 L1/N1, j2 L2/N2, j3 L3/N3) for integer index triples."""
    idx = np.asarray(idx, float)
    return idx * (np.asarray(L, float) / np.asarray(grid, float))


def test_density_parseval(si8):
    """sum_r rho(r) = N_r sum_n f_n sum_G |c_nG|^2 for the unnormalised inverse transform."""
    cell, model = si8[0], si8[1]
    rng = np.random.default_rng(5)
    X = rng.standard_normal((model.npw, 5)) + 1j * rng.standard_normal((model.npw, 5))
    occ = np.array([2.0, 2.0, 1.0, 0.5, 0.0])
    rho = O.density(X, occ, model.miller, model.grid)
    nr = float(np.prod(model.grid))
    want = nr * float(np.sum(occ * np.sum(np.abs(X) ** 2, axis=0)))
    assert abs(rho.sum() - want) <= 1e-12 * want
    assert rho.min() >= 0.0


def test_density_two_plane_waves_closed_form(si8):
    """Two plane waves a e^{iG1.r} + b e^{iG2.r}: |psi|^2 = |a|^2 + |b|^2 + 2 Re(a b* e^{i(G1-G2).r}),
    evaluated from the formula at every grid point (pins axis order and the transform sign)."""
    cell, model = si8[0], si8[1]
    m = model.miller
    i1 = int(np.flatnonzero((m == [1, 2, -1]).all(axis=1))[0])
    i2 = int(np.flatnonzero((m == [-2, 0, 1]).all(axis=1))[0])
    a, b = 0.7 - 0.2j, -0.3 + 0.9j
    X = np.zeros((model.npw, 1), complex)
    X[i1, 0], X[i2, 0] = a, b
    rho = O.density(X, np.array([1.0]), m, model.grid)
    N = model.grid
    j = np.stack(np.meshgrid(*[np.arange(n) for n in N], indexing="ij"), axis=-1).reshape(-1, 3)
    r = _grid_points(model.L, N, j)
    dG = 2 * np.pi * (np.array([1, 2, -1]) - np.array([-2, 0, 1])) / np.asarray(model.L, float)
    want = abs(a) ** 2 + abs(b) ** 2 + 2 * np.real(a * np.conj(b) * np.exp(1j * r @ dG))
    assert np.abs(rho.reshape(-1) - want).max() < 1e-12


def test_density_direct_sum_at_points(si8):
    """rho at a few grid points equals the weighted |sum_G c_G e^{iG.r}|^2 summed by brute force."""
    cell, model = si8[0], si8[1]
    rng = np.random.default_rng(9)
    X = rng.standard_normal((model.npw, 3)) + 1j * rng.standard_normal((model.npw, 3))
    occ = np.array([2.0, 1.0, 0.5])
    rho = O.density(X, occ, model.miller, model.grid)
    G = 2 * np.pi * model.miller / np.asarray(model.L, float)
    for idx in [(0, 0, 0), (3, 5, 7), (model.grid[0] - 1, 1, model.grid[2] // 2)]:
        r = _grid_points(model.L, model.grid, idx)
        psi = np.exp(1j * (G @ r)) @ X
        want = float(np.sum(occ * np.abs(psi) ** 2))
        assert abs(rho[idx] - want) < 1e-10 * want


# --- LOBPCG step ------------------------------------------------------------------------------
def test_lobpcg_ritz_values_bounded(si8):
    """Ritz values on span[X, R] lie above the exact eigenvalues (Courant-Fischer) and below the
    Rayleigh-Ritz values of span X alone, which the larger space contains."""
    cell, model, H, lam, V = si8
    hop = lambda Y: H @ Y
    rng = np.random.default_rng(11)
    X = rng.standard_normal((model.npw, 6)) + 1j * rng.standard_normal((model.npw, 6))
    X, _ = np.linalg.qr(X)
    r = O.lobpcg_step(hop, X, None, model.kin)
    rr = np.linalg.eigvalsh(X.conj().T @ H @ X)
    assert np.all(r.eig >= lam[:6] - 1e-10)
    assert np.all(r.eig <= rr + 1e-10)
    assert np.abs(r.X.conj().T @ r.X - np.eye(6)).max() < 1e-10
    # residual norms of the input block, from their definition
    th = np.real(np.diag(X.conj().T @ H @ X))
    assert np.allclose(r.resid, np.linalg.norm(H @ X - X * th, axis=0), rtol=1e-12)


def test_lobpcg_converges_to_dense(si8):
    """Repeated steps from a random orthonormal block reach the dense spectrum."""
    cell, model, H, lam, V = si8
    hop = lambda Y: H @ Y
    nb = 10
    rng = np.random.default_rng(12)
    X = rng.standard_normal((model.npw, nb)) + 1j * rng.standard_normal((model.npw, nb))
    X, _ = np.linalg.qr(X)
    P = None
    for _ in range(60):
        r = O.lobpcg_step(hop, X, P, model.kin)
        X, P = r.X, r.P
        if r.resid[:8].max() < 1e-9:
            break
    assert np.abs(r.eig[:8] - lam[:8]).max() < 1e-8


def test_lanczos_bound_brackets_the_top_of_the_spectrum(si8):
    """The Lanczos estimate (largest Ritz value plus the last off-diagonal) bounds lambda_max of the
    dense H from above (the Ritz value interlaces below it; the residual term covers the gap); on a
    Krylov space that is the whole space it is lambda_max itself."""
    cell, model, H, lam, V = si8
    hop = lambda x: H @ x
    for steps, seed in ((20, 1), (80, 2)):
        assert O.lanczos_max(hop, model.npw, steps, seed=seed) >= lam[-1] - 1e-9
    # a Krylov space that is the whole space gives lambda_max exactly (the off-diagonal vanishes)
    small = H[:6, :6]
    ev = np.linalg.eigvalsh(small)
    assert abs(O.lanczos_max(lambda x: small @ x, 6, 6, seed=3) - ev[-1]) < 1e-8
