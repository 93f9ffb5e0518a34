"""Pins of the oracle's basis-selecting Rayleigh-Ritz (SVQB with truncation), of the LOBPCG step on
a singular basis, and of the PPCG step (Section II-A names CG, PPCG and LOBPCG as inner solvers).

Each pin holds for the mathematics, not for the code: a library generalised eigensolver on a
well-conditioned basis, the span argument on planted dependent bases, the single-vector case in
which PPCG and LOBPCG search the same three-dimensional space, the variational bound on each column,
and convergence to the dense spectrum (faster with the search directions than without)."""
import numpy as np
import pytest
import scipy.linalg

from oracle import pw_oracle as O
from paper_2406_10765_amd import synth


@pytest.fixture(scope="module")
def si8_dense():
    cell = synth.make_cell("si8")
    model = O.model_from_cell(cell)
    H = O.dense_h(model)
    return model, H, np.linalg.eigvalsh(H)


def _herm(rng, n):
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return 0.5 * (A + A.conj().T)


def test_svqb_equals_generalised_eigensolver_on_an_independent_basis():
    rng = np.random.default_rng(3)
    n, k = 60, 12
    Y = rng.standard_normal((n, k)) + 1j * rng.standard_normal((n, k))
    Y *= np.linspace(0.1, 10.0, k)[None, :]  # columns of very different length
    H = _herm(rng, n)
    S, Hs = Y.conj().T @ Y, Y.conj().T @ H @ Y
    S, Hs = 0.5 * (S + S.conj().T), 0.5 * (Hs + Hs.conj().T)
    lam, C, kept = O.svqb_rayleigh_ritz(S, Hs, 1e-12)
    assert kept == k
    ref = scipy.linalg.eigh(Hs, S, eigvals_only=True)
    assert np.abs(lam - ref).max() < 1e-10 * np.abs(ref).max()
    assert np.abs(C.conj().T @ S @ C - np.eye(k)).max() < 1e-10
    assert np.abs(C.conj().T @ Hs @ C - np.diag(lam)).max() < 1e-9


def test_svqb_drops_exactly_the_dependent_directions():
    """[Y, Y B] spans what Y spans: the kept count is the rank and the Ritz values are those of Y."""
    rng = np.random.default_rng(4)
    n, k, extra = 50, 8, 5
    Y = rng.standard_normal((n, k)) + 1j * rng.standard_normal((n, k))
    B = rng.standard_normal((k, extra)) + 1j * rng.standard_normal((k, extra))
    Z = np.hstack([Y, Y @ B])
    H = _herm(rng, n)
    S, Hs = Z.conj().T @ Z, Z.conj().T @ H @ Z
    lam, C, kept = O.svqb_rayleigh_ritz(0.5 * (S + S.conj().T), 0.5 * (Hs + Hs.conj().T), 1e-10)
    assert kept == k
    ref = scipy.linalg.eigh(Y.conj().T @ H @ Y, Y.conj().T @ Y, eigvals_only=True)
    assert np.abs(lam - ref).max() < 1e-8 * np.abs(ref).max()
    # the Ritz vectors Z C are orthonormal and lie in span Y
    V = Z @ C
    assert np.abs(V.conj().T @ V - np.eye(k)).max() < 1e-8
    Q, _ = np.linalg.qr(Y)
    assert np.abs(V - Q @ (Q.conj().T @ V)).max() < 1e-8


def test_lobpcg_with_directions_inside_span_x_equals_the_step_without(si8_dense):
    """P = X makes [X R P] singular: Cholesky fails, the truncated Rayleigh-Ritz keeps the 2 nb
    independent directions, and the step equals the step on [X R]."""
    model, H, lam = si8_dense
    hop = lambda Y: H @ Y
    rng = np.random.default_rng(31)
    nb = 8
    X, _ = np.linalg.qr(rng.standard_normal((model.npw, nb)) + 1j * rng.standard_normal((model.npw, nb)))
    with pytest.raises(np.linalg.LinAlgError):
        O.lobpcg_step(hop, X, X.copy(), model.kin)  # no tolerance: the singular basis is an error
    a = O.lobpcg_step(hop, X, X.copy(), model.kin, drop_tol=1e-10)
    b = O.lobpcg_step(hop, X, None, model.kin)
    assert a.kept == 2 * nb and b.kept == 2 * nb
    assert np.abs(a.eig - b.eig).max() < 1e-10
    assert O.subspace_sin(b.X, a.X) < 1e-8
    # X' - P' still lies in span X
    Q, _ = np.linalg.qr(X)
    D = a.X - a.P
    assert np.abs(D - Q @ (Q.conj().T @ D)).max() < 1e-9


def test_ppcg_single_vector_is_lobpcg(si8_dense):
    """For one vector both methods take the lowest Ritz vector of H on span{x, K r, p}: the new
    iterates agree up to a phase (both have unit length)."""
    model, H, lam = si8_dense
    hop = lambda Y: H @ Y
    rng = np.random.default_rng(5)
    x = rng.standard_normal((model.npw, 1)) + 1j * rng.standard_normal((model.npw, 1))
    x /= np.linalg.norm(x)
    lo = O.lobpcg_step(hop, x, None, model.kin)
    pp = O.ppcg_step(hop, x, None, model.kin, 1e-10)
    assert abs(abs(np.vdot(lo.X[:, 0], pp.X[:, 0])) - 1.0) < 1e-10
    assert abs(np.linalg.norm(pp.X) - 1.0) < 1e-10
    # second step, with directions (each method's own)
    lo2 = O.lobpcg_step(hop, lo.X, lo.P, model.kin)
    pp2 = O.ppcg_step(hop, pp.X, pp.P, model.kin, 1e-10)
    assert abs(abs(np.vdot(lo2.X[:, 0], pp2.X[:, 0])) - 1.0) < 1e-9
    assert abs(pp2.eig[0] - lo.eig[0]) < 1e-10  # the Ritz value of the iterate entering step 2


def test_ppcg_columns_never_rise(si8_dense):
    """Each column's new vector minimises the Rayleigh quotient over a space that contains the Ritz
    vector x_j: its quotient is at most lam_j, and the coefficients are consistent with the output."""
    model, H, lam = si8_dense
    hop = lambda Y: H @ Y
    rng = np.random.default_rng(6)
    nb = 10
    X = rng.standard_normal((model.npw, nb)) + 1j * rng.standard_normal((model.npw, nb))
    r = O.ppcg_step(hop, X, None, model.kin, 1e-10)
    r2 = O.ppcg_step(hop, r.X, r.P, model.kin, 1e-10)
    for res in (r, r2):
        q = np.real(np.sum(res.X.conj() * (H @ res.X), axis=0)) / np.real(np.sum(res.X.conj() * res.X, axis=0))
        assert np.all(q <= res.eig + 1e-10)
        assert np.all(q < res.eig - 1e-6)  # and they move
        assert np.all(np.abs(np.imag(res.coef[:, 0])) < 1e-14) and np.all(np.real(res.coef[:, 0]) >= 0.0)
    # the second step's Ritz values lie at or below the first's (Rayleigh-Ritz on better vectors)
    assert np.all(r2.eig[:8] <= r.eig[:8] + 1e-10)


def test_ppcg_converges_to_dense_and_directions_help(si8_dense):
    model, H, lam = si8_dense
    hop = lambda Y: H @ Y
    nb, nconv, tol = 10, 8, 1e-8

    def steps(use_p):
        rng = np.random.default_rng(12)
        X = rng.standard_normal((model.npw, nb)) + 1j * rng.standard_normal((model.npw, nb))
        P = None
        for it in range(1, 400):
            r = O.ppcg_step(hop, X, P if use_p else None, model.kin, 1e-10)
            X, P = r.X, r.P
            if r.resid[:nconv].max() < tol:
                assert np.abs(r.eig[:nconv] - lam[:nconv]).max() < 1e-9
                return it
        return 400

    with_p, without_p = steps(True), steps(False)
    assert with_p < 400
    assert with_p <= 0.75 * without_p, (with_p, without_p)


def test_ppcg_new_directions_are_orthogonal_to_span_x(si8_dense):
    """w_j and p_j are projected against span X before the small problems, so P' = beta W + gamma P
    is orthogonal to the input span, and X' - P' = X diag(alpha) lies in it."""
    model, H, lam = si8_dense
    hop = lambda Y: H @ Y
    rng = np.random.default_rng(8)
    nb = 10
    X = rng.standard_normal((model.npw, nb)) + 1j * rng.standard_normal((model.npw, nb))
    r1 = O.ppcg_step(hop, X, None, model.kin, 1e-10)
    r2 = O.ppcg_step(hop, r1.X, r1.P, model.kin, 1e-10)
    for prev, res in ((X, r1), (r1.X, r2)):
        Q, _ = np.linalg.qr(prev)
        assert np.abs(Q.conj().T @ res.P).max() < 1e-10 * max(1.0, np.abs(res.P).max())
        D = res.X - res.P
        assert np.abs(D - Q @ (Q.conj().T @ D)).max() < 1e-10
        assert np.linalg.norm(res.P) > 1e-3
