"""Host-side accuracy measures (paper_2406_10765_amd.accuracy): clusters, principal angles and the
Davis-Kahan bound, on matrices whose answers are known in closed form."""
import numpy as np

from paper_2406_10765_amd import accuracy as A


def test_clusters_split_at_gaps():
    eig = np.array([0.0, 0.0005, 0.002, 0.0024, 1.0])
    assert A.clusters(eig, 1e-3) == [(0, 2), (2, 4), (4, 5)]


def test_largest_angle_of_a_known_rotation():
    rng = np.random.default_rng(0)
    Q, _ = np.linalg.qr(rng.standard_normal((40, 6)) + 1j * rng.standard_normal((40, 6)))
    for th in (1e-9, 1e-4, 0.3, 1.2):
        B = Q[:, :2].copy()
        B[:, 1] = np.cos(th) * Q[:, 1] + np.sin(th) * Q[:, 5]  # one direction turned by th out of span
        assert abs(A.largest_angle(Q[:, :2], B) - th) < 1e-12 + 1e-9 * th
        # the same span in another basis: angle 0
    C = Q[:, :3] @ (rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3)))
    assert A.largest_angle(Q[:, :3], C) < 1e-12


def test_davis_kahan_bounds_the_angle_of_perturbed_eigenvectors():
    """H diagonal with a known spectrum; V spans a perturbed cluster; the Ritz pairs of V obey
    sin(angle to the exact eigenvectors) <= ||R||_F / delta."""
    rng = np.random.default_rng(1)
    n = 30
    lam = np.sort(rng.uniform(-1, 1, n))
    lam[10] = lam[9] + 1e-5  # a cluster 9..10
    H = np.diag(lam).astype(complex)
    E = np.eye(n, dtype=complex)
    for eps in (1e-8, 1e-5, 1e-3):
        V = E[:, 9:11] + eps * (rng.standard_normal((n, 2)) + 1j * rng.standard_normal((n, 2)))
        Q, _ = np.linalg.qr(V)
        th, W = np.linalg.eigh(Q.conj().T @ H @ Q)
        X = Q @ W
        R = H @ X - X * th[None, :]
        res = np.zeros(n)
        res[9:11] = np.linalg.norm(R, axis=0)
        ritz = np.array(lam)
        ritz[9:11] = th
        bound = A.davis_kahan(res, ritz, lam, 9, 11)
        ang = A.largest_angle(X, E[:, 9:11])
        assert np.sin(ang) <= bound * (1 + 1e-9)
        assert bound < 1e3 * np.sin(ang) + 1e-14  # and it is not vacuous


def test_cluster_report_skips_a_cluster_at_the_block_edge():
    n, nb = 12, 6
    lam = np.linspace(0, 1, n)
    lam[5] = lam[4] + 1e-6  # cluster 4..5 reaches the last column of the block
    X = np.eye(n, dtype=complex)[:, :nb]
    rows = A.cluster_report(X, lam, np.zeros(nb), X, lam[:nb], np.zeros(nb), nocc=6)
    assert [r[:2] for r in rows] == [(0, 1), (1, 2), (2, 3), (3, 4)]
    assert all(r[2] < 1e-12 and r[3] == 0.0 for r in rows)
