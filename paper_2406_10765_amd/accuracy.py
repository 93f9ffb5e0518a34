"""Accuracy measures of a computed block of eigenvectors (host side, numpy): clusters of nearly
degenerate eigenvalues, the largest principal angle between two spans, and the Davis-Kahan
sin(theta) bound ||R|| / delta of a cluster of Ritz pairs.

Eigenvectors of (nearly) degenerate eigenvalues are not individually defined, so vectors are
compared cluster by cluster: eigenvalues closer than `gap` join one cluster, and two blocks agree
on a cluster when the spans of its columns do.  For Ritz pairs (V, theta) with residual block
R = H V - V diag(theta), the Davis-Kahan theorem bounds the sine of the largest angle between
span V and the exact invariant subspace of the cluster by ||R||_F / delta, where delta separates
the cluster's Ritz values from the eigenvalues outside it.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np


def clusters(eig: np.ndarray, gap: float = 1e-3) -> List[Tuple[int, int]]:
    """Index ranges [lo, hi) of consecutive eigenvalues whose neighbours are closer than gap."""
    out = []
    lo = 0
    for i in range(1, len(eig) + 1):
        if i == len(eig) or eig[i] - eig[i - 1] >= gap:
            out.append((lo, i))
            lo = i
    return out


def largest_angle(A: np.ndarray, B: np.ndarray) -> float:
    """Largest principal angle (radians) between the column spans of A and B (same row count)."""
    qa, _ = np.linalg.qr(A)
    qb, _ = np.linalg.qr(B)
    s = np.linalg.svd(qa.conj().T @ qb, compute_uv=False)
    c = float(min(1.0, s.min()))
    # for small angles arccos loses precision; use the sine from the projection residual
    resid = qb - qa @ (qa.conj().T @ qb)
    sn = float(np.linalg.norm(resid, 2))
    return float(np.arcsin(min(1.0, sn))) if sn < 0.5 else float(np.arccos(c))


def davis_kahan(resid: np.ndarray, ritz: np.ndarray, outside: np.ndarray, lo: int, hi: int) -> float:
    """||R_cluster||_F / delta for the Ritz pairs lo..hi-1 (residual norms resid, Ritz values ritz)
    against the eigenvalues `outside` of the cluster (the reference spectrum with lo..hi-1 left
    out); inf when delta is 0."""
    rnorm = float(np.sqrt(np.sum(np.asarray(resid[lo:hi]) ** 2)))
    rest = np.concatenate([outside[:lo], outside[hi:]])
    if rest.size == 0:
        return float("inf")
    delta = float(np.min(np.abs(rest[None, :] - np.asarray(ritz[lo:hi])[:, None])))
    return rnorm / delta if delta > 0 else float("inf")


def cluster_report(X: np.ndarray, ritz: np.ndarray, resid: np.ndarray, Xref: np.ndarray, eig_ref: np.ndarray,
                   resid_ref: np.ndarray, nocc: int, gap: float = 1e-3):
    """Per occupied cluster of eig_ref (a cluster that reaches the last column is left out, since
    it may continue past the block): (lo, hi, largest angle between X and Xref, bound), where the
    bound is the sum of the Davis-Kahan bounds of (X, ritz, resid) and of (Xref, eig_ref,
    resid_ref): each bounds the angle to the exact invariant subspace, so their sum bounds the
    angle between the two blocks."""
    nb = X.shape[1]
    rows = []
    for lo, hi in clusters(eig_ref[:nb], gap):
        if lo >= nocc:
            break
        if hi >= nb:
            continue
        ang = largest_angle(X[:, lo:hi], Xref[:, lo:hi])
        bound = davis_kahan(resid, ritz, eig_ref[:nb], lo, hi) + davis_kahan(resid_ref, eig_ref, eig_ref[:nb], lo, hi)
        rows.append((lo, hi, ang, bound))
    return rows
