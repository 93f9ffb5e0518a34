"""Seeded synthetic inputs shared by the GPU path, the tests and the bench.

This module holds only input recipes: the silicon supercell geometry with
seeded displacements, the seeded smooth perturbation modes of the effective
potential, the seeded starting block of wavefunction coefficients and the
named workloads.  It computes nothing of the Hamiltonian or the eigensolver.

The paper studies bulk silicon supercells (Section IV-A, "Setup of the Test
Physical Systems") and states that every silicon atom contributes two
occupied wavefunctions (Section III-B3).  The sizes, cutoffs, band counts
and the analytic pseudopotential parameters below define the synthetic
stand-ins for the paper's crystal inputs, whose pseudopotential files are
not part of the paper.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence, Tuple

import numpy as np

# Fractional coordinates of the 8 atoms of the conventional diamond cell.
DIAMOND_SITES = np.array(
    [
        [0.00, 0.00, 0.00],
        [0.00, 0.50, 0.50],
        [0.50, 0.00, 0.50],
        [0.50, 0.50, 0.00],
        [0.25, 0.25, 0.25],
        [0.25, 0.75, 0.75],
        [0.75, 0.25, 0.75],
        [0.75, 0.75, 0.25],
    ]
)

A0_BOHR = 10.26

# Base seeds; each workload adds its index.
SEED_DISP = 2406107650
SEED_MODES = 2406107660
SEED_X0 = 2406107670
SEED_ARRIVALS = 2406107680
SEED_REQUEST = 2406107700


@dataclasses.dataclass(frozen=True)
class Pseudo:
    """Analytic synthetic pseudopotential (one species, silicon-like)."""

    zval: float = 4.0  # valence charge of the local part
    rc: float = 1.0  # Gaussian width of the local part (bohr)
    gauss_c: float = 2.0  # short-range Gaussian coefficient of the local part
    beta_sigma: float = 0.8  # projector Gaussian width (bohr)
    d0: float = 1.5  # KB energy of the l=0 projector (Ha)
    d1: float = -0.7  # KB energy of each l=1 projector (Ha)


@dataclasses.dataclass(frozen=True)
class Modes:
    """Smooth perturbation dV(r) = sum_k amp_k cos(G_k . r + phase_k)."""

    miller: np.ndarray  # (K, 3) int
    amp: np.ndarray  # (K,) float, Ha
    phase: np.ndarray  # (K,) float, rad

    @staticmethod
    def empty() -> "Modes":
        return Modes(np.zeros((0, 3), np.int64), np.zeros(0), np.zeros(0))


@dataclasses.dataclass(frozen=True)
class Cell:
    """Orthorhombic cell, atoms in Cartesian bohr, cutoff and band count."""

    L: Tuple[float, float, float]
    tau: np.ndarray  # (natoms, 3)
    ecut: float
    nbands: int
    pseudo: Pseudo = Pseudo()
    modes: Modes = dataclasses.field(default_factory=Modes.empty)

    @property
    def natoms(self) -> int:
        return int(self.tau.shape[0])

    @property
    def nocc(self) -> int:
        # Two occupied wavefunctions per silicon atom (Section III-B3).
        return 2 * self.natoms


def silicon_atoms(ncells: Sequence[int], a0: float = A0_BOHR, seed: Optional[int] = None,
                  disp: float = 0.05) -> Tuple[Tuple[float, float, float], np.ndarray]:
    """Diamond-cubic silicon replicated ncells times; uniform +-disp bohr per component.

    Displacements are drawn from numpy's PCG64 in atom order, x then y then z.
    """
    nx, ny, nz = (int(c) for c in ncells)
    frac = []
    for i in range(nx):
        for j in range(ny):
            for k in range(nz):
                frac.append(DIAMOND_SITES + np.array([i, j, k], float))
    frac = np.concatenate(frac, axis=0)
    tau = frac * a0
    if seed is not None and disp > 0:
        rng = np.random.Generator(np.random.PCG64(seed))
        tau = tau + rng.uniform(-disp, disp, size=tau.shape)
    L = (nx * a0, ny * a0, nz * a0)
    return L, tau


def potential_modes(L: Sequence[float], seed: int, nmodes: int = 32, gmax: float = 2.0,
                    amp: float = 0.05) -> Modes:
    """Draw nmodes distinct reciprocal-lattice vectors with 0 < |G| < gmax.

    Candidates are restricted to the half-space whose first non-zero Miller
    component is positive, so +G and -G are never both drawn.  Phases are
    uniform in [0, 2 pi).
    """
    L = np.asarray(L, float)
    nmax = [int(math.floor(gmax * L[i] / (2 * math.pi))) + 1 for i in range(3)]
    cand = []
    for a in range(-nmax[0], nmax[0] + 1):
        for b in range(-nmax[1], nmax[1] + 1):
            for c in range(-nmax[2], nmax[2] + 1):
                n = (a, b, c)
                first = next((v for v in n if v != 0), 0)
                if first <= 0:
                    continue
                g2 = sum((2 * math.pi * n[i] / L[i]) ** 2 for i in range(3))
                if g2 < gmax * gmax:
                    cand.append(n)
    cand = np.array(cand, np.int64)
    rng = np.random.Generator(np.random.PCG64(seed))
    pick = rng.choice(len(cand), size=min(nmodes, len(cand)), replace=False)
    phase = rng.uniform(0.0, 2 * math.pi, size=len(pick))
    return Modes(cand[pick], np.full(len(pick), amp), phase)


def lexsort_millers(miller: np.ndarray) -> np.ndarray:
    """Permutation that sorts Miller triples lexicographically (n1, then n2, then n3)."""
    m = np.asarray(miller)
    return np.lexsort((m[:, 2], m[:, 1], m[:, 0]))


def initial_block(miller: np.ndarray, L: Sequence[float], nbands: int, seed: int) -> np.ndarray:
    """Seeded starting coefficients, identical for any ordering of `miller`.

    Values are complex standard normal drawn in lexicographic Miller order,
    damped by 1/(1 + |G|^2) and normalised per column, then returned in the
    order of `miller`.
    """
    m = np.asarray(miller, np.int64)
    order = lexsort_millers(m)
    rng = np.random.Generator(np.random.PCG64(seed))
    npw = m.shape[0]
    z = rng.standard_normal((npw, nbands)) + 1j * rng.standard_normal((npw, nbands))
    Lv = np.asarray(L, float)
    gs = (2 * np.pi * m[order] / Lv) ** 2
    w = 1.0 / (1.0 + gs.sum(axis=1))
    z *= w[:, None]
    z /= np.linalg.norm(z, axis=0, keepdims=True)
    out = np.empty_like(z)
    out[order] = z
    return out


def random_block(npw: int, nbands: int, seed: int) -> np.ndarray:
    """Plain complex normal block (for operator tests)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((npw, nbands)) + 1j * rng.standard_normal((npw, nbands))


# Named workloads: (cells, ecut, nbands, perturbation on)
WORKLOADS = {
    "si8": dict(index=0, ncells=(1, 1, 1), ecut=10.0, nbands=20, modes=False),
    "si64": dict(index=1, ncells=(2, 2, 2), ecut=20.0, nbands=144, modes=True),
    "si512": dict(index=2, ncells=(4, 4, 4), ecut=20.0, nbands=1088, modes=True),
    "si4096": dict(index=3, ncells=(8, 8, 8), ecut=10.0, nbands=8256, modes=True),
}


def make_cell(name: str, ecut: Optional[float] = None, nbands: Optional[int] = None,
              modes: Optional[bool] = None, disp_seed: Optional[int] = None,
              pseudo: Pseudo = Pseudo()) -> Cell:
    """Build a named silicon workload with its seeded displacements and modes."""
    w = WORKLOADS[name]
    idx = w["index"]
    L, tau = silicon_atoms(w["ncells"], seed=SEED_DISP + idx if disp_seed is None else disp_seed)
    use_modes = w["modes"] if modes is None else modes
    md = potential_modes(L, SEED_MODES + idx) if use_modes else Modes.empty()
    return Cell(L=L, tau=tau, ecut=w["ecut"] if ecut is None else ecut,
                nbands=w["nbands"] if nbands is None else nbands, pseudo=pseudo, modes=md)


def silicon_cell(ncells: Sequence[int], ecut: float, nbands: Optional[int] = None,
                 disp_seed: Optional[int] = None, modes_seed: Optional[int] = None,
                 pseudo: Pseudo = Pseudo()) -> Cell:
    """Arbitrary silicon supercell (used by the serving mix and small tests)."""
    L, tau = silicon_atoms(ncells, seed=disp_seed)
    md = potential_modes(L, modes_seed) if modes_seed is not None else Modes.empty()
    nat = tau.shape[0]
    return Cell(L=L, tau=tau, ecut=ecut, nbands=2 * nat + 8 if nbands is None else nbands,
                pseudo=pseudo, modes=md)


SERVING_CELLS = {"si8": (1, 1, 1), "si16": (1, 1, 2), "si64": (2, 2, 2), "si216": (3, 3, 3)}


def serving_mix(n_requests: int = 200, rate: float = 20.0, seed: int = SEED_ARRIVALS):
    """Poisson arrivals (mean `rate` per second) of eigen-solves; each request draws its cell
    uniformly from Si8, Si16, Si64, Si216, its cutoff uniformly from {10, 15, 20} Ha, and has
    2 N + 8 bands and its own seeded displacements."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    t = np.cumsum(gaps)
    names = list(SERVING_CELLS)
    which = rng.integers(0, len(names), size=n_requests)
    ecut = rng.choice(np.array([10.0, 15.0, 20.0]), size=n_requests)
    out = []
    for i in range(n_requests):
        name = names[int(which[i])]
        cell = silicon_cell(SERVING_CELLS[name], float(ecut[i]), disp_seed=SEED_REQUEST + i)
        out.append({"t_arrive": float(t[i]), "name": name, "cell": cell, "seed": SEED_REQUEST + i})
    return out
