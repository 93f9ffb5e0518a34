"""ctypes binding of libpw.so (argument marshalling only).

Every computation runs inside the HIP library.  torch provides the device
memory (the arena and the wavefunction blocks) and the stream.  If the
library has not been built this module raises on first use; there is no
fallback path.

Block convention on the Python side: a torch tensor of shape (nb, ld) with
contiguous rows is the column-major npw x nb block of the C ABI (row b is band
b, first npw entries used).  complex128 for FP64 handles, complex64 for mixed.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpw.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "pw.h")

PW_OK, PW_PENDING, PW_EINVAL, PW_ENOMEM, PW_EDEVICE = 0, 1, -1, -2, -3
PW_ENOTPD, PW_ENUMERIC, PW_ENOTCONV, PW_EBUSY = -4, -5, -6, -7
PW_FP64, PW_MIXED = 0, 1


class CellDesc(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_double * 3),
        ("natoms", ctypes.c_int),
        ("tau", ctypes.POINTER(ctypes.c_double)),
        ("ecut", ctypes.c_double),
        ("nbands", ctypes.c_int),
        ("zval", ctypes.c_double),
        ("rc", ctypes.c_double),
        ("gauss_c", ctypes.c_double),
        ("beta_sigma", ctypes.c_double),
        ("d0", ctypes.c_double),
        ("d1", ctypes.c_double),
        ("nmodes", ctypes.c_int),
        ("mode_miller", ctypes.POINTER(ctypes.c_int)),
        ("mode_amp", ctypes.POINTER(ctypes.c_double)),
        ("mode_phase", ctypes.POINTER(ctypes.c_double)),
        ("fft_n", ctypes.c_int * 3),
        ("prec", ctypes.c_int),
        ("flags", ctypes.c_uint),
        ("filter_block", ctypes.c_int),
        ("proj_form", ctypes.c_int),
        ("rs_radius", ctypes.c_double),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("npw", ctypes.c_longlong),
        ("nst", ctypes.c_longlong),
        ("nr", ctypes.c_longlong),
        ("nproj", ctypes.c_longlong),
        ("footprint_bytes", ctypes.c_size_t),
        ("fft_n", ctypes.c_int * 3),
        ("nbands", ctypes.c_int),
        ("prec", ctypes.c_int),
        ("fused_planes", ctypes.c_int),
        ("filter_block", ctypes.c_int),
    ]


class StepParams(ctypes.Structure):
    _fields_ = [
        ("degree", ctypes.c_int),
        ("a_lo", ctypes.c_double),
        ("a", ctypes.c_double),
        ("b", ctypes.c_double),
        ("want_hx", ctypes.c_int),
    ]


PHASES = ["sticks_inv", "plane", "pencil_yinv", "pencil_x", "pencil_yfwd", "sticks_fwd", "proj", "proj_reduce",
          "nl", "gram", "gram_reduce", "eigsolve", "rotate", "resid", "other"]


class PhaseStat(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_longlong), ("ms", ctypes.c_double)]


PW_SERVER_DRY_RUN = 1


class ServerCfg(ctypes.Structure):
    _fields_ = [("arena_dev", ctypes.c_void_p), ("arena_bytes", ctypes.c_size_t), ("max_slots", ctypes.c_int),
                ("flags", ctypes.c_uint), ("hip_stream", ctypes.c_void_p)]


class Request(ctypes.Structure):
    _fields_ = [("cell", CellDesc), ("seed", ctypes.c_ulonglong), ("tol", ctypes.c_double),
                ("max_steps", ctypes.c_int), ("degree", ctypes.c_int), ("nconv", ctypes.c_int)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("nbands", ctypes.c_int), ("steps", ctypes.c_int),
                ("eig", ctypes.POINTER(ctypes.c_double)), ("resid", ctypes.POINTER(ctypes.c_double)),
                ("t_arrive", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
                ("message", ctypes.c_char * 256), ("retried", ctypes.c_int)]


class PWError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_lib = None


def declared_functions() -> List[str]:
    """Names of every function include/pw.h declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pw_[a-z_0-9]+)\s*\(", text)))


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run paper_2406_10765_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    sig = {
        "pw_plan": ([P(CellDesc), P(Info)]),
        "pw_plan_gvectors": ([P(CellDesc), P(ctypes.c_int)]),
        "pw_setup": ([P(CellDesc), vp, ctypes.c_size_t, vp, P(vp)]),
        "pw_query": ([vp, P(Info)]),
        "pw_get_gvectors": ([vp, P(ctypes.c_int)]),
        "pw_apply_h": ([vp, vp, vp, ctypes.c_int, ctypes.c_int]),
        "pw_apply_h_noalloc": ([vp, vp, vp, ctypes.c_int, ctypes.c_int]),
        "pw_density": ([vp, vp, ctypes.c_int, ctypes.c_int, P(ctypes.c_double), vp]),
        "pw_lobpcg_step": ([vp, vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, P(ctypes.c_double),
                            P(ctypes.c_double), P(ctypes.c_int)]),
        "pw_ppcg_step": ([vp, vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, P(ctypes.c_double),
                          P(ctypes.c_double)]),
        "pw_eig_step": ([vp, vp, vp, ctypes.c_int, ctypes.c_int, P(StepParams), P(ctypes.c_double),
                         P(ctypes.c_double), P(ctypes.c_double)]),
        "pw_solve": ([vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                      ctypes.c_double, P(ctypes.c_double), P(ctypes.c_double), P(ctypes.c_int)]),
        "pw_spectrum_bound": ([vp, ctypes.c_int, ctypes.c_ulonglong, P(ctypes.c_double)]),
        "pw_set_timing": ([vp, ctypes.c_int]),
        "pw_get_stats": ([vp, P(PhaseStat)]),
        "pw_reset_stats": ([vp]),
        "pw_random_block": ([vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_ulonglong]),
        "pw_destroy": ([vp]),
        "pw_server_create": ([P(ServerCfg), P(vp)]),
        "pw_submit": ([vp, P(Request), ctypes.c_double, P(ctypes.c_ulonglong)]),
        "pw_poll": ([vp, ctypes.c_ulonglong, P(Result)]),
        "pw_server_destroy": ([vp]),
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.pw_solve_retries.argtypes = [vp, P(ctypes.c_char_p)]
    L.pw_solve_retries.restype = ctypes.c_int
    L.pw_server_clock.argtypes = [vp]
    L.pw_server_clock.restype = ctypes.c_double
    L.pw_last_error.argtypes = [vp]
    L.pw_last_error.restype = ctypes.c_char_p
    L.pw_status_string.argtypes = [ctypes.c_int]
    L.pw_status_string.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(status: int, handle=None):
    if status != PW_OK:
        msg = lib().pw_last_error(handle)
        raise PWError(status, (msg or b"").decode() or lib().pw_status_string(status).decode())


PW_FLAG_PENCIL_FFT = 1
PW_FLAG_BF16_GRAM = 2
PW_FLAG_BF16_KB = 4
PW_FLAG_BF16_ROT = 8
PW_FLAG_BF16_ALL = PW_FLAG_BF16_GRAM | PW_FLAG_BF16_KB | PW_FLAG_BF16_ROT
PW_FLAG_BETA_OTF = 16
PW_FLAG_LOBPCG = 32
PW_FLAG_RSPACE_KB = 64
PW_PROJ_GSPACE, PW_PROJ_LOCALIZED = 0, 1
# fraction of the largest scaled Gram eigenvalue below which basis directions are dropped
PW_DROP_TOL_FP64 = 1e-10
PW_DROP_TOL_MIXED = 1e-5


def make_desc(cell, prec: int = PW_FP64, nbands: Optional[int] = None,
              fft_n: Sequence[int] = (0, 0, 0), flags: int = 0, filter_block: int = 0,
              proj_form: int = PW_PROJ_GSPACE, rs_radius: float = 0.0):
    """CellDesc from a synth.Cell; returns (desc, keepalive)."""
    p = cell.pseudo
    tau = np.ascontiguousarray(np.asarray(cell.tau, np.float64).reshape(-1))
    mm = np.ascontiguousarray(np.asarray(cell.modes.miller, np.int32).reshape(-1))
    ma = np.ascontiguousarray(np.asarray(cell.modes.amp, np.float64))
    mp = np.ascontiguousarray(np.asarray(cell.modes.phase, np.float64))
    d = CellDesc()
    d.L[:] = [float(x) for x in cell.L]
    d.natoms = int(cell.natoms)
    d.tau = tau.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if tau.size else None
    d.ecut = float(cell.ecut)
    d.nbands = int(cell.nbands if nbands is None else nbands)
    d.zval, d.rc, d.gauss_c = p.zval, p.rc, p.gauss_c
    d.beta_sigma, d.d0, d.d1 = p.beta_sigma, p.d0, p.d1
    d.nmodes = int(ma.size)
    d.mode_miller = mm.ctypes.data_as(ctypes.POINTER(ctypes.c_int)) if ma.size else None
    d.mode_amp = ma.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if ma.size else None
    d.mode_phase = mp.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if ma.size else None
    d.fft_n[:] = [int(x) for x in fft_n]
    d.prec = int(prec)
    d.flags = int(flags)
    d.filter_block = int(filter_block)
    d.proj_form = int(proj_form)
    d.rs_radius = float(rs_radius)
    return d, (tau, mm, ma, mp)


def plan(cell, prec: int = PW_FP64, nbands: Optional[int] = None, fft_n=(0, 0, 0), flags: int = 0,
         filter_block: int = 0, proj_form: int = PW_PROJ_GSPACE, rs_radius: float = 0.0) -> Info:
    d, keep = make_desc(cell, prec, nbands, fft_n, flags, filter_block, proj_form, rs_radius)
    info = Info()
    _check(lib().pw_plan(ctypes.byref(d), ctypes.byref(info)))
    return info


def plan_gvectors(cell, nbands: Optional[int] = None, fft_n=(0, 0, 0)) -> np.ndarray:
    info = plan(cell, PW_FP64, nbands, fft_n)
    d, keep = make_desc(cell, PW_FP64, nbands, fft_n)
    out = np.empty((info.npw, 3), np.int32)
    _check(lib().pw_plan_gvectors(ctypes.byref(d), out.ctypes.data_as(ctypes.POINTER(ctypes.c_int))))
    return out


class Handle:
    """A set-up cell on the current torch CUDA device and stream."""

    def __init__(self, cell, prec: int = PW_FP64, nbands: Optional[int] = None, fft_n=(0, 0, 0),
                 device=None, stream=None, flags: int = 0, filter_block: int = 0,
                 proj_form: int = PW_PROJ_GSPACE, rs_radius: float = 0.0):
        import torch

        self._torch = torch
        self.prec = prec
        self.dtype = torch.complex128 if prec == PW_FP64 else torch.complex64
        d, self._keep = make_desc(cell, prec, nbands, fft_n, flags, filter_block, proj_form, rs_radius)
        self.info = Info()
        _check(lib().pw_plan(ctypes.byref(d), ctypes.byref(self.info)))
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.arena = torch.empty(int(self.info.footprint_bytes), dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device) if stream is None else stream
        h = ctypes.c_void_p()
        _check(lib().pw_setup(ctypes.byref(d), ctypes.c_void_p(self.arena.data_ptr()),
                              ctypes.c_size_t(self.arena.numel()), ctypes.c_void_p(self.stream.cuda_stream),
                              ctypes.byref(h)))
        self._h = h
        _check(lib().pw_query(self._h, ctypes.byref(self.info)), self._h)
        self.npw = int(self.info.npw)
        self.nbands = int(self.info.nbands)

    def close(self):
        if getattr(self, "_h", None):
            lib().pw_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def gvectors(self) -> np.ndarray:
        out = np.empty((self.npw, 3), np.int32)
        _check(lib().pw_get_gvectors(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int))), self._h)
        return out

    @property
    def ld(self) -> int:
        """Default leading dimension: npw rounded up to 16 (aligned 16-byte loads in every column)."""
        return (self.npw + 15) // 16 * 16

    def empty_block(self, nb: int, ld: Optional[int] = None):
        ld = self.ld if ld is None else ld
        return self._torch.empty((nb, ld), dtype=self.dtype, device=self.device)

    def to_device(self, X: np.ndarray, ld: Optional[int] = None):
        """numpy (npw, nb) in this handle's plane-wave order -> device block (nb, ld)."""
        nb = X.shape[1]
        t = self._torch.zeros((nb, self.ld if ld is None else ld), dtype=self.dtype)
        t[:, : self.npw] = self._torch.from_numpy(np.ascontiguousarray(X.T)).to(self.dtype)
        return t.to(self.device)

    def to_host(self, T) -> np.ndarray:
        """device block (nb, ld) -> numpy (npw, nb) complex128."""
        return T[:, : self.npw].cpu().numpy().astype(np.complex128).T.copy()

    def _check_block(self, T):
        torch = self._torch
        if T.dtype != self.dtype or T.device != self.device or T.dim() != 2 or T.stride(1) != 1:
            raise ValueError("block must be a (nb, ld) row-contiguous tensor of the handle's dtype and device")
        return int(T.shape[0]), int(T.stride(0))

    def apply_h(self, X, HX=None):
        nb, ld = self._check_block(X)
        if HX is None:
            HX = self._torch.zeros_like(X)
        nb2, ld2 = self._check_block(HX)
        if nb2 != nb or ld2 != ld:
            raise ValueError("X and HX must have the same shape and stride")
        _check(lib().pw_apply_h(self._h, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(HX.data_ptr()), nb, ld),
               self._h)
        return HX

    def apply_h_noalloc(self, X, HX):
        """HX = H X through pw_apply_h_noalloc (work buffers in the library's static array)."""
        nb, ld = self._check_block(X)
        nb2, ld2 = self._check_block(HX)
        if nb2 != nb or ld2 != ld:
            raise ValueError("X and HX must have the same shape and stride")
        _check(lib().pw_apply_h_noalloc(self._h, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(HX.data_ptr()), nb,
                                        ld), self._h)
        return HX

    def density(self, X, occ, rho=None):
        """rho(r) = sum_n occ[n] |psi_n(r)|^2 on the FFT grid: float64 device tensor (N3, N2, N1)."""
        nb, ld = self._check_block(X)
        w = np.ascontiguousarray(np.asarray(occ, dtype=np.float64))
        if w.shape != (nb,):
            raise ValueError("occ must hold one weight per band")
        n1, n2, n3 = (int(v) for v in self.info.fft_n)
        if rho is None:
            rho = self._torch.empty((n3, n2, n1), dtype=self._torch.float64, device=self.device)
        if rho.dtype != self._torch.float64 or rho.device != self.device or not rho.is_contiguous() \
                or rho.numel() != n1 * n2 * n3:
            raise ValueError("rho must be a contiguous float64 device tensor of N1 N2 N3 entries")
        _check(lib().pw_density(self._h, ctypes.c_void_p(X.data_ptr()), nb, ld,
                                w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.c_void_p(rho.data_ptr())),
               self._h)
        return rho

    def lobpcg_step(self, X, P, have_p: bool, info: Optional[dict] = None):
        """One LOBPCG step on X and the directions P (both in place; P's input ignored when
        not have_p).  Returns (Ritz values, residual norms of the input X) as numpy arrays;
        info["kept"] is the dimension of the span the Rayleigh-Ritz used (3 nb or 2 nb unless
        dependent directions were dropped)."""
        nb, ld = self._check_block(X)
        nb2, ld2 = self._check_block(P)
        if nb2 != nb or ld2 != ld:
            raise ValueError("X and P must have the same shape and stride")
        eig = np.empty(nb)
        res = np.empty(nb)
        dp = ctypes.POINTER(ctypes.c_double)
        kept = ctypes.c_int(0)
        _check(lib().pw_lobpcg_step(self._h, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(P.data_ptr()), nb, ld,
                                    1 if have_p else 0, eig.ctypes.data_as(dp), res.ctypes.data_as(dp),
                                    ctypes.byref(kept)), self._h)
        if info is not None:
            info["kept"] = int(kept.value)
        return eig, res

    def ppcg_step(self, X, P, have_p: bool):
        """One PPCG step on X and the directions P (both in place).  Returns (Ritz values of the
        input block, residual norms of its Ritz vectors) as numpy arrays."""
        nb, ld = self._check_block(X)
        nb2, ld2 = self._check_block(P)
        if nb2 != nb or ld2 != ld:
            raise ValueError("X and P must have the same shape and stride")
        eig = np.empty(nb)
        res = np.empty(nb)
        dp = ctypes.POINTER(ctypes.c_double)
        _check(lib().pw_ppcg_step(self._h, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(P.data_ptr()), nb, ld,
                                  1 if have_p else 0, eig.ctypes.data_as(dp), res.ctypes.data_as(dp)), self._h)
        return eig, res

    def eig_step(self, X, degree: int, a_lo: float = float("nan"), a: float = float("nan"),
                 b: float = float("nan"), HX=None):
        """One step on X (in place).  Returns (eig, resid, bounds) as numpy arrays."""
        nb, ld = self._check_block(X)
        p = StepParams(int(degree), float(a_lo), float(a), float(b), 1 if HX is not None else 0)
        eig = np.empty(nb)
        res = np.empty(nb)
        bnd = np.empty(3)
        dp = ctypes.POINTER(ctypes.c_double)
        _check(lib().pw_eig_step(self._h, ctypes.c_void_p(X.data_ptr()),
                                 ctypes.c_void_p(HX.data_ptr() if HX is not None else 0), nb, ld, ctypes.byref(p),
                                 eig.ctypes.data_as(dp), res.ctypes.data_as(dp), bnd.ctypes.data_as(dp)), self._h)
        return eig, res, bnd

    def random_block(self, nb: int, seed: int, ld: Optional[int] = None):
        """Seeded starting block generated on the device."""
        X = self.empty_block(nb, ld)
        _check(lib().pw_random_block(self._h, ctypes.c_void_p(X.data_ptr()), nb, int(X.stride(0)), seed), self._h)
        return X

    def spectrum_bound(self, steps: int = 20, seed: int = 1) -> float:
        out = ctypes.c_double()
        _check(lib().pw_spectrum_bound(self._h, steps, seed, ctypes.byref(out)), self._h)
        return out.value

    def set_timing(self, on: bool):
        _check(lib().pw_set_timing(self._h, 1 if on else 0), self._h)

    def reset_stats(self):
        _check(lib().pw_reset_stats(self._h), self._h)

    def stats(self) -> dict:
        """Per-phase {launches, ms} measured with HIP events on the handle's stream."""
        arr = (PhaseStat * len(PHASES))()
        _check(lib().pw_get_stats(self._h, arr), self._h)
        return {name: {"launches": int(arr[i].launches), "ms": float(arr[i].ms)} for i, name in enumerate(PHASES)}

    def solve(self, X, nocc: int, tol: float, degree: int = 10, max_steps: int = 200, b: Optional[float] = None):
        """pw_solve: a degree-0 step, then degree-m steps until max residual over the lowest nocc bands
        <= tol.  Returns (eig, resid, steps, converged)."""
        nb, ld = self._check_block(X)
        eig = np.empty(nb)
        res = np.empty(nb)
        steps = ctypes.c_int(0)
        dp = ctypes.POINTER(ctypes.c_double)
        st = lib().pw_solve(self._h, ctypes.c_void_p(X.data_ptr()), nb, ld, int(nocc), float(tol), int(degree),
                            int(max_steps), float("nan") if b is None else float(b), eig.ctypes.data_as(dp),
                            res.ctypes.data_as(dp), ctypes.byref(steps))
        if st not in (PW_OK, PW_ENOTCONV):
            _check(st, self._h)
        self.last_solve_retries = int(lib().pw_solve_retries(self._h, None))
        return eig, res, int(steps.value), st == PW_OK


def permutation_to(miller_from: np.ndarray, miller_to: np.ndarray) -> np.ndarray:
    """Index array p with miller_from[p] == miller_to (row order conversion between bases)."""
    key = lambda m: ((m[:, 0].astype(np.int64) + 4096) * 8192 + (m[:, 1] + 4096)) * 8192 + (m[:, 2] + 4096)
    kf, kt = key(np.asarray(miller_from)), key(np.asarray(miller_to))
    order = np.argsort(kf)
    pos = np.searchsorted(kf[order], kt)
    p = order[pos]
    if not np.array_equal(kf[p], kt):
        raise ValueError("Miller sets differ")
    return p


class Server:
    """Request loop (pw_server_*).  The arena is a torch uint8 device tensor unless dry_run."""

    def __init__(self, arena_bytes: int, max_slots: int, dry_run: bool = False):
        self._arena = None
        stream = None
        if dry_run:
            ptr = 1 << 20  # never dereferenced
        else:
            import torch

            self._arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device="cuda")
            ptr = self._arena.data_ptr()
            stream = torch.cuda.current_stream().cuda_stream
        cfg = ServerCfg(ctypes.c_void_p(ptr), ctypes.c_size_t(int(arena_bytes)), int(max_slots),
                        PW_SERVER_DRY_RUN if dry_run else 0, ctypes.c_void_p(stream))
        s = ctypes.c_void_p()
        _check(lib().pw_server_create(ctypes.byref(cfg), ctypes.byref(s)))
        self._s = s
        self._nbands = {}

    def clock(self) -> float:
        return float(lib().pw_server_clock(self._s))

    def submit(self, cell, prec: int = PW_MIXED, flags: int = 0, seed: int = 1, tol: float = 1e-4,
               max_steps: int = 200, degree: int = 10, nconv: int = 0, t_arrive: float = float("nan"),
               nbands: Optional[int] = None) -> int:
        d, keep = make_desc(cell, prec, nbands, (0, 0, 0), flags)
        r = Request(d, seed, tol, max_steps, degree, nconv)
        t = ctypes.c_ulonglong()
        _check(lib().pw_submit(self._s, ctypes.byref(r), float(t_arrive), ctypes.byref(t)))
        self._nbands[int(t.value)] = int(d.nbands)
        return int(t.value)

    def poll(self, ticket: int, nbands: Optional[int] = None):
        """None while pending; else a dict with status, eig, resid, steps, times and message.  The
        result buffers hold the request's own band count (the nbands argument is only a lower bound)."""
        nbands = max(int(nbands or 0), self._nbands.get(int(ticket), 0))
        eig = np.empty(nbands)
        res = np.empty(nbands)
        out = Result()
        dp = ctypes.POINTER(ctypes.c_double)
        out.eig = eig.ctypes.data_as(dp)
        out.resid = res.ctypes.data_as(dp)
        st = lib().pw_poll(self._s, ticket, ctypes.byref(out))
        if st == PW_PENDING:
            return None
        _check(st)
        return {"status": out.status, "eig": eig[: out.nbands], "resid": res[: out.nbands], "steps": out.steps,
                "t_arrive": out.t_arrive, "t_admit": out.t_admit, "t_done": out.t_done,
                "message": out.message.decode(errors="replace"), "retried": int(out.retried)}

    def close(self):
        if getattr(self, "_s", None):
            lib().pw_server_destroy(self._s)
            self._s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
