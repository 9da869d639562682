"""ctypes loader for the C oracle (TEST INFRASTRUCTURE ONLY).

Arrays are numpy float64 in C order with shape (ny, nx) in 2-D or
(nz, ny, nx) in 3-D, i.e. x fastest, the layout the C file indexes.
"""
import ctypes
import os

import numpy as np

from . import build as _build

BC = {"periodic": 0, "insulating": 1, "dirichlet": 2}
LIMITER = {"vanleer": 0, "minmod": 1, "mc": 2, "linear": 3}

_dp = ctypes.POINTER(ctypes.c_double)


class _OrcGrid(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int),
        ("n", ctypes.c_long * 3),
        ("h", ctypes.c_double * 3),
        ("bc", ctypes.c_int),
        ("limiter", ctypes.c_int),
        ("chi_par", ctypes.c_double),
        ("chi_perp", ctypes.c_double),
        ("b", _dp * 3),
        ("chi", _dp),
        ("chi_exp", ctypes.c_double),
        ("chi_tref", ctypes.c_double),
        ("src", _dp),
    ]


_libs = {}


def lib(omp=False):
    """Load liborc.so (omp: liborc_omp.so, the OpenMP build), building it
    with gcc only when it is missing."""
    if omp not in _libs:
        path = _build.LIB_OMP if omp else _build.LIB
        if not os.path.exists(path):
            _build.build(omp=omp)
        L = ctypes.CDLL(path)
        L.orc_lim2.restype = ctypes.c_double
        L.orc_lim2.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double]
        L.orc_lim4.restype = ctypes.c_double
        L.orc_lim4.argtypes = [ctypes.c_int] + [ctypes.c_double] * 4
        for name in ("orc_thomas", "orc_cyclic"):
            f = getattr(L, name)
            f.restype = ctypes.c_int
            f.argtypes = [ctypes.c_long, _dp, _dp, _dp, _dp, _dp]
        L.orc_sweep.restype = ctypes.c_int
        L.orc_sweep.argtypes = [ctypes.POINTER(_OrcGrid), ctypes.c_int, ctypes.c_double, _dp, _dp]
        L.orc_sweep2.restype = ctypes.c_int
        L.orc_sweep2.argtypes = [ctypes.POINTER(_OrcGrid), ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp, _dp]
        L.orc_sweep3.restype = ctypes.c_int
        L.orc_sweep3.argtypes = [ctypes.POINTER(_OrcGrid), ctypes.c_int] + [ctypes.c_double] * 3 + [_dp, _dp]
        for name in ("orc_step_si", "orc_step_si4", "orc_step_explicit"):
            f = getattr(L, name)
            f.restype = ctypes.c_int
            f.argtypes = [ctypes.POINTER(_OrcGrid), ctypes.c_double, ctypes.c_int, _dp, _dp]
        L.orc_step_si_ex.restype = ctypes.c_int
        L.orc_step_si_ex.argtypes = [ctypes.POINTER(_OrcGrid), ctypes.c_double, ctypes.c_int, _dp, _dp, ctypes.c_int]
        L.orc_energy.restype = ctypes.c_double
        L.orc_energy.argtypes = [ctypes.POINTER(_OrcGrid), _dp]
        L.orc_dt_from_ncfl.restype = ctypes.c_double
        L.orc_dt_from_ncfl.argtypes = [ctypes.POINTER(_OrcGrid), ctypes.c_double]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_num_threads.argtypes = []
        L.orc_grid_sizeof.restype = ctypes.c_long
        assert L.orc_grid_sizeof() == ctypes.sizeof(_OrcGrid), "orc_grid layout mismatch"
        _libs[omp] = L
    return _libs[omp]


def num_threads(omp=False):
    """Threads the oracle's sweeps use."""
    return lib(omp).orc_num_threads()


def _ptr(a):
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleGrid:
    """A grid description for the oracle.

    b: sequence of ndim cell-centred arrays (bx, by[, bz]), each of shape
       (ny, nx) or (nz, ny, nx).  h: cell widths (hx, hy[, hz]).
    """

    def __init__(self, b, h, bc="periodic", limiter="vanleer", chi_par=1.0, chi_perp=0.0, chi=None,
                 chi_exp=0.0, chi_tref=1.0, src=None, omp=False):
        """chi_exp != 0: temperature-dependent chi_par(T) = chi_par (T / chi_tref)^chi_exp
        from the state each sweep (or explicit step) reads (chi must then be None).
        bc "dirichlet": T = 0 on the boundary faces.  src: per-cell source Q,
        dt Q added to the first sweep of each step.  omp: run on the OpenMP
        build (same results, lines shared out over the host's cores)."""
        self._L = lib(omp)
        self.b = [_f64(c) for c in b]
        self.ndim = len(self.b)
        if self.ndim not in (2, 3):
            raise ValueError("ndim must be 2 or 3")
        self.shape = self.b[0].shape
        if len(self.shape) != self.ndim or any(c.shape != self.shape for c in self.b):
            raise ValueError("b components must share one (ny,nx) or (nz,ny,nx) shape")
        self.h = tuple(float(x) for x in h)
        self.bc = bc
        self.limiter = limiter
        self.chi_par = float(chi_par)
        self.chi_perp = float(chi_perp)
        self.chi = None if chi is None else _f64(chi)
        if self.chi is not None and self.chi.shape != self.shape:
            raise ValueError("chi must have the grid shape")
        self.src = None if src is None else _f64(src)
        if self.src is not None and self.src.shape != self.shape:
            raise ValueError("src must have the grid shape")
        s = _OrcGrid()
        s.ndim = self.ndim
        nxyz = tuple(reversed(self.shape)) + (1,) * (3 - self.ndim)
        for q in range(3):
            s.n[q] = nxyz[q]
            s.h[q] = self.h[q] if q < self.ndim else 1.0
            s.b[q] = _ptr(self.b[q]) if q < self.ndim else _dp()
        s.bc = BC[bc]
        s.limiter = LIMITER[limiter]
        s.chi_par = self.chi_par
        s.chi_perp = self.chi_perp
        s.chi = _ptr(self.chi) if self.chi is not None else _dp()
        s.chi_exp = float(chi_exp)
        s.chi_tref = float(chi_tref)
        s.src = _ptr(self.src) if self.src is not None else _dp()
        self.chi_exp, self.chi_tref = float(chi_exp), float(chi_tref)
        self._s = s

    @property
    def ncells(self):
        return int(np.prod(self.shape))

    def _check(self, T):
        T = _f64(T)
        if T.shape != self.shape:
            raise ValueError(f"field shape {T.shape} != grid shape {self.shape}")
        return T

    def sweep(self, axis, dt, U):
        """One directional sweep along axis (0=x, 1=y, 2=z); returns a new array."""
        U = self._check(U)
        out = np.empty_like(U)
        rc = self._L.orc_sweep(ctypes.byref(self._s), int(axis), float(dt), _ptr(U), _ptr(out))
        if rc != 0:
            raise RuntimeError(f"orc_sweep failed ({rc})")
        return out

    def sweep2(self, axis, dt_normal, dt_transverse, U):
        """Sweep with the normal (implicit) part at dt_normal and the
        transverse (explicit) part at dt_transverse (0: a pure solve)."""
        U = self._check(U)
        out = np.empty_like(U)
        rc = self._L.orc_sweep2(ctypes.byref(self._s), int(axis), float(dt_normal), float(dt_transverse),
                              _ptr(U), _ptr(out))
        if rc != 0:
            raise RuntimeError(f"orc_sweep2 failed ({rc})")
        return out

    def sweep3(self, axis, dt_normal, dt_transverse, dt_source, U):
        """sweep2 plus dt_source Q on the right-hand side."""
        U = self._check(U)
        out = np.empty_like(U)
        rc = self._L.orc_sweep3(ctypes.byref(self._s), int(axis), float(dt_normal), float(dt_transverse),
                              float(dt_source), _ptr(U), _ptr(out))
        if rc != 0:
            raise RuntimeError(f"orc_sweep3 failed ({rc})")
        return out

    def step_si(self, T, dt, nsteps=1, energy=False, four_step=False, reverse=False):
        """nsteps semi-implicit steps (the 2-step scheme, or the 4-step
        scheme of Eq. 4step; sweeps x, y (, z), or in reverse order);
        returns T (and energies if asked)."""
        T = self._check(T).copy()
        e = np.empty(nsteps + 1) if energy else None
        flags = (1 if four_step else 0) | (2 if reverse else 0)
        rc = self._L.orc_step_si_ex(ctypes.byref(self._s), float(dt), int(nsteps), _ptr(T),
                                  _ptr(e) if e is not None else _dp(), flags)
        if rc != 0:
            raise RuntimeError(f"orc_step_si failed ({rc})")
        return (T, e) if energy else T

    def step_si_stored(self, T, dt, nsteps=1, store=np.float32, rounding_seed=None):
        """step_si (2-step scheme, sweeps x, y (, z), no source term) with the
        state rounded to the type `store` after every sweep: the method as
        an implementation computes it that keeps its state in that type but
        evaluates each sweep exactly (in FP64).  Its difference from step_si
        is the part of a reduced-precision run's error that the storage
        alone causes.  rounding_seed: None rounds to nearest; an integer
        rounds faithfully in seeded random directions (round_to), another
        equally valid run of that precision."""
        if self.src is not None:
            raise ValueError("step_si_stored takes no source term")
        rng = None if rounding_seed is None else np.random.default_rng(rounding_seed)
        T = self._check(T).astype(store).astype(np.float64)
        for _ in range(nsteps):
            for axis in range(self.ndim):
                T = round_to(self.sweep(axis, dt, T), store, rng)
        return T

    def step_si_noisy(self, T, dt, nsteps=1, seed=0, ulps=1):
        """step_si (2-step scheme, sweeps x, y (, z), no source term) with
        every value moved by a random whole number of units in the last place
        (uniform in -ulps .. ulps, seeded) after every sweep: an FP64 run
        whose arithmetic rounds differently.  Its difference from step_si
        measures how far the method itself carries FP64 rounding noise."""
        if self.src is not None:
            raise ValueError("step_si_noisy takes no source term")
        rng = np.random.default_rng(seed)
        T = self._check(T).copy()
        for _ in range(nsteps):
            for axis in range(self.ndim):
                T = self.sweep(axis, dt, T)
                k = rng.integers(-ulps, ulps + 1, T.shape)
                for j in range(ulps):
                    T = np.where(k > j, np.nextafter(T, np.inf), T)
                    T = np.where(k < -j, np.nextafter(T, -np.inf), T)
        return T

    def step_explicit(self, T, dt, nsteps=1, energy=False):
        """nsteps explicit limited steps; returns T (and energies if asked)."""
        T = self._check(T).copy()
        e = np.empty(nsteps + 1) if energy else None
        rc = self._L.orc_step_explicit(ctypes.byref(self._s), float(dt), int(nsteps), _ptr(T),
                                     _ptr(e) if e is not None else _dp())
        if rc != 0:
            raise RuntimeError(f"orc_step_explicit failed ({rc})")
        return (T, e) if energy else T

    def energy(self, T):
        T = self._check(T)
        return self._L.orc_energy(ctypes.byref(self._s), _ptr(T))

    def dt_from_ncfl(self, ncfl):
        return self._L.orc_dt_from_ncfl(ctypes.byref(self._s), float(ncfl))


def round_to(x, store, rng=None):
    """x (FP64) rounded to the floating type `store`, returned as FP64.
    rng None: to nearest.  Otherwise faithfully, in a random direction per
    value: to the neighbour of `store` below or above x, each with
    probability 1/2 (a value of `store` stays as it is)."""
    f = x.astype(store)
    if rng is None:
        return f.astype(np.float64)
    fd = f.astype(np.float64)
    lo = np.where(fd > x, np.nextafter(f, store(-np.inf)), f)
    hi = np.where(fd < x, np.nextafter(f, store(np.inf)), f)
    return np.where(rng.random(x.shape) < 0.5, lo, hi).astype(np.float64)


def lim2(limiter, a, b):
    return lib().orc_lim2(LIMITER[limiter], float(a), float(b))


def lim4(limiter, a, b, c, d):
    return lib().orc_lim4(LIMITER[limiter], float(a), float(b), float(c), float(d))


def thomas(lo, di, up, r):
    lo, di, up, r = (_f64(v) for v in (lo, di, up, r))
    x = np.empty_like(r)
    if lib().orc_thomas(len(r), _ptr(lo), _ptr(di), _ptr(up), _ptr(r), _ptr(x)) != 0:
        raise RuntimeError("orc_thomas failed")
    return x


def cyclic(lo, di, up, r):
    lo, di, up, r = (_f64(v) for v in (lo, di, up, r))
    x = np.empty_like(r)
    if lib().orc_cyclic(len(r), _ptr(lo), _ptr(di), _ptr(up), _ptr(r), _ptr(x)) != 0:
        raise RuntimeError("orc_cyclic failed")
    return x
