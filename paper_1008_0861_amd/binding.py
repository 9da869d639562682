"""ctypes binding of libasd (include/asd.h).

Argument marshalling only: every step of the scheme runs in the HIP kernels
of libasd.so.  torch provides device memory (tensors, workspace) and the
stream; nothing here computes any part of the scheme.  If the compiled
library is missing, loading fails loudly: there is no fallback.
"""
import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libasd.so")

# status codes
OK = 0
ERRORS = {
    -1: "EINVAL", -2: "ESHAPE", -3: "EDTYPE", -4: "ENOTSET", -5: "EWORKSPACE",
    -6: "EUNSTABLE", -7: "EHIP", -8: "EUNSUPPORTED",
}
BC = {"periodic": 0, "insulating": 1, "dirichlet": 2}
LIMITER = {"vanleer": 0, "minmod": 1, "mc": 2, "linear": 3}
F32, F64 = 0, 1
FIELD = {"T": 0, "bx": 1, "by": 2, "bz": 3, "chi": 4, "Q": 5}
FLAG_PER_CELL_CHI = 1
FLAG_ALLOW_UNSTABLE = 2
FLAG_FOUR_STEP = 4
FLAG_REVERSE_ORDER = 8
STATUS_NONFINITE, STATUS_NEG_T, STATUS_ENERGY_DRIFT = 1, 2, 4
GRAPHS_OFF, GRAPHS_AUTO, GRAPHS_ALWAYS = 0, 1, 2

# every entry point of include/asd.h and include/asd_extra.h
EXPORTED = [
    "asd_last_error", "asd_workspace_bytes", "asd_init_grid", "asd_set_field",
    "asd_step_semi_implicit", "asd_step_explicit_limited", "asd_step_series", "asd_adjoint_workspace_bytes",
    "asd_adjoint_step", "asd_adjoint_forward", "asd_adjoint_step_stored", "asd_status", "asd_destroy",
    "asd_batch_workspace_bytes", "asd_batch_init", "asd_batch_set_problem", "asd_batch_step",
    "asd_batch_destroy", "asd_batch_set_block", "asd_batch_set_variant", "asd_batch_get_variant", "asd_batch_tune",
    "asd_batch_set_capacity",
    "asd_batch_step_energy", "asd_batch_status",
    "asd_batch_set_graphs",
    "asd_get_sweep_config", "asd_set_sweep_config", "asd_set_sweep_shape", "asd_get_sweep_io",
    "asd_set_sweep_kernel", "asd_get_sweep_variant", "asd_tune",
    "asd_set_graphs",
    "asd_bench_sweep", "asd_bench_copy", "asd_bench_copy_wide",
    "asd_noalloc_scratch_bytes", "asd_step_semi_implicit_noalloc",
]


class AsdError(RuntimeError):
    def __init__(self, code, msg):
        self.code = code
        self.name = ERRORS.get(code, str(code))
        super().__init__(f"{self.name}: {msg}")


class Desc(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("bc", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("limiter", ctypes.c_int32),
        ("n", ctypes.c_int64 * 3),
        ("h", ctypes.c_double * 3),
        ("chi_par", ctypes.c_double),
        ("chi_perp", ctypes.c_double),
        ("flags", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
        ("chi_exp", ctypes.c_double),
        ("chi_tref", ctypes.c_double),
    ]


_lib = None


def lib():
    """Load libasd.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not built: run python -m paper_1008_0861_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
        P = ctypes.POINTER
        sig = {
            "asd_last_error": (ctypes.c_char_p, []),
            "asd_workspace_bytes": (ctypes.c_int, [P(Desc), P(sz)]),
            "asd_init_grid": (ctypes.c_int, [P(Desc), vp, sz, vp, P(vp)]),
            "asd_set_field": (ctypes.c_int, [vp, i32, vp, i64, i32]),
            "asd_step_semi_implicit": (ctypes.c_int, [vp, dbl, i32, vp]),
            "asd_step_explicit_limited": (ctypes.c_int, [vp, dbl, i32, vp]),
            "asd_step_series": (ctypes.c_int, [vp, i32, dbl, i32, vp]),
            "asd_adjoint_workspace_bytes": (ctypes.c_int, [vp, i32, i32, P(sz)]),
            "asd_adjoint_step": (ctypes.c_int, [vp, dbl, i32, i32, vp, vp, vp, vp, vp, sz]),
            "asd_adjoint_forward": (ctypes.c_int, [vp, dbl, i32, i32, vp, sz]),
            "asd_adjoint_step_stored": (ctypes.c_int, [vp, dbl, i32, i32, vp, vp, vp, vp, sz]),
            "asd_status": (ctypes.c_int, [vp, P(ctypes.c_uint32), P(dbl)]),
            "asd_destroy": (ctypes.c_int, [vp]),
            "asd_batch_workspace_bytes": (ctypes.c_int, [P(Desc), i32, P(sz)]),
            "asd_batch_init": (ctypes.c_int, [P(Desc), i32, vp, sz, vp, P(vp)]),
            "asd_batch_set_problem": (ctypes.c_int, [vp, i32, vp, vp, vp, dbl]),
            "asd_batch_step": (ctypes.c_int, [vp, i32, i32]),
            "asd_batch_destroy": (ctypes.c_int, [vp]),
            "asd_batch_set_block": (ctypes.c_int, [vp, i32]),
            "asd_batch_set_variant": (ctypes.c_int, [vp, i32]),
            "asd_batch_set_capacity": (ctypes.c_int, [vp, i32]),
            "asd_batch_get_variant": (ctypes.c_int, [vp, P(i32)]),
            "asd_batch_tune": (ctypes.c_int, [vp, i32, P(i32), P(i32)]),
            "asd_batch_step_energy": (ctypes.c_int, [vp, i32, i32, vp]),
            "asd_batch_status": (ctypes.c_int, [vp, P(ctypes.c_uint32), P(dbl)]),
            "asd_batch_set_graphs": (ctypes.c_int, [vp, i32]),
            "asd_get_sweep_config": (ctypes.c_int, [vp, i32, P(i32), P(i32), P(i32), P(i32)]),
            "asd_set_sweep_config": (ctypes.c_int, [vp, i32, i32, i32]),
            "asd_set_sweep_shape": (ctypes.c_int, [vp, i32, i32, i32, i32]),
            "asd_get_sweep_io": (ctypes.c_int, [vp, i32, P(i32)]),
            "asd_set_sweep_kernel": (ctypes.c_int, [vp, i32, i32, i32, i32, i32]),
            "asd_get_sweep_variant": (ctypes.c_int, [vp, i32, P(i32)]),
            "asd_tune": (ctypes.c_int, [vp, dbl, i32]),
            "asd_set_graphs": (ctypes.c_int, [vp, i32]),
            "asd_bench_sweep": (ctypes.c_int, [vp, i32, dbl, i32]),
            "asd_bench_copy": (ctypes.c_int, [vp, vp, sz, vp]),
            "asd_bench_copy_wide": (ctypes.c_int, [vp, vp, sz, vp]),
            "asd_noalloc_scratch_bytes": (sz, []),
            "asd_step_semi_implicit_noalloc": (ctypes.c_int, [P(Desc), vp, vp, vp, vp, vp, dbl, i32, vp, vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def last_error():
    return lib().asd_last_error().decode(errors="replace")


def check(rc):
    if rc != OK:
        raise AsdError(rc, last_error())
    return rc


def _dtype_code(dtype):
    if dtype == torch.float32:
        return F32
    if dtype == torch.float64:
        return F64
    raise TypeError(f"unsupported dtype {dtype}")


def make_desc(shape, h, bc="periodic", dtype=torch.float32, limiter="vanleer", chi_par=1.0, chi_perp=0.0,
              per_cell_chi=False, allow_unstable=False, four_step=False, reverse_order=False, chi_exp=0.0,
              chi_tref=1.0):
    """Build an asd_desc.  shape is (ny, nx) or (nz, ny, nx), h is (hx, hy[, hz]).
    chi_exp != 0: chi_par(T) = chi_par (T / chi_tref)^chi_exp."""
    d = Desc()
    d.ndim = len(shape)
    d.bc = BC[bc]
    d.dtype = _dtype_code(dtype)
    d.limiter = LIMITER[limiter]
    nxyz = list(reversed(shape)) + [1] * (3 - len(shape))
    for q in range(3):
        d.n[q] = int(nxyz[q])
        d.h[q] = float(h[q]) if q < len(h) else 1.0
    d.chi_par = float(chi_par)
    d.chi_perp = float(chi_perp)
    d.flags = ((FLAG_PER_CELL_CHI if per_cell_chi else 0) | (FLAG_ALLOW_UNSTABLE if allow_unstable else 0)
               | (FLAG_FOUR_STEP if four_step else 0) | (FLAG_REVERSE_ORDER if reverse_order else 0))
    d.reserved = 0
    d.chi_exp = float(chi_exp)
    d.chi_tref = float(chi_tref)
    return d


def workspace_bytes(desc):
    n = ctypes.c_size_t()
    check(lib().asd_workspace_bytes(ctypes.byref(desc), ctypes.byref(n)))
    return n.value


def _stream_handle(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream), stream


class Grid:
    """A problem on the GPU: owns the workspace tensor and the library handle.

    Fields are torch tensors on the GPU with the grid's dtype and shape
    (ny, nx) / (nz, ny, nx), contiguous.  The handle keeps references to them.
    """

    def __init__(self, shape, h, bc="periodic", dtype=torch.float32, limiter="vanleer", chi_par=1.0,
                 chi_perp=0.0, per_cell_chi=False, allow_unstable=False, device="cuda", stream=None,
                 four_step=False, reverse_order=False, chi_exp=0.0, chi_tref=1.0):
        self.shape = tuple(int(s) for s in shape)
        self.dtype = dtype
        self.device = torch.device(device)
        self.desc = make_desc(self.shape, h, bc, dtype, limiter, chi_par, chi_perp, per_cell_chi, allow_unstable,
                              four_step, reverse_order, chi_exp, chi_tref)
        nbytes = workspace_bytes(self.desc)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._stream_ptr, self.stream = _stream_handle(stream)
        h_out = ctypes.c_void_p()
        check(lib().asd_init_grid(ctypes.byref(self.desc), ctypes.c_void_p(self.workspace.data_ptr()),
                                  nbytes, self._stream_ptr, ctypes.byref(h_out)))
        self.handle = h_out
        self.fields = {}

    @property
    def ncells(self):
        n = 1
        for s in self.shape:
            n *= s
        return n

    def _check_tensor(self, t):
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
            raise TypeError("fields must be CUDA tensors")
        if t.dtype != self.dtype or tuple(t.shape) != self.shape or not t.is_contiguous():
            raise ValueError(f"field must be contiguous {self.dtype} of shape {self.shape}")

    def set_field(self, name, t):
        self._check_tensor(t)
        check(lib().asd_set_field(self.handle, FIELD[name], ctypes.c_void_p(t.data_ptr()), t.numel(),
                                  _dtype_code(t.dtype)))
        self.fields[name] = t

    def set_b(self, *comps):
        for name, c in zip(("bx", "by", "bz"), comps):
            self.set_field(name, c)

    @property
    def T(self):
        return self.fields["T"]

    def _energy_buf(self, nsteps, energy, out):
        if out is not None:
            if out.dtype != torch.float64 or out.device.type != "cuda" or out.numel() < nsteps + 1:
                raise ValueError("out must be a CUDA float64 tensor of at least nsteps+1 entries")
            return out
        if energy:
            return torch.empty(nsteps + 1, dtype=torch.float64, device=self.device)
        return None

    def step_semi_implicit(self, dt, nsteps=1, energy=False, out=None):
        """nsteps semi-implicit steps of T in place.  With energy=True (or an
        FP64 buffer `out` of nsteps+1 entries, reused across calls so that the
        captured step graph is replayed) returns sum T dV per step."""
        e = self._energy_buf(nsteps, energy, out)
        check(lib().asd_step_semi_implicit(self.handle, float(dt), int(nsteps),
                                           ctypes.c_void_p(e.data_ptr()) if e is not None else None))
        return e

    def step_explicit(self, dt, nsteps=1, energy=False, out=None):
        e = self._energy_buf(nsteps, energy, out)
        check(lib().asd_step_explicit_limited(self.handle, float(dt), int(nsteps),
                                              ctypes.c_void_p(e.data_ptr()) if e is not None else None))
        return e

    def step_series(self, scheme, dt, nsteps):
        """nsteps steps of scheme "si" or "ex"; returns a device FP64 tensor
        (nsteps+1, 3) of (energy, min T, max T) for the initial state and
        after every step."""
        s = torch.empty((int(nsteps) + 1, 3), dtype=torch.float64, device=self.device)
        code = {"si": 0, "ex": 1}[scheme]
        check(lib().asd_step_series(self.handle, code, float(dt), int(nsteps), ctypes.c_void_p(s.data_ptr())))
        return s

    def status(self):
        f = ctypes.c_uint32()
        st = (ctypes.c_double * 3)()
        check(lib().asd_status(self.handle, ctypes.byref(f), st))
        return f.value, (st[0], st[1], st[2])

    def adjoint(self, dt, nsteps, ckpt_every, T0, lam, grad_chi=True):
        """dL/dT0 (and dL/dchi) of nsteps semi-implicit steps from T0, given lam = dL/dT_N."""
        self._check_tensor(T0)
        self._check_tensor(lam)
        gT = torch.empty_like(T0)
        gC = torch.empty_like(T0) if grad_chi else None
        n = ctypes.c_size_t()
        check(lib().asd_adjoint_workspace_bytes(self.handle, int(nsteps), int(ckpt_every), ctypes.byref(n)))
        ws = torch.empty(max(n.value, 1), dtype=torch.uint8, device=self.device)
        check(lib().asd_adjoint_step(self.handle, float(dt), int(nsteps), int(ckpt_every),
                                     ctypes.c_void_p(T0.data_ptr()), ctypes.c_void_p(lam.data_ptr()),
                                     ctypes.c_void_p(gT.data_ptr()),
                                     ctypes.c_void_p(gC.data_ptr()) if gC is not None else None,
                                     ctypes.c_void_p(ws.data_ptr()), n.value))
        self._adj_ws = ws  # keep alive until the stream has used it
        return gT, gC

    def adjoint_workspace(self, nsteps, ckpt_every):
        """A device workspace of asd_adjoint_workspace_bytes bytes."""
        n = ctypes.c_size_t()
        check(lib().asd_adjoint_workspace_bytes(self.handle, int(nsteps), int(ckpt_every), ctypes.byref(n)))
        return torch.empty(max(n.value, 1), dtype=torch.uint8, device=self.device)

    def adjoint_forward(self, dt, nsteps, ckpt_every, ws=None):
        """nsteps semi-implicit steps of T in place, storing the reverse
        pass's checkpoints in ws (allocated if None); returns ws."""
        if ws is None:
            ws = self.adjoint_workspace(nsteps, ckpt_every)
        check(lib().asd_adjoint_forward(self.handle, float(dt), int(nsteps), int(ckpt_every),
                                        ctypes.c_void_p(ws.data_ptr()), ws.numel()))
        return ws

    def adjoint_stored(self, dt, nsteps, ckpt_every, ws, lam, grad_chi=True):
        """dL/dT0 (and dL/dchi) from the checkpoints adjoint_forward left in ws."""
        self._check_tensor(lam)
        gT = torch.empty_like(lam)
        gC = torch.empty_like(lam) if grad_chi else None
        check(lib().asd_adjoint_step_stored(self.handle, float(dt), int(nsteps), int(ckpt_every),
                                            ctypes.c_void_p(lam.data_ptr()), ctypes.c_void_p(gT.data_ptr()),
                                            ctypes.c_void_p(gC.data_ptr()) if gC is not None else None,
                                            ctypes.c_void_p(ws.data_ptr()), ws.numel()))
        return gT, gC

    def sweep_config(self, axis):
        w, l, p, m, io, v = (ctypes.c_int32() for _ in range(6))
        check(lib().asd_get_sweep_config(self.handle, int(axis), ctypes.byref(w), ctypes.byref(l),
                                         ctypes.byref(p), ctypes.byref(m)))
        check(lib().asd_get_sweep_io(self.handle, int(axis), ctypes.byref(io)))
        check(lib().asd_get_sweep_variant(self.handle, int(axis), ctypes.byref(v)))
        return dict(wpl=w.value, lpw=l.value, P=p.value, mmax=m.value, io=io.value, variant=v.value)

    def set_sweep_config(self, axis, wpl, lpw, io=1, variant=0):
        """variant 0: face-slot tile body, 1: cell-slot tile body."""
        check(lib().asd_set_sweep_kernel(self.handle, int(axis), int(wpl), int(lpw), int(io), int(variant)))

    def tune(self, dt, reps=20):
        check(lib().asd_tune(self.handle, float(dt), int(reps)))
        return [self.sweep_config(a) for a in range(len(self.shape))]

    def set_graphs(self, mode):
        """Graph capture of step calls: False (never), "auto" (the default:
        calls of 64 steps or more), True (every call of 2 steps or more)."""
        code = {False: GRAPHS_OFF, "auto": GRAPHS_AUTO, True: GRAPHS_ALWAYS}[mode]
        check(lib().asd_set_graphs(self.handle, code))

    def bench_sweep(self, axis, dt, reps):
        """Enqueue reps launches of one sweep kernel (T -> scratch) for timing."""
        check(lib().asd_bench_sweep(self.handle, int(axis), float(dt), int(reps)))

    def close(self):
        if getattr(self, "handle", None):
            lib().asd_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent 2-D problems advanced together (asd_batch_*).

    problems: sequence of dicts with keys shape (ny, nx), h, chi_par, dt and
    tensors T, bx, by (contiguous CUDA, the batch dtype).  T is advanced in
    place.  bc, dtype and limiter are shared."""

    def __init__(self, problems, bc="periodic", dtype=torch.float32, limiter="vanleer", stream=None):
        self.descs = (Desc * len(problems))()
        for i, pr in enumerate(problems):
            self.descs[i] = make_desc(pr["shape"], pr["h"], bc, dtype, limiter, pr.get("chi_par", 1.0),
                                      pr.get("chi_perp", 0.0))
        n = ctypes.c_size_t()
        check(lib().asd_batch_workspace_bytes(self.descs, len(problems), ctypes.byref(n)))
        self.workspace = torch.empty(n.value, dtype=torch.uint8, device="cuda")
        self._stream_ptr, self.stream = _stream_handle(stream)
        h = ctypes.c_void_p()
        check(lib().asd_batch_init(self.descs, len(problems), ctypes.c_void_p(self.workspace.data_ptr()), n.value,
                                   self._stream_ptr, ctypes.byref(h)))
        self.handle = h
        self.problems = list(problems)
        for i, pr in enumerate(problems):
            for name in ("T", "bx", "by"):
                t = pr[name]
                if t.dtype != dtype or tuple(t.shape) != tuple(pr["shape"]) or not t.is_contiguous():
                    raise ValueError(f"problem {i}: {name} must be contiguous {dtype} of shape {pr['shape']}")
            check(lib().asd_batch_set_problem(h, i, ctypes.c_void_p(pr["T"].data_ptr()),
                                              ctypes.c_void_p(pr["bx"].data_ptr()),
                                              ctypes.c_void_p(pr["by"].data_ptr()), float(pr["dt"])))

    def step(self, nsteps, mode=-1, energy=False):
        """nsteps steps of every problem; energy=True returns a device FP64
        tensor (nprob, nsteps + 1) of every problem's sum T dV."""
        e = torch.empty((len(self.problems), nsteps + 1), dtype=torch.float64, device="cuda") if energy else None
        check(lib().asd_batch_step_energy(self.handle, int(nsteps), int(mode),
                                          ctypes.c_void_p(e.data_ptr()) if e is not None else None))
        return e

    def status(self):
        """(flags per problem, stats (nprob, 3) of the last energy-producing call)."""
        import numpy as np
        n = len(self.problems)
        fl = (ctypes.c_uint32 * n)()
        st = (ctypes.c_double * (3 * n))()
        check(lib().asd_batch_status(self.handle, fl, st))
        return np.array(fl[:], dtype=np.uint32), np.array(st[:]).reshape(n, 3)

    def set_graphs(self, on):
        check(lib().asd_batch_set_graphs(self.handle, int(on)))

    def set_block(self, nthreads):
        check(lib().asd_batch_set_block(self.handle, int(nthreads)))

    def set_variant(self, variant):
        """Tile body of the batch kernels: 0 face slots, 1 cell slots."""
        check(lib().asd_batch_set_variant(self.handle, int(variant)))

    def set_capacity(self, mmax):
        """Per-lane capacity of the batch kernels (4, 8 or 16 cells; 16 on
        the face body runs lines of 32-512 cells two per wave)."""
        check(lib().asd_batch_set_capacity(self.handle, int(mmax)))

    def variant(self):
        v = ctypes.c_int32()
        check(lib().asd_batch_get_variant(self.handle, ctypes.byref(v)))
        return v.value

    def tune(self, probe_steps=2):
        m, t = ctypes.c_int32(), ctypes.c_int32()
        check(lib().asd_batch_tune(self.handle, int(probe_steps), ctypes.byref(m), ctypes.byref(t)))
        return m.value, t.value

    def close(self):
        if getattr(self, "handle", None):
            lib().asd_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bench_copy(src, dst, stream=None, wide=False):
    """Device copy kernel of src.numel()*itemsize bytes: the plain one
    (counter calibration) or, wide=True, the 16-byte streaming copy (the
    practical bandwidth ceiling)."""
    sp, _ = _stream_handle(stream)
    f = lib().asd_bench_copy_wide if wide else lib().asd_bench_copy
    check(f(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), src.numel() * src.element_size(), sp))


def noalloc_scratch_bytes():
    """Bytes of the static device scratch behind step_semi_implicit_noalloc."""
    return int(lib().asd_noalloc_scratch_bytes())


def step_semi_implicit_noalloc(T, b, h, dt, nsteps, bc="periodic", limiter="vanleer", chi_par=1.0, chi_perp=0.0,
                               chi=None, energy=None, stream=None):
    """nsteps semi-implicit steps of T in place through the no-allocation
    entry point (static scratch, no handle, no workspace).  b: (bx, by[, bz])
    device tensors of T's shape and dtype; chi: per-cell chi or None;
    energy: None or a device FP64 tensor of nsteps + 1 entries."""
    shape = tuple(T.shape)
    desc = make_desc(shape, h, bc=bc, dtype=T.dtype, limiter=limiter, chi_par=chi_par, chi_perp=chi_perp,
                     per_cell_chi=chi is not None)
    sp, _ = _stream_handle(stream)
    ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)  # noqa: E731
    bz = b[2] if len(b) == 3 else None
    check(lib().asd_step_semi_implicit_noalloc(ctypes.byref(desc), ptr(T), ptr(b[0]), ptr(b[1]), ptr(bz), ptr(chi),
                                               float(dt), int(nsteps), ptr(energy), sp))
