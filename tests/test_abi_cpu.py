"""C ABI checks that run without a GPU: the library loads, exports every
entry point the headers declare, and rejects invalid calls with the
documented status codes before making any HIP call."""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def asd():
    from paper_1008_0861_amd import binding
    binding.lib()
    return binding


def _declared():
    names = set()
    for h in ("asd.h", "asd_extra.h"):
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(asd_[a-z_0-9]+)\s*\(", src))
    return names


def test_every_declared_symbol_is_exported(asd):
    L = asd.lib()
    declared = _declared()
    assert len(declared) >= 20
    for name in sorted(declared):
        assert hasattr(L, name), name
    assert declared == set(asd.EXPORTED)


def test_header_constants_match_binding(asd):
    src = open(os.path.join(ROOT, "include", "asd.h")).read()
    consts = dict(re.findall(r"#define (ASD_\w+) \(?(-?\d+)u?\)?", src))
    assert int(consts["ASD_BC_PERIODIC"]) == asd.BC["periodic"]
    assert int(consts["ASD_BC_INSULATING"]) == asd.BC["insulating"]
    assert int(consts["ASD_BC_DIRICHLET"]) == asd.BC["dirichlet"]
    assert int(consts["ASD_FIELD_Q"]) == asd.FIELD["Q"]
    assert int(consts["ASD_LIM_MC"]) == asd.LIMITER["mc"]
    assert int(consts["ASD_FIELD_CHI"]) == asd.FIELD["chi"]
    for code, name in asd.ERRORS.items():
        assert int(consts["ASD_" + name]) == code
    assert ctypes.sizeof(asd.Desc) == 4 * 4 + 8 * 3 + 8 * 3 + 8 * 2 + 4 * 2 + 8 * 2


def _desc(asd, **kw):
    args = dict(shape=(64, 48), h=(1 / 48, 1 / 64))
    args.update(kw)
    return asd.make_desc(**args)


def _rc_ws(asd, d):
    n = ctypes.c_size_t()
    return asd.lib().asd_workspace_bytes(ctypes.byref(d), ctypes.byref(n)), n.value


def test_workspace_bytes_valid(asd):
    rc, n = _rc_ws(asd, _desc(asd))
    assert rc == 0 and n >= 2 * 64 * 48 * 4 + 2 * 64 * 48 * 4
    rc3, n3 = _rc_ws(asd, _desc(asd, shape=(8, 9, 10), h=(0.1, 0.1, 0.1), dtype=__import__("torch").float64))
    assert rc3 == 0 and n3 >= 2 * 720 * 8 + 6 * 720 * 8


@pytest.mark.parametrize("mutate,code", [
    (lambda d: setattr(d, "ndim", 4), -1),
    (lambda d: setattr(d, "bc", 7), -1),
    (lambda d: setattr(d, "dtype", 5), -1),
    (lambda d: setattr(d, "limiter", 9), -1),
    (lambda d: setattr(d, "reserved", 1), -1),
    (lambda d: setattr(d, "flags", 64), -1),
    (lambda d: d.h.__setitem__(0, 0.0), -1),
    (lambda d: d.h.__setitem__(1, math.nan), -1),
    (lambda d: setattr(d, "chi_par", -1.0), -1),
    (lambda d: setattr(d, "chi_perp", 5.0), -1),
    (lambda d: d.n.__setitem__(0, 2), -2),     # periodic needs n >= 3
    (lambda d: d.n.__setitem__(2, 3), -2),     # 2-D needs n[2] == 1
    (lambda d: d.n.__setitem__(0, 200000), -8),  # line does not fit in LDS
    (lambda d: setattr(d, "chi_exp", -1.0), -1),
    (lambda d: setattr(d, "chi_exp", 9.0), -1),
    (lambda d: setattr(d, "chi_exp", math.inf), -1),
    (lambda d: (setattr(d, "chi_exp", 2.5), setattr(d, "chi_tref", 0.0)), -1),
    (lambda d: (setattr(d, "chi_exp", 2.5), setattr(d, "flags", 1)), -1),  # with per-cell chi
])
def test_bad_descriptions(asd, mutate, code):
    d = _desc(asd)
    mutate(d)
    rc, _ = _rc_ws(asd, d)
    assert rc == code, asd.last_error()
    assert asd.last_error()


@pytest.mark.parametrize("ndim,dtype,nmax", [(2, "float32", 16109), (3, "float32", 16109),
                                             (2, "float64", 4096), (3, "float64", 4096)])
def test_longest_line(asd, ndim, dtype, nmax):
    """The documented maximum line length is accepted on every axis and one
    more cell is refused with EUNSUPPORTED (the line no longer fits in LDS)."""
    import torch
    dt = getattr(torch, dtype)
    for axis in range(ndim):
        for n, code in ((nmax, 0), (nmax + 1, -8)):
            shape = [4] * ndim
            shape[ndim - 1 - axis] = n
            rc, _ = _rc_ws(asd, _desc(asd, shape=tuple(shape), h=(1.0,) * ndim, dtype=dt))
            assert rc == code, (axis, n, asd.last_error())


def test_longest_aligned_fp32_line(asd):
    """16384 cells (16 per lane of 1024 segments) fit in FP32 as well."""
    import torch
    for shape in ((4, 16384), (16384, 4)):
        rc, _ = _rc_ws(asd, _desc(asd, shape=shape, h=(1.0, 1.0), dtype=torch.float32))
        assert rc == 0, asd.last_error()


def test_insulating_allows_two_cells(asd):
    rc, _ = _rc_ws(asd, _desc(asd, shape=(2, 2), h=(1.0, 1.0), bc="insulating"))
    assert rc == 0


def _fake_grid(asd, **kw):
    """A handle over a fake device address: valid for calls that fail in
    validation, which must not touch the device."""
    d = _desc(asd, **kw)
    rc, n = _rc_ws(asd, d)
    assert rc == 0
    h = ctypes.c_void_p()
    rc = asd.lib().asd_init_grid(ctypes.byref(d), ctypes.c_void_p(1 << 20), n, None, ctypes.byref(h))
    assert rc == 0, asd.last_error()
    return h, d, n


def test_init_grid_workspace_errors(asd):
    d = _desc(asd)
    rc, n = _rc_ws(asd, d)
    h = ctypes.c_void_p()
    L = asd.lib()
    assert L.asd_init_grid(ctypes.byref(d), None, n, None, ctypes.byref(h)) == -5
    assert L.asd_init_grid(ctypes.byref(d), ctypes.c_void_p(4096 + 8), n, None, ctypes.byref(h)) == -5
    assert L.asd_init_grid(ctypes.byref(d), ctypes.c_void_p(4096), n - 1, None, ctypes.byref(h)) == -5
    assert L.asd_init_grid(ctypes.byref(d), ctypes.c_void_p(4096), n, None, None) == -1


def test_set_field_and_step_validation(asd):
    import torch
    L = asd.lib()
    h, d, _ = _fake_grid(asd)
    N = 64 * 48
    fake = ctypes.c_void_p(1 << 24)
    assert L.asd_set_field(h, 0, fake, N, asd.F64) == -3       # dtype mismatch
    assert L.asd_set_field(h, 0, fake, N + 1, asd.F32) == -2   # size mismatch
    assert L.asd_set_field(h, 0, None, N, asd.F32) == -1       # null pointer
    assert L.asd_set_field(h, 9, fake, N, asd.F32) == -1       # unknown field
    assert L.asd_set_field(h, 3, fake, N, asd.F32) == -1       # bz on a 2-D grid
    assert L.asd_set_field(h, 4, fake, N, asd.F32) == -1       # chi without the flag
    # step before the fields are set
    assert L.asd_step_semi_implicit(h, 1e-3, 1, None) == -4
    assert L.asd_set_field(h, 0, fake, N, asd.F32) == 0
    assert L.asd_set_field(h, 1, fake, N, asd.F32) == 0
    assert L.asd_step_semi_implicit(h, 1e-3, 1, None) == -4     # by missing
    assert "by" in asd.last_error()
    for bad_dt in (0.0, -1.0, math.nan, math.inf):
        assert L.asd_step_semi_implicit(h, bad_dt, 1, None) == -1
        assert L.asd_step_explicit_limited(h, bad_dt, 1, None) == -1
    assert L.asd_step_semi_implicit(h, 1e-3, -1, None) == -1
    # explicit step beyond the 2-D limit chi dt (1/hx^2 + 1/hy^2) <= 1
    assert L.asd_set_field(h, 2, fake, N, asd.F32) == 0
    dt_bad = 1.01 / (48 ** 2 + 64 ** 2)
    assert L.asd_step_explicit_limited(h, dt_bad, 1, None) == -6
    assert L.asd_destroy(h) == 0
    assert L.asd_destroy(None) == -1
    del torch


def test_3d_stability_limits_are_enforced(asd):
    import torch
    L = asd.lib()
    h, d, _ = _fake_grid(asd, shape=(8, 8, 8), h=(0.1, 0.1, 0.1), dtype=torch.float64)
    fake = ctypes.c_void_p(1 << 24)
    for f in range(4):
        assert L.asd_set_field(h, f, fake, 512, asd.F64) == 0
    assert L.asd_step_semi_implicit(h, 8.3 * 0.01, 1, None) == -6      # > 8.25
    assert L.asd_step_explicit_limited(h, 0.45 * 0.01, 1, None) == -6  # > 0.444
    L.asd_destroy(h)
    d = _desc(asd, shape=(8, 8, 8), h=(0.1, 0.1, 0.1), dtype=torch.float64, allow_unstable=True)
    assert d.flags & asd.FLAG_ALLOW_UNSTABLE


def test_sweep_config_api(asd):
    L = asd.lib()
    h, d, _ = _fake_grid(asd, shape=(64, 1024), h=(1 / 1024, 1 / 64))
    w, l, p, m = (ctypes.c_int32() for _ in range(4))
    assert L.asd_get_sweep_config(h, 0, ctypes.byref(w), ctypes.byref(l), ctypes.byref(p), ctypes.byref(m)) == 0
    assert p.value <= 64 * w.value and p.value & (p.value - 1) == 0
    assert m.value * p.value >= 1024
    assert L.asd_set_sweep_config(h, 0, 2, 2) == 0
    assert L.asd_get_sweep_config(h, 0, ctypes.byref(w), ctypes.byref(l), ctypes.byref(p), ctypes.byref(m)) == 0
    assert (w.value, l.value) == (2, 2)
    assert L.asd_set_sweep_config(h, 0, 3, 1) == -1
    assert L.asd_set_sweep_config(h, 0, 1, 64) == -8
    assert L.asd_set_sweep_config(h, 5, 1, 1) == -1
    # tile bodies: face slots (0, default) and cell slots (1, io = 1 only)
    v = ctypes.c_int32()
    assert L.asd_get_sweep_variant(h, 0, ctypes.byref(v)) == 0 and v.value == 0
    assert L.asd_set_sweep_kernel(h, 0, 2, 4, 1, 1) == 0
    assert L.asd_get_sweep_variant(h, 0, ctypes.byref(v)) == 0 and v.value == 1
    assert L.asd_get_sweep_config(h, 0, ctypes.byref(w), ctypes.byref(l), ctypes.byref(p), ctypes.byref(m)) == 0
    assert (w.value, l.value) == (2, 4)
    assert L.asd_set_sweep_kernel(h, 0, 2, 4, 2, 1) == -1  # io 2 is face-slot only
    assert L.asd_set_sweep_kernel(h, 0, 2, 4, 1, 2) == -1  # no such body
    assert L.asd_set_sweep_kernel(h, 0, 1, 64, 1, 1) == -8  # does not fit
    assert L.asd_set_sweep_shape(h, 0, 2, 2, 1) == 0       # back to face slots
    assert L.asd_get_sweep_variant(h, 0, ctypes.byref(v)) == 0 and v.value == 0
    L.asd_destroy(h)


def test_cell_body_longest_lines(asd):
    """The cell-slot body stages 16 bytes per cell in FP32 (twice the face
    slots): its longest 2-D FP32 line is 8192 cells, and longer lines refuse
    it while the face-slot body takes them."""
    L = asd.lib()
    for n, fits in ((8192, True), (16109, False)):
        h, d, _ = _fake_grid(asd, shape=(4, n), h=(1 / n, 1 / 4))
        ok = False
        for wpl in (1, 2, 4, 8, 16):
            ok = ok or L.asd_set_sweep_kernel(h, 0, wpl, 1, 1, 1) == 0
        assert ok == fits, n
        assert L.asd_set_sweep_kernel(h, 0, 16, 1, 1, 0) == 0 or L.asd_set_sweep_kernel(h, 0, 8, 1, 1, 0) == 0
        L.asd_destroy(h)


def test_batch_refuses_chi_of_T(asd):
    descs = (asd.Desc * 2)(_desc(asd), _desc(asd, chi_exp=2.5, chi_tref=1.0))
    n = ctypes.c_size_t()
    assert asd.lib().asd_batch_workspace_bytes(descs, 2, ctypes.byref(n)) == -8
    assert "constant chi_par" in asd.last_error()
    rc, _ = _rc_ws(asd, _desc(asd, chi_exp=2.5, chi_tref=1.0))
    assert rc == 0


def test_batch_boundary_conditions(asd):
    # T = 0 walls are accepted; every problem of a batch takes problem 0's bc
    n = ctypes.c_size_t()
    descs = (asd.Desc * 2)(_desc(asd, bc="dirichlet"), _desc(asd, bc="dirichlet", shape=(7, 5)))
    assert asd.lib().asd_batch_workspace_bytes(descs, 2, ctypes.byref(n)) == 0
    assert n.value > 0
    descs = (asd.Desc * 2)(_desc(asd), _desc(asd, bc="dirichlet"))
    assert asd.lib().asd_batch_workspace_bytes(descs, 2, ctypes.byref(n)) == -1
    assert "must match problem 0" in asd.last_error()


def test_noalloc_validation_before_any_gpu_call(asd):
    """The no-allocation entry point checks its arguments and the static
    scratch's capacity before any HIP call (no device is needed here)."""
    import ctypes
    import torch
    fake = ctypes.c_void_p(256)
    big = _desc(asd, shape=(1800, 1800), h=(1 / 1800, 1 / 1800), dtype=torch.float32)
    rc = asd.lib().asd_step_semi_implicit_noalloc(ctypes.byref(big), fake, fake, fake, None, None, 1e-6, 1, None,
                                                  None)
    assert rc == -8 and "scratch" in asd.last_error()
    small = _desc(asd, shape=(64, 64), h=(1 / 64, 1 / 64), dtype=torch.float32)
    rc = asd.lib().asd_step_semi_implicit_noalloc(ctypes.byref(small), fake, fake, fake, None, None, 1e-6, -1,
                                                  None, None)
    assert rc == -1
    rc = asd.lib().asd_step_semi_implicit_noalloc(ctypes.byref(small), fake, None, fake, None, None, 1e-6, 1, None,
                                                  None)
    assert rc == -1
    assert asd.noalloc_scratch_bytes() == 64 << 20


def test_adjoint_entry_points_validate_before_any_gpu_call(asd):
    """asd_adjoint_step, asd_adjoint_forward and asd_adjoint_step_stored share
    one validation: null grid or pointers, bad dt or counts, workspace
    missing / misaligned / too small, grad_chi without per-cell chi, fields
    not set; all are refused before the device is touched."""
    L = asd.lib()
    h, d, _ = _fake_grid(asd)
    fake = ctypes.c_void_p(1 << 24)
    ws_n = ctypes.c_size_t()
    field = (64 * 48 * 4 + 255) // 256 * 256
    # one segment: one set of segment states
    assert L.asd_adjoint_workspace_bytes(h, 5, 5, ctypes.byref(ws_n)) == 0
    assert ws_n.value == (1 + 10 + 4) * field
    # 3 checkpoints + 2 sets of 2 x 5 segment states + 4 work fields of 64 x 48 FP32
    assert L.asd_adjoint_workspace_bytes(h, 12, 5, ctypes.byref(ws_n)) == 0
    assert ws_n.value == (3 + 20 + 4) * field
    ws, n = ctypes.c_void_p(1 << 26), ws_n.value
    assert L.asd_adjoint_forward(None, 1e-3, 12, 5, ws, n) == -1
    assert L.asd_adjoint_step_stored(None, 1e-3, 12, 5, fake, fake, None, ws, n) == -1
    for bad_dt in (0.0, -1.0, math.nan, math.inf):
        assert L.asd_adjoint_forward(h, bad_dt, 12, 5, ws, n) == -1
        assert L.asd_adjoint_step_stored(h, bad_dt, 12, 5, fake, fake, None, ws, n) == -1
    assert L.asd_adjoint_forward(h, 1e-3, -1, 5, ws, n) == -1
    assert L.asd_adjoint_forward(h, 1e-3, 12, 0, ws, n) == -1
    assert L.asd_adjoint_step_stored(h, 1e-3, 12, 5, None, fake, None, ws, n) == -1
    assert L.asd_adjoint_step_stored(h, 1e-3, 12, 5, fake, None, None, ws, n) == -1
    assert L.asd_adjoint_step_stored(h, 1e-3, 12, 5, fake, fake, fake, ws, n) == -1  # grad_chi, no per-cell chi
    assert L.asd_adjoint_forward(h, 1e-3, 12, 5, None, n) == -5
    assert L.asd_adjoint_forward(h, 1e-3, 12, 5, ctypes.c_void_p((1 << 26) + 64), n) == -5
    assert L.asd_adjoint_forward(h, 1e-3, 12, 5, ws, n - 1) == -5
    assert L.asd_adjoint_step_stored(h, 1e-3, 12, 5, fake, fake, None, ws, n - 1) == -5
    assert L.asd_adjoint_forward(h, 1e-3, 12, 5, ws, n) == -4  # T, b not set
    assert L.asd_adjoint_step_stored(h, 1e-3, 12, 5, fake, fake, None, ws, n) == -4
    assert L.asd_destroy(h) == 0


def test_graph_mode_validation(asd):
    """asd_set_graphs takes ASD_GRAPHS_OFF / _AUTO / _ALWAYS (the values the
    header defines) and refuses anything else; no device work."""
    src = open(os.path.join(ROOT, "include", "asd_extra.h")).read()
    consts = dict(re.findall(r"#define (ASD_GRAPHS_\w+) (\d+)", src))
    assert {k: int(v) for k, v in consts.items()} == {
        "ASD_GRAPHS_OFF": asd.GRAPHS_OFF, "ASD_GRAPHS_AUTO": asd.GRAPHS_AUTO, "ASD_GRAPHS_ALWAYS": asd.GRAPHS_ALWAYS}
    L = asd.lib()
    h, _, _ = _fake_grid(asd)
    for m in (asd.GRAPHS_OFF, asd.GRAPHS_AUTO, asd.GRAPHS_ALWAYS):
        assert L.asd_set_graphs(h, m) == 0
    for m in (-1, 3, 7):
        assert L.asd_set_graphs(h, m) == -1
    assert L.asd_set_graphs(None, 1) == -1
    assert L.asd_destroy(h) == 0


def test_batch_capacity_validation(asd):
    L = asd.lib()
    assert L.asd_batch_set_capacity(None, 16) == -1
