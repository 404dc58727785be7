"""The C ABI without a GPU: every symbol declared in include/demag.h is
exported, and argument checking happens on the host before any HIP call."""
import ctypes
import os
import re

import pytest

from paper_2008_02478_amd import lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        from paper_2008_02478_amd import build_lib
        build_lib.build()
    return L.load()


def declared():
    text = open(os.path.join(ROOT, "include", "demag.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(demag_\w+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert "demag_field" in names and "demag_setup" in names
    for name in names:
        assert hasattr(lib, name), name


def setup(lib, *args):
    p = ctypes.c_void_p()
    rc = lib.demag_setup(ctypes.byref(p), *args)
    return rc, p


@pytest.mark.parametrize("args,code", [
    ((0, 4, 4, 1e-9, 1e-9, 1e-9, 0, 0), L.EINVAL),
    ((4, -1, 4, 1e-9, 1e-9, 1e-9, 0, 0), L.EINVAL),
    ((4, 4, 4, 0.0, 1e-9, 1e-9, 0, 0), L.EINVAL),
    ((4, 4, 4, 1e-9, float("nan"), 1e-9, 0, 0), L.EINVAL),
    ((4, 4, 4, 1e-9, 1e-9, float("inf"), 0, 0), L.EINVAL),
    ((4, 4, 4, 1e-9, 1e-9, 1e-9, 8, 0), L.EINVAL),
    ((4, 4, 4, 1e-9, 1e-9, 1e-9, L.PBC_X, 1001), L.EINVAL),
    ((4, 4, 257, 1e-9, 1e-9, 1e-9, 0, 0), L.EUNSUPPORTED),
    ((4, 1025, 4, 1e-9, 1e-9, 1e-9, 0, 0), L.EUNSUPPORTED),
    ((2049, 4, 4, 1e-9, 1e-9, 1e-9, 0, 0), L.EUNSUPPORTED),
])
def test_setup_rejects(lib, args, code):
    rc, p = setup(lib, *args)
    assert rc == code
    assert not p.value
    assert len(lib.demag_last_error()) > 0


def test_setup_null_out(lib):
    assert lib.demag_setup(None, 4, 4, 4, 1e-9, 1e-9, 1e-9, 0, 0) == L.EINVAL


@pytest.mark.parametrize("n,padded", [((64, 64, 1), (128, 128, 1)), ((512, 512, 16), (1024, 1024, 32)),
                                      ((1, 1, 1), (1, 1, 1)), ((5, 3, 2), (16, 8, 4)),
                                      ((1024, 1024, 4), (2048, 2048, 8))])
def test_geometry_and_buffer_sizes(lib, n, padded):
    rc, p = setup(lib, *n, 2e-9, 2e-9, 1e-9, 0, 0)
    assert rc == L.OK
    try:
        dims = [ctypes.c_int() for _ in range(3)]
        assert lib.demag_padded_dims(p, *[ctypes.byref(d) for d in dims]) == L.OK
        assert tuple(d.value for d in dims) == padded
        kb, wb = ctypes.c_size_t(), ctypes.c_size_t()
        assert lib.demag_buffer_bytes(p, ctypes.byref(kb), ctypes.byref(wb)) == L.OK
        Nx, Ny, Nz = padded
        Kx = Nx // 2 + 1 if Nx > 1 else 1
        Ky = Ny // 2 + 1 if Ny > 1 else 1
        Kz = Nz // 2 + 1 if Nz > 1 else 1
        assert kb.value >= 6 * Kx * Ky * Kz * 4 + 4096 * 8
        tiles = (Kx + 7) // 8
        assert wb.value >= 3 * Nz * tiles * 8 * n[1] * 8
        assert kb.value % 256 == 0 and wb.value % 256 == 0
    finally:
        assert lib.demag_destroy(p) == L.OK


def test_calls_before_bind_are_state_errors(lib):
    rc, p = setup(lib, 8, 8, 2, 1e-9, 1e-9, 1e-9, 0, 0)
    assert rc == L.OK
    try:
        dummy = ctypes.c_void_p(256)
        assert lib.demag_field(p, dummy, None, 1.0, dummy, 0, None, None) == L.ESTATE
        assert lib.demag_energy(p, dummy, None, 1.0, dummy, dummy, None) == L.ESTATE
        assert lib.demag_backward(p, dummy, None, 1.0, None, None, dummy, 0, None) == L.ESTATE
        # bind validates its buffers before touching the device
        assert lib.demag_bind(p, None, dummy, None) == L.EINVAL
        assert lib.demag_bind(p, ctypes.c_void_p(257), dummy, None) == L.EINVAL
    finally:
        lib.demag_destroy(p)


def test_null_plan_and_destroy(lib):
    assert lib.demag_destroy(None) == L.OK
    assert lib.demag_field(None, None, None, 1.0, None, 0, None, None) == L.EINVAL
    assert lib.demag_buffer_bytes(None, None, None) == L.EINVAL
    assert lib.demag_set_timing_events(None, None, 0) == L.EINVAL


def test_timing_event_validation(lib):
    rc, p = setup(lib, 8, 8, 2, 1e-9, 1e-9, 1e-9, 0, 0)
    try:
        arr = (ctypes.c_void_p * 4)(1, 2, 3, 4)
        assert lib.demag_set_timing_events(p, arr, 3) == L.EINVAL
        bad = (ctypes.c_void_p * 4)(1, None, 3, 4)
        assert lib.demag_set_timing_events(p, bad, 4) == L.EINVAL
        assert lib.demag_set_timing_events(p, None, 0) == L.OK
    finally:
        lib.demag_destroy(p)


def test_batch_setup_and_layout(lib):
    import numpy as np
    dims = (ctypes.c_int * 9)(4, 3, 2, 8, 8, 1, 4, 3, 2)
    cells = (ctypes.c_double * 9)(1e-9, 1e-9, 1e-9, 5e-9, 5e-9, 3e-9, 1e-9, 1e-9, 1e-9)
    p = ctypes.c_void_p()
    assert lib.demag_setup_batch(ctypes.byref(p), 3, dims, cells, None, None, 0, 0) == L.OK
    try:
        nm, tot = ctypes.c_int(), ctypes.c_size_t()
        offs = (ctypes.c_longlong * 3)()
        assert lib.demag_batch_layout(p, ctypes.byref(nm), offs, ctypes.byref(tot)) == L.OK
        assert nm.value == 3
        assert list(offs) == [0, 3 * 24, 3 * 24 + 3 * 64]
        assert tot.value == 3 * (24 + 64 + 24)
        dummy = ctypes.c_void_p(256)
        # single-mesh entry points refuse batch plans, batch calls need a bind first
        assert lib.demag_field(p, dummy, None, 1.0, dummy, 0, None, None) == L.EINVAL
        assert lib.demag_field_batch(p, dummy, None, 1.0, dummy, 0, None, None) == L.ESTATE
    finally:
        lib.demag_destroy(p)


@pytest.mark.parametrize("n,code", [(0, L.EINVAL), (2, L.EUNSUPPORTED)])
def test_batch_setup_rejects(lib, n, code):
    dims = (ctypes.c_int * 6)(4, 3, 2, 4, 3, 257)
    cells = (ctypes.c_double * 6)(1e-9, 1e-9, 1e-9, 1e-9, 1e-9, 1e-9)
    p = ctypes.c_void_p()
    assert lib.demag_setup_batch(ctypes.byref(p), n, dims, cells, None, None, 0, 0) == code
    assert not p.value


def test_single_plan_refuses_batch_calls(lib):
    p = ctypes.c_void_p()
    assert lib.demag_setup(ctypes.byref(p), 8, 8, 2, 1e-9, 1e-9, 1e-9, 0, 0) == L.OK
    try:
        dummy = ctypes.c_void_p(256)
        assert lib.demag_field_batch(p, dummy, None, 1.0, dummy, 0, None, None) == L.EINVAL
        assert lib.demag_backward_batch(p, dummy, None, 1.0, None, None, dummy, 0, None) == L.EINVAL
    finally:
        lib.demag_destroy(p)


def test_coupled_group_validation(lib):
    dims = (ctypes.c_int * 9)(8, 8, 2, 8, 8, 1, 4, 4, 3)
    ok_cells = (ctypes.c_double * 9)(1e-9, 1e-9, 1e-9, 1e-9, 1e-9, 1e-9, 2e-9, 2e-9, 2e-9)
    origins = (ctypes.c_double * 9)(0, 0, 0, 0, 0, 3e-9, 0, 0, 7e-9)
    groups = (ctypes.c_int * 3)(0, 0, 0)
    p = ctypes.c_void_p()
    assert lib.demag_setup_batch(ctypes.byref(p), 3, dims, ok_cells, origins, groups, 0, 0) == L.OK
    lib.demag_destroy(p)
    # non power-of-two in-plane ratio
    bad = (ctypes.c_double * 9)(1e-9, 1e-9, 1e-9, 1e-9, 1e-9, 1e-9, 3e-9, 3e-9, 2e-9)
    assert lib.demag_setup_batch(ctypes.byref(p), 3, dims, bad, origins, groups, 0, 0) == L.EUNSUPPORTED
    # origin off the fine lattice
    off = (ctypes.c_double * 9)(0, 0, 0, 0.3e-9, 0, 3e-9, 0, 0, 7e-9)
    assert lib.demag_setup_batch(ctypes.byref(p), 3, dims, ok_cells, off, groups, 0, 0) == L.EUNSUPPORTED
    # too many planes (2 + 1 + 6 > 8)
    dims9 = (ctypes.c_int * 9)(8, 8, 2, 8, 8, 1, 4, 4, 6)
    assert lib.demag_setup_batch(ctypes.byref(p), 3, dims9, ok_cells, origins, groups, 0, 0) == L.EUNSUPPORTED
    # groups without origins
    assert lib.demag_setup_batch(ctypes.byref(p), 3, dims, ok_cells, None, groups, 0, 0) == L.EINVAL


def _sched(lib, p, part):
    yg, kw, r = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    rc = lib.demag_get_schedule(p, part, ctypes.byref(yg), ctypes.byref(kw), ctypes.byref(r))
    return rc, (yg.value, kw.value, r.value)


def test_schedule_defaults_and_parts(lib):
    rc, p = setup(lib, 512, 512, 16, 2e-9, 2e-9, 1e-9, 0, 0)
    assert rc == L.OK
    n = ctypes.c_int()
    assert lib.demag_schedule_count(p, ctypes.byref(n)) == L.OK and n.value == 1
    rc, s = _sched(lib, p, 0)
    # 16 rows of one y line fill a 512-thread workgroup; Ny/2 = 512 points per y line at radix 8
    assert rc == L.OK and s == (1, 4, 8)
    assert _sched(lib, p, 1)[0] == L.EINVAL
    assert _sched(lib, p, -1)[0] == L.EINVAL
    lib.demag_destroy(p)
    # batch: two geometries of independent meshes, then one coupled group
    k = 4
    dims = (ctypes.c_int * (3 * k))(64, 64, 1, 32, 32, 2, 64, 64, 1, 64, 64, 2)
    cells = (ctypes.c_double * (3 * k))(*([1e-9] * (3 * k)))
    orig = (ctypes.c_double * (3 * k))(*([0.0] * 9 + [0.0, 0.0, 5e-9]))
    grp = (ctypes.c_int * k)(-1, -1, 0, 0)
    p = ctypes.c_void_p()
    assert lib.demag_setup_batch(ctypes.byref(p), k, dims, cells, orig, grp, 0, 0) == L.OK
    assert lib.demag_schedule_count(p, ctypes.byref(n)) == L.OK and n.value == 3
    assert _sched(lib, p, 2)[1][0] == 0   # coupled groups have no x-pass rows to tune
    lib.demag_destroy(p)


@pytest.mark.parametrize("n,yg,kw,radix,code", [
    ((512, 512, 16), 0, 2, 0, L.OK),
    ((512, 512, 16), 0, 8, 16, L.OK),        # 2 x 8 lines x 32 lanes = 512 threads
    ((512, 512, 16), 2, 0, 0, L.OK),         # two 16-row y lines in 144 KiB of LDS
    ((512, 512, 16), 3, 0, 0, L.EINVAL),     # beyond 160 KiB
    ((512, 512, 16), 0, 3, 0, L.EINVAL),
    ((512, 512, 16), 0, 0, 4, L.EUNSUPPORTED),   # 128 lanes per 512-point line
    ((512, 512, 16), 0, 0, 32, L.EUNSUPPORTED),
    ((200, 200, 2), 0, 8, 4, L.OK),          # 256-point lines at radix 4: 1024 threads
    ((200, 200, 2), 0, 0, 16, L.OK),
    ((200, 200, 2), 201, 0, 0, L.EINVAL),    # more rows than ny
    ((100, 1000, 1), 0, 8, 0, L.EUNSUPPORTED),   # 1024-point lines at radix 16 with 8 lines
    ((100, 1000, 1), 0, 0, 8, L.EUNSUPPORTED),
    ((64, 64, 1), 0, 0, 16, L.EUNSUPPORTED),
])
def test_set_schedule_validation(lib, n, yg, kw, radix, code):
    rc, p = setup(lib, *n, 1e-9, 1e-9, 1e-9, 0, 0)
    assert rc == L.OK
    before = _sched(lib, p, 0)[1]
    rc = lib.demag_set_schedule(p, 0, yg, kw, radix)
    assert rc == code, lib.demag_last_error()
    after = _sched(lib, p, 0)[1]
    if code == L.OK:
        want = tuple(v if v else b for v, b in zip((yg, kw, radix), before))
        assert after == want
    else:
        assert after == before and len(lib.demag_last_error()) > 0
    lib.demag_destroy(p)


def test_set_schedule_group_rules(lib):
    k = 2
    dims = (ctypes.c_int * (3 * k))(64, 64, 1, 64, 64, 1)
    cells = (ctypes.c_double * (3 * k))(*([1e-9] * (3 * k)))
    orig = (ctypes.c_double * (3 * k))(0.0, 0.0, 0.0, 0.0, 0.0, 3e-9)
    grp = (ctypes.c_int * k)(0, 0)
    p = ctypes.c_void_p()
    assert lib.demag_setup_batch(ctypes.byref(p), k, dims, cells, orig, grp, 0, 0) == L.OK
    assert lib.demag_set_schedule(p, 0, 1, 0, 0) == L.EINVAL
    assert lib.demag_set_schedule(p, 0, 0, 2, 0) == L.OK
    assert _sched(lib, p, 0)[1][1] == 2
    assert lib.demag_set_schedule(p, 1, 0, 4, 0) == L.EINVAL
    assert lib.demag_set_schedule(None, 0, 0, 4, 0) == L.EINVAL
    lib.demag_destroy(p)


def test_autotune_host_checks(lib, tmp_path):
    rc, p = setup(lib, 64, 64, 1, 5e-9, 5e-9, 3e-9, 0, 0)
    assert rc == L.OK
    n = ctypes.c_int(7)
    assert lib.demag_autotune(None, None, None, None, 0, ctypes.byref(n), None) == L.EINVAL
    assert lib.demag_autotune(p, None, None, None, 4, ctypes.byref(n), None) == L.EINVAL
    for bad in ('{"entries": {}}', '{"format": "demag-schedule-cache/1", "entries": [1]}', "{", "[]",
                '{"format": "demag-schedule-cache/1", "entries": {"k": {"kw": }}}',
                '{"format": "demag-schedule-cache/1"} trailing'):
        f = tmp_path / "bad.json"
        f.write_text(bad)
        assert lib.demag_autotune(p, None, None, str(f).encode(), 0, ctypes.byref(n), None) == L.EINVAL, bad
        assert b"schedule cache" in lib.demag_last_error()
    assert n.value == 0
    lib.demag_destroy(p)


@pytest.mark.parametrize("flags,images", [(L.PBC_X, 3), (L.PBC_Y, 0), (L.PBC_X | L.PBC_Y, -5),
                                          (L.PBC_Z, 1000), (7, 2)])
def test_periodic_setup_accepted(lib, flags, images):
    rc, p = setup(lib, 20, 12, 2, 2e-9, 2e-9, 1e-9, flags, images)
    assert rc == L.OK, lib.demag_last_error()
    lib.demag_destroy(p)


def test_periodic_batch_rules(lib):
    k = 3
    dims = (ctypes.c_int * (3 * k))(16, 16, 1, 16, 16, 1, 8, 8, 2)
    cells = (ctypes.c_double * (3 * k))(*([1e-9] * (3 * k)))
    orig = (ctypes.c_double * (3 * k))(0.0, 0.0, 0.0, 0.0, 0.0, 3e-9, 0.0, 0.0, 0.0)
    p = ctypes.c_void_p()
    grp = (ctypes.c_int * k)(0, 0, -1)
    # coupled groups: periodic x and y, not z
    assert lib.demag_setup_batch(ctypes.byref(p), k, dims, cells, orig, grp, L.PBC_X, 4) == L.OK
    lib.demag_destroy(p)
    assert lib.demag_setup_batch(ctypes.byref(p), k, dims, cells, orig, grp, L.PBC_X | L.PBC_Y, 0) == L.OK
    lib.demag_destroy(p)
    assert lib.demag_setup_batch(ctypes.byref(p), k, dims, cells, orig, grp, L.PBC_Z, 4) == L.EUNSUPPORTED
    assert not p.value
    # along a periodic axis every mesh of the group spans the whole group
    dims2 = (ctypes.c_int * (3 * k))(16, 16, 1, 12, 16, 1, 8, 8, 2)
    assert lib.demag_setup_batch(ctypes.byref(p), k, dims2, cells, orig, grp, L.PBC_X, 4) == L.EUNSUPPORTED
    assert lib.demag_setup_batch(ctypes.byref(p), k, dims2, cells, orig, grp, L.PBC_Y, 4) == L.OK
    lib.demag_destroy(p)
    orig2 = (ctypes.c_double * (3 * k))(0.0, 0.0, 0.0, 0.0, 2e-9, 3e-9, 0.0, 0.0, 0.0)
    dims3 = (ctypes.c_int * (3 * k))(16, 18, 1, 16, 16, 1, 8, 8, 2)
    assert lib.demag_setup_batch(ctypes.byref(p), k, dims3, cells, orig2, grp, L.PBC_Y, 4) == L.EUNSUPPORTED
    grp = (ctypes.c_int * k)(-1, -1, -1)
    assert lib.demag_setup_batch(ctypes.byref(p), k, dims, cells, orig, grp, L.PBC_X | L.PBC_Y, 4) == L.OK
    lib.demag_destroy(p)
    assert lib.demag_setup_batch(ctypes.byref(p), k, dims, cells, orig, grp, 8, 4) == L.EINVAL


def test_llg_and_two_sublattice_host_checks(lib):
    rc, p = setup(lib, 16, 8, 1, 5e-9, 5e-9, 3e-9, 0, 0)
    assert rc == L.OK
    nb = ctypes.c_size_t()
    assert lib.demag_llg_workspace_bytes(p, ctypes.byref(nb)) == L.OK
    assert nb.value >= 4 * 3 * 16 * 8 * 4
    d = ctypes.c_void_p(256)
    prm = L.LlgParams(8e5, 1.3e-11, 0.02, 0.0, 1e-13, (ctypes.c_float * 3)(0.0, 0.0, 1e4))
    # not bound yet
    assert lib.demag_llg_rk4(p, d, ctypes.byref(prm), d, None) == L.ESTATE
    assert lib.demag_llg_rk4(p, None, ctypes.byref(prm), d, None) == L.EINVAL
    assert lib.demag_llg_rk4(p, d, None, d, None) == L.EINVAL
    assert lib.demag_field_2sub(p, d, d, 1.0, 1.0, d, 0, None, None) == L.ESTATE
    # unbound plans report the state before argument pointers
    assert lib.demag_field_2sub(p, d, None, 1.0, 1.0, d, 0, None, None) == L.ESTATE
    assert lib.demag_field_2sub(None, d, d, 1.0, 1.0, d, 0, None, None) == L.EINVAL
    bad = L.LlgParams(-1.0, 1.3e-11, 0.02, 0.0, 1e-13, (ctypes.c_float * 3)(0.0, 0.0, 0.0))
    assert lib.demag_llg_rk4(None, d, ctypes.byref(bad), d, None) == L.EINVAL
    lib.demag_destroy(p)
    k = 2
    dims = (ctypes.c_int * (3 * k))(8, 8, 1, 8, 8, 1)
    cells = (ctypes.c_double * (3 * k))(*([1e-9] * (3 * k)))
    q = ctypes.c_void_p()
    assert lib.demag_setup_batch(ctypes.byref(q), k, dims, cells, None, None, 0, 0) == L.OK
    assert lib.demag_llg_workspace_bytes(q, ctypes.byref(nb)) == L.EINVAL
    assert lib.demag_llg_rk4(q, d, ctypes.byref(prm), d, None) == L.EINVAL
    assert lib.demag_field_2sub(q, d, d, 1.0, 1.0, d, 0, None, None) == L.EINVAL
    lib.demag_destroy(q)


def test_oersted_plan_host_checks(lib):
    p = ctypes.c_void_p()
    assert lib.demag_setup_oersted(None, 8, 8, 1, 1e-9, 1e-9, 1e-9, 0, 0) == L.EINVAL
    assert lib.demag_setup_oersted(ctypes.byref(p), 0, 8, 1, 1e-9, 1e-9, 1e-9, 0, 0) == L.EINVAL
    assert lib.demag_setup_oersted(ctypes.byref(p), 8, 8, 1, 1e-9, -1e-9, 1e-9, 0, 0) == L.EINVAL
    assert lib.demag_setup_oersted(ctypes.byref(p), 8, 8, 257, 1e-9, 1e-9, 1e-9, 0, 0) == L.EUNSUPPORTED
    assert lib.demag_setup_oersted(ctypes.byref(p), 8, 8, 1, 1e-9, 1e-9, 1e-9, 8, 0) == L.EINVAL
    assert lib.demag_setup_oersted(ctypes.byref(p), 8, 8, 1, 1e-9, 1e-9, 1e-9, L.PBC_X, 1001) == L.EINVAL
    assert lib.demag_setup_oersted(ctypes.byref(p), 8, 8, 1, 1e-9, 1e-9, 1e-9, L.PBC_X | L.PBC_Y, 0) == L.OK
    lib.demag_destroy(p)
    assert lib.demag_setup_oersted(ctypes.byref(p), 40, 30, 5, 2e-9, 2e-9, 1e-9, 0, 0) == L.OK
    kb, wb = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.demag_buffer_bytes(p, ctypes.byref(kb), ctypes.byref(wb)) == L.OK
    rc, q = setup(lib, 40, 30, 5, 2e-9, 2e-9, 1e-9, 0, 0)
    assert rc == L.OK
    kq, wq = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.demag_buffer_bytes(q, ctypes.byref(kq), ctypes.byref(wq)) == L.OK
    # three kernel rows per (kz, kx) instead of six; the same work buffer
    assert kb.value < kq.value and wb.value == wq.value
    d = ctypes.c_void_p(256)
    prm = L.LlgParams(8e5, 1.3e-11, 0.02, 0.0, 1e-13, (ctypes.c_float * 3)(0.0, 0.0, 0.0))
    nb = ctypes.c_size_t()
    # the demagnetizing calls refuse an Oersted plan, before the bind state
    assert lib.demag_field(p, d, None, 1.0, d, 0, None, None) == L.EINVAL
    assert lib.demag_field_2sub(p, d, d, 1.0, 1.0, d, 0, None, None) == L.EINVAL
    assert lib.demag_energy(p, d, None, 1.0, d, d, None) == L.EINVAL
    assert lib.demag_backward(p, d, None, 1.0, None, None, d, 0, None) == L.EINVAL
    assert lib.demag_llg_workspace_bytes(p, ctypes.byref(nb)) == L.EINVAL
    assert lib.demag_llg_rk4(p, d, ctypes.byref(prm), d, None) == L.EINVAL
    # and the Oersted call refuses a demagnetizing plan
    assert lib.demag_oersted_field(q, d, 1.0, d, 0, None) == L.EINVAL
    assert lib.demag_oersted_field(None, d, 1.0, d, 0, None) == L.EINVAL
    assert lib.demag_oersted_field(p, d, 1.0, d, 0, None) == L.ESTATE
    n = ctypes.c_int()
    assert lib.demag_schedule_count(p, ctypes.byref(n)) == L.OK and n.value == 1
    lib.demag_destroy(p)
    lib.demag_destroy(q)


def test_stream_copy_host_checks(lib):
    d = ctypes.c_void_p(256)
    assert lib.demag_stream_copy(None, d, 16, None) == L.EINVAL
    assert lib.demag_stream_copy(d, None, 16, None) == L.EINVAL
    assert lib.demag_stream_copy(d, d, 20, None) == L.EINVAL
    assert lib.demag_stream_copy(ctypes.c_void_p(264), d, 16, None) == L.EINVAL


def test_padded_dims_refuses_batch_plans(lib):
    # a batch whose meshes all belong to one coupled group has no single padded size
    dims = (ctypes.c_int * 6)(8, 8, 1, 8, 8, 1)
    cells = (ctypes.c_double * 6)(1e-9, 1e-9, 1e-9, 1e-9, 1e-9, 1e-9)
    origin = (ctypes.c_double * 6)(0, 0, 0, 0, 0, 2e-9)
    group = (ctypes.c_int * 2)(0, 0)
    p = ctypes.c_void_p()
    assert lib.demag_setup_batch(ctypes.byref(p), 2, dims, cells, origin, group, 0, 0) == L.OK
    try:
        a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        assert lib.demag_padded_dims(p, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)) == L.EINVAL
    finally:
        lib.demag_destroy(p)
    # independent meshes of two geometries: also refused
    dims = (ctypes.c_int * 6)(8, 8, 1, 4, 4, 2)
    assert lib.demag_setup_batch(ctypes.byref(p), 2, dims, cells, None, None, 0, 0) == L.OK
    try:
        assert lib.demag_padded_dims(p, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)) == L.EINVAL
    finally:
        lib.demag_destroy(p)


def test_xpass_classes_skipped_on_the_gpu_are_rejected_for_every_mesh(lib):
    # tests/test_gpu_xpass.py runs one mesh per (log2 Nx, log2 Nz) class the
    # library accepts; a class whose representative is rejected must be
    # rejected for every nx and nz in it (the limits only grow with nx, nz)
    from tests.xpass_classes import representatives, padded

    def ok(nx, ny, nz):
        p = ctypes.c_void_p()
        rc = lib.demag_setup(ctypes.byref(p), nx, ny, nz, 3e-9, 2e-9, 1e-9, 0, 0)
        if rc == L.OK:
            lib.demag_destroy(p)
        return rc == L.OK

    n_acc = 0
    for (a, b), (nx, ny, nz) in representatives():
        assert padded(nx) == 1 << a and padded(nz) == 1 << b
        lo_x = 1 if a == 0 else (2 if a == 2 else (1 << (a - 2)) + 1)
        lo_z = 1 if b == 0 else (2 if b == 2 else (1 << (b - 2)) + 1)
        assert nz == lo_z
        if ok(nx, ny, nz):
            n_acc += 1
            continue
        for x in (lo_x, nx, 1 << max(a - 1, 0)):
            for z in (lo_z, 1 << max(b - 1, 0)):
                if padded(x) == 1 << a and padded(z) == 1 << b:
                    assert not ok(x, ny, z), (a, b, x, z)
    assert n_acc >= 70


def test_noalloc_host_checks(lib):
    p = ctypes.c_void_p()
    dummy = ctypes.c_void_p(256)
    # work space beyond the static scratch: refused before the bind state
    assert lib.demag_setup(ctypes.byref(p), 512, 512, 16, 2e-9, 2e-9, 1e-9, 0, 0) == L.OK
    try:
        kb, wb = ctypes.c_size_t(), ctypes.c_size_t()
        assert lib.demag_buffer_bytes(p, ctypes.byref(kb), ctypes.byref(wb)) == L.OK
        assert wb.value > L.NOALLOC_WORK_BYTES
        assert lib.demag_field_noalloc(p, dummy, None, 1.0, dummy, 0, None, None) == L.EUNSUPPORTED
        assert b"static scratch" in lib.demag_last_error()
    finally:
        lib.demag_destroy(p)
    assert lib.demag_setup(ctypes.byref(p), 64, 48, 3, 5e-9, 5e-9, 3e-9, 0, 0) == L.OK
    try:
        assert lib.demag_field_noalloc(p, dummy, None, 1.0, dummy, 0, None, None) == L.ESTATE
        assert lib.demag_bind(p, None, None, None) == L.EINVAL
    finally:
        lib.demag_destroy(p)
    assert lib.demag_field_noalloc(None, dummy, None, 1.0, dummy, 0, None, None) == L.EINVAL
    dims = (ctypes.c_int * 6)(8, 8, 1, 4, 4, 2)
    cells = (ctypes.c_double * 6)(1e-9, 1e-9, 1e-9, 1e-9, 1e-9, 1e-9)
    assert lib.demag_setup_batch(ctypes.byref(p), 2, dims, cells, None, None, 0, 0) == L.OK
    try:
        assert lib.demag_field_noalloc(p, dummy, None, 1.0, dummy, 0, None, None) == L.EINVAL
        # batch plans always need their work buffer
        assert lib.demag_bind(p, dummy, None, None) == L.EINVAL
    finally:
        lib.demag_destroy(p)


@pytest.mark.parametrize("n,fused,separate", [
    ((4, 4, 1), True, False),        # no z transform at all
    ((512, 512, 16), True, True),
    ((256, 256, 64), True, True),
    ((4, 4, 65), False, True),
    ((300, 4, 33), False, True),
    ((600, 4, 17), False, True),
    ((2048, 4, 16), False, True),    # the 16 rows of a y line exceed LDS
    ((1024, 1024, 32), False, True),
    ((8, 8, 256), False, True),
])
def test_z_pass_forms(lib, n, fused, separate):
    rc, p = setup(lib, *n, 2e-9, 2e-9, 1e-9, 0, 0)
    assert rc == L.OK
    try:
        v = ctypes.c_int()
        assert lib.demag_get_z_passes(p, 0, ctypes.byref(v)) == L.OK
        assert v.value == (0 if fused else 1)        # the fused form wherever it exists
        assert lib.demag_set_z_passes(p, 0, 1) == (L.OK if separate else L.EUNSUPPORTED)
        assert lib.demag_set_z_passes(p, 0, 0) == (L.OK if fused else L.EUNSUPPORTED)
        assert lib.demag_set_z_passes(p, 0, 2) == L.EINVAL
        assert lib.demag_set_z_passes(p, 1, 0) == L.EINVAL
        assert lib.demag_get_z_passes(p, 0, None) == L.EINVAL
        # yg of the schedule follows the form: flattened rows with separate z passes
        if separate:
            assert lib.demag_set_z_passes(p, 0, 1) == L.OK
            yg = ctypes.c_int()
            kw, r = ctypes.c_int(), ctypes.c_int()
            assert lib.demag_get_schedule(p, 0, ctypes.byref(yg), ctypes.byref(kw), ctypes.byref(r)) == L.OK
            assert 1 <= yg.value <= n[1] * n[2]
            assert lib.demag_set_schedule(p, 0, n[1] * n[2] + 1, 0, 0) == L.EINVAL
    finally:
        lib.demag_destroy(p)


def test_z_passes_refused_for_coupled_groups(lib):
    dims = (ctypes.c_int * 6)(8, 8, 1, 8, 8, 1)
    cells = (ctypes.c_double * 6)(1e-9, 1e-9, 1e-9, 1e-9, 1e-9, 1e-9)
    origin = (ctypes.c_double * 6)(0, 0, 0, 0, 0, 2e-9)
    group = (ctypes.c_int * 2)(0, 0)
    p = ctypes.c_void_p()
    assert lib.demag_setup_batch(ctypes.byref(p), 2, dims, cells, origin, group, 0, 0) == L.OK
    try:
        assert lib.demag_set_z_passes(p, 0, 1) == L.EUNSUPPORTED
    finally:
        lib.demag_destroy(p)
