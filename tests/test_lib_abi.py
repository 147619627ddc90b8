"""The C ABI library loads without a GPU, exports every declared symbol, and
rejects invalid requests on the host before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "empso.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(empso_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_1905_12795_amd import _lib
    return _lib


def test_every_declared_symbol_is_exported_and_bound(L):
    names = _declared()
    assert len(names) >= 14
    raw = ctypes.CDLL(L.LIB_PATH)
    for n in names:
        assert hasattr(raw, n), n
        assert n in L.SIGNATURES, n


def test_status_strings(L):
    for code, name in L.STATUS.items():
        assert L.lib.empso_status_string(code).decode() == name


def test_stable_dt_host(L):
    out = ctypes.c_double()
    assert L.lib.empso_stable_dt(6000.0, 10.0, 10.0, ctypes.byref(out)) == 0
    assert out.value == pytest.approx(2.0 / (6000.0 * np.sqrt(2048 / 315 * 0.02)), rel=1e-14)
    assert L.lib.empso_stable_dt(-1.0, 10.0, 10.0, ctypes.byref(out)) == -1
    assert L.lib.empso_stable_dt(1.0, 10.0, 10.0, None) == -1


def _geom(L, **kw):
    src = np.array([[0.0, 500.0]])
    rec = np.array([[0.0, 10.0 * j] for j in range(101)])
    g = L.Geometry()
    g.nz = g.nx = 101
    g.dz = g.dx = 10.0
    g.nbl = 40
    g.dt = 0.4 * 0.554632 * 10 / 2700
    g.nt = 100
    g.f0 = 10.0
    g.nshots, g.nrec = 1, 101
    g.ncz, g.ncx = 2, 3
    g.vmin, g.vmax, g.damp_R = 1400.0, 2700.0, 1e-3
    for k, v in kw.items():
        if k == "src":
            src = np.asarray(v, dtype=np.float64)
        elif k == "rec":
            rec = np.asarray(v, dtype=np.float64)
        elif k == "levels":                               # (node_z, level_nodes, node_x)
            z, n, x = (np.asarray(v[0], np.float64), np.asarray(v[1], np.int32), np.asarray(v[2], np.float64))
            g._lv = (z, n, x)
            g.ncz = len(z)
            g.node_z = z.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            g.level_nodes = n.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            g.node_x = x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        else:
            setattr(g, k, v)
    g.nshots, g.nrec = len(src), len(rec)
    g._keep = (src, rec)
    g.src_zx = src.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    g.rec_zx = rec.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return g


@pytest.mark.parametrize("kw,status", [
    (dict(dt=1.01 * 0.554632 * 10 / 2700), -2),           # above the stability limit
    (dict(nz=1), -1),
    (dict(ncz=1), -1),
    (dict(vmin=3000.0), -1),                              # vmin > vmax
    (dict(damp_R=1.5), -1),
    (dict(rec=[[0.0, 15.0]]), -6),                        # receiver off the grid
    (dict(rec=[[0.0, 10.0], [10.0, 20.0]]), -6),          # receivers on two rows
    (dict(rec=[[0.0, 10.0], [0.0, 10.0]]), -6),           # two receivers on one point
    (dict(src=[[0.0, 2000.0]]), -6),                      # source outside the grid
    (dict(levels=([100.0, 50.0], [2, 2], [0, 500, 0, 500])), -1),          # levels not increasing
    (dict(levels=([0.0, 500.0], [2, 1], [0, 500, 0])), -1),                # a level with one node
    (dict(levels=([0.0, 500.0], [2, 2], [0, 500, 500, 0])), -1),          # x not increasing in a level
    (dict(levels=([0.0, 500.0], [2, 2], [0, np.nan, 0, 500])), -1),       # non-finite position
    (dict(water_rows=101), -1),                                             # water_rows >= nz
    (dict(water_rows=-1), -1),
    (dict(water_rows=4, v_water=1000.0), -1),                               # water velocity below vmin
    (dict(misfit=2), -1),                                                   # unknown misfit
    (dict(misfit=-1), -1),
])
def test_problem_create_rejects_on_host(L, kw, status):
    g = _geom(L, **kw)
    h = ctypes.c_void_p(123)
    assert L.lib.empso_problem_create(ctypes.byref(g), ctypes.byref(h)) == status
    assert h.value is None
    assert len(L.lib.empso_last_error()) > 0


def test_null_arguments(L):
    assert L.lib.empso_problem_create(None, None) == -1
    assert L.lib.empso_fitness_batch(None, 1, None, None, 1, None, 1, None, None, 0, None, None) == -1
    assert L.lib.empso_misfit(None, None, 10, None, None, 0, None) == -1
    assert L.lib.empso_fitness_workspace_bytes(None, 1, None, 1) == 0
    t = L.Tuning()
    assert L.lib.empso_default_tuning(ctypes.byref(t)) == 0
    assert t.tsteps >= 1 and t.bz > 0


def test_grid_above_the_32_bit_field_limit_is_rejected(L):
    # 16352 stored rows (ring included) of 8192 floats fill 2^29 bytes: four
    # such fields no longer fit 32-bit byte offsets below 2^31
    g = _geom(L, nz=16352, nx=8160, nbl=0)
    h = ctypes.c_void_p(123)
    assert L.lib.empso_problem_create(ctypes.byref(g), ctypes.byref(h)) == -6
    assert h.value is None
    assert b"512 MiB" in L.lib.empso_last_error()
    # one row less passes the size check (it then needs a device for its tables)
    g = _geom(L, nz=16351, nx=8160, nbl=0)
    rc = L.lib.empso_problem_create(ctypes.byref(g), ctypes.byref(h))
    assert rc != -6, L.lib.empso_last_error()
    if rc == 0:
        L.lib.empso_problem_destroy(h)


def test_fitness_steps_null_and_empty(L):
    args = (None, 1, None, None, 1, None, 1, None, 0, 10, None, 0, None, None)
    assert L.lib.empso_fitness_batch_steps(*args) == -1
    assert L.lib.empso_fitness_batch_steps(None, 0, None, None, 0, None, 0, None, 0, 0, None, 0, None, None) == 0


def test_empty_batch_is_a_no_op(L):
    # np = 0: nothing to evaluate, nothing enqueued and no device call made
    assert L.lib.empso_fitness_batch(None, 0, None, None, 0, None, 0, None, None, 0, None, None) == 0
    assert L.lib.empso_fitness_batch(None, 1, None, None, -1, None, 1, None, None, 0, None, None) == -1
    assert L.lib.empso_fitness_workspace_bytes(None, 1, None, 0) == 0
    assert L.lib.empso_forward_shots(None, None, 0, 0, None, None, 0, None, None) == -1      # no problem


def test_gradient_null_arguments(L):
    assert L.lib.empso_gradient_workspace_bytes(None, 0) == 0
    assert L.lib.empso_gradient(None, None, None, None, None, None, 0, None, 0, None) == -1


def test_traces_misfit_null_arguments(L):
    assert L.lib.empso_traces_misfit_workspace_bytes(None, 1) == 0
    assert L.lib.empso_traces_misfit(None, None, None, 0, None, None, 0, None) == -1


def test_geometry_struct_matches_the_header(L):
    """The binding's struct ends with the misfit selector, after v_water."""
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "empso.h")).read()
    body = hdr[hdr.index("typedef struct {\n    int32_t nz, nx;"):hdr.index("} empso_geometry;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = re.findall(r"(\w+)\s*[,;]", body)
    assert names == [f for f, _ in L.Geometry._fields_]
    assert (L.MISFITS["l2"], L.MISFITS["trace_normalised"]) == (0, 1)
    assert "#define EMPSO_MISFIT_L2 0" in hdr and "#define EMPSO_MISFIT_TRACE_NORMALISED 1" in hdr


def test_mlp_shape_limits_on_the_host(L):
    """The network's shape bounds (1 <= D, H <= 4096, 1 <= n <= 2^22) are checked
    before anything reaches the device: sizes outside them have no workspace,
    and the calls refuse them with EINVAL."""
    ok = L.lib.empso_mlp_workspace_bytes(60, 256, 1 << 22)
    assert ok > 0 and ok % 256 == 0
    assert L.lib.empso_mlp_workspace_bytes(60, 256, 1) > 0
    for D, H, n in ((60, 256, (1 << 22) + 1), (60, 256, 0), (0, 256, 8), (4097, 256, 8), (60, 4097, 8), (60, 0, 8)):
        assert L.lib.empso_mlp_workspace_bytes(D, H, n) == 0, (D, H, n)
    p = ctypes.c_void_p(256)                        # never dereferenced: the shape check comes first
    assert L.lib.empso_mlp_predict(60, 256, p, p, p, p, p, (1 << 22) + 1, p, p, 1 << 40, None) == -1
    assert b"bad shape" in L.lib.empso_last_error()
    assert L.lib.empso_mlp_param_count(60, 256) == 256 * 60 + 256 + 2 * (256 * 256 + 256) + 256 + 1
