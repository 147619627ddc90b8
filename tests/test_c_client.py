"""The C ABI from a C program: include/empso.h compiles as strict C99, a
client links against libempso.so, the struct layouts seen by C match the
Python binding's field by field, and host-only entry points behave as the
header states (no GPU needed)."""
import ctypes
import json
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1905_12795_amd")

STRUCTS = {
    "empso_geometry": ["nz", "nx", "dz", "dx", "nbl", "dt", "nt", "f0", "nshots", "src_zx", "nrec", "rec_zx",
                       "ncz", "ncx", "vmin", "vmax", "damp_R", "node_z", "level_nodes", "node_x", "water_rows",
                       "v_water", "misfit"],
    "empso_problem_info": ["nz", "nx", "nbl", "nt", "nshots", "nrec", "ncz", "ncx", "Nz", "Nx", "row_stride",
                           "updates_per_run", "D"],
    "empso_tuning": ["variant", "bz", "tsteps", "prefetch", "use_graph"],
}


def _client_source():
    lines = ["#include <stdio.h>", "#include <stddef.h>", "#include <string.h>", '#include "empso.h"', "",
             "int main(void) {", '    printf("{");']
    for st, fields in STRUCTS.items():
        lines.append('    printf("\\"%s\\": {\\"size\\": %%zu", sizeof(%s));' % (st, st))
        for f in fields:
            lines.append('    printf(", \\"%s\\": %%zu", offsetof(%s, %s));' % (f, st, f))
        lines.append('    printf("}, ");')
    lines += [
        "    double dt = 0.0;",
        "    int rc = empso_stable_dt(6000.0, 10.0, 10.0, &dt);",
        '    printf("\\"stable_dt\\": [%d, %.17g], ", rc, dt);',
        "    double src[2] = {0.0, 500.0}, rec[4] = {0.0, 0.0, 0.0, 10.0};",
        "    empso_geometry g;",
        "    memset(&g, 0, sizeof g);",
        "    g.nz = 101; g.nx = 101; g.dz = 10.0; g.dx = 10.0; g.nbl = 40; g.nt = 100; g.f0 = 10.0;",
        "    g.nshots = 1; g.src_zx = src; g.nrec = 2; g.rec_zx = rec; g.ncz = 2; g.ncx = 3;",
        "    g.vmin = 1400.0; g.vmax = 2700.0; g.damp_R = 1e-3; g.misfit = EMPSO_MISFIT_L2;",
        "    g.dt = 1.01 * 0.554632 * 10.0 / 2700.0;            /* above the stability limit */",
        "    empso_problem *p = (empso_problem *)&g;             /* must be overwritten with NULL */",
        "    rc = empso_problem_create(&g, &p);",
        '    printf("\\"create_cfl\\": [%d, %d, \\"%s\\"], ", rc, p == NULL, empso_status_string(rc));',
        '    printf("\\"create_null\\": %d, ", empso_problem_create(NULL, &p));',
        '    printf("\\"mlp\\": [%zu, %zu, %zu], ", empso_mlp_param_count(60, 256), empso_mlp_bf16_count(60, 256),',
        "           empso_mlp_workspace_bytes(60, 256, 0));",
        '    printf("\\"ok\\": \\"%s\\"}\\n", empso_status_string(EMPSO_OK));',
        "    return 0;",
        "}",
    ]
    return "\n".join(lines) + "\n"


@pytest.fixture(scope="module")
def client(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    lib = os.path.join(PKG, "libempso.so")
    assert os.path.exists(lib), "build the library first (__graft_entry__.build())"
    d = tmp_path_factory.mktemp("c_client")
    src, exe = d / "client.c", d / "client"
    src.write_text(_client_source())
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic", "-I",
                           os.path.join(ROOT, "include"), str(src), "-o", str(exe), "-L", PKG, "-l:libempso.so",
                           "-Wl,-rpath," + PKG])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120, check=True).stdout
    return json.loads(out)


def test_struct_layouts_match_the_binding(client):
    from paper_1905_12795_amd import _lib as L
    for st, cls in (("empso_geometry", L.Geometry), ("empso_problem_info", L.ProblemInfo),
                    ("empso_tuning", L.Tuning)):
        c = client[st]
        assert c["size"] == ctypes.sizeof(cls), st
        assert [f for f, _ in cls._fields_] == STRUCTS[st], st
        for f, _ in cls._fields_:
            assert c[f] == getattr(cls, f).offset, (st, f)


def test_host_entry_points_from_c(client):
    rc, dt = client["stable_dt"]
    assert rc == 0 and dt == pytest.approx(2.0 / (6000.0 * (2048 / 315 * 0.02) ** 0.5), rel=1e-14)
    rc, nulled, name = client["create_cfl"]
    assert (rc, nulled, name) == (-2, 1, "EMPSO_ECFL")
    assert client["create_null"] == -1
    P, PB, ws0 = client["mlp"]
    assert P == 256 * 60 + 256 + 2 * (256 * 256 + 256) + 256 + 1
    assert PB == 256 * 60 + 2 * 256 * 256 and ws0 == 0
    assert client["ok"] == "EMPSO_OK"
