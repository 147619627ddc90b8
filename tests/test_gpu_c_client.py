"""The library from a C program without PyTorch (run on an MI355X).

The boundary is a C ABI over plain device pointers: a C99 client that
allocates with the HIP runtime's C API, builds the tiny workload's problem,
interpolates a true model from its nodes, models its shot
(empso_forward_shots) and scores four particles against those traces
(empso_fitness_batch, library-default tuning, default stream), gets the
fitness values that the Python binding gets for the same inputs bit for bit;
the true particle's fitness is exactly zero (the same kernels made its data).
"""
import json
import os
import shutil
import subprocess

import numpy as np
import pytest
import torch

from workloads.configs import config

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1905_12795_amd")
X = [[1500.0, 1500.0, 1500.0, 2500.0, 2500.0, 2500.0],
     [1600.0, 1700.0, 1800.0, 2300.0, 2400.0, 2600.0],
     [1450.0, 2000.0, 1450.0, 2650.0, 1900.0, 2650.0],
     [2000.0, 2000.0, 2000.0, 2000.0, 2000.0, 2000.0]]

CLIENT = r"""
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <hip/hip_runtime_api.h>
#include "empso.h"

#define CHECK(x) do { int rc_ = (x); if (rc_) { fprintf(stderr, "%s: %d %s\n", #x, rc_, empso_last_error()); return 1; } } while (0)
#define HCHECK(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) { fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_)); return 1; } } while (0)

int main(int argc, char **argv) {
    if (argc != 3) return 2;
    const double dt = strtod(argv[1], NULL);
    const int nt = atoi(argv[2]);
    double src[2] = {0.0, 500.0}, rec[2 * 101];
    for (int j = 0; j < 101; ++j) { rec[2 * j] = 0.0; rec[2 * j + 1] = 10.0 * j; }
    empso_geometry g;
    memset(&g, 0, sizeof g);
    g.nz = 101; g.nx = 101; g.dz = 10.0; g.dx = 10.0; g.nbl = 40; g.dt = dt; g.nt = nt; g.f0 = 10.0;
    g.nshots = 1; g.src_zx = src; g.nrec = 101; g.rec_zx = rec; g.ncz = 2; g.ncx = 3;
    g.vmin = 1400.0; g.vmax = 2700.0; g.damp_R = 1e-3; g.misfit = EMPSO_MISFIT_L2;
    empso_problem *p = NULL;
    CHECK(empso_problem_create(&g, &p));

    const float truth[6] = {1500.f, 1500.f, 1500.f, 2500.f, 2500.f, 2500.f};
    float *nodes_d = NULL, *vp_d = NULL, *tr_d = NULL, *fit_d = NULL;
    void *ws = NULL, *ws2 = NULL;
    HCHECK(hipMalloc((void **)&nodes_d, sizeof truth));
    HCHECK(hipMemcpy(nodes_d, truth, sizeof truth, hipMemcpyHostToDevice));
    HCHECK(hipMalloc((void **)&vp_d, sizeof(float) * 101 * 101));
    CHECK(empso_vp_from_nodes(p, 1, nodes_d, vp_d, NULL));
    const size_t wb = empso_forward_workspace_bytes(p, 1);
    HCHECK(hipMalloc(&ws, wb));
    HCHECK(hipMalloc((void **)&tr_d, sizeof(float) * (size_t)nt * 101));
    CHECK(empso_forward_shots(p, vp_d, 0, 1, tr_d, ws, wb, NULL, NULL));

    const double X[4][6] = {%X%};
    const int32_t pop[4] = {0, 0, 0, 0};
    const empso_problem *probs[1] = {p};
    const float *obs[1] = {tr_d};
    const size_t wb2 = empso_fitness_workspace_bytes(probs, 1, pop, 4);
    HCHECK(hipMalloc(&ws2, wb2));
    HCHECK(hipMalloc((void **)&fit_d, 4 * sizeof(float)));
    CHECK(empso_fitness_batch(probs, 1, obs, pop, 4, &X[0][0], 6, fit_d, ws2, wb2, NULL, NULL));
    float fit[4];
    HCHECK(hipMemcpy(fit, fit_d, sizeof fit, hipMemcpyDeviceToHost));
    float *tr = (float *)malloc(sizeof(float) * (size_t)nt * 101);
    HCHECK(hipMemcpy(tr, tr_d, sizeof(float) * (size_t)nt * 101, hipMemcpyDeviceToHost));
    double energy = 0.0;
    for (size_t k = 0; k < (size_t)nt * 101; ++k) energy += (double)tr[k] * tr[k];
    printf("{\"fitness_bits\": [");
    for (int k = 0; k < 4; ++k) {
        uint32_t b;
        memcpy(&b, &fit[k], 4);
        printf("%s%u", k ? ", " : "", (unsigned)b);
    }
    printf("], \"trace_energy\": %.17g}\n", energy);
    free(tr);
    HCHECK(hipFree(fit_d)); HCHECK(hipFree(ws2)); HCHECK(hipFree(tr_d)); HCHECK(hipFree(ws));
    HCHECK(hipFree(vp_d)); HCHECK(hipFree(nodes_d));
    empso_problem_destroy(p);
    return 0;
}
"""


def test_c_client_equals_the_python_binding(tmp_path):
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    from paper_1905_12795_amd import fd
    g = config("tiny")
    gp = fd.Problem(g)
    src = tmp_path / "client.c"
    exe = tmp_path / "client"
    src.write_text(CLIENT.replace("%X%", ", ".join("{%s}" % ", ".join(repr(v) for v in row) for row in X)))
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
                           "-I", "/opt/rocm/include", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe),
                           "-L", PKG, "-l:libempso.so", "-Wl,-rpath," + PKG,
                           "-L", "/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"])
    r = subprocess.run([str(exe), repr(gp.dt), str(gp.nt)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    c = json.loads(r.stdout)

    truth = torch.tensor([X[0]], dtype=torch.float32, device="cuda")
    vp = fd.vp_from_nodes(gp, truth)[0].contiguous()
    tr = fd.forward_shots(gp, vp)
    f = fd.FitnessBatch([gp], [tr], [0] * 4)(np.array(X)).cpu().numpy()
    energy = float(np.sum(tr.cpu().numpy().astype(np.float64) ** 2))
    print("C client fitness", np.array(c["fitness_bits"], np.uint32).view(np.float32), "binding", f, flush=True)
    assert np.array_equal(np.array(c["fitness_bits"], np.uint32), f.view(np.uint32))
    assert f[0] == 0.0 and np.all(f[1:] > 0)
    assert c["trace_energy"] == pytest.approx(energy, rel=1e-12) and energy > 0
