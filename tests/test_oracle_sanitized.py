"""The oracle's C time loops built with AddressSanitizer and
UndefinedBehaviorSanitizer (host code only) run the brute-force,
reciprocity, causality and adjoint pins without a report: no out-of-bounds
access, use after free or undefined arithmetic in the code the parity tests
trust. The sanitized library runs in a child Python process with the ASan
runtime preloaded."""
import os
import subprocess
import sys

import pytest

from oracle import build as obuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r'''
import ctypes, sys
sys.path.insert(0, sys.argv[1])
from oracle import fd
real = fd._load()
lib = ctypes.CDLL(sys.argv[2])
for fn in ("oracle_forward_run", "oracle_gradient_run"):
    getattr(lib, fn).restype = ctypes.c_int
    getattr(lib, fn).argtypes = getattr(real, fn).argtypes
fd._lib = lib
from tests import test_oracle_forward as F, test_oracle_gradient as G
F.test_brute_force_dense_matrices()
F.test_reciprocity_heterogeneous_with_damping()
F.test_causality_exact_zeros()
g, op = G._problem()
vp, truth = G._models(op)
dobs = fd.forward_shots(op, truth)
J, grad = fd.gradient(op, vp, dobs)
setup = (op, vp, dobs, J, grad)
G.test_misfit_matches_forward(setup)
G.test_directional_derivative_matches_central_differences(setup, 0)
G.test_pointwise_derivative_matches_central_differences(setup, (0, 0))
G.test_zero_residual_gives_zero_gradient(setup)
print("SANITIZED_PINS_OK", flush=True)
'''


def _asan_runtime():
    out = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


@pytest.mark.timeout(600)
def test_oracle_pins_pass_under_asan_and_ubsan(tmp_path):
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("no ASan runtime for gcc on this host")
    so = tmp_path / "liboracle_fd_asan.so"
    subprocess.check_call(["gcc", "-O1", "-g", "-fPIC", "-shared", "-std=c99", "-fno-fast-math", "-ffp-contract=off",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                           "-o", str(so), obuild.SRC])
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT, str(so)], env=env, capture_output=True, text=True,
                       timeout=560)
    assert r.returncode == 0 and "SANITIZED_PINS_OK" in r.stdout, (r.returncode, r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
