"""ctypes binding of libempso.so (include/empso.h). Argument marshalling only.

Every numerical step runs in the HIP library. PyTorch supplies device memory
(tensor data pointers) and the current HIP stream. If the library has not been
built this module raises ImportError: there is no fallback path.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libempso.so")

EMPSO_OK = 0
STATUS = {0: "EMPSO_OK", -1: "EMPSO_EINVAL", -2: "EMPSO_ECFL", -3: "EMPSO_ERANGE",
          -4: "EMPSO_EWORKSPACE", -5: "EMPSO_EHIP", -6: "EMPSO_ENOTSUP"}


class EmpsoError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class Geometry(ctypes.Structure):
    _fields_ = [("nz", ctypes.c_int32), ("nx", ctypes.c_int32),
                ("dz", ctypes.c_double), ("dx", ctypes.c_double),
                ("nbl", ctypes.c_int32), ("dt", ctypes.c_double), ("nt", ctypes.c_int32),
                ("f0", ctypes.c_double), ("nshots", ctypes.c_int32),
                ("src_zx", ctypes.POINTER(ctypes.c_double)), ("nrec", ctypes.c_int32),
                ("rec_zx", ctypes.POINTER(ctypes.c_double)),
                ("ncz", ctypes.c_int32), ("ncx", ctypes.c_int32),
                ("vmin", ctypes.c_double), ("vmax", ctypes.c_double), ("damp_R", ctypes.c_double),
                ("node_z", ctypes.POINTER(ctypes.c_double)), ("level_nodes", ctypes.POINTER(ctypes.c_int32)),
                ("node_x", ctypes.POINTER(ctypes.c_double)), ("water_rows", ctypes.c_int32),
                ("v_water", ctypes.c_double), ("misfit", ctypes.c_int32)]


# Values of empso_geometry.misfit by the workload key "misfit".
MISFITS = {"l2": 0, "trace_normalised": 1}


class ProblemInfo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in
                ("nz", "nx", "nbl", "nt", "nshots", "nrec", "ncz", "ncx", "Nz", "Nx", "row_stride")] + \
               [("updates_per_run", ctypes.c_int64), ("D", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("bz", ctypes.c_int32),
                ("tsteps", ctypes.c_int32), ("prefetch", ctypes.c_int32), ("use_graph", ctypes.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


# Every exported symbol of include/empso.h with (restype, argtypes).
_vp = ctypes.c_void_p
_P = ctypes.POINTER
SIGNATURES = {
    "empso_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "empso_last_error": (ctypes.c_char_p, []),
    "empso_stable_dt": (ctypes.c_int, [ctypes.c_double, ctypes.c_double, ctypes.c_double, _P(ctypes.c_double)]),
    "empso_problem_create": (ctypes.c_int, [_P(Geometry), _P(_vp)]),
    "empso_problem_destroy": (None, [_vp]),
    "empso_problem_get_info": (ctypes.c_int, [_vp, _P(ProblemInfo)]),
    "empso_vp_from_nodes": (ctypes.c_int, [_vp, ctypes.c_int32, _vp, _vp, _vp]),
    "empso_forward_workspace_bytes": (ctypes.c_size_t, [_vp, ctypes.c_int32]),
    "empso_forward_shots": (ctypes.c_int, [_vp, _vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp,
                                           ctypes.c_size_t, _P(Tuning), _vp]),
    "empso_misfit_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int64]),
    "empso_gradient_workspace_bytes": (ctypes.c_size_t, [_vp, ctypes.c_int32]),
    "empso_gradient": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, ctypes.c_int32, _vp, ctypes.c_size_t, _vp]),
    "empso_misfit": (ctypes.c_int, [_vp, _vp, ctypes.c_int64, _vp, _vp, ctypes.c_size_t, _vp]),
    "empso_traces_misfit_workspace_bytes": (ctypes.c_size_t, [_vp, ctypes.c_int32]),
    "empso_traces_misfit": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int32, _vp, _vp, ctypes.c_size_t, _vp]),
    "empso_traces_misfit_noalloc": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int32, _vp, _vp]),
    "empso_fitness_workspace_bytes": (ctypes.c_size_t, [_P(_vp), ctypes.c_int32, _P(ctypes.c_int32),
                                                        ctypes.c_int32]),
    "empso_fitness_batch": (ctypes.c_int, [_P(_vp), ctypes.c_int32, _P(_vp), _P(ctypes.c_int32),
                                           ctypes.c_int32, _P(ctypes.c_double), ctypes.c_int32, _vp,
                                           _vp, ctypes.c_size_t, _P(Tuning), _vp]),
    "empso_fitness_batch_steps": (ctypes.c_int, [_P(_vp), ctypes.c_int32, _P(_vp), _P(ctypes.c_int32),
                                                 ctypes.c_int32, _P(ctypes.c_double), ctypes.c_int32, _vp,
                                                 ctypes.c_int32, ctypes.c_int32, _vp, ctypes.c_size_t, _P(Tuning),
                                                 _vp]),
    "empso_default_tuning": (ctypes.c_int, [_P(Tuning)]),
    "empso_mlp_param_count": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32]),
    "empso_mlp_bf16_count": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32]),
    "empso_mlp_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "empso_mlp_sync_bf16": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp]),
    "empso_mlp_predict": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp,
                                         ctypes.c_int32, _vp, _vp, ctypes.c_size_t, _vp]),
    "empso_mlp_grad": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                      ctypes.c_int32, ctypes.c_float, ctypes.c_float, _vp, _vp, _vp,
                                      ctypes.c_size_t, _vp]),
    "empso_mlp_train_step": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp, _vp, ctypes.c_int32,
                                            ctypes.c_float, _vp, _vp, _vp, _vp, _vp, ctypes.c_int32,
                                            ctypes.c_float, ctypes.c_float, _vp, _vp, ctypes.c_size_t, _vp]),
    "empso_autotune_fitness": (ctypes.c_int, [_P(_vp), ctypes.c_int32, _P(_vp), _P(ctypes.c_int32),
                                              ctypes.c_int32, _P(ctypes.c_double), ctypes.c_int32, _vp,
                                              ctypes.c_size_t, _P(Tuning), _P(ctypes.c_float), _vp]),
    "empso_time_tuning": (ctypes.c_int, [_P(_vp), ctypes.c_int32, _P(_vp), _P(ctypes.c_int32),
                                         ctypes.c_int32, _P(ctypes.c_double), ctypes.c_int32, _vp,
                                         ctypes.c_size_t, _P(Tuning), ctypes.c_int32, _P(ctypes.c_float), _vp]),
}


def load(path=LIB_PATH):
    if not os.path.exists(path):
        raise ImportError("libempso.so is not built (%s); run __graft_entry__.build()" % path)
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = load()


def check(status):
    if status != EMPSO_OK:
        raise EmpsoError(status, lib.empso_last_error().decode(errors="replace"))
    return status
