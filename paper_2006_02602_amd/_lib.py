"""ctypes declarations of libcavity.so (include/cavity.h).

Loading fails loudly when the library has not been built: there is no
fallback implementation of any call.
"""
import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
# CAVITY_LIB selects another build of the same library (e.g. for A/B timing)
LIB_PATH = os.environ.get("CAVITY_LIB") or os.path.join(PKG, "libcavity.so")

CAV_OK = 0
CAV_EINVAL = -1
CAV_ESIZE = -2
CAV_EHIP = -3
CAV_ENONFINITE = -4
CAV_ENOSYS = -5
CAV_F64 = 0
CAV_F32 = 1
CAV_NOALLOC_MAX_SWEEP_BLOCKS = 32768

ERROR_NAMES = {CAV_EINVAL: "CAV_EINVAL", CAV_ESIZE: "CAV_ESIZE", CAV_EHIP: "CAV_EHIP",
               CAV_ENONFINITE: "CAV_ENONFINITE", CAV_ENOSYS: "CAV_ENOSYS"}

# every function include/cavity.h declares
EXPORTS = ("cavity_layout", "cavity_state_elems", "cavity_workspace_bytes", "halo_buffer_bytes", "cavity_init",
           "cavity_step", "cavity_step_from", "cavity_step_noalloc", "cavity_step_overlap", "halo_pack", "halo_unpack", "cavity_residual_norm", "cavity_nusselt",
           "cavity_adjoint_workspace_bytes", "cavity_nusselt_adjoint", "cavity_adjoint_step",
           "cavity_batch_table_bytes", "cavity_batch_build", "cavity_batch_step", "cavity_batch_graph_create",
           "cavity_batch_graph_launch", "cavity_batch_graph_destroy",
           "cavity_stream_copy", "cavity_selftest_math", "cavity_last_error", "cavity_timing_enable", "cavity_timing_read")


class CavGrid(ctypes.Structure):
    _fields_ = [("ni", ctypes.c_int32), ("nj", ctypes.c_int32), ("nk", ctypes.c_int32),
                ("ng", ctypes.c_int32), ("dtype", ctypes.c_int32)]


class CavParams(ctypes.Structure):
    _fields_ = [("Ra", ctypes.c_double), ("Pr", ctypes.c_double), ("cfl", ctypes.c_double),
                ("eps4", ctypes.c_double), ("kappa", ctypes.c_double), ("u_ref", ctypes.c_double),
                ("t_hot", ctypes.c_double), ("t_cold", ctypes.c_double), ("t_inf", ctypes.c_double),
                ("t_hot_field", ctypes.c_void_p)]


class CavHalo(ctypes.Structure):
    _fields_ = [("split", ctypes.c_int32 * 3), ("width", ctypes.c_int32 * 5)]


class CavLayout(ctypes.Structure):
    _fields_ = [("lead", ctypes.c_int64), ("sj", ctypes.c_int64), ("sk", ctypes.c_int64),
                ("sf", ctypes.c_int64), ("origin", ctypes.c_int64)]


class CavBatchMember(ctypes.Structure):
    _fields_ = [("grid", CavGrid), ("params", CavParams), ("q", ctypes.c_void_p), ("q_tmp", ctypes.c_void_p),
                ("ws", ctypes.c_void_p), ("ws_bytes", ctypes.c_size_t), ("kc", ctypes.c_int32),
                ("ti", ctypes.c_int32)]


class CavBatch(ctypes.Structure):
    _fields_ = [("table", ctypes.c_void_p), ("members", ctypes.c_int32), ("items", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("parity", ctypes.c_int32), ("cells", ctypes.c_uint64),
                ("shapes", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class CavKernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double)]


class CavError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (ERROR_NAMES.get(code, "?"), code, msg))
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libcavity.so is not built (%s); run __graft_entry__.build() or "
                          "python paper_2006_02602_amd/build.py" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    vp, sz, i32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32
    G, Pp, H = ctypes.POINTER(CavGrid), ctypes.POINTER(CavParams), ctypes.POINTER(CavHalo)
    dp = ctypes.POINTER(ctypes.c_double)
    L.cavity_layout.restype = ctypes.c_int
    L.cavity_layout.argtypes = [G, ctypes.POINTER(CavLayout)]
    L.cavity_state_elems.restype = sz
    L.cavity_state_elems.argtypes = [G]
    L.cavity_workspace_bytes.restype = sz
    L.cavity_workspace_bytes.argtypes = [G]
    L.halo_buffer_bytes.restype = sz
    L.halo_buffer_bytes.argtypes = [G, H]
    L.cavity_init.restype = ctypes.c_int
    L.cavity_init.argtypes = [G, Pp, ctypes.c_uint64, ctypes.c_double, vp, vp]
    L.cavity_step.restype = ctypes.c_int
    L.cavity_step.argtypes = [G, Pp, H, vp, vp, vp, sz, vp, sz, i32, vp]
    L.cavity_step_from.restype = ctypes.c_int
    L.cavity_step_from.argtypes = [G, Pp, vp, vp, vp, sz, vp]
    L.cavity_step_noalloc.restype = ctypes.c_int
    L.cavity_step_noalloc.argtypes = [G, Pp, H, vp, vp, vp, sz, vp, i32, vp]
    L.cavity_step_overlap.restype = ctypes.c_int
    L.cavity_step_overlap.argtypes = [G, Pp, H, vp, vp, vp, sz, vp, sz, i32, vp, vp]
    L.halo_pack.restype = ctypes.c_int
    L.halo_pack.argtypes = [G, H, vp, vp, sz, vp]
    L.halo_unpack.restype = ctypes.c_int
    L.halo_unpack.argtypes = [G, H, vp, sz, vp, vp]
    L.cavity_residual_norm.restype = ctypes.c_int
    L.cavity_residual_norm.argtypes = [G, vp, sz, dp, vp]
    L.cavity_nusselt.restype = ctypes.c_int
    L.cavity_nusselt.argtypes = [G, Pp, vp, vp, sz, dp, vp]
    L.cavity_adjoint_workspace_bytes.restype = sz
    L.cavity_adjoint_workspace_bytes.argtypes = [G]
    L.cavity_nusselt_adjoint.restype = ctypes.c_int
    L.cavity_nusselt_adjoint.argtypes = [G, Pp, vp, vp, vp]
    L.cavity_adjoint_step.restype = ctypes.c_int
    L.cavity_adjoint_step.argtypes = [G, Pp, vp, vp, vp, vp, sz, vp, vp, vp]
    BM, BP = ctypes.POINTER(CavBatchMember), ctypes.POINTER(CavBatch)
    L.cavity_batch_table_bytes.restype = sz
    L.cavity_batch_table_bytes.argtypes = [i32, BM]
    L.cavity_batch_build.restype = ctypes.c_int
    L.cavity_batch_build.argtypes = [i32, BM, vp, sz, BP, vp]
    L.cavity_batch_step.restype = ctypes.c_int
    L.cavity_batch_step.argtypes = [BP, i32, i32, vp]
    L.cavity_batch_graph_create.restype = ctypes.c_int
    L.cavity_batch_graph_create.argtypes = [BP, i32, i32, vp, ctypes.POINTER(ctypes.c_void_p)]
    L.cavity_batch_graph_launch.restype = ctypes.c_int
    L.cavity_batch_graph_launch.argtypes = [BP, vp, vp]
    L.cavity_batch_graph_destroy.restype = ctypes.c_int
    L.cavity_batch_graph_destroy.argtypes = [vp]
    L.cavity_stream_copy.restype = ctypes.c_int
    L.cavity_stream_copy.argtypes = [G, vp, vp, vp]
    L.cavity_selftest_math.restype = ctypes.c_int
    L.cavity_selftest_math.argtypes = [vp, vp, i32, vp]
    L.cavity_last_error.restype = ctypes.c_char_p
    L.cavity_last_error.argtypes = []
    L.cavity_timing_enable.restype = ctypes.c_int
    L.cavity_timing_enable.argtypes = [i32]
    L.cavity_timing_read.restype = ctypes.c_int
    L.cavity_timing_read.argtypes = [ctypes.POINTER(CavKernelTime), i32, ctypes.POINTER(i32)]
    _lib = L
    return L


def check(rc):
    if rc != CAV_OK:
        raise CavError(rc, lib().cavity_last_error().decode(errors="replace"))
    return rc
