"""ctypes declarations of the C ABI in include/vbd.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libvbd.so")

VBD_OK = 0
STATUS_NAMES = {0: "VBD_OK", -1: "VBD_E_INVALID_ARG", -2: "VBD_E_TOPOLOGY", -3: "VBD_E_NOT_COLORED",
                -4: "VBD_E_NO_WORKSPACE", -5: "VBD_E_HIP", -6: "VBD_E_UNSUPPORTED",
                -7: "VBD_E_NONFINITE", -8: "VBD_E_DEVICE"}

LAUNCH_PLAIN, LAUNCH_GRAPH, LAUNCH_PERSISTENT, LAUNCH_PERSISTENT_GRAPH = 0, 1, 2, 3
COLOR_ID_ORDER, COLOR_SMALLEST_LAST, COLOR_DSATUR = 0, 1, 2

(Q_COUNTS, Q_COLORS, Q_PERM, Q_COLOR_OFFSETS, Q_TET_ROWS, Q_TET_ENTRIES, Q_SPRING_ROWS,
 Q_SPRING_NBRS, Q_MASS, Q_DMINV, Q_VOLUME, Q_PHASE_BYTES, Q_TET_ORDER, Q_REST_FRAME, Q_SURFACE,
 Q_SURFACE_COUNTS, Q_SNAPSHOT_REGION, Q_ADJ_PHASE_BYTES, Q_PHASE_COUNTS, Q_SURFACE_EDGES,
 Q_XCD_SPLIT) = range(21)

# every symbol include/vbd.h declares
EXPORTS = ["vbd_build_topology", "vbd_color", "vbd_color_greedy", "vbd_color_given", "vbd_workspace_size", "vbd_bind_workspace",
           "vbd_topology_query", "vbd_topology_destroy", "vbd_step", "vbd_step_static", "vbd_step_record", "vbd_step_backward",
           "vbd_get_launch_config", "vbd_set_launch_config", "vbd_autotune",
           "vbd_profile_enable", "vbd_profile_read", "vbd_check", "vbd_probe_copy", "vbd_probe_read",
           "vbd_detect_contacts", "vbd_detect_edges", "vbd_read_counters", "vbd_last_error"]


class MeshDesc(C.Structure):
    _fields_ = [("n_verts", C.c_int32), ("n_tets", C.c_int32), ("n_springs", C.c_int32),
                ("n_meshes", C.c_int32), ("vert_offsets", C.c_void_p), ("tet_offsets", C.c_void_p),
                ("tets", C.c_void_p), ("springs", C.c_void_p), ("rest_pos", C.c_void_p),
                ("spring_rest", C.c_void_p), ("spring_k", C.c_double), ("mass", C.c_void_p),
                ("density", C.c_double), ("poisson_nu", C.c_double), ("pinned", C.c_void_p)]


class StepParamsC(C.Structure):
    _fields_ = [("h", C.c_float), ("n_iters", C.c_int32), ("gravity", C.c_float * 3),
                ("init_mode", C.c_int32), ("det_eps_rel", C.c_float), ("contact_k", C.c_float),
                ("contact_thickness", C.c_float), ("n_spheres", C.c_int32), ("spheres", C.c_void_p),
                ("n_planes", C.c_int32), ("planes", C.c_void_p), ("kd", C.c_float),
                ("cheb_rho", C.c_float), ("friction_mu", C.c_float), ("friction_eps_v", C.c_float),
                ("spring_psd", C.c_int32), ("launch_mode", C.c_int32),
                ("mesh_contacts", C.c_int32), ("collision_radius", C.c_float), ("n_col", C.c_int32),
                ("backward_recorded", C.c_int32), ("check_finite", C.c_int32),
                ("self_contact", C.c_int32), ("self_exclusion", C.c_float),
                ("edge_contacts", C.c_int32)]


class LaunchConfig(C.Structure):
    _fields_ = [("lanes_per_vertex", C.c_int32), ("block_size", C.c_int32),
                ("xcd_remap", C.c_int32), ("blocks_per_cu", C.c_int32), ("tet_unroll", C.c_int32),
                ("compact_records", C.c_int32)]


class ProfileStats(C.Structure):
    _fields_ = [("n_launches", C.c_int64), ("total_ms", C.c_double), ("total_bytes", C.c_double),
                ("n_vertex_updates", C.c_int64)]


class Counters(C.Structure):
    _fields_ = [("n_skips", C.c_int64), ("n_nonfinite", C.c_int64)]


class VBDError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libvbd.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2403_06321_amd.build.build() "
                          "(or __graft_entry__.build())")
    L = C.CDLL(LIB_PATH)
    p, i32, sz = C.c_void_p, C.c_int32, C.c_size_t
    L.vbd_build_topology.argtypes = [C.POINTER(MeshDesc), C.POINTER(C.c_void_p)]
    L.vbd_color.argtypes = [p, C.POINTER(i32), p]
    L.vbd_color_given.argtypes = [p, p]
    L.vbd_color_greedy.argtypes = [p, i32, C.POINTER(i32), p]
    L.vbd_workspace_size.argtypes = [p, i32, C.POINTER(sz)]
    L.vbd_bind_workspace.argtypes = [p, p, sz, p]
    L.vbd_topology_query.argtypes = [p, i32, p, sz]
    L.vbd_topology_destroy.argtypes = [p]
    L.vbd_step.argtypes = [p, C.POINTER(StepParamsC), p, p, p, p, p]
    L.vbd_step_static.argtypes = [p, C.POINTER(StepParamsC), p, p, p, p, p]
    L.vbd_step_record.argtypes = [p, C.POINTER(StepParamsC), p, p, p, p, p]
    L.vbd_step_backward.argtypes = [p, C.POINTER(StepParamsC)] + [p] * 12
    L.vbd_get_launch_config.argtypes = [p, C.POINTER(LaunchConfig)]
    L.vbd_set_launch_config.argtypes = [p, C.POINTER(LaunchConfig)]
    L.vbd_autotune.argtypes = [p, C.POINTER(StepParamsC), p, p, p, p, p]
    L.vbd_profile_enable.argtypes = [p, i32]
    L.vbd_profile_read.argtypes = [p, C.POINTER(ProfileStats), i32]
    L.vbd_check.argtypes = [p, p]
    L.vbd_probe_copy.argtypes = [p, p, sz, p]
    L.vbd_probe_read.argtypes = [p, sz, p, i32, p]
    L.vbd_detect_contacts.argtypes = [p, C.POINTER(StepParamsC), p, p, p]
    L.vbd_detect_edges.argtypes = [p, C.POINTER(StepParamsC), p, p, p, p]
    L.vbd_read_counters.argtypes = [p, C.POINTER(Counters), i32, p]
    L.vbd_last_error.argtypes = []
    L.vbd_last_error.restype = C.c_char_p
    for name in EXPORTS:
        if name != "vbd_last_error":
            getattr(L, name).restype = i32
    _lib = L
    return L


def check(status):
    if status != VBD_OK:
        msg = lib().vbd_last_error()
        raise VBDError(status, msg.decode() if msg else "")
