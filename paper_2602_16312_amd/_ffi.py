"""ctypes mirror of include/dgmg.h and loading of the in-tree libdgmg.so."""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# DGMG_LIB selects another build of the same library (the host-sanitizer build)
LIB_PATH = os.environ.get("DGMG_LIB") or os.path.join(HERE, "libdgmg.so")

MAX_LEVELS = 8
MULTI_RHS = 8          # DGMG_MULTI_RHS
OK, NOT_CONVERGED = 0, 1
ERRORS = {-1: "EINVAL", -2: "ENOTSPD", -3: "ENAN", -4: "EHIP", -5: "ENOMEM",
          -6: "EUNSUPPORTED"}

# every symbol declared in include/dgmg.h
EXPORTS = [
    "dgmg_build_hierarchy", "dgmg_hierarchy_info", "dgmg_hierarchy_parents", "dgmg_hierarchy_boxes",
    "dgmg_destroy_hierarchy", "dgmg_setup_levels", "dgmg_destroy_solver",
    "dgmg_get_info", "dgmg_pcg_solve", "dgmg_ionic_step", "dgmg_time_step",
    "dgmg_pcg_solve_multi", "dgmg_time_step_multi", "dgmg_apply_multi", "dgmg_vcycle_multi",
    "dgmg_apply", "dgmg_vcycle", "dgmg_mass_apply", "dgmg_export_level",
    "dgmg_profile_begin", "dgmg_profile_end", "dgmg_kernel_bench", "dgmg_last_error",
    "dgmg_set_sensors", "dgmg_sensor_misfit", "dgmg_adjoint_step", "dgmg_grad_accumulate",
    "dgmg_pcg_solve_noalloc", "dgmg_set_phase_timing", "dgmg_step_phase_ms",
]

dp = C.POINTER(C.c_double)
i64p = C.POINTER(C.c_int64)


class Mesh(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_vert", C.c_int64), ("xyz", dp),
                ("n_cells", C.c_int64), ("cell_vtx", i64p)]


class AggloOpts(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("method", C.c_int32),
                ("grid_bins", (C.c_int32 * 3) * MAX_LEVELS),
                ("rtree_fanout", C.c_int32),
                ("user_parents", C.POINTER(i64p))]


class Disc(C.Structure):
    _fields_ = [("p", C.c_int32), ("penalty_mode", C.c_int32), ("eta", C.c_double)]


class Physics(C.Structure):
    _fields_ = [("chi", C.c_double), ("Cm", C.c_double), ("dt", C.c_double),
                ("bdf", C.c_int32), ("D_cell", dp), ("cell_scale", dp),
                ("model", C.c_int32), ("n_params", C.c_int32), ("params", dp)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


class MGOpts(C.Structure):
    _fields_ = [("cheb_degree", C.c_int32), ("cheb_sweeps", C.c_int32),
                ("lanczos_steps", C.c_int32), ("lam_safety", C.c_double),
                ("smooth_range", C.c_double), ("lam_override", dp),
                ("precision", C.c_int32), ("device_setup", C.c_int32),
                ("adjoint", C.c_int32), ("max_rhs", C.c_int32),
                ("mfma", C.c_int32), ("fine_layout", C.c_int32),
                ("setup_on_device", C.c_int32), ("allocator", C.POINTER(Allocator)),
                ("jacobi", C.c_int32)]


class SolverInfo(C.Structure):
    _fields_ = [("dim", C.c_int32), ("p", C.c_int32), ("b", C.c_int32),
                ("n_levels", C.c_int32), ("precision", C.c_int32),
                ("model", C.c_int32), ("n_gates", C.c_int32),
                ("n_dofs", C.c_int64),
                ("n_cells", C.c_int64 * MAX_LEVELS),
                ("n_faces", C.c_int64 * MAX_LEVELS),
                ("lam_lo", C.c_double * MAX_LEVELS),
                ("lam_hi", C.c_double * MAX_LEVELS),
                ("op_complexity", C.c_double),
                ("t_assembly", C.c_double), ("t_hierarchy", C.c_double),
                ("t_transfer", C.c_double), ("t_galerkin", C.c_double),
                ("t_smoother", C.c_double), ("t_coarse", C.c_double),
                ("t_upload", C.c_double), ("device_bytes", C.c_int64),
                ("fine_layout", C.c_int32),
                ("level_layout", C.c_int32 * MAX_LEVELS),
                ("prolong_types", C.c_int32 * MAX_LEVELS),
                ("level_grouped", C.c_int32 * MAX_LEVELS),
                ("sparse_faces", C.c_int32)]


class PCGOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("tol_mode", C.c_int32),
                ("max_it", C.c_int32), ("flexible", C.c_int32)]


class PCGStats(C.Structure):
    _fields_ = [("its", C.c_int32), ("converged", C.c_int32),
                ("r0", C.c_double), ("rfin", C.c_double)]


class State(C.Structure):
    _fields_ = [("U", C.c_void_p), ("Uprev", C.c_void_p), ("W", C.c_void_p),
                ("Wprev", C.c_void_p), ("g", C.c_void_p)]


_lib = None


def lib():
    """The loaded library; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2602_16312_amd.build` first")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.dgmg_build_hierarchy.argtypes = [C.POINTER(Mesh), C.POINTER(AggloOpts), C.POINTER(vp)]
        L.dgmg_hierarchy_info.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32), i64p]
        L.dgmg_hierarchy_parents.argtypes = [vp, C.c_int32, i64p]
        L.dgmg_hierarchy_boxes.argtypes = [vp, C.c_int32, dp, dp]
        L.dgmg_destroy_hierarchy.argtypes = [vp]
        L.dgmg_destroy_hierarchy.restype = None
        L.dgmg_setup_levels.argtypes = [vp, C.POINTER(Disc), C.POINTER(Physics),
                                        C.POINTER(MGOpts), C.POINTER(vp)]
        L.dgmg_destroy_solver.argtypes = [vp]
        L.dgmg_destroy_solver.restype = None
        L.dgmg_get_info.argtypes = [vp, C.POINTER(SolverInfo)]
        L.dgmg_pcg_solve.argtypes = [vp, vp, vp, C.POINTER(PCGOpts), C.POINTER(PCGStats), vp]
        L.dgmg_pcg_solve_noalloc.argtypes = [vp, vp, vp, C.POINTER(PCGOpts), C.POINTER(PCGStats), vp]
        L.dgmg_ionic_step.argtypes = [vp] * 7 + [vp]
        L.dgmg_time_step.argtypes = [vp, C.POINTER(State), C.c_double, vp,
                                     C.POINTER(PCGOpts), C.POINTER(PCGStats), vp]
        L.dgmg_apply.argtypes = [vp, C.c_int32, C.c_int32, vp, vp, vp]
        L.dgmg_vcycle.argtypes = [vp, vp, vp, vp]
        L.dgmg_mass_apply.argtypes = [vp, vp, vp, vp]
        L.dgmg_export_level.argtypes = [vp, C.c_int32, dp, i64p, dp, dp, i64p]
        L.dgmg_profile_begin.argtypes = [vp, C.c_int32, C.c_int32]
        L.dgmg_set_phase_timing.argtypes = [vp, C.c_int32]
        L.dgmg_step_phase_ms.argtypes = [vp, dp]
        L.dgmg_profile_end.argtypes = [vp, i64p, dp]
        L.dgmg_kernel_bench.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, vp, dp]
        L.dgmg_pcg_solve_multi.argtypes = [vp, C.c_int32, vp, vp, C.POINTER(PCGOpts),
                                           C.POINTER(PCGStats), vp]
        L.dgmg_time_step_multi.argtypes = [vp, C.c_int32, C.POINTER(State), C.c_double, vp,
                                           C.POINTER(PCGOpts), C.POINTER(PCGStats), vp]
        L.dgmg_apply_multi.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, vp, vp, vp]
        L.dgmg_vcycle_multi.argtypes = [vp, C.c_int32, vp, vp, vp]
        L.dgmg_set_sensors.argtypes = [vp, C.c_int32, i64p, dp]
        L.dgmg_sensor_misfit.argtypes = [vp, vp, vp, vp, vp, vp]
        L.dgmg_adjoint_step.argtypes = [vp] * 12
        L.dgmg_grad_accumulate.argtypes = [vp, vp, vp, vp, vp]
        L.dgmg_last_error.restype = C.c_char_p
        _lib = L
    return _lib


class DGMGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


def check(rc):
    if rc < 0:
        raise DGMGError(rc, lib().dgmg_last_error().decode())
    return rc
