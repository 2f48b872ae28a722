"""ctypes declarations of the C ABI in include/mpm.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpm.so")

MPM_OK, MPM_EINVAL, MPM_ENOMEM, MPM_EBUDGET, MPM_EDOMAIN, MPM_ENOCONV, MPM_ENONFINITE, MPM_EHIP = range(8)
STATUS_NAMES = {0: "MPM_OK", 1: "MPM_EINVAL", 2: "MPM_ENOMEM", 3: "MPM_EBUDGET", 4: "MPM_EDOMAIN",
                5: "MPM_ENOCONV", 6: "MPM_ENONFINITE", 7: "MPM_EHIP"}
MPM_FP64, MPM_MIXED = 0, 1
(F_MASS, F_MOM, F_W, F_WT, F_E, F_ET, F_VN, F_TN, F_FREE, F_HEAT_RHS, F_HEAT_DIAG, F_VHAT, F_THAT,
 F_PARENT, F_COUNT, F_KSURF, F_MOM_DIAG, F_PERM) = range(18)


class MpmParams(C.Structure):
    _fields_ = [(k, C.c_int32) for k in (
        "dim", "n", "precision", "hess_mode", "term_mask", "momentum_fix", "wall_layers", "slab",
        "slab_axis", "heat", "gamma_by_label", "newton_max", "cg_max", "ls_max", "heat_max", "krylov")] + [
        ("dx", C.c_double), ("dt", C.c_double), ("gravity", C.c_double * 3), ("bulk", C.c_double),
        ("mu0", C.c_double), ("mu_k", C.c_double), ("mu_T0", C.c_double),
        ("g0", C.c_double), ("g1", C.c_double), ("gT0", C.c_double), ("gmin", C.c_double), ("gmax", C.c_double),
        ("gamma_label", C.c_double * 4),
        ("cp", C.c_double), ("K", C.c_double), ("h", C.c_double), ("T_amb", C.c_double), ("b", C.c_double),
        ("H", C.c_double), ("slab_lo", C.c_double * 3), ("slab_hi", C.c_double * 3),
        ("newton_tol", C.c_double), ("cg_rel", C.c_double), ("ls_c1", C.c_double), ("heat_tol", C.c_double),
        ("cfl", C.c_double), ("dt_min", C.c_double), ("dt_max", C.c_double),
        ("n_planes", C.c_int32), ("pad0_", C.c_int32), ("plane_o", (C.c_double * 3) * 4),
        ("plane_n", (C.c_double * 3) * 4), ("plane_mu", C.c_double * 4),
        ("T_melt", C.c_double), ("muh0", C.c_double), ("lamh0", C.c_double), ("kh", C.c_double),
        ("Th0", C.c_double)]


class MpmParticles(C.Structure):
    _fields_ = [("n", C.c_int64)] + [(k, C.c_void_p) for k in ("x", "v", "A", "J", "V0", "m", "T", "gradT", "F")]


class MpmSurface(C.Structure):
    _fields_ = [("n", C.c_int64), ("s", C.c_void_p), ("dA", C.c_void_p), ("label", C.c_void_p)]


class MpmStats(C.Structure):
    _fields_ = [(k, C.c_int32) for k in (
        "newton_iters", "cg_iters", "heat_iters", "line_search_halvings", "energy_evals", "hessvecs",
        "converged", "status")] + [
        ("g0", C.c_double), ("gnorm", C.c_double), ("phi", C.c_double), ("heat_res", C.c_double),
        ("momentum", C.c_double * 3), ("n_part", C.c_int64), ("n_surf", C.c_int64), ("n_dof", C.c_int64),
        ("n_tiles", C.c_int64), ("dt", C.c_double), ("host_waits", C.c_int64)]


class MpmTuning(C.Structure):
    _fields_ = [("run", C.c_int32 * 3), ("ncand", C.c_int32), ("cand", C.c_int32 * 8), ("us", (C.c_double * 8) * 3)]


class MpmRequest(C.Structure):
    _fields_ = [("id", C.c_int64), ("params", MpmParams), ("n_steps", C.c_int32), ("implicit", C.c_int32),
                ("keep_result", C.c_int32), ("borrow", C.c_int32), ("n_part", C.c_int64), ("seed", C.c_uint64),
                ("first_step", C.c_uint64), ("ls_radius", C.c_double), ("sample_density", C.c_double),
                ("label_lo", C.c_double * 3), ("label_hi", C.c_double * 3)] + [
        (k, C.c_void_p) for k in ("x", "v", "A", "J", "V0", "m", "T", "gradT")]


class MpmCompletion(C.Structure):
    _fields_ = [("id", C.c_int64), ("status", C.c_int32), ("steps_done", C.c_int32), ("t_submit", C.c_double),
                ("t_admit", C.c_double), ("t_done", C.c_double), ("n_part", C.c_int64), ("n_surf", C.c_int64),
                ("bytes", C.c_int64), ("newton_iters", C.c_int32), ("cg_iters", C.c_int32)]


class MpmServerInfo(C.Structure):
    _fields_ = [(k, C.c_int64) for k in ("submitted", "completed", "rejected", "queued", "running", "arena_bytes",
                                         "bytes_in_use", "peak_bytes")] + [("peak_running", C.c_int32),
                                                                          ("pad_", C.c_int32)]


EXPORTS = {
    "mpm_params_default": (C.c_int, [C.POINTER(MpmParams), C.c_int32, C.c_int32]),
    "mpm_workspace_bytes": (C.c_int, [C.POINTER(MpmParams), C.c_int64, C.c_int64, C.POINTER(C.c_size_t)]),
    "mpm_ctx_create": (C.c_int, [C.POINTER(MpmParams), C.c_void_p, C.c_size_t, C.c_int64, C.c_int64,
                                 C.POINTER(C.c_void_p)]),
    "mpm_ctx_destroy": (C.c_int, [C.c_void_p]),
    "mpm_last_error": (C.c_char_p, [C.c_void_p]),
    "mpm_ctx_set_params": (C.c_int, [C.c_void_p, C.POINTER(MpmParams)]),
    "mpm_p2g": (C.c_int, [C.c_void_p, C.POINTER(MpmParticles), C.POINTER(MpmSurface), C.c_void_p]),
    "mpm_energy_grad": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mpm_hessvec": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p]),
    "mpm_heat_apply": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mpm_g2p": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(MpmParticles), C.c_void_p]),
    "mpm_solve_momentum": (C.c_int, [C.c_void_p, C.c_void_p]),
    "mpm_solve_heat": (C.c_int, [C.c_void_p, C.c_void_p]),
    "mpm_step": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(C.POINTER(MpmParticles)),
                           C.POINTER(C.POINTER(MpmSurface)), C.c_int32, C.c_int32, C.c_void_p]),
    "mpm_batch_config": (C.c_int, [C.c_int32]),
    "mpm_step_noalloc": (C.c_int, [C.POINTER(MpmParams), C.POINTER(MpmParticles), C.POINTER(MpmSurface), C.c_int32,
                                   C.c_void_p, C.POINTER(C.c_size_t)]),
    "mpm_grid_view": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p)]),
    "mpm_get_stats": (C.c_int, [C.c_void_p, C.POINTER(MpmStats)]),
    "mpm_timing": (C.c_int, [C.c_void_p, C.c_int32]),
    "mpm_timing_read": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mpm_scene_status": (C.c_int, [C.c_void_p, C.c_void_p]),
    "mpm_server_clock": (C.c_double, []),
    "mpm_server_create": (C.c_int, [C.c_void_p, C.c_size_t, C.c_int32, C.POINTER(C.c_void_p)]),
    "mpm_server_submit": (C.c_int, [C.c_void_p, C.POINTER(MpmRequest)]),
    "mpm_server_poll": (C.c_int, [C.c_void_p, C.POINTER(MpmCompletion), C.c_int32, C.POINTER(C.c_int32)]),
    "mpm_server_wait": (C.c_int, [C.c_void_p, C.c_double]),
    "mpm_server_result": (C.c_int, [C.c_void_p, C.c_int64] + [C.c_void_p] * 6),
    "mpm_server_info_get": (C.c_int, [C.c_void_p, C.POINTER(MpmServerInfo)]),
    "mpm_server_destroy": (C.c_int, [C.c_void_p]),
    "mpm_sample_surface": (C.c_int, [C.c_int32, C.c_int32, C.c_void_p, C.c_int64, C.c_double, C.c_double,
                                     C.c_uint64, C.c_uint64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_int64, C.POINTER(C.c_int64)]),
    "mpm_autotune": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "mpm_tuning_set": (C.c_int, [C.c_void_p, C.c_void_p]),
    "mpm_sample_surface_dev": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_uint64, C.c_uint64,
                                         C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                         C.POINTER(C.c_int64), C.c_void_p]),
}

KERNEL_CLASSES = ["sort", "setup", "p2g", "energy_int", "energy_surf", "energy_node", "hess_int",
                  "hess_surf", "hess_node", "heat_pt", "heat_node", "g2p_split", "g2p", "blas", "p2g_node",
                  "sample"]

_lib = None


def load(path=LIB_PATH):
    """Loads libmpm.so; raises if it was not built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2101_12408_amd.build`")
    # torch ships its own HIP runtime; loading it first makes libmpm.so bind to that same
    # runtime instead of pulling a second copy into the process.
    import torch  # noqa: F401
    lib = C.CDLL(path)
    for name, (res, args) in EXPORTS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib
