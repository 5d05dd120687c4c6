"""ctypes declarations of the C ABI in include/mrcm.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_float, c_int32, c_int64, c_uint32, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmrcm.so")

STATUS = {0: "MRCM_OK", -1: "MRCM_EINVAL", -2: "MRCM_ENOMEM", -3: "MRCM_ENOTSPD",
          -4: "MRCM_ENOCONV", -5: "MRCM_ESINGULAR", -6: "MRCM_EHIP", -7: "MRCM_EUNSUPPORTED"}

# Every entry point declared in include/mrcm.h.
EXPORTS = [
    "mrcm_build_mbfs", "mrcm_assemble_interface", "mrcm_solve_interface", "mrcm_reconstruct",
    "mrcm_query", "mrcm_get_subdomain", "mrcm_copy_mbfs", "mrcm_copy_flux", "mrcm_copy_factor",
    "mrcm_interface_dims", "mrcm_copy_interface", "mrcm_interface_query", "mrcm_postprocess_mean",
    "mrcm_transport_step", "mrcm_transport_dt", "mrcm_transport_advance", "mrcm_transport_marks_bytes",
    "mrcm_transport_mark_sources", "mrcm_mobility_scale", "mrcm_impes_run",
    "mrcm_mbfs_destroy", "mrcm_interface_destroy",
    "mrcm_status_string", "mrcm_last_error", "mrcm_profile_enable", "mrcm_profile_reset",
    "mrcm_profile_get", "mrcm_autotune", "mrcm_autotune_cached", "mrcm_graph_capture", "mrcm_graph_launch", "mrcm_graph_check", "mrcm_graph_destroy",
    # mrcm_nn.h
    "mrcm_conv3d_max_channels", "mrcm_conv3d_forward", "mrcm_conv3d_backward", "mrcm_mse", "mrcm_mse_noalloc",
    "mrcm_adam_step",
    "mrcm_nn_features", "mrcm_nn_scatter",
    "mrcm_unet_max_channels", "mrcm_unet_padded", "mrcm_unet_pack", "mrcm_unet_conv", "mrcm_unet_wgrad_workspace",
    "mrcm_unet_wgrad", "mrcm_unet_pool", "mrcm_unet_upsample", "mrcm_unet_relu_mask", "mrcm_nn_channels_last",
]

STAGES = ["coef", "factor", "rhs", "solve", "residual", "refine", "flux", "assemble", "lu", "sweep",
          "reconstruct", "pcg", "fallback", "solve_rest", "mean", "transport"]


class CProblem(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("nz", c_int32),
                ("hx", c_double), ("hy", c_double), ("hz", c_double),
                ("kx", c_void_p), ("ky", c_void_p), ("kz", c_void_p), ("q", c_void_p),
                ("wall_type", c_int32 * 6), ("wall_value", c_void_p * 6),
                ("pin_cell", c_int64)]


class CPartition(ctypes.Structure):
    _fields_ = [("ndx", c_int32), ("ndy", c_int32), ("ndz", c_int32),
                ("cut_x", POINTER(c_int32)), ("cut_y", POINTER(c_int32)), ("cut_z", POINTER(c_int32))]


class CIfaceSpace(ctypes.Structure):
    _fields_ = [("uniform_split", (c_int32 * 2) * 3), ("split", POINTER(c_int32))]


class COptions(ctypes.Structure):
    _fields_ = [("alpha", c_double), ("precision", c_int32), ("ir_tol", c_double),
                ("ir_max_iter", c_int32), ("fp64_refine", c_int32), ("pcg_max_iter", c_int32),
                ("pcg_x0", ctypes.c_void_p), ("pcg_x0_scale", c_int32), ("solve_tiles", c_int32),
                ("solve_group", c_int32), ("beta_mode", c_int32), ("keep", c_uint32), ("iface_panel", c_int32),
                ("launch_mode", c_int32)]


class CTwoPhase(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("nz", c_int32), ("hx", c_double), ("hy", c_double),
                ("hz", c_double), ("mu_w", c_double), ("mu_o", c_double)]


class CImpesOptions(ctypes.Structure):
    _fields_ = [("skip", c_int32), ("max_steps", c_int32), ("t_end", c_double), ("cfl", c_double),
                ("dt_max", c_double), ("refine", c_int32)]


class CImpesStats(ctypes.Structure):
    _fields_ = [("darcy_solves", c_int32), ("steps", c_int32), ("t", c_double), ("ms_darcy", c_double),
                ("ms_darcy_first", c_double), ("ms_mean", c_double), ("ms_transport", c_double)]


class CIfaceInfo(ctypes.Structure):
    _fields_ = [("n", c_int32), ("nodes", c_int32), ("levels", c_int32), ("max_front", c_int32),
                ("front_bytes", c_int64), ("factor_flops", c_double), ("factor_launches", c_int32),
                ("bandwidth", c_int32), ("device_bytes", c_int64), ("method", c_int32),
                ("refine_iters", c_int32), ("rel_residual", c_double)]


class CInfo(ctypes.Structure):
    _fields_ = [("n_sub", c_int32), ("n_patch", c_int32), ("n_cells", c_int64),
                ("n_mbfs", c_int64), ("n_rhs", c_int64), ("max_band", c_int32),
                ("max_rhs", c_int32), ("precision", c_int32), ("ir_iters", c_int32),
                ("ir_residual", c_double), ("factor_flops", c_double), ("solve_flops", c_double),
                ("device_bytes", c_int64), ("pcg_fallback", c_int32), ("pcg_iters", c_int64)]


class CProfile(ctypes.Structure):
    _fields_ = [("ms", c_double * 16), ("count", c_int64 * 16)]


class CSubInfo(ctypes.Structure):
    _fields_ = [("lo", c_int32 * 3), ("ext", c_int32 * 3), ("ax", c_int32 * 3),
                ("n_cells", c_int32), ("band", c_int32), ("n_rhs", c_int32),
                ("n_patch", c_int32), ("pin_local", c_int32), ("solve_group", c_int32)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libmrcm.so and declare its signatures.  Raises if it is missing:
    there is no other implementation to fall back to."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run paper_2103_08513_amd.build.build() first")
    lib = ctypes.CDLL(path)
    P = POINTER
    sigs = {
        "mrcm_build_mbfs": ([P(CProblem), P(CPartition), P(CIfaceSpace), P(COptions), c_void_p,
                             P(c_void_p)], c_int32),
        "mrcm_assemble_interface": ([c_void_p, c_void_p, P(c_void_p)], c_int32),
        "mrcm_solve_interface": ([c_void_p, c_int32, c_double, c_int32, c_void_p, c_void_p, P(c_int32),
                                  P(c_double)], c_int32),
        "mrcm_interface_query": ([c_void_p, P(CIfaceInfo)], c_int32),
        "mrcm_reconstruct": ([c_void_p, c_void_p, c_void_p, c_void_p, c_void_p], c_int32),
        "mrcm_postprocess_mean": ([c_void_p, c_void_p, c_void_p, c_void_p, c_void_p], c_int32),
        "mrcm_transport_step": ([P(CTwoPhase), c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p], c_int32),
        "mrcm_transport_advance": ([P(CTwoPhase)] + [c_void_p] * 5 + [c_double, c_double] + [c_void_p] * 3, c_int32),
        "mrcm_transport_marks_bytes": ([P(CTwoPhase)], c_int64),
        "mrcm_transport_mark_sources": ([P(CTwoPhase), c_void_p, c_void_p, c_void_p], c_int32),
        "mrcm_transport_dt": ([P(CTwoPhase), c_void_p, c_void_p, c_double, c_double, c_void_p, c_void_p], c_int32),
        "mrcm_mobility_scale": ([P(CTwoPhase)] + [c_void_p] * 8, c_int32),
        "mrcm_impes_run": ([P(CProblem), P(CPartition), P(CIfaceSpace), P(COptions), P(CTwoPhase), P(CImpesOptions),
                            c_void_p, c_void_p, P(CImpesStats)], c_int32),
        "mrcm_query": ([c_void_p, P(CInfo)], c_int32),
        "mrcm_get_subdomain": ([c_void_p, c_int32, P(CSubInfo)], c_int32),
        "mrcm_copy_mbfs": ([c_void_p, c_int32, c_void_p], c_int32),
        "mrcm_copy_flux": ([c_void_p, c_int32, c_void_p, c_void_p, c_void_p], c_int32),
        "mrcm_copy_factor": ([c_void_p, c_int32, c_void_p], c_int32),
        "mrcm_interface_dims": ([c_void_p, P(c_int32), P(c_int32)], c_int32),
        "mrcm_copy_interface": ([c_void_p, c_void_p, c_void_p], c_int32),
        "mrcm_mbfs_destroy": ([c_void_p], None),
        "mrcm_interface_destroy": ([c_void_p], None),
        "mrcm_status_string": ([c_int32], c_char_p),
        "mrcm_last_error": ([], c_char_p),
        "mrcm_profile_enable": ([c_int32], None),
        "mrcm_profile_reset": ([], None),
        "mrcm_profile_get": ([P(CProfile)], c_int32),
        "mrcm_autotune": ([P(CProblem), P(CPartition), P(CIfaceSpace), P(COptions), c_void_p, P(COptions),
                           P(c_double), P(c_double)], c_int32),
        "mrcm_autotune_cached": ([P(CProblem), P(CPartition), P(CIfaceSpace), P(COptions), c_void_p, ctypes.c_char_p,
                                  P(COptions), P(c_double), P(c_double), P(c_int32)], c_int32),
        "mrcm_graph_capture": ([P(CProblem), P(CPartition), P(CIfaceSpace), P(COptions), c_void_p, c_void_p,
                                c_int32, c_void_p, c_void_p, c_void_p, c_void_p, P(c_void_p)], c_int32),
        "mrcm_graph_launch": ([c_void_p, c_void_p], c_int32),
        "mrcm_graph_check": ([c_void_p, c_void_p], c_int32),
        "mrcm_graph_destroy": ([c_void_p], None),
        "mrcm_conv3d_max_channels": ([], c_int32),
        "mrcm_conv3d_forward": ([c_void_p] * 5 + [c_int32] * 8 + [c_void_p], c_int32),
        "mrcm_conv3d_backward": ([c_void_p] * 8 + [c_int32] * 7 + [c_void_p], c_int32),
        "mrcm_mse": ([c_void_p] * 5 + [c_int64, c_void_p], c_int32),
        "mrcm_mse_noalloc": ([c_void_p] * 4 + [c_int64, c_void_p], c_int32),
        "mrcm_unet_max_channels": ([], c_int32),
        "mrcm_unet_padded": ([c_int32], c_int32),
        "mrcm_unet_pack": ([c_void_p] * 3 + [c_int32, c_int32, c_void_p], c_int32),
        "mrcm_unet_conv": ([c_void_p] * 5 + [c_int32] * 7 + [c_void_p], c_int32),
        "mrcm_unet_wgrad_workspace": ([c_int32] * 6, c_int64),
        "mrcm_unet_wgrad": ([c_void_p] * 5 + [c_int32] * 6 + [c_void_p], c_int32),
        "mrcm_unet_pool": ([c_void_p] * 2 + [c_int32] * 6 + [c_void_p], c_int32),
        "mrcm_unet_upsample": ([c_void_p] * 2 + [c_int32] * 6 + [c_void_p], c_int32),
        "mrcm_unet_relu_mask": ([c_void_p] * 2 + [c_int64, c_void_p], c_int32),
        "mrcm_nn_channels_last": ([c_void_p] * 2 + [c_int32, c_int32, c_int64, c_void_p], c_int32),
        "mrcm_adam_step": ([c_void_p] * 4 + [c_int32, c_int32, c_float, c_float, c_float, c_float, c_void_p],
                           c_int32),
        "mrcm_nn_features": ([c_void_p, P(c_int32), c_int32, c_void_p, c_void_p, c_void_p], c_int32),
        "mrcm_nn_scatter": ([c_void_p, P(c_int32), c_int32, c_void_p, c_void_p, c_void_p], c_int32),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


class MRCMError(RuntimeError):
    def __init__(self, code, where, detail):
        self.code = code
        super().__init__(f"{where}: {STATUS.get(code, code)}: {detail}")


def check(code, where):
    if code != 0:
        detail = _lib.mrcm_last_error().decode(errors="replace") if _lib else ""
        raise MRCMError(code, where, detail)
