"""ctypes loader of libpme.so: the C ABI declared in include/pme.h.

Argument marshalling only.  The library must have been built in-tree
(``python -m paper_2606_01598_amd.build``); without it every entry point
raises, there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpme.so")

PME_OK = 0
PME_EINVAL = -1
PME_EORDER = -2
PME_EMESH = -3
PME_EALPHA = -4
PME_ECAPACITY = -5
PME_ENOMEM = -6
PME_EHIP = -7
PME_ENONFINITE = -8
PME_ESCRATCH = -9
PME_NOALLOC_SCRATCH_BYTES = 64 << 20

PME_F_KEEP_PHI = 1
PME_F_CONCURRENT = 2
PME_F_OPT_INFLUENCE = 4
PME_F_SEPARATE_SPREAD = 8

PME_SPREAD_TILE = 0
PME_SPREAD_BAND = 1
PME_SPREAD_FUSED = 2

PME_MESH_POW2 = 0
PME_MESH_SMOOTH = 1
PME_MESH_CEIL = 2

# every symbol include/pme.h declares
EXPORTS = ("pme_mesh_dims", "pme_plan", "pme_plan_destroy", "pme_plan_workspace_bytes",
           "pme_plan_phi_id", "pme_plan_drop_phi", "pme_forward_noalloc",
           "pme_forward", "pme_forward_cell", "pme_forward_quad", "pme_backward", "pme_step", "pme_step_capture", "pme_step_replay", "pme_status", "pme_strerror", "pme_last_hip_error",
           "pme_plan_phi", "pme_plan_rho", "pme_plan_spread_kind", "pme_plan_timer",
           "pme_plan_timer_read",
           "pol_plan_create", "pol_plan_destroy", "pol_real", "pol_real_mixed", "pol_model",
           "pol_model_hvp", "pol_scf", "dip_plan_create", "dip_plan_destroy", "dip_features",
           "dip_forward", "dip_backward", "dip_position_vjp", "dip_features_jvp", "dip_charges",
           "dip_forward_jvp", "dip_backward_jvp", "dip_loss", "dip_adam", "pme_batch_plan", "pme_batch_destroy",
           "pme_batch_forward", "pme_batch_backward", "pme_batch_graph_capture", "pme_batch_graph_launch",
           "pme_batch_status", "pme_lds_probe", "pme_halo_probe")

DIP_NFEAT, DIP_NCH, DIP_HIDDEN, DIP_NPARAM, DIP_NQPARAM = 34, 16, 64, 7440, 2304

# launch-timer kinds (PME_K_* of include/pme.h)
KERNEL_KINDS = ("bin", "bin_tangent", "spread", "spread_tangent", "fft_r2c", "fft_x",
                "fft_c2r", "gather", "gather_hvp")


class PMEDesc(ctypes.Structure):
    _fields_ = [("mesh", ctypes.c_int32 * 3),
                ("order", ctypes.c_int32),
                ("max_atoms", ctypes.c_int32),
                ("flags", ctypes.c_int32),
                ("alpha", ctypes.c_double),
                ("influence_power", ctypes.c_double),
                ("prefactor", ctypes.c_double),
                ("tile", ctypes.c_int32 * 3),
                ("fft_lines", ctypes.c_int32)]


class BatchStep(ctypes.Structure):
    _fields_ = [(name, ctypes.c_void_p) for name in (
        "pos", "q", "mu", "box", "energy", "dE_dpos", "dE_dq", "dE_dmu", "v_pos", "v_q", "v_mu",
        "g_pos", "g_q", "g_mu", "vf_pos", "gf_pos", "gf_q", "gf_mu")]


class PolDesc(ctypes.Structure):
    _fields_ = [("max_atoms", ctypes.c_int32),
                ("flags", ctypes.c_int32),
                ("box", ctypes.c_double * 9),
                ("alpha", ctypes.c_double),
                ("cutoff", ctypes.c_double),
                ("thole_a", ctypes.c_double),
                ("prefactor", ctypes.c_double)]


POL_F_WARM_START = 1
POL_F_FIXED_ITERS = 2

PME_PROBE_LDS_READ = 0
PME_PROBE_LDS_ATOMIC = 1
PME_PROBE_HALO_ATOMIC = 2
PME_PROBE_HALO_WRITE = 3
PME_PROBE_HALO_FOLD = 4


class DipDesc(ctypes.Structure):
    _fields_ = [("max_atoms", ctypes.c_int32),
                ("flags", ctypes.c_int32),
                ("box", ctypes.c_double * 9),
                ("cutoff", ctypes.c_double)]


class PMEError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(msg)
        self.code = code


_lib = None


def load():
    """Load libpme.so once; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2606_01598_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    lib.pme_mesh_dims.argtypes = [ctypes.POINTER(f64), f64, ctypes.c_int, ctypes.POINTER(i32)]
    lib.pme_mesh_dims.restype = ctypes.c_int
    lib.pme_plan.argtypes = [ctypes.POINTER(PMEDesc), ctypes.POINTER(vp)]
    lib.pme_plan.restype = ctypes.c_int
    lib.pme_plan_destroy.argtypes = [vp]
    lib.pme_plan_destroy.restype = None
    lib.pme_plan_workspace_bytes.argtypes = [vp]
    lib.pme_plan_workspace_bytes.restype = ctypes.c_int64
    lib.pme_plan_phi_id.argtypes = [vp]
    lib.pme_plan_phi_id.restype = ctypes.c_int64
    lib.pme_plan_drop_phi.argtypes = [vp]
    lib.pme_plan_drop_phi.restype = ctypes.c_int
    lib.pme_forward.argtypes = [vp, vp, i32, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.pme_forward_noalloc.argtypes = [ctypes.POINTER(PMEDesc), vp, i32, vp, vp, vp, vp, vp, vp,
                                        vp, vp]
    lib.pme_forward_noalloc.restype = ctypes.c_int
    lib.pme_forward.restype = ctypes.c_int
    lib.pme_forward_cell.argtypes = [vp, vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.pme_forward_cell.restype = ctypes.c_int
    lib.pme_forward_quad.argtypes = [vp, vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.pme_forward_quad.restype = ctypes.c_int
    lib.pme_backward.argtypes = [vp, vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.pme_backward.restype = ctypes.c_int
    lib.pme_step.argtypes = [vp, vp, i32] + [vp] * 14
    lib.pme_step.restype = ctypes.c_int
    lib.pme_step_capture.argtypes = [vp, i32, i32] + [vp] * 14
    lib.pme_step_capture.restype = ctypes.c_int
    lib.pme_step_replay.argtypes = [vp, vp]
    lib.pme_step_replay.restype = ctypes.c_int
    lib.pme_status.argtypes = [vp, vp]
    lib.pme_status.restype = ctypes.c_int
    lib.pme_strerror.argtypes = [ctypes.c_int]
    lib.pme_strerror.restype = ctypes.c_char_p
    lib.pme_last_hip_error.argtypes = []
    lib.pme_last_hip_error.restype = ctypes.c_char_p
    lib.pme_plan_phi.argtypes = [vp]
    lib.pme_plan_phi.restype = vp
    lib.pme_plan_rho.argtypes = [vp]
    lib.pme_plan_rho.restype = vp
    lib.pme_plan_spread_kind.argtypes = [vp]
    lib.pme_plan_spread_kind.restype = ctypes.c_int
    lib.pme_plan_timer.argtypes = [vp, ctypes.c_int]
    lib.pme_plan_timer.restype = ctypes.c_int
    lib.pme_plan_timer_read.argtypes = [vp, ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_double)]
    lib.pme_plan_timer_read.restype = ctypes.c_int
    lib.pol_plan_create.argtypes = [ctypes.POINTER(PolDesc), ctypes.POINTER(vp)]
    lib.pol_plan_create.restype = ctypes.c_int
    lib.pol_plan_destroy.argtypes = [vp]
    lib.pol_plan_destroy.restype = None
    lib.pol_real.argtypes = [vp, vp, i32, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.pol_real.restype = ctypes.c_int
    lib.pol_real_mixed.argtypes = [vp, vp, i32, vp, vp, vp, vp, vp, vp]
    lib.pol_real_mixed.restype = ctypes.c_int
    lib.pol_model.argtypes = [vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.pol_model.restype = ctypes.c_int
    lib.pol_model_hvp.argtypes = [vp, vp, vp, i32] + [vp] * 10
    lib.pol_model_hvp.restype = ctypes.c_int
    lib.pol_scf.argtypes = [vp, vp, vp, i32, vp, vp, vp, vp, f64, i32, vp,
                            ctypes.POINTER(i32), ctypes.POINTER(f64)]
    lib.pol_scf.restype = ctypes.c_int
    lib.pme_batch_plan.argtypes = [ctypes.POINTER(PMEDesc), i32, ctypes.POINTER(i32),
                                   ctypes.POINTER(vp)]
    lib.pme_batch_plan.restype = ctypes.c_int
    lib.pme_batch_destroy.argtypes = [vp]
    lib.pme_batch_destroy.restype = None
    lib.pme_batch_forward.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.pme_batch_forward.restype = ctypes.c_int
    lib.pme_batch_backward.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.pme_batch_backward.restype = ctypes.c_int
    lib.pme_batch_graph_capture.argtypes = [vp, ctypes.POINTER(BatchStep)]
    lib.pme_batch_graph_capture.restype = ctypes.c_int
    lib.pme_batch_graph_launch.argtypes = [vp, vp]
    lib.pme_batch_graph_launch.restype = ctypes.c_int
    lib.pme_batch_status.argtypes = [vp, vp]
    lib.pme_batch_status.restype = ctypes.c_int
    lib.pme_lds_probe.argtypes = [vp, i32, i32, i32, vp]
    lib.pme_lds_probe.restype = ctypes.c_int
    lib.pme_halo_probe.argtypes = [vp, i32, vp, vp, i32, vp, vp]
    lib.pme_halo_probe.restype = ctypes.c_int
    lib.dip_plan_create.argtypes = [ctypes.POINTER(DipDesc), ctypes.POINTER(vp)]
    lib.dip_plan_create.restype = ctypes.c_int
    lib.dip_plan_destroy.argtypes = [vp]
    lib.dip_plan_destroy.restype = None
    lib.dip_features.argtypes = [vp, vp, i32, vp, vp, vp, vp]
    lib.dip_features.restype = ctypes.c_int
    lib.dip_forward.argtypes = [vp, vp, i32, vp, vp, vp, vp]
    lib.dip_forward.restype = ctypes.c_int
    lib.dip_backward.argtypes = [vp, vp, i32, vp, vp, vp, vp, vp, vp, vp]
    lib.dip_backward.restype = ctypes.c_int
    lib.dip_position_vjp.argtypes = [vp, vp, i32] + [vp] * 10
    lib.dip_position_vjp.restype = ctypes.c_int
    lib.dip_features_jvp.argtypes = [vp, vp, i32] + [vp] * 6
    lib.dip_features_jvp.restype = ctypes.c_int
    lib.dip_charges.argtypes = [vp, vp, i32] + [vp] * 6
    lib.dip_charges.restype = ctypes.c_int
    lib.dip_forward_jvp.argtypes = [vp, vp, i32] + [vp] * 7
    lib.dip_forward_jvp.restype = ctypes.c_int
    lib.dip_backward_jvp.argtypes = [vp, vp, i32] + [vp] * 14
    lib.dip_backward_jvp.restype = ctypes.c_int
    lib.dip_loss.argtypes = [vp, vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, f64, f64, f64, vp, vp,
                             vp, vp]
    lib.dip_loss.restype = ctypes.c_int
    lib.dip_adam.argtypes = [vp, i32, i32, f64, f64, f64, f64, vp, vp, vp, vp]
    lib.dip_adam.restype = ctypes.c_int
    _lib = lib
    return lib


def check(rc: int) -> None:
    if rc != PME_OK:
        lib = load()
        msg = lib.pme_strerror(rc).decode()
        if rc == PME_EHIP:
            msg += ": " + lib.pme_last_hip_error().decode()
        raise PMEError(rc, msg)
