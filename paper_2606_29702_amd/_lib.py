"""ctypes loader for libpinnjet.so (the gfx950 HIP library) and its C ABI.

Argument marshalling only: every step of the computation runs in the HIP
kernels behind include/pinn_jet.h.  If the library is missing this module
raises at import time; there is no fallback implementation.
"""
import ctypes
import os

# torch brings its own HIP runtime (soname libamdhip64.so.7).  Loading torch
# first makes the library bind to that same runtime, so that torch's streams
# and device memory are valid handles inside the library.  Loading the library
# first would map a second runtime into the process.
import torch  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpinnjet.so")

PINN_OK = 0
PINN_ERR_ARG, PINN_ERR_UNSUPPORTED = -1, -2
STATUS_NAMES = {0: "PINN_OK", -1: "PINN_ERR_ARG", -2: "PINN_ERR_UNSUPPORTED", -3: "PINN_ERR_NOMEM",
                -4: "PINN_ERR_DEVICE", -5: "PINN_ERR_STATE", -6: "PINN_ERR_CAP"}
KINDS = {"burgers": 1, "ns": 2, "ks": 3, "heat": 4, "aniso": 5, "burgers_bc": 6}
PRECISIONS = {"fp32": 0, "bf16": 1, "fp16": 2}
PINN_VERIFY_F64 = 1
PINN_BATCH_GRAPH, PINN_BATCH_PER_NETWORK, PINN_BATCH_WIDTH_LANES = 1, 2, 4

# Every symbol the public header declares.
EXPORTS = ["pinn_plan_create", "pinn_plan_destroy", "pinn_plan_memory", "pinn_jet_forward",
           "pinn_jet_residual", "pinn_jet_backward", "pinn_last_error", "pinn_pde_channels",
           "pinn_pde_residuals", "pinn_plan_profile", "pinn_plan_profile_read", "pinn_plan_get_tuning",
           "pinn_plan_set_tuning", "pinn_plan_autotune", "pinn_batch_create", "pinn_batch_destroy",
           "pinn_batch_configure", "pinn_batch_step", "pinn_batch_autotune", "pinn_graph_capture",
           "pinn_graph_launch", "pinn_graph_destroy", "pinn_adam_step", "pinn_graph_capture_train",
           "pinn_jet_step_noalloc", "pinn_jet_backward_cot", "pinn_batch_train_step", "pinn_batch_launches",
           "pinn_batch_profile", "pinn_batch_profile_read", "pinn_batch_get_tuning", "pinn_batch_set_tuning",
           "pinn_tuning_cache_clear", "pinn_tuning_cache_size", "pinn_tuning_cache_save", "pinn_tuning_cache_load",
           "pinn_jet_loss", "pinn_jet_loss_backward", "pinn_batch_get_config", "pinn_plan_create_modified",
           "pinn_batch_schedule_classes"]
KERNEL_CLASSES = {"layer_fwd": 1, "layer_bwd": 2, "dw_hidden": 3, "out_fwd": 4, "out_bwd": 5,
                  "seed_fwd": 6, "other": 7, "bwd_dw": 8}


class PinnError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class Net(ctypes.Structure):
    _fields_ = [("n_layers", ctypes.c_int32), ("dims", ctypes.POINTER(ctypes.c_int32)),
                ("W", ctypes.POINTER(ctypes.c_void_p)), ("b", ctypes.POINTER(ctypes.c_void_p))]


class Pde(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("coef", ctypes.c_double * 4)]


class Segment(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int32), ("data", ctypes.c_int32), ("begin", ctypes.c_int64),
                ("count", ctypes.c_int64), ("weight", ctypes.c_double), ("mask", ctypes.c_uint32),
                ("param", ctypes.c_double * 4), ("values", ctypes.c_void_p)]


SEG_TYPES = {"pde": 0, "dirichlet": 1, "periodic": 2}
SEG_DATA = {"zero": 0, "const": 1, "sin": 2, "values": 3}


class Modified(ctypes.Structure):
    _fields_ = [("hidden", ctypes.c_int32), ("width", ctypes.c_int32), ("harmonics", ctypes.c_int32),
                ("period", ctypes.c_double)]


class Adam(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_double), ("beta1", ctypes.c_double), ("beta2", ctypes.c_double),
                ("eps", ctypes.c_double)]


class Tuning(ctypes.Structure):
    _fields_ = [("dw_splits", ctypes.c_int32), ("fwd_points", ctypes.c_int32), ("bwd_fused", ctypes.c_int32),
                ("bwd_points", ctypes.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc for gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    pp = ctypes.POINTER(ctypes.c_void_p)
    NetP, PdeP = ctypes.POINTER(Net), ctypes.POINTER(Pde)
    lib.pinn_plan_create.argtypes = [NetP, PdeP, i64, i32, ctypes.c_uint32, ctypes.c_size_t, pp]
    lib.pinn_plan_destroy.argtypes = [vp]
    lib.pinn_plan_memory.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]
    lib.pinn_jet_forward.argtypes = [vp, NetP, vp, i64, vp, vp]
    lib.pinn_jet_residual.argtypes = [vp, NetP, PdeP, vp, i64, vp, vp, vp, vp, vp]
    lib.pinn_jet_backward.argtypes = [vp, NetP, PdeP, vp, i64, vp, pp, pp, pp, pp, vp]
    lib.pinn_jet_backward_cot.argtypes = [vp, NetP, PdeP, vp, i64, vp, vp, pp, pp, pp, pp, vp]
    lib.pinn_plan_profile.argtypes = [vp, i32]
    lib.pinn_plan_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    TuneP = ctypes.POINTER(Tuning)
    dptr = ctypes.POINTER(ctypes.c_double)
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.pinn_plan_get_tuning.argtypes = [vp, TuneP]
    lib.pinn_plan_set_tuning.argtypes = [vp, TuneP]
    lib.pinn_plan_autotune.argtypes = [vp, NetP, PdeP, vp, i64, i32, TuneP, dptr, vp]
    lib.pinn_batch_create.argtypes = [i32, NetP, PdeP, i64p, i32, ctypes.c_uint32, pp]
    lib.pinn_batch_destroy.argtypes = [vp]
    lib.pinn_batch_configure.argtypes = [vp, i32, i32]
    lib.pinn_batch_step.argtypes = [vp, NetP, PdeP, pp, i64p, vp, pp, pp, vp]
    lib.pinn_batch_train_step.argtypes = [vp, NetP, PdeP, pp, i64p, vp, pp, pp, pp, pp, pp, pp, ctypes.POINTER(Adam),
                                          vp, vp]
    SegP = ctypes.POINTER(Segment)
    lib.pinn_jet_loss.argtypes = [vp, NetP, PdeP, SegP, i32, vp, i64, vp, vp, vp]
    lib.pinn_jet_loss_backward.argtypes = [vp, NetP, PdeP, SegP, i32, vp, i64, pp, pp, vp]
    lib.pinn_batch_launches.argtypes = [vp, i64p]
    lib.pinn_plan_create_modified.argtypes = [ctypes.POINTER(Modified), PdeP, i64, i32, ctypes.c_uint32, pp]
    lib.pinn_batch_get_config.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.pinn_batch_schedule_classes.argtypes = [vp, ctypes.POINTER(i32), i64, i64p]
    lib.pinn_batch_get_tuning.argtypes = [vp, i32, TuneP]
    lib.pinn_batch_set_tuning.argtypes = [vp, i32, TuneP]
    lib.pinn_batch_profile.argtypes = [vp, i32]
    lib.pinn_batch_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    lib.pinn_tuning_cache_clear.argtypes = []
    lib.pinn_tuning_cache_size.argtypes = [i64p]
    lib.pinn_tuning_cache_save.argtypes = [ctypes.c_char_p]
    lib.pinn_tuning_cache_load.argtypes = [ctypes.c_char_p]
    lib.pinn_batch_autotune.argtypes = [vp, NetP, PdeP, pp, i64p, vp, pp, pp, i32,
                                        ctypes.POINTER(ctypes.c_int32), dptr, vp]
    lib.pinn_graph_capture.argtypes = [vp, NetP, PdeP, vp, i64, vp, vp, pp, pp, pp]
    lib.pinn_graph_launch.argtypes = [vp, vp]
    lib.pinn_graph_destroy.argtypes = [vp]
    lib.pinn_adam_step.argtypes = [i32, ctypes.POINTER(ctypes.c_int32), pp, pp, pp, pp, pp, pp, pp, pp, i64,
                                   ctypes.POINTER(Adam), vp]
    lib.pinn_graph_capture_train.argtypes = [vp, NetP, PdeP, vp, i64, vp, vp, pp, pp, pp, pp, pp, pp,
                                             ctypes.POINTER(Adam), vp, pp]
    lib.pinn_jet_step_noalloc.argtypes = [NetP, PdeP, i32, vp, i64, vp, vp, pp, pp, vp]
    lib.pinn_last_error.restype = ctypes.c_char_p
    lib.pinn_last_error.argtypes = []
    lib.pinn_pde_channels.argtypes = [i32]
    lib.pinn_pde_residuals.argtypes = [i32]
    for name in ("pinn_plan_create", "pinn_plan_destroy", "pinn_plan_memory", "pinn_jet_forward",
                 "pinn_jet_residual", "pinn_jet_backward", "pinn_pde_channels", "pinn_pde_residuals",
                 "pinn_plan_profile", "pinn_plan_profile_read", "pinn_plan_get_tuning", "pinn_plan_set_tuning",
                 "pinn_plan_autotune", "pinn_batch_create", "pinn_batch_destroy", "pinn_batch_configure",
                 "pinn_batch_step", "pinn_batch_autotune", "pinn_graph_capture", "pinn_graph_launch",
                 "pinn_graph_destroy", "pinn_adam_step", "pinn_graph_capture_train", "pinn_jet_step_noalloc",
                 "pinn_jet_backward_cot", "pinn_batch_train_step", "pinn_batch_launches", "pinn_batch_profile",
                 "pinn_batch_profile_read", "pinn_batch_get_tuning", "pinn_batch_set_tuning", "pinn_tuning_cache_clear",
                 "pinn_tuning_cache_size", "pinn_tuning_cache_save", "pinn_tuning_cache_load", "pinn_jet_loss",
                 "pinn_jet_loss_backward", "pinn_batch_get_config", "pinn_plan_create_modified",
                 "pinn_batch_schedule_classes"):
        getattr(lib, name).restype = ctypes.c_int32
    return lib


lib = _load()


def check(status: int) -> None:
    if status != PINN_OK:
        raise PinnError(status, lib.pinn_last_error().decode())


def ptr_array(ptrs):
    arr = (ctypes.c_void_p * len(ptrs))(*[ctypes.c_void_p(p) if p else None for p in ptrs])
    return ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p)), arr
