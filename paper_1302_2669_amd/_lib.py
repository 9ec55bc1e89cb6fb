"""ctypes binding of libmcmcdec.so (C-ABI in include/mcmcdec.h).

Argument marshalling only: every step of the decode runs in the library's HIP
kernels.  torch is used for device memory and streams.  If the shared library
is missing this module raises; there is no fallback path.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmcmcdec.so")

MCMC_OK = 0
STATUS = {0: "MCMC_OK", -1: "MCMC_EINVAL", -2: "MCMC_ERANGE", -3: "MCMC_ENOMEM",
          -4: "MCMC_EDEVICE", -5: "MCMC_EWORKSPACE"}
MCMC_L_MIN, MCMC_L_MAX = 2, 25
MCMC_TEMPS_MAX = 64
MCMC_TRACE, MCMC_RESUME, MCMC_RANDOM_SCAN = 1, 2, 4
MCMC_INIT_CANONICAL, MCMC_INIT_MATCHING, MCMC_INIT_MWPM = 0, 1, 2
MCMC_NOISE_DEPOLARIZING, MCMC_NOISE_BITPHASE = 0, 1
MCMC_CNN_BATCH_MAX = 1 << 24
MCMC_ROUNDS_MAX = 64


class McmcError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)} ({_lib().mcmc_strerror(status).decode()})")


class Params(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int32),
        ("n_temps", ctypes.c_int32),
        ("chains", ctypes.c_int32),
        ("burn", ctypes.c_int32),
        ("sweeps", ctypes.c_int32),
        ("sweep_begin", ctypes.c_int32),
        ("p", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("flags", ctypes.c_uint32),
        ("init", ctypes.c_uint32),
        ("noise", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
        ("beta_scale", ctypes.c_double),
    ]


class Item(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int32),
        ("sweeps", ctypes.c_int32),
        ("burn", ctypes.c_int32),
        ("chains", ctypes.c_int32),
        ("n_temps", ctypes.c_int32),
        ("syndrome_id", ctypes.c_uint32),
        ("p", ctypes.c_double),
        ("syn_offset", ctypes.c_int64),
        ("corr_offset", ctypes.c_int64),
        ("noise", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
        ("beta_scale", ctypes.c_double),
    ]


class SpaceTimeParams(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int32),
        ("rounds", ctypes.c_int32),
        ("chains", ctypes.c_int32),
        ("burn", ctypes.c_int32),
        ("sweeps", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("p", ctypes.c_double),
        ("p_m", ctypes.c_double),
        ("seed", ctypes.c_uint64),
    ]


class Tuning(ctypes.Structure):
    _fields_ = [
        ("wg_narrow", ctypes.c_int32),
        ("occ_narrow", ctypes.c_int32),
        ("wg_wide", ctypes.c_int32),
        ("occ_wide", ctypes.c_int32),
        ("concurrent", ctypes.c_int32),
        ("pair_small", ctypes.c_int32),
    ]


class GateConfig(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int32),
        ("n_temps", ctypes.c_int32),
        ("chains", ctypes.c_int32),
        ("burn", ctypes.c_int32),
        ("sweeps_short", ctypes.c_int32),
        ("sweeps_full", ctypes.c_int32),
        ("p", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("init", ctypes.c_uint32),
        ("threshold", ctypes.c_float),
        ("escalate", ctypes.c_float),
        ("max_batch", ctypes.c_int64),
        ("class_route", ctypes.c_int32),
    ]


class TrainConfig(ctypes.Structure):
    _fields_ = [
        ("lr", ctypes.c_float),
        ("lr_final", ctypes.c_float),
        ("beta1", ctypes.c_float),
        ("beta2", ctypes.c_float),
        ("eps", ctypes.c_float),
        ("budget_weight", ctypes.c_float),
        ("batch", ctypes.c_int64),
        ("total_steps", ctypes.c_int64),
        ("seed", ctypes.c_uint64),
    ]


_P = ctypes.c_void_p
_I32, _I64, _U32, _U64, _D, _SZ = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                   ctypes.c_uint64, ctypes.c_double, ctypes.c_size_t)
_PI32 = ctypes.POINTER(ctypes.c_int32)
_PSZ = ctypes.POINTER(ctypes.c_size_t)
_PPRM = ctypes.POINTER(Params)

_SIGNATURES = {
    "mcmc_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "mcmc_abi_version": (_I32, []),
    "mcmc_geometry": (ctypes.c_int, [_I32, _PI32, _PI32]),
    "mcmc_lattice": (ctypes.c_int, [_I32, _P, _P, _P]),
    "mcmc_acceptance_table": (ctypes.c_int, [_D, _I32, _P]),
    "mcmc_params_table": (ctypes.c_int, [_PPRM, _P]),
    "mcmc_workspace_size": (ctypes.c_int, [_PPRM, _I64, _PSZ]),
    "mcmc_chain_state_size": (ctypes.c_int, [_PPRM, _I64, _PSZ]),
    "mcmc_decode_batch": (ctypes.c_int, [_P, _P, _I64, _PPRM, _P, _P, _P, _P, _P, _P, _P, _P,
                                         _P, _SZ, _P]),
    "mcmc_decode_batch_noalloc": (ctypes.c_int, [_P, _P, _I64, _PPRM, _P, _P, _P, _P, _P, _P,
                                                 _P, _P, _P]),
    "mcmc_init_representatives": (ctypes.c_int, [_I32, _U32, _P, _I64, _P, _P]),
    "mcmc_start_weights": (ctypes.c_int, [_I32, _U32, _P, _I64, _P, _P]),
    "mcmc_unpack_chain_state": (ctypes.c_int, [_PPRM, _I64, _P, _P, _P, _P]),
    "mcmc_sample_errors": (ctypes.c_int, [_I32, _D, _U64, _P, _U32, _I64, _P, _P, _P, _P]),
    "mcmc_sample_errors_model": (ctypes.c_int,
                                 [_I32, _U32, _D, _U64, _P, _U32, _I64, _P, _P, _P, _P]),
    "mcmc_plan_create": (ctypes.c_int, [ctypes.POINTER(Item), _I64, _U64, _U32,
                                        ctypes.POINTER(_P)]),
    "mcmc_plan_destroy": (ctypes.c_int, [_P]),
    "mcmc_plan_rebuild": (ctypes.c_int, [_P, ctypes.POINTER(Item), _I64]),
    "mcmc_plan_info": (ctypes.c_int, [_P, ctypes.POINTER(_I64), _PSZ, ctypes.POINTER(_I64)]),
    "mcmc_plan_get_tuning": (ctypes.c_int, [_P, ctypes.POINTER(Tuning)]),
    "mcmc_plan_set_tuning": (ctypes.c_int, [_P, ctypes.POINTER(Tuning)]),
    "mcmc_plan_execute": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _P, _P, _SZ, _P]),
    "mcmc_plan_graph_launch": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _P, _P, _SZ, _P]),
    "mcmc_plan_sample": (ctypes.c_int, [_P, _U64, _P, _P, _P]),
    "mcmc_plan_autotune": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _P, _P, _SZ, _P,
                                          ctypes.c_char_p, ctypes.POINTER(Tuning)]),
    "mcmc_cnn_param_count": (ctypes.c_int, [_I32, ctypes.POINTER(_I64)]),
    "mcmc_cnn_workspace_size": (ctypes.c_int, [_I32, _I64, _PSZ]),
    "mcmc_cnn_workspace_offsets": (ctypes.c_int, [_I32, _I64, ctypes.POINTER(_I64)]),
    "mcmc_cnn_forward": (ctypes.c_int, [_I32, _I64, _P, _P, _P, _P, _P, _SZ, _P]),
    "mcmc_cnn_infer_workspace_size": (ctypes.c_int, [_I32, _PSZ]),
    "mcmc_cnn_infer": (ctypes.c_int, [_I32, _I64, _P, _P, _P, _P, _P, _SZ, _P]),
    "mcmc_cnn_backward": (ctypes.c_int, [_I32, _I64, _P, _P, _P, _P, ctypes.c_float, _P, _P, _P,
                                         _SZ, _P]),
    "mcmc_cnn_step": (ctypes.c_int, [_I64, _I64, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                     ctypes.c_float, _P, _P, _P, _P, _P]),
    "mcmc_cnn_gate": (ctypes.c_int, [_I64, _P, ctypes.c_float, _I32, _P, _P, _P, _P]),
    "mcmc_cnn_init": (ctypes.c_int, [_I32, _U64, _P, _P]),
    "mcmc_gate_budget_labels": (ctypes.c_int, [_I64, _P, _P, _P, _P, _P]),
    "mcmc_gate_fit_gap_table": (ctypes.c_int, [_I64, _P, _P, _P, ctypes.c_double, _I32, _P, _P]),
    "mcmc_gate_relative_targets": (ctypes.c_int, [_I64, _P, _P, _P, _P]),
    "mcmc_cnn_permutation": (ctypes.c_int, [_I64, _U64, _U32, _P, _P]),
    "mcmc_cnn_train_workspace_size": (ctypes.c_int, [_I32, _I64, _I64, _PSZ]),
    "mcmc_cnn_train_epoch": (ctypes.c_int, [_I32, _I64, ctypes.POINTER(TrainConfig), _U32,
                                            ctypes.POINTER(ctypes.c_int64), _P, _P, _P, _P, _P,
                                            _P, _P, _P, _P, _SZ, _P]),
    "mcmc_gated_create": (ctypes.c_int, [ctypes.POINTER(GateConfig), ctypes.POINTER(_P)]),
    "mcmc_gated_destroy": (ctypes.c_int, [_P]),
    "mcmc_gated_workspace_size": (ctypes.c_int, [_P, _PSZ]),
    "mcmc_gated_plan": (ctypes.c_int, [_P, ctypes.POINTER(_P)]),
    "mcmc_gated_set_gap_table": (ctypes.c_int, [_P, _P]),
    "mcmc_gated_decode": (ctypes.c_int, [_P, _P, _P, _P, _P, _I64, _P, _P, _P, _P,
                                         ctypes.POINTER(_I64), _P, _SZ, _P]),
    "mcmc_spacetime_workspace_size": (ctypes.c_int, [ctypes.POINTER(SpaceTimeParams), _I64, _PSZ]),
    "mcmc_spacetime_tables": (ctypes.c_int, [ctypes.POINTER(SpaceTimeParams), _P, _P, _P, _P]),
    "mcmc_decode_spacetime": (ctypes.c_int, [_P, _P, _I64, ctypes.POINTER(SpaceTimeParams), _P,
                                             _P, _P, _P, _P, _P, _P, _P, _P, _SZ, _P]),
    "mcmc_sample_spacetime": (ctypes.c_int, [_I32, _I32, _D, _D, _U64, _U32, _I64, _P, _P, _P]),
}

_handle = None


# layout of the structures below (mcmc_params, mcmc_item, ...)
ABI_VERSION = 0x00010500


def _lib():
    global _handle
    if _handle is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1302_2669_amd.build` "
                "(the decoder has no CPU fallback)")
        h = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        if h.mcmc_abi_version() != ABI_VERSION:
            raise ImportError(f"{LIB_PATH} has ABI {h.mcmc_abi_version():#010x}, this binding "
                              f"expects {ABI_VERSION:#010x}: rebuild the library")
        _handle = h
    return _handle


def exported_symbols():
    return sorted(_SIGNATURES)


def check(status, where):
    if status != MCMC_OK:
        raise McmcError(status, where)
