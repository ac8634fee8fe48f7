"""ctypes declarations of the C ABI in include/nqs.h (argument marshalling only)."""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnqs.so")

NQS_OK = 0
STATUS_NAMES = {0: "NQS_OK", 1: "NQS_ERR_INVALID_ARGUMENT", 2: "NQS_ERR_UNSUPPORTED",
                3: "NQS_ERR_NOT_HERMITIAN", 4: "NQS_ERR_WORKSPACE_TOO_SMALL", 5: "NQS_ERR_HIP",
                6: "NQS_ERR_DEVICE"}
NQS_H_CONSERVES_SPIN_SECTORS = 1
NQS_H_TABLES = 2
NQS_PLAN_DEDUP_ON = 1
NQS_PLAN_DEDUP_OFF = 2
NQS_PLAN_DEDUP_AUTO = 4
NQS_NOALLOC_SCRATCH_BYTES = 256 << 20
NQS_TUNE_FORCE = 1
NQS_TUNE_CACHE_ONLY = 2
NQS_TUNE_MAX_CANDIDATES = 32
NQS_DEV_ZERO_AMPLITUDE = 1
NQS_DEV_ENTRY_OVERFLOW = 2
NQS_DEV_HASH_OVERFLOW = 4
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2, "bf16x3": 3, "bf16w": 4}


class PauliTerms(C.Structure):
    _fields_ = [("n_qubits", C.c_int), ("n_terms", C.c_int64),
                ("x_mask", C.c_void_p), ("z_mask", C.c_void_p),
                ("coeff", C.c_void_p), ("coeff_imag", C.c_void_p),
                ("drop_tol", C.c_double), ("flags", C.c_uint32)]


class NetDesc(C.Structure):
    _fields_ = [("n_qubits", C.c_int), ("n_layers", C.c_int), ("width", C.c_int),
                ("order", C.c_void_p), ("n_up", C.c_int), ("n_dn", C.c_int),
                ("precision", C.c_int), ("phase_mode", C.c_int)]


class Profile(C.Structure):
    _fields_ = [("calls", C.c_int64), ("forward_launches", C.c_int64), ("call_ms", C.c_double),
                ("eloc_ms", C.c_double), ("forward_ms", C.c_double), ("forward_rows", C.c_double),
                ("forward_flops", C.c_double), ("forward_flops_executed", C.c_double)]


class TuneCandidate(C.Structure):
    _fields_ = [("waves_per_block", C.c_int), ("rows_per_block", C.c_int), ("dedup", C.c_int),
                ("chunk_samples", C.c_int64), ("resident", C.c_int), ("ms", C.c_double)]


class TuneReport(C.Structure):
    _fields_ = [("n_candidates", C.c_int), ("chosen", C.c_int), ("from_cache", C.c_int),
                ("probe_samples", C.c_int64), ("cand", TuneCandidate * NQS_TUNE_MAX_CANDIDATES)]


class Instance(C.Structure):
    _fields_ = [("plan", C.c_void_p), ("d_params", C.c_void_p), ("d_samples", C.c_void_p),
                ("d_weights", C.c_void_p), ("B", C.c_int64), ("d_eloc", C.c_void_p),
                ("d_energy", C.c_void_p), ("d_grad", C.c_void_p)]


_P = C.c_void_p
_I64 = C.c_int64
_SZ = C.c_size_t
SIGNATURES = {
    "nqs_status_str": (C.c_char_p, [C.c_int]),
    "nqs_last_error": (_SZ, [C.c_char_p, _SZ]),
    "nqs_version": (C.c_int, []),
    "nqs_source_hash": (C.c_char_p, []),
    "nqs_ctx_create": (C.c_int, [C.c_int, _P, C.POINTER(_P)]),
    "nqs_ctx_set_stream": (C.c_int, [_P, _P]),
    "nqs_ctx_destroy": (None, [_P]),
    "nqs_ham_create": (C.c_int, [C.POINTER(PauliTerms), C.POINTER(_P)]),
    "nqs_ham_info": (C.c_int, [_P, C.POINTER(_I64), C.POINTER(_I64), C.POINTER(_SZ),
                               C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "nqs_ham_upload": (C.c_int, [_P, _P, _P, _SZ]),
    "nqs_ham_export": (C.c_int, [_P, _P, _P, _P, _P, _P]),
    "nqs_ham_table_info": (C.c_int, [_P, C.POINTER(_I64), C.POINTER(_I64)]),
    "nqs_ham_export_tables": (C.c_int, [_P, _P, _P, _P, _P, _P, _P]),
    "nqs_ham_destroy": (None, [_P]),
    "nqs_net_param_count": (C.c_int, [C.POINTER(NetDesc), C.POINTER(_I64)]),
    "nqs_plan_create": (C.c_int, [_P, _P, C.POINTER(NetDesc), _I64, C.c_uint32, _I64, C.POINTER(_P)]),
    "nqs_plan_workspace_size": (C.c_int, [_P, _I64, C.POINTER(_SZ)]),
    "nqs_plan_info": (C.c_int, [_P, C.POINTER(_I64), C.POINTER(_I64), C.POINTER(C.c_int),
                                C.POINTER(_I64)]),
    "nqs_plan_destroy": (None, [_P]),
    "nqs_plan_configure": (C.c_int, [_P, C.c_int, C.c_int, C.c_int, _I64, C.c_int]),
    "nqs_plan_kernel_info": (C.c_int, [_P, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
                                       C.POINTER(C.c_int)]),
    "nqs_plan_autotune": (C.c_int, [_P, _P, _P, _I64, _P, _SZ, C.c_uint32, C.POINTER(TuneReport)]),
    "nqs_tune_db_save": (C.c_int, [C.c_char_p]),
    "nqs_tune_db_load": (C.c_int, [C.c_char_p, C.POINTER(C.c_int)]),
    "nqs_log_psi": (C.c_int, [_P, _P, _P, _I64, _P, _P, _SZ]),
    "nqs_local_energy": (C.c_int, [_P, _P, _P, _I64, _P, _P, _SZ]),
    "nqs_energy_grad": (C.c_int, [_P, _P, _P, _P, _I64, _P, _P, _P, _P, _SZ]),
    "nqs_energy_grad_noalloc": (C.c_int, [_P, _P, _P, _P, _I64, _P, _P, _P, _P]),
    "nqs_multi_workspace_size": (C.c_int, [C.c_int, C.POINTER(Instance), C.POINTER(_SZ)]),
    "nqs_energy_grad_multi": (C.c_int, [C.c_int, C.POINTER(Instance), _P, _SZ]),
    "nqs_sample_workspace_size": (C.c_int, [_P, _I64, C.POINTER(_SZ)]),
    "nqs_sample": (C.c_int, [_P, _P, _I64, C.c_uint64, _I64, _P, _P, _P, _P, _SZ]),
    "nqs_connected": (C.c_int, [_P, _P, _I64, _I64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _SZ]),
    "nqs_reduce_table": (C.c_int, [_P, _I64, _P, _P, _P, _P, _P, _I64, _P, _P, _SZ]),
    "nqs_adam_step": (C.c_int, [_P, _I64, _P, _P, _P, _P, _I64, C.c_double, C.c_double, C.c_double,
                                C.c_double]),
    "nqs_device_status": (C.c_int, [_P, _P, C.POINTER(C.c_uint32)]),
    "nqs_multi_device_status": (C.c_int, [C.c_int, C.POINTER(Instance), _P, C.POINTER(C.c_uint32)]),
    "nqs_plan_profile": (C.c_int, [_P, C.c_int]),
    "nqs_plan_profile_read": (C.c_int, [_P, _P, C.POINTER(Profile)]),
}

_lib = None


class NQSError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__(f"{what}: {STATUS_NAMES.get(status, status)}: {last_error()}")


def load():
    """Load libnqs.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library {LIB_PATH} is missing; build it with "
                          "python -m paper_2208_05637_amd.build")
    lib = C.CDLL(LIB_PATH)
    lib.nqs_source_hash.restype = C.c_char_p
    lib.nqs_source_hash.argtypes = []
    from .build import source_hash
    built, now = lib.nqs_source_hash().decode(), source_hash()
    if built != now:
        raise ImportError(f"HIP library {LIB_PATH} was built from other sources ({built[:12]}) than the "
                          f"tree holds ({now[:12]}); rebuild it with python -m paper_2208_05637_amd.build")
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def last_error():
    lib = load()
    buf = C.create_string_buffer(1024)
    lib.nqs_last_error(buf, 1024)
    return buf.value.decode(errors="replace")


def check(status, what):
    if status != NQS_OK:
        raise NQSError(status, what)
