"""ctypes binding of libffst.so: the C ABI declared in include/ffst.h, one
Python function per C entry point, with the same names. Argument
marshalling only; every step of the transform runs in the HIP kernels of
the library. Fails loudly when the library is missing."""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# FFST_LIBRARY may name another build of the same sources (the host-sanitizer
# build libffst_asan.so); its build id is checked like the default library's.
LIB_PATH = os.environ.get("FFST_LIBRARY") or os.path.join(HERE, "libffst.so")

FFST_OK = 0
FFST_EINVAL = 1
FFST_EUNSUPPORTED = 2
FFST_ENOMEM = 3
FFST_EDEVICE = 4
FFST_EBADPLAN = 5

FFST_SHEARLET_MEYER = 0
FFST_SHEARLET_MEYER_SMOOTH = 1

FFST_KIND_LOWPASS = 0
FFST_KIND_HORIZONTAL = 1
FFST_KIND_VERTICAL = 2
FFST_KIND_SEAM = 3
KIND_NAMES = {FFST_KIND_LOWPASS: "lowpass", FFST_KIND_HORIZONTAL: "horizontal", FFST_KIND_VERTICAL: "vertical",
              FFST_KIND_SEAM: "seam"}

EXPORTED = [
    "ffst_spectra", "ffst_spectra_ex", "ffst_plan_info", "ffst_workspace_size",
    "ffst_get_spectra", "ffst_plan_windows", "ffst_forward", "ffst_forward_noalloc",
    "ffst_adjoint",
    "ffst_inverse", "ffst_adjoint_sign", "ffst_forward_complex", "ffst_adjoint_complex", "ffst_inverse_complex",
    "ffst_scale_shear", "ffst_shearlet_index",
    "ffst_set_tuning", "ffst_get_tuning", "ffst_set_tuning_ex", "ffst_get_tuning_ex", "ffst_tune",
    "ffst_batch_create", "ffst_batch_info", "ffst_batch_class", "ffst_batch_layout",
    "ffst_batch_workspace_size", "ffst_batch_forward", "ffst_batch_adjoint", "ffst_batch_inverse",
    "ffst_batch_tune", "ffst_batch_destroy",
    "ffst_destroy", "ffst_last_error", "ffst_build_id", "ffst_device_bytes", "ffst_profile_enable",
    "ffst_profile_read", "ffst_profile_reset", "ffst_num_kernels", "ffst_kernel_name",
]


class FfstError(RuntimeError):
    def __init__(self, status, where, message):
        super().__init__(f"{where} failed with status {status}: {message}")
        self.status = status


class ffst_tuning(ctypes.Structure):
    _fields_ = [("nparts", ctypes.c_int), ("blocks_per_cu", ctypes.c_int), ("col_values", ctypes.c_int),
                ("row_block", ctypes.c_int), ("fwd_nparts", ctypes.c_int)]


class ffst_options(ctypes.Structure):
    _fields_ = [("max_scale_min", ctypes.c_int), ("shearlet", ctypes.c_int),
                ("complex_shearlets", ctypes.c_int), ("aux_order", ctypes.c_int)]


_lib = None


def check_build_id(lib_id, tree_id):
    """Refuse a library whose compiled-in build id differs from the hash of
    the sources next to it (a stale or foreign libffst.so)."""
    if lib_id != tree_id:
        raise ImportError(f"{LIB_PATH} was built from other sources (library build id {lib_id}, "
                          f"sources {tree_id}): rebuild with `python -m paper_1202_1773_amd.build`")


def load():
    """Load libffst.so (built in-tree by paper_1202_1773_amd.build) after
    checking that it was built from the sources in this tree."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1202_1773_amd.build` (there is no fallback path)")
    from .build import build_id
    lib = ctypes.CDLL(LIB_PATH)
    lib.ffst_build_id.restype = ctypes.c_char_p
    lib.ffst_build_id.argtypes = []
    check_build_id(lib.ffst_build_id().decode(), build_id())
    P = ctypes.c_void_p
    I = ctypes.c_int
    sig = {
        "ffst_spectra": (I, [I, I, I, ctypes.POINTER(P)]),
        "ffst_spectra_ex": (I, [I, I, I, ctypes.POINTER(ffst_options), ctypes.POINTER(P)]),
        "ffst_plan_info": (I, [P, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I)]),
        "ffst_workspace_size": (ctypes.c_size_t, [P, I]),
        "ffst_get_spectra": (I, [P, P, I]),
        "ffst_plan_windows": (I, [P, ctypes.POINTER(I), ctypes.POINTER(I)]),
        "ffst_forward": (I, [P, P, P, I, P, P]),
        "ffst_forward_noalloc": (I, [P, P, P, I, P]),
        "ffst_adjoint": (I, [P, P, P, I, P, P]),
        "ffst_inverse": (I, [P, P, P, I, P, P]),
        "ffst_adjoint_sign": (I, [P, P, P, I, P, P, P]),
        "ffst_forward_complex": (I, [P, P, P, I, P, P]),
        "ffst_adjoint_complex": (I, [P, P, P, I, P, P]),
        "ffst_inverse_complex": (I, [P, P, P, I, P, P]),
        "ffst_scale_shear": (I, [I, I, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I)]),
        "ffst_shearlet_index": (I, [I, I, I, I, ctypes.POINTER(I)]),
        "ffst_set_tuning": (I, [P, I, I]),
        "ffst_get_tuning": (I, [P, ctypes.POINTER(I), ctypes.POINTER(I)]),
        "ffst_set_tuning_ex": (I, [P, ctypes.POINTER(ffst_tuning)]),
        "ffst_get_tuning_ex": (I, [P, ctypes.POINTER(ffst_tuning)]),
        "ffst_tune": (I, [P, P, P, P, I, P, ctypes.c_size_t, P, ctypes.POINTER(ctypes.c_double)]),
        "ffst_batch_create": (I, [I, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I),
                                  ctypes.POINTER(ffst_options), ctypes.POINTER(P)]),
        "ffst_batch_info": (I, [P, ctypes.POINTER(I), ctypes.POINTER(I)]),
        "ffst_batch_class": (I, [P, I, ctypes.POINTER(P), ctypes.POINTER(I)]),
        "ffst_batch_layout": (I, [P, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_longlong),
                                  ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_longlong)]),
        "ffst_batch_workspace_size": (ctypes.c_size_t, [P]),
        "ffst_batch_forward": (I, [P, P, P, P, P]),
        "ffst_batch_adjoint": (I, [P, P, P, P, P]),
        "ffst_batch_inverse": (I, [P, P, P, P, P]),
        "ffst_batch_tune": (I, [P, P, P, P, P, P]),
        "ffst_batch_destroy": (None, [P]),
        "ffst_destroy": (None, [P]),
        "ffst_last_error": (ctypes.c_char_p, []),
        "ffst_build_id": (ctypes.c_char_p, []),
        "ffst_device_bytes": (ctypes.c_size_t, []),
        "ffst_profile_enable": (I, [ctypes.c_uint]),
        "ffst_profile_read": (I, [I, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_longlong)]),
        "ffst_profile_reset": (I, []),
        "ffst_num_kernels": (I, []),
        "ffst_kernel_name": (ctypes.c_char_p, [I]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status, where):
    if status != FFST_OK:
        msg = load().ffst_last_error().decode()
        raise FfstError(status, where, msg)


# ---- thin wrappers with the C names ------------------------------------

def aux_order(aux):
    """C value of the auxiliary-function choice: 3 -> 0 (eq. (v), the default),
    k -> k, "inf" -> -1."""
    if aux == "inf":
        return -1
    if isinstance(aux, int) and 1 <= aux <= 10:
        return 0 if aux == 3 else aux
    raise ValueError("aux must be an int in [1, 10] or 'inf'")


def ffst_spectra(M, N, J=0, max_scale="max", shearlet=FFST_SHEARLET_MEYER, complex_shearlets=False, aux=3):
    """Create a plan and generate its spectra; returns the opaque handle."""
    lib = load()
    out = ctypes.c_void_p()
    opt = ffst_options(1 if max_scale == "min" else 0, int(shearlet), 1 if complex_shearlets else 0,
                       aux_order(aux))
    _check(lib.ffst_spectra_ex(int(M), int(N), int(J), ctypes.byref(opt), ctypes.byref(out)), "ffst_spectra")
    return out.value


def ffst_plan_info(plan):
    vals = [ctypes.c_int() for _ in range(4)]
    _check(load().ffst_plan_info(plan, *[ctypes.byref(v) for v in vals]), "ffst_plan_info")
    return tuple(v.value for v in vals)


def ffst_workspace_size(plan, batch):
    return int(load().ffst_workspace_size(plan, int(batch)))


def ffst_scale_shear(J, i):
    """(kind, j, k) of coefficient plane i of a J-scale transform."""
    kind, j, k = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(load().ffst_scale_shear(int(J), int(i), ctypes.byref(kind), ctypes.byref(j), ctypes.byref(k)),
           "ffst_scale_shear")
    return kind.value, j.value, k.value


def ffst_shearlet_index(J, kind, j, k):
    """Index of the plane (kind, j, k) of a J-scale transform."""
    i = ctypes.c_int()
    _check(load().ffst_shearlet_index(int(J), int(kind), int(j), int(k), ctypes.byref(i)), "ffst_shearlet_index")
    return i.value


def ffst_get_spectra(plan, dst_ptr, full_plane=0):
    _check(load().ffst_get_spectra(plan, ctypes.c_void_p(dst_ptr), int(full_plane)), "ffst_get_spectra")


def ffst_plan_windows(plan, eta):
    lo = (ctypes.c_int * eta)()
    hi = (ctypes.c_int * eta)()
    _check(load().ffst_plan_windows(plan, lo, hi), "ffst_plan_windows")
    return list(lo), list(hi)


def ffst_forward(plan, f_ptr, c_ptr, batch, ws_ptr, stream_ptr):
    _check(load().ffst_forward(plan, ctypes.c_void_p(f_ptr), ctypes.c_void_p(c_ptr), int(batch),
                               ctypes.c_void_p(ws_ptr), ctypes.c_void_p(stream_ptr)), "ffst_forward")


def ffst_forward_noalloc(plan, f_ptr, c_ptr, batch, stream_ptr):
    _check(load().ffst_forward_noalloc(plan, ctypes.c_void_p(f_ptr), ctypes.c_void_p(c_ptr), int(batch),
                                       ctypes.c_void_p(stream_ptr)), "ffst_forward_noalloc")



def ffst_adjoint(plan, c_ptr, f_ptr, batch, ws_ptr, stream_ptr):
    _check(load().ffst_adjoint(plan, ctypes.c_void_p(c_ptr), ctypes.c_void_p(f_ptr), int(batch),
                               ctypes.c_void_p(ws_ptr), ctypes.c_void_p(stream_ptr)), "ffst_adjoint")


def ffst_adjoint_sign(plan, c_ptr, f_ptr, batch, scale_ptr, ws_ptr, stream_ptr):
    _check(load().ffst_adjoint_sign(plan, ctypes.c_void_p(c_ptr), ctypes.c_void_p(f_ptr), int(batch),
                                    ctypes.c_void_p(scale_ptr), ctypes.c_void_p(ws_ptr), ctypes.c_void_p(stream_ptr)),
           "ffst_adjoint_sign")


def ffst_inverse(plan, c_ptr, f_ptr, batch, ws_ptr, stream_ptr):
    _check(load().ffst_inverse(plan, ctypes.c_void_p(c_ptr), ctypes.c_void_p(f_ptr), int(batch),
                               ctypes.c_void_p(ws_ptr), ctypes.c_void_p(stream_ptr)), "ffst_inverse")


def ffst_forward_complex(plan, f_ptr, c_ptr, batch, ws_ptr, stream_ptr):
    _check(load().ffst_forward_complex(plan, ctypes.c_void_p(f_ptr), ctypes.c_void_p(c_ptr), int(batch),
                                       ctypes.c_void_p(ws_ptr), ctypes.c_void_p(stream_ptr)), "ffst_forward_complex")


def ffst_adjoint_complex(plan, c_ptr, f_ptr, batch, ws_ptr, stream_ptr):
    _check(load().ffst_adjoint_complex(plan, ctypes.c_void_p(c_ptr), ctypes.c_void_p(f_ptr), int(batch),
                                       ctypes.c_void_p(ws_ptr), ctypes.c_void_p(stream_ptr)), "ffst_adjoint_complex")


def ffst_inverse_complex(plan, c_ptr, f_ptr, batch, ws_ptr, stream_ptr):
    _check(load().ffst_inverse_complex(plan, ctypes.c_void_p(c_ptr), ctypes.c_void_p(f_ptr), int(batch),
                                       ctypes.c_void_p(ws_ptr), ctypes.c_void_p(stream_ptr)), "ffst_inverse_complex")


def ffst_set_tuning(plan, nparts, blocks_per_cu):
    _check(load().ffst_set_tuning(plan, int(nparts), int(blocks_per_cu)), "ffst_set_tuning")


def ffst_get_tuning(plan):
    n = ctypes.c_int()
    b = ctypes.c_int()
    _check(load().ffst_get_tuning(plan, ctypes.byref(n), ctypes.byref(b)), "ffst_get_tuning")
    return n.value, b.value


def ffst_set_tuning_ex(plan, nparts=0, blocks_per_cu=0, col_values=0, row_block=0, fwd_nparts=0):
    t = ffst_tuning(int(nparts), int(blocks_per_cu), int(col_values), int(row_block), int(fwd_nparts))
    _check(load().ffst_set_tuning_ex(plan, ctypes.byref(t)), "ffst_set_tuning_ex")


def ffst_get_tuning_ex(plan):
    """dict(nparts, blocks_per_cu, col_values, row_block, fwd_nparts) of a plan."""
    t = ffst_tuning()
    _check(load().ffst_get_tuning_ex(plan, ctypes.byref(t)), "ffst_get_tuning_ex")
    return {k: getattr(t, k) for k, _ in ffst_tuning._fields_}


def ffst_tune(plan, f_ptr, c_ptr, out_ptr, batch, ws_ptr, ws_size, stream_ptr):
    best = ctypes.c_double()
    _check(load().ffst_tune(plan, ctypes.c_void_p(f_ptr), ctypes.c_void_p(c_ptr), ctypes.c_void_p(out_ptr),
                            int(batch), ctypes.c_void_p(ws_ptr), ctypes.c_size_t(ws_size),
                            ctypes.c_void_p(stream_ptr), ctypes.byref(best)), "ffst_tune")
    return best.value


def ffst_batch_create(Ms, Ns, Js, max_scale="max", shearlet=FFST_SHEARLET_MEYER, complex_shearlets=False, aux=3):
    n = len(Ms)
    arr = ctypes.c_int * n
    opt = ffst_options(1 if max_scale == "min" else 0, int(shearlet), 1 if complex_shearlets else 0,
                       aux_order(aux))
    out = ctypes.c_void_p()
    _check(load().ffst_batch_create(n, arr(*Ms), arr(*Ns), arr(*Js), ctypes.byref(opt), ctypes.byref(out)),
           "ffst_batch_create")
    return out.value


def ffst_batch_info(batch):
    c = ctypes.c_int()
    k = ctypes.c_int()
    _check(load().ffst_batch_info(batch, ctypes.byref(c), ctypes.byref(k)), "ffst_batch_info")
    return c.value, k.value


def ffst_batch_class(batch, cls):
    p = ctypes.c_void_p()
    n = ctypes.c_int()
    _check(load().ffst_batch_class(batch, int(cls), ctypes.byref(p), ctypes.byref(n)), "ffst_batch_class")
    return p.value, n.value


def ffst_batch_layout(batch, count):
    io = (ctypes.c_longlong * count)()
    co = (ctypes.c_longlong * count)()
    it = ctypes.c_longlong()
    ct = ctypes.c_longlong()
    _check(load().ffst_batch_layout(batch, io, co, ctypes.byref(it), ctypes.byref(ct)), "ffst_batch_layout")
    return list(io), list(co), it.value, ct.value


def ffst_batch_workspace_size(batch):
    return int(load().ffst_batch_workspace_size(batch))


def ffst_batch_forward(batch, f_ptr, c_ptr, ws_ptr, stream_ptr):
    _check(load().ffst_batch_forward(batch, ctypes.c_void_p(f_ptr), ctypes.c_void_p(c_ptr), ctypes.c_void_p(ws_ptr),
                                     ctypes.c_void_p(stream_ptr)), "ffst_batch_forward")


def ffst_batch_adjoint(batch, c_ptr, f_ptr, ws_ptr, stream_ptr):
    _check(load().ffst_batch_adjoint(batch, ctypes.c_void_p(c_ptr), ctypes.c_void_p(f_ptr), ctypes.c_void_p(ws_ptr),
                                     ctypes.c_void_p(stream_ptr)), "ffst_batch_adjoint")


def ffst_batch_inverse(batch, c_ptr, f_ptr, ws_ptr, stream_ptr):
    _check(load().ffst_batch_inverse(batch, ctypes.c_void_p(c_ptr), ctypes.c_void_p(f_ptr), ctypes.c_void_p(ws_ptr),
                                     ctypes.c_void_p(stream_ptr)), "ffst_batch_inverse")


def ffst_batch_tune(batch, f_ptr, c_ptr, out_ptr, ws_ptr, stream_ptr):
    _check(load().ffst_batch_tune(batch, ctypes.c_void_p(f_ptr), ctypes.c_void_p(c_ptr), ctypes.c_void_p(out_ptr),
                                  ctypes.c_void_p(ws_ptr), ctypes.c_void_p(stream_ptr)), "ffst_batch_tune")


def ffst_batch_destroy(batch):
    if batch:
        load().ffst_batch_destroy(batch)


def ffst_destroy(plan):
    if plan:
        load().ffst_destroy(plan)


def ffst_last_error():
    return load().ffst_last_error().decode()


def ffst_build_id():
    return load().ffst_build_id().decode()


def ffst_device_bytes():
    return int(load().ffst_device_bytes())


def ffst_profile_enable(mask):
    _check(load().ffst_profile_enable(ctypes.c_uint(mask)), "ffst_profile_enable")


def ffst_profile_read(kernel_id):
    ms = ctypes.c_double()
    n = ctypes.c_longlong()
    _check(load().ffst_profile_read(int(kernel_id), ctypes.byref(ms), ctypes.byref(n)), "ffst_profile_read")
    return ms.value, n.value


def ffst_profile_reset():
    _check(load().ffst_profile_reset(), "ffst_profile_reset")


def ffst_num_kernels():
    return int(load().ffst_num_kernels())


def ffst_kernel_name(kernel_id):
    return load().ffst_kernel_name(int(kernel_id)).decode()
