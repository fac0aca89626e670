"""Python binding of the C ABI in include/kifmm_mi355x.h (argument marshalling only).

Every function here forwards to the entry point of the same name in
``libkifmm_mi355x.so``; no step of the FMM runs in Python.  Importing works
without the library; the first call raises ``RuntimeError`` if it is not built
(``python -m paper_2604_19243_amd.build``).  Device buffers are passed as torch
CUDA (HIP) tensors or raw integer addresses; PyTorch provides device memory and
streams only.
"""

import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libkifmm_mi355x.so")

KIFMM_OK = 0
KIFMM_E_INVALID = -1
KIFMM_E_NOMEM = -2
KIFMM_E_DEVICE = -3
KIFMM_E_NUMERIC = -4
KIFMM_E_STATE = -5
KIFMM_MAX_DEPTH = 10

KIFMM_POTENTIAL = 1
KIFMM_GRADIENT = 2
KIFMM_POT = KIFMM_POTENTIAL
KIFMM_GRAD = KIFMM_GRADIENT
KIFMM_M2L_BF16X3 = 4
KIFMM_SERIAL = 8
KIFMM_M2L_BF16X6 = 16
KIFMM_VJP = 32
KIFMM_M2L_BLOCKED = 64
KIFMM_M2L_GATHER = 128
KIFMM_UPPER_STREAM = 256
KIFMM_NO_UPPER_STREAM = 512
KIFMM_LEAF_THREADS_256 = 1024
KIFMM_LEAF_THREADS_320 = 2048
KIFMM_LEAF_QUEUE = 4096
KIFMM_LEAF_BLOCKS = 8192
KIFMM_NO_AUTOTUNE = 16384
KIFMM_N_STATS = 29
KIFMM_NOALLOC_MAX_POINTS = 2097152

ALPHA_INNER = 1.05
ALPHA_OUTER = 2.95

(KIFMM_OP_SURFACE, KIFMM_OP_UC2E, KIFMM_OP_DC2E, KIFMM_OP_M2M, KIFMM_OP_L2L, KIFMM_OP_M2L_U, KIFMM_OP_M2L_V,
 KIFMM_OP_M2L_CORE, KIFMM_OP_M2L_OFFSET, KIFMM_OP_M2L_POST) = range(10)

STAGES = ["permute", "p2m", "uc2e", "m2m", "compress", "m2l", "l2l", "p2p", "l2p"]
KIFMM_N_STAGES = len(STAGES)


class KifmmError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"kifmm status {status}: {message}")
        self.status = status


class TreeStats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nonempty_leaves", ctypes.c_int64), ("max_leaf", ctypes.c_int64),
                ("nonempty_boxes", ctypes.c_int64 * 16), ("center", ctypes.c_double * 3),
                ("half_width", ctypes.c_double), ("depth", ctypes.c_int)]


class OpsInfo(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("n_surface", ctypes.c_int32), ("rank_m2l", ctypes.c_int32),
                ("rank_c2e", ctypes.c_int32), ("n_m2l_offsets", ctypes.c_int32), ("eps_pinv", ctypes.c_double),
                ("eps_svd", ctypes.c_double), ("alpha_inner", ctypes.c_double), ("alpha_outer", ctypes.c_double)]


_lib = None
_VP = ctypes.c_void_p


def library():
    """The loaded C library (raises RuntimeError when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                           "python -m paper_2604_19243_amd.build")
    # The library and torch must share one HIP runtime (torch's tensors and streams are
    # passed in).  Both name it libamdhip64.so.7, and the first one loaded is the one the
    # process keeps: torch's is loaded first, so that torch keeps the runtime it was built
    # for and the library binds to it.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "kifmm_abi_version": (ctypes.c_int, []),
        "kifmm_last_error": (ctypes.c_char_p, []),
        "kifmm_tree_build": (ctypes.c_int, [_VP, ctypes.c_int64, ctypes.c_int, _VP, _VP, ctypes.POINTER(_VP)]),
        "kifmm_tree_build_host": (ctypes.c_int, [_VP, ctypes.c_int64, ctypes.c_int, _VP, ctypes.POINTER(_VP)]),
        "kifmm_tree_stats_get": (ctypes.c_int, [_VP, ctypes.POINTER(TreeStats)]),
        "kifmm_tree_get_order": (ctypes.c_int, [_VP, _VP]),
        "kifmm_tree_get_leaf_coords": (ctypes.c_int, [_VP, _VP]),
        "kifmm_tree_destroy": (ctypes.c_int, [_VP]),
        "kifmm_ops_precompute": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                                ctypes.c_double, ctypes.POINTER(_VP)]),
        "kifmm_ops_get_info": (ctypes.c_int, [_VP, ctypes.POINTER(OpsInfo)]),
        "kifmm_ops_get_matrix": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, _VP, ctypes.c_int64]),
        "kifmm_ops_destroy": (ctypes.c_int, [_VP]),
        "kifmm_plan_create": (ctypes.c_int, [_VP, _VP, ctypes.c_int, ctypes.c_uint, _VP, ctypes.POINTER(_VP)]),
        "kifmm_plan_workspace_bytes": (ctypes.c_int, [_VP, _VP, ctypes.c_int, ctypes.c_uint, _VP]),
        "kifmm_set_device_memory_limit": (ctypes.c_int, [ctypes.c_int64]),
        "kifmm_evaluate": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP]),
        "kifmm_evaluate_vjp": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP, _VP]),
        "kifmm_evaluate_vjp_noalloc": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP, _VP]),
        "kifmm_plan_destroy": (ctypes.c_int, [_VP]),
        "kifmm_plan_set_timing": (ctypes.c_int, [_VP, ctypes.c_int]),
        "kifmm_plan_get_stage_times": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int]),
        "kifmm_plan_get_stats": (ctypes.c_int, [_VP, _VP, ctypes.c_int]),
        "kifmm_plan_read_density": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, _VP, ctypes.c_int64]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status):
    if status != KIFMM_OK:
        msg = library().kifmm_last_error()
        raise KifmmError(status, msg.decode() if msg else "")


def _host_ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def _dev_ptr(x):
    """Device address of a torch tensor or an integer address (None -> NULL)."""
    if x is None:
        return None
    if isinstance(x, int):
        return ctypes.c_void_p(x)
    if not x.is_contiguous():
        raise ValueError("device buffers must be contiguous")
    return ctypes.c_void_p(x.data_ptr())


# ----------------------------------------------------------------------- C names

def kifmm_abi_version():
    return library().kifmm_abi_version()


def _stream(stream):
    return None if stream is None else ctypes.c_void_p(int(stream))


def _cube(cube):
    return None if cube is None else np.ascontiguousarray(cube, dtype=np.float64)


def kifmm_tree_build(xyz, depth, cube=None, stream=None):
    """xyz: device [n,3] float32 tensor (or (address, n)); cube: (cx, cy, cz, half) or None; stream: int or None."""
    if isinstance(xyz, tuple):
        ptr, n = ctypes.c_void_p(int(xyz[0])), int(xyz[1])
    else:
        if xyz.ndim != 2 or xyz.shape[1] != 3:
            raise ValueError("xyz must have shape [n, 3]")
        ptr, n = _dev_ptr(xyz), int(xyz.shape[0])
    c = _cube(cube)
    out = ctypes.c_void_p()
    _check(library().kifmm_tree_build(ptr, n, int(depth), None if c is None else _host_ptr(c), _stream(stream),
                                      ctypes.byref(out)))
    return out


def kifmm_tree_build_host(xyz, depth, cube=None):
    """xyz: host [n,3] float32 array; cube: (cx, cy, cz, half) or None. Returns a tree handle."""
    x = np.ascontiguousarray(xyz, dtype=np.float32)
    if x.ndim != 2 or x.shape[1] != 3:
        raise ValueError("xyz must have shape [n, 3]")
    c = _cube(cube)
    out = ctypes.c_void_p()
    _check(library().kifmm_tree_build_host(_host_ptr(x), x.shape[0], int(depth), None if c is None else _host_ptr(c),
                                           ctypes.byref(out)))
    return out


def kifmm_tree_stats_get(tree):
    st = TreeStats()
    _check(library().kifmm_tree_stats_get(tree, ctypes.byref(st)))
    return {"n": st.n, "depth": st.depth, "max_leaf": st.max_leaf, "nonempty_leaves": st.nonempty_leaves,
            "nonempty_boxes": [st.nonempty_boxes[l] for l in range(st.depth + 1)],
            "center": tuple(st.center), "half_width": st.half_width}


def kifmm_tree_get_order(tree, n):
    out = np.empty(n, dtype=np.int64)
    _check(library().kifmm_tree_get_order(tree, _host_ptr(out)))
    return out


def kifmm_tree_get_leaf_coords(tree, n):
    out = np.empty((n, 3), dtype=np.int32)
    _check(library().kifmm_tree_get_leaf_coords(tree, _host_ptr(out)))
    return out


def kifmm_tree_destroy(tree):
    _check(library().kifmm_tree_destroy(tree))


def kifmm_ops_precompute(p, alpha_inner=ALPHA_INNER, alpha_outer=ALPHA_OUTER, eps_pinv=1e-7, eps_svd=1e-6):
    """eps_svd in (0, 1): compression cutoff; a negative integer -k gives the rank k."""
    out = ctypes.c_void_p()
    _check(library().kifmm_ops_precompute(int(p), float(alpha_inner), float(alpha_outer), float(eps_pinv),
                                          float(eps_svd), ctypes.byref(out)))
    return out


def kifmm_ops_get_info(ops):
    info = OpsInfo()
    _check(library().kifmm_ops_get_info(ops, ctypes.byref(info)))
    return {f: getattr(info, f) for f, _ in OpsInfo._fields_}


def kifmm_ops_get_matrix(ops, which, index, shape):
    out = np.empty(shape, dtype=np.float64)
    _check(library().kifmm_ops_get_matrix(ops, int(which), int(index), _host_ptr(out), out.size))
    return out


def kifmm_ops_destroy(ops):
    _check(library().kifmm_ops_destroy(ops))


def kifmm_plan_create(tree, ops, nrhs=1, flags=KIFMM_POTENTIAL | KIFMM_GRADIENT, stream=None):
    out = ctypes.c_void_p()
    _check(library().kifmm_plan_create(tree, ops, int(nrhs), int(flags), _stream(stream), ctypes.byref(out)))
    return out


def kifmm_plan_workspace_bytes(tree, ops, nrhs=1, flags=KIFMM_POTENTIAL | KIFMM_GRADIENT):
    out = ctypes.c_int64()
    _check(library().kifmm_plan_workspace_bytes(tree, ops, int(nrhs), int(flags), ctypes.byref(out)))
    return out.value


def kifmm_set_device_memory_limit(nbytes):
    _check(library().kifmm_set_device_memory_limit(int(nbytes)))


def kifmm_evaluate(plan, charges, potential=None, gradient=None, stream=None):
    """charges [n] (device), potential [n] / gradient [n,3] device outputs or None; stream: int handle or None."""
    _check(library().kifmm_evaluate(plan, _dev_ptr(charges), _dev_ptr(potential), _dev_ptr(gradient), _stream(stream)))


def kifmm_evaluate_vjp(plan, charges, weights, field=None, grad_charges=None, grad_points=None, stream=None):
    """Vector-Jacobian product of the evaluate for L = sum_i w_i f_i (device arrays; see the header)."""
    _check(library().kifmm_evaluate_vjp(plan, _dev_ptr(charges), _dev_ptr(weights), _dev_ptr(field),
                                        _dev_ptr(grad_charges), _dev_ptr(grad_points), _stream(stream)))


def kifmm_evaluate_vjp_noalloc(plan, charges, weights, field=None, grad_charges=None, grad_points=None,
                               stream=None):
    """kifmm_evaluate_vjp with its workspace in the library's static device array (no allocation)."""
    _check(library().kifmm_evaluate_vjp_noalloc(plan, _dev_ptr(charges), _dev_ptr(weights), _dev_ptr(field),
                                                _dev_ptr(grad_charges), _dev_ptr(grad_points), _stream(stream)))


def kifmm_plan_destroy(plan):
    _check(library().kifmm_plan_destroy(plan))


def kifmm_plan_set_timing(plan, enable):
    _check(library().kifmm_plan_set_timing(plan, int(bool(enable))))


def kifmm_plan_get_stage_times(plan, reset=True):
    ms = np.zeros(KIFMM_N_STAGES, dtype=np.float64)
    counts = np.zeros(KIFMM_N_STAGES, dtype=np.int64)
    _check(library().kifmm_plan_get_stage_times(plan, _host_ptr(ms), _host_ptr(counts), int(bool(reset))))
    return {s: (float(ms[i]), int(counts[i])) for i, s in enumerate(STAGES)}


STATS_KEYS = ["p2p_pairs", "m2l_pairs", "leaf_slots", "m2l_targets", "k", "n", "nrhs", "m2l_form",
              "m2l_stage_pairs", "upper_stream", "m2l_lds_slab", "p2p_threads", "leaf_queue", "leaf_tiles",
              "tune_us_single_256", "tune_us_single_320", "tune_us_upper_256", "tune_us_upper_320",
              "tune_us_m2l_blocked", "tune_us_m2l_gathered", "tune_us_leaf_blocks", "tune_us_leaf_queue",
              "m2l_pairs_leaf", "tuned_from_cache", "queue_per_cu", "tune_us_slab_24", "tune_us_slab_32",
              "tune_us_slab_40", "tune_us_slab_48"]


def kifmm_plan_get_stats(plan):
    out = np.zeros(KIFMM_N_STATS, dtype=np.int64)
    _check(library().kifmm_plan_get_stats(plan, _host_ptr(out), KIFMM_N_STATS))
    return dict(zip(STATS_KEYS, (int(v) for v in out)))


def kifmm_plan_read_density(plan, kind, level, boxes, n):
    out = np.empty((boxes, n), dtype=np.float32)
    _check(library().kifmm_plan_read_density(plan, int(kind), int(level), _host_ptr(out), out.size))
    return out


# ------------------------------------------------------------------ convenience

class FMM:
    """Tree + operators + plan for one point set on one device (owns the three handles)."""

    def __init__(self, points, depth, p, cube=None, eps_pinv=1e-7, eps_svd=1e-6, rank=0,
                 flags=KIFMM_POTENTIAL | KIFMM_GRADIENT, nrhs=1, stream=None, alpha_inner=ALPHA_INNER,
                 alpha_outer=ALPHA_OUTER):
        """points: host [n,3] float32 array, or a device tensor (tree built from device memory)."""
        self.n = int(points.shape[0])
        if isinstance(points, np.ndarray):
            self.tree = kifmm_tree_build_host(points, depth, cube)
        else:
            self.tree = kifmm_tree_build(points, depth, cube, stream)
        self.ops = kifmm_ops_precompute(p, alpha_inner, alpha_outer, eps_pinv, -float(rank) if rank else eps_svd)
        self.plan = kifmm_plan_create(self.tree, self.ops, nrhs, flags, stream)

    def evaluate(self, charges, potential=None, gradient=None, stream=None):
        kifmm_evaluate(self.plan, charges, potential, gradient, stream)

    def vjp(self, charges, weights, field=None, grad_charges=None, grad_points=None, stream=None):
        kifmm_evaluate_vjp(self.plan, charges, weights, field, grad_charges, grad_points, stream)

    def close(self):
        for attr, fn in (("plan", kifmm_plan_destroy), ("ops", kifmm_ops_destroy), ("tree", kifmm_tree_destroy)):
            h = getattr(self, attr, None)
            if h is not None:
                fn(h)
                setattr(self, attr, None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
