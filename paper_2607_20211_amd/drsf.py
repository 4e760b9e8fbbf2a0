"""ctypes binding of libdrsf.so (include/drsf.h).

Argument marshalling only: every step of a batch update runs in the HIP
kernels of libdrsf.so.  Inputs may be numpy arrays (host memory) or torch
tensors on the GPU (device memory, ``inputs_on_device=1``).  There is no CPU
fallback: if the library is missing or no GPU is present, calls fail.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("DRSF_LIB") or os.path.join(_HERE, "libdrsf.so")

DRSF_INSERT, DRSF_DELETE = 0, 1
DRSF_OK, DRSF_E_ARG, DRSF_E_NOMEM, DRSF_E_FOREST = 0, -1, -2, -3
DRSF_E_BATCH, DRSF_E_CAPACITY, DRSF_E_DEVICE, DRSF_E_STATE = -4, -5, -6, -7
DRSF_E_BUDGET = -8
DRSF_SERVER_DIGESTS, DRSF_SERVER_SERIAL, DRSF_SERVER_COALESCE = 1, 2, 4
PHASES = ("validate", "update_graph", "root_finding", "orphan_list", "orphan_scan",
          "store_sweep", "batch_and_inserted_scan", "replacement_edges", "superforest_rooting",
          "reversal_and_labels", "host_continuation")
# the entry after the phases in drsf_phase_times: two events back to back (the fixed cost
# of the event record that every phase time includes)
EVENT_BRACKET = "event_bracket"


class drsf_opts(ctypes.Structure):
    _fields_ = [("stream", ctypes.c_void_p),
                ("inputs_on_device", ctypes.c_int),
                ("validate_forest", ctypes.c_int),
                ("profile", ctypes.c_int),
                ("max_batch", ctypes.c_int64),
                ("delta_capacity", ctypes.c_int64),
                ("sweep_mode", ctypes.c_int),
                ("rounds_queued", ctypes.c_int),
                ("levels_queued", ctypes.c_int),
                ("reverse_mode", ctypes.c_int),
                ("replacement_mode", ctypes.c_int),
                ("dev_alloc", ctypes.c_void_p),
                ("dev_free", ctypes.c_void_p),
                ("alloc_user", ctypes.c_void_p),
                ("small_graph_vertices", ctypes.c_int),
                ("small_threads", ctypes.c_int),
                ("validate_batches", ctypes.c_int),
                ("launch_mode", ctypes.c_int),
                ("walk_limit", ctypes.c_int)]


# device allocator hooks of drsf_opts
DEV_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
DEV_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class drsf_view(ctypes.Structure):
    _fields_ = [("parent", ctypes.c_void_p),
                ("label", ctypes.c_void_p),
                ("n", ctypes.c_int32),
                ("num_edges", ctypes.c_int64),
                ("num_key_cross", ctypes.c_int64),
                ("num_replacement", ctypes.c_int64),
                ("num_pieces", ctypes.c_int64),
                ("num_paths", ctypes.c_int64),
                ("num_orphans", ctypes.c_int64),
                ("orphan_slots", ctypes.c_int64),
                ("scan_orphans", ctypes.c_int32),
                ("host_finished", ctypes.c_int32),
                ("jump_rounds", ctypes.c_int32)]


class DrsfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"drsf error {code}: {msg}")
        self.code = code


# every symbol include/drsf.h declares
EXPORTS = ("drsf_default_opts", "drsf_create", "drsf_apply", "drsf_apply_async", "drsf_wait",
           "drsf_copy_out", "drsf_get_view", "drsf_num_edges", "drsf_export_edges",
           "drsf_snapshot_take", "drsf_snapshot_restore", "drsf_snapshot_free",
           "drsf_phase_times", "drsf_destroy", "drsf_last_error", "drsf_version",
           "drsf_multi_create", "drsf_multi_apply", "drsf_multi_apply_async", "drsf_multi_wait",
           "drsf_multi_num_edges", "drsf_num_graphs", "drsf_set_tuning", "drsf_set_small_schedule",
           "drsf_digest",
           "drsf_device_bytes", "drsf_footprint", "drsf_server_create", "drsf_server_admit",
           "drsf_server_submit", "drsf_server_release", "drsf_server_start",
           "drsf_server_wait_all", "drsf_server_result", "drsf_server_batch", "drsf_server_stats",
           "drsf_server_tenant_state", "drsf_server_copy_out", "drsf_server_error", "drsf_server_destroy",
           "drsf_static_forest", "drsf_static_forest_noalloc")

_lib = None


def load():
    """Load libdrsf.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built (run __graft_entry__.build())")
    # One HIP runtime per process: torch's wheel ships its own libamdhip64
    # with the same soname.  Loading torch first makes libdrsf.so bind to that
    # copy; loading libdrsf.so first would let torch load a second runtime
    # later, and two runtimes cannot share the device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, c_int = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int
    lib.drsf_default_opts.argtypes = [ctypes.POINTER(drsf_opts)]
    lib.drsf_default_opts.restype = None
    lib.drsf_create.argtypes = [i32, vp, vp, vp, ctypes.POINTER(drsf_opts), ctypes.POINTER(vp)]
    lib.drsf_create.restype = c_int
    lib.drsf_apply.argtypes = [vp, vp, i64, c_int, ctypes.POINTER(drsf_view)]
    lib.drsf_apply.restype = c_int
    lib.drsf_apply_async.argtypes = [vp, vp, i64, c_int]
    lib.drsf_apply_async.restype = c_int
    lib.drsf_wait.argtypes = [vp, ctypes.POINTER(drsf_view)]
    lib.drsf_wait.restype = c_int
    lib.drsf_copy_out.argtypes = [vp, vp, vp]
    lib.drsf_copy_out.restype = c_int
    lib.drsf_get_view.argtypes = [vp, ctypes.POINTER(drsf_view)]
    lib.drsf_get_view.restype = c_int
    lib.drsf_num_edges.argtypes = [vp]
    lib.drsf_num_edges.restype = i64
    lib.drsf_export_edges.argtypes = [vp, vp, i64, ctypes.POINTER(i64)]
    lib.drsf_export_edges.restype = c_int
    lib.drsf_snapshot_take.argtypes = [vp, ctypes.POINTER(vp)]
    lib.drsf_snapshot_take.restype = c_int
    lib.drsf_snapshot_restore.argtypes = [vp, vp]
    lib.drsf_snapshot_restore.restype = c_int
    lib.drsf_snapshot_free.argtypes = [vp]
    lib.drsf_snapshot_free.restype = None
    lib.drsf_phase_times.argtypes = [vp, ctypes.POINTER(ctypes.c_float), c_int]
    lib.drsf_phase_times.restype = c_int
    lib.drsf_destroy.argtypes = [vp]
    lib.drsf_destroy.restype = None
    lib.drsf_last_error.argtypes = [vp]
    lib.drsf_last_error.restype = ctypes.c_char_p
    lib.drsf_version.argtypes = []
    lib.drsf_version.restype = ctypes.c_char_p
    lib.drsf_multi_create.argtypes = [i32, vp, vp, vp, vp, ctypes.POINTER(drsf_opts), ctypes.POINTER(vp)]
    lib.drsf_multi_create.restype = c_int
    lib.drsf_multi_apply.argtypes = [vp, vp, vp, vp, vp]
    lib.drsf_multi_apply.restype = c_int
    lib.drsf_multi_apply_async.argtypes = [vp, vp, vp, vp]
    lib.drsf_multi_apply_async.restype = c_int
    lib.drsf_multi_wait.argtypes = [vp, vp]
    lib.drsf_multi_wait.restype = c_int
    lib.drsf_multi_num_edges.argtypes = [vp, vp]
    lib.drsf_multi_num_edges.restype = c_int
    lib.drsf_num_graphs.argtypes = [vp]
    lib.drsf_num_graphs.restype = c_int
    lib.drsf_set_tuning.argtypes = [vp, c_int, c_int, c_int]
    lib.drsf_set_tuning.restype = c_int
    lib.drsf_set_small_schedule.argtypes = [vp, c_int, c_int]
    lib.drsf_set_small_schedule.restype = c_int
    lib.drsf_digest.argtypes = [vp, vp]
    lib.drsf_digest.restype = c_int
    lib.drsf_device_bytes.argtypes = [vp]
    lib.drsf_device_bytes.restype = i64
    lib.drsf_footprint.argtypes = [i32, i64, ctypes.POINTER(drsf_opts)]
    lib.drsf_footprint.restype = i64
    lib.drsf_static_forest.argtypes = [i32, vp, vp, vp, vp, vp, ctypes.POINTER(i32)]
    lib.drsf_static_forest.restype = c_int
    lib.drsf_static_forest_noalloc.argtypes = [i32, vp, vp, vp, vp, vp, ctypes.POINTER(i32)]
    lib.drsf_static_forest_noalloc.restype = c_int
    lib.drsf_server_create.argtypes = [i64, ctypes.POINTER(drsf_opts), c_int, ctypes.POINTER(vp)]
    lib.drsf_server_create.restype = c_int
    lib.drsf_server_admit.argtypes = [vp, i32, vp, vp, vp, i64, ctypes.POINTER(i32)]
    lib.drsf_server_admit.restype = c_int
    lib.drsf_server_submit.argtypes = [vp, i32, vp, i64, c_int, i64, ctypes.POINTER(i64)]
    lib.drsf_server_submit.restype = c_int
    lib.drsf_server_release.argtypes = [vp, i32]
    lib.drsf_server_release.restype = c_int
    lib.drsf_server_start.argtypes = [vp]
    lib.drsf_server_start.restype = c_int
    lib.drsf_server_wait_all.argtypes = [vp]
    lib.drsf_server_wait_all.restype = c_int
    lib.drsf_server_result.argtypes = [vp, i64, ctypes.POINTER(i32), vp, vp]
    lib.drsf_server_result.restype = c_int
    lib.drsf_server_batch.argtypes = [vp, i64, ctypes.POINTER(i64)]
    lib.drsf_server_batch.restype = c_int
    lib.drsf_server_stats.argtypes = [vp, vp]
    lib.drsf_server_stats.restype = c_int
    lib.drsf_server_tenant_state.argtypes = [vp, i32]
    lib.drsf_server_tenant_state.restype = i32
    lib.drsf_server_copy_out.argtypes = [vp, i32, vp, vp]
    lib.drsf_server_copy_out.restype = c_int
    lib.drsf_server_error.argtypes = [vp]
    lib.drsf_server_error.restype = ctypes.c_char_p
    lib.drsf_server_destroy.argtypes = [vp]
    lib.drsf_server_destroy.restype = None
    _lib = lib
    return lib


def _ptr(x):
    """Raw pointer of a numpy array (host) or a torch tensor (host or device)."""
    if x is None:
        return None
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    return x.ctypes.data


_TORCH_DTYPE_NAMES = {np.dtype(np.int8): "torch.int8", np.dtype(np.int32): "torch.int32",
                      np.dtype(np.int64): "torch.int64"}


def _arr(x, dtype, on_device: bool, what: str, count: int | None = None):
    """Checks that an input is what the library will read through its
    pointer — the element type, C-contiguous memory, at least `count`
    elements, and host memory (numpy array, CPU tensor) for a context whose
    inputs are host memory or a GPU tensor for one whose inputs are device
    memory — and returns the pointer; raises DrsfError (DRSF_E_ARG) before
    any library call otherwise.  Nothing is converted."""
    dtype = np.dtype(dtype)
    if hasattr(x, "data_ptr") and hasattr(x, "is_cuda"):  # torch tensor
        if str(x.dtype) != _TORCH_DTYPE_NAMES[dtype]:
            raise DrsfError(DRSF_E_ARG, f"{what}: dtype {x.dtype}, expected {_TORCH_DTYPE_NAMES[dtype]}")
        if not x.is_contiguous():
            raise DrsfError(DRSF_E_ARG, f"{what}: tensor is not contiguous")
        if bool(x.is_cuda) != bool(on_device):
            raise DrsfError(DRSF_E_ARG, f"{what}: a {'GPU' if x.is_cuda else 'CPU'} tensor given to a context "
                                        f"whose inputs are {'device' if on_device else 'host'} memory")
        size = x.numel()
    elif isinstance(x, np.ndarray):
        if on_device:
            raise DrsfError(DRSF_E_ARG, f"{what}: a host (numpy) array given to a context whose inputs are "
                                        "device memory")
        if x.dtype != dtype:
            raise DrsfError(DRSF_E_ARG, f"{what}: dtype {x.dtype}, expected {dtype}")
        if not x.flags.c_contiguous:
            raise DrsfError(DRSF_E_ARG, f"{what}: array is not C-contiguous")
        size = x.size
    else:
        raise DrsfError(DRSF_E_ARG, f"{what}: expected a numpy array or a torch tensor, got {type(x).__name__}")
    if count is not None and size < count:
        raise DrsfError(DRSF_E_ARG, f"{what}: {size} elements, needs {count}")
    return x.data_ptr() if hasattr(x, "data_ptr") else x.ctypes.data


def _host_input(x, dtype):
    """Host-memory input of a host-input context: numpy arrays are converted
    (values, not bytes) to the dtype the library reads; tensors pass as they
    are and are checked by _arr."""
    if isinstance(x, np.ndarray) or isinstance(x, (list, tuple)):
        return np.ascontiguousarray(x, dtype=dtype)
    return x


def _batch(x, on_device: bool):
    """(array, b) of a batch of edge pairs: numpy input of a host-input
    context is converted to int32 pairs; anything else must already be an
    int32 array of 2b entries."""
    if not on_device and (isinstance(x, np.ndarray) or isinstance(x, (list, tuple))):
        x = np.ascontiguousarray(x, dtype=np.int32).reshape(-1, 2)
    size = x.numel() if hasattr(x, "numel") else getattr(x, "size", 0)
    if size % 2:
        raise DrsfError(DRSF_E_ARG, f"edges: {size} entries, expected pairs")
    _arr(x, np.int32, on_device, "edges")
    return x, size // 2


class TorchAllocator:
    """drsf_opts allocator hooks that take the context's device memory from
    torch's caching allocator (torch.cuda.caching_allocator_alloc / _delete),
    optionally failing every allocation after the first `limit` (to exercise
    DRSF_E_NOMEM).  Counts live blocks and bytes.  Must outlive the context
    and its snapshots."""

    def __init__(self, limit: int | None = None):
        self.limit = limit
        self.calls = 0
        self.live = {}
        self._alloc = DEV_ALLOC_FN(self._do_alloc)
        self._free = DEV_FREE_FN(self._do_free)

    def _do_alloc(self, nbytes, user):
        try:
            self.calls += 1
            if self.limit is not None and self.calls > self.limit:
                return None
            import torch
            p = int(torch.cuda.caching_allocator_alloc(int(nbytes)))
            self.live[p] = int(nbytes)
            return p
        except Exception:
            return None

    def _do_free(self, p, user):
        try:
            import torch
            if p in self.live:
                del self.live[p]
                torch.cuda.caching_allocator_delete(int(p))
        except Exception:
            pass

    def install(self, o: drsf_opts) -> None:
        o.dev_alloc = ctypes.cast(self._alloc, ctypes.c_void_p)
        o.dev_free = ctypes.cast(self._free, ctypes.c_void_p)
        o.alloc_user = None


def _check(rc: int, ctx=None):
    if rc != DRSF_OK:
        msg = load().drsf_last_error(ctx)
        raise DrsfError(rc, msg.decode() if msg else "")


# ---- functions with the names of the C ABI --------------------------------

def drsf_default_opts() -> drsf_opts:
    o = drsf_opts()
    load().drsf_default_opts(ctypes.byref(o))
    return o


def drsf_create(n: int, row_ptr, col, parent, opts: drsf_opts | None = None):
    o = opts if opts is not None else drsf_default_opts()
    out = ctypes.c_void_p()
    _check(load().drsf_create(n, _ptr(row_ptr), _ptr(col), _ptr(parent), ctypes.byref(o),
                              ctypes.byref(out)))
    return out


def drsf_apply(ctx, edges, b: int, op: int) -> drsf_view:
    v = drsf_view()
    _check(load().drsf_apply(ctx, _ptr(edges), b, op, ctypes.byref(v)), ctx)
    return v


def drsf_apply_async(ctx, edges, b: int, op: int) -> None:
    _check(load().drsf_apply_async(ctx, _ptr(edges), b, op), ctx)


def drsf_wait(ctx) -> drsf_view:
    v = drsf_view()
    _check(load().drsf_wait(ctx, ctypes.byref(v)), ctx)
    return v


def drsf_copy_out(ctx, parent_host=None, label_host=None) -> None:
    _check(load().drsf_copy_out(ctx, _ptr(parent_host), _ptr(label_host)), ctx)


def drsf_num_edges(ctx) -> int:
    return int(load().drsf_num_edges(ctx))


def drsf_export_edges(ctx) -> np.ndarray:
    m = drsf_num_edges(ctx)
    keys = np.empty(max(m, 1), dtype=np.uint64)
    got = ctypes.c_int64()
    _check(load().drsf_export_edges(ctx, keys.ctypes.data, len(keys), ctypes.byref(got)), ctx)
    return keys[: got.value]


def drsf_snapshot_take(ctx):
    s = ctypes.c_void_p()
    _check(load().drsf_snapshot_take(ctx, ctypes.byref(s)), ctx)
    return s


def drsf_snapshot_restore(ctx, snap) -> None:
    _check(load().drsf_snapshot_restore(ctx, snap), ctx)


def drsf_snapshot_free(snap) -> None:
    load().drsf_snapshot_free(snap)


def drsf_phase_times(ctx) -> dict:
    names = PHASES + (EVENT_BRACKET,)
    buf = (ctypes.c_float * len(names))()
    k = load().drsf_phase_times(ctx, buf, len(names))
    return {names[i]: float(buf[i]) for i in range(k)}


def drsf_multi_create(G: int, n_off, row_ptr, col, parent, opts: drsf_opts | None = None):
    o = opts if opts is not None else drsf_default_opts()
    n_off = np.ascontiguousarray(n_off, dtype=np.int32)
    out = ctypes.c_void_p()
    _check(load().drsf_multi_create(G, _ptr(n_off), _ptr(row_ptr), _ptr(col), _ptr(parent),
                                    ctypes.byref(o), ctypes.byref(out)))
    return out


def drsf_multi_apply_async(ctx, edges, b_off, op) -> None:
    b_off = np.ascontiguousarray(b_off, dtype=np.int64)
    op = np.ascontiguousarray(op, dtype=np.int8)
    _check(load().drsf_multi_apply_async(ctx, _ptr(edges), _ptr(b_off), _ptr(op)), ctx)


def drsf_multi_wait(ctx, G: int) -> np.ndarray:
    st = np.zeros(G, dtype=np.int32)
    _check(load().drsf_multi_wait(ctx, _ptr(st)), ctx)
    return st


def drsf_multi_apply(ctx, edges, b_off, op) -> np.ndarray:
    b_off = np.ascontiguousarray(b_off, dtype=np.int64)
    op = np.ascontiguousarray(op, dtype=np.int8)
    st = np.zeros(len(op), dtype=np.int32)
    _check(load().drsf_multi_apply(ctx, _ptr(edges), _ptr(b_off), _ptr(op), _ptr(st)), ctx)
    return st


def drsf_multi_num_edges(ctx, G: int) -> np.ndarray:
    m = np.zeros(G, dtype=np.int64)
    _check(load().drsf_multi_num_edges(ctx, _ptr(m)), ctx)
    return m


def drsf_num_graphs(ctx) -> int:
    return int(load().drsf_num_graphs(ctx))


def drsf_set_tuning(ctx, rounds_queued: int = 0, levels_queued: int = 0, sweep_mode: int = 0) -> None:
    _check(load().drsf_set_tuning(ctx, rounds_queued, levels_queued, sweep_mode), ctx)


def drsf_set_small_schedule(ctx, threads: int = 0, workgroups: int = 0) -> None:
    _check(load().drsf_set_small_schedule(ctx, threads, workgroups), ctx)


def drsf_digest(ctx) -> tuple:
    out = np.zeros(2, dtype=np.uint64)
    _check(load().drsf_digest(ctx, out.ctypes.data), ctx)
    return int(out[0]), int(out[1])


def drsf_device_bytes(ctx) -> int:
    return int(load().drsf_device_bytes(ctx))


def drsf_static_forest(n: int, row_ptr, col, parent_out, label_out, stream=None) -> int:
    """Static rebuild (no context): device CSR in, device parent and label
    out (torch tensors or raw pointers); returns the breadth-first levels."""
    lv = ctypes.c_int32(0)
    rc = load().drsf_static_forest(n, _ptr(row_ptr), _ptr(col), _ptr(parent_out), _ptr(label_out),
                                   stream, ctypes.byref(lv))
    _check(rc)
    return int(lv.value)


def drsf_static_forest_noalloc(n: int, row_ptr, col, parent_out, label_out, stream=None) -> int:
    """drsf_static_forest without any allocation (the library's fixed
    per-device scratch); returns the breadth-first levels."""
    lv = ctypes.c_int32(0)
    rc = load().drsf_static_forest_noalloc(n, _ptr(row_ptr), _ptr(col), _ptr(parent_out), _ptr(label_out),
                                           stream, ctypes.byref(lv))
    _check(rc)
    return int(lv.value)


def drsf_footprint(n: int, nnz: int, opts: drsf_opts | None = None) -> int:
    o = opts if opts is not None else drsf_default_opts()
    return int(load().drsf_footprint(n, nnz, ctypes.byref(o)))


def drsf_destroy(ctx) -> None:
    load().drsf_destroy(ctx)


def drsf_version() -> str:
    return load().drsf_version().decode()


# ---- convenience wrapper -----------------------------------------------------

class Forest:
    """A graph and its rooted spanning forest resident on the GPU."""

    ctx = None

    def __init__(self, n: int, row_ptr, col, parent, *, max_batch: int = 1 << 20,
                 stream=None, inputs_on_device: bool = False, validate: bool = True,
                 profile: bool = False, delta_capacity: int = 0, sweep_mode: int = 0,
                 rounds_queued: int = 0, levels_queued: int = 0, reverse_mode: int = 0,
                 replacement_mode: int = 0, allocator: TorchAllocator | None = None,
                 validate_batches: bool = True, launch_mode: int = 0, walk_limit: int = 0):
        self.on_device = bool(inputs_on_device)
        if not self.on_device:
            row_ptr = _host_input(row_ptr, np.int64)
            col = _host_input(col, np.int32)
            parent = _host_input(parent, np.int32)
        self.n = n
        _arr(row_ptr, np.int64, self.on_device, "row_ptr", n + 1)
        _arr(col, np.int32, self.on_device, "col",
             None if self.on_device else int(np.asarray(row_ptr)[n]) if n >= 0 else None)
        _arr(parent, np.int32, self.on_device, "parent", n)
        o = drsf_default_opts()
        o.max_batch = max_batch
        o.inputs_on_device = int(inputs_on_device)
        o.validate_forest = int(validate)
        o.profile = int(profile)
        o.delta_capacity = delta_capacity
        o.sweep_mode = sweep_mode
        o.rounds_queued = rounds_queued
        o.levels_queued = levels_queued
        o.reverse_mode = reverse_mode
        o.replacement_mode = replacement_mode
        o.validate_batches = int(validate_batches)
        o.launch_mode = launch_mode
        o.walk_limit = walk_limit
        if stream is not None:
            o.stream = stream
        self.allocator = allocator
        if allocator is not None:
            allocator.install(o)
        self._keep = (row_ptr, col, parent)
        self.ctx = drsf_create(n, row_ptr, col, parent, o)
        self._keep = None

    def apply(self, edges, op: int) -> dict:
        edges, b = _batch(edges, self.on_device)
        v = drsf_apply(self.ctx, edges, b, op)
        return self._stats(v)

    def apply_async(self, edges, op: int) -> None:
        """Queues an update (up to two run back to back on a device-input
        context; see drsf_apply_async); the batch is kept alive until its
        wait."""
        edges, b = _batch(edges, self.on_device)
        if not hasattr(self, "_pending_edges"):
            self._pending_edges = []
        drsf_apply_async(self.ctx, edges, b, op)
        self._pending_edges.append(edges)
        del self._pending_edges[:-2]  # the library keeps at most two queued

    def wait(self) -> dict:
        """Waits for the oldest queued update and returns its statistics."""
        try:
            return self._stats(drsf_wait(self.ctx))
        finally:
            if getattr(self, "_pending_edges", None):
                self._pending_edges.pop(0)

    @staticmethod
    def _stats(v: drsf_view) -> dict:
        return {"num_edges": v.num_edges, "num_key_cross": v.num_key_cross,
                "num_replacement": v.num_replacement, "num_pieces": v.num_pieces,
                "num_paths": v.num_paths, "num_orphans": v.num_orphans,
                "orphan_slots": v.orphan_slots, "scan_orphans": v.scan_orphans,
                "host_finished": v.host_finished, "jump_rounds": v.jump_rounds}

    def parent(self) -> np.ndarray:
        p = np.empty(self.n, dtype=np.int32)
        drsf_copy_out(self.ctx, p, None)
        return p

    def label(self) -> np.ndarray:
        lab = np.empty(self.n, dtype=np.int32)
        drsf_copy_out(self.ctx, None, lab)
        return lab

    def edges(self) -> np.ndarray:
        return drsf_export_edges(self.ctx)

    def phase_times(self) -> dict:
        return drsf_phase_times(self.ctx)

    def digest(self) -> tuple:
        return drsf_digest(self.ctx)

    def device_bytes(self) -> int:
        return drsf_device_bytes(self.ctx)

    def set_tuning(self, rounds_queued: int = 0, levels_queued: int = 0, sweep_mode: int = 0) -> None:
        drsf_set_tuning(self.ctx, rounds_queued, levels_queued, sweep_mode)

    def snapshot(self):
        return drsf_snapshot_take(self.ctx)

    def restore(self, snap) -> None:
        drsf_snapshot_restore(self.ctx, snap)

    def close(self) -> None:
        if self.ctx is not None:
            drsf_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MultiForest(Forest):
    """Several independent graphs in one context (global vertex ids
    n_off[g] .. n_off[g + 1] - 1 belong to graph g), updated together: one
    batch and op per graph per call."""

    def __init__(self, n_off, row_ptr, col, parent, *, max_batch: int = 1 << 20,
                 stream=None, inputs_on_device: bool = False, validate: bool = True,
                 profile: bool = False, delta_capacity: int = 0, sweep_mode: int = 0,
                 rounds_queued: int = 0, levels_queued: int = 0, reverse_mode: int = 0,
                 replacement_mode: int = 0, allocator: TorchAllocator | None = None,
                 small_graph_vertices: int = 0, small_threads: int = 0, validate_batches: bool = True,
                 launch_mode: int = 0, walk_limit: int = 0):
        self.on_device = bool(inputs_on_device)
        if not self.on_device:
            row_ptr = _host_input(row_ptr, np.int64)
            col = _host_input(col, np.int32)
            parent = _host_input(parent, np.int32)
        self.n_off = np.ascontiguousarray(n_off, dtype=np.int32)
        self.G = len(self.n_off) - 1
        self.n = int(self.n_off[-1])
        _arr(row_ptr, np.int64, self.on_device, "row_ptr", self.n + 1)
        _arr(col, np.int32, self.on_device, "col", None if self.on_device else int(np.asarray(row_ptr)[self.n]))
        _arr(parent, np.int32, self.on_device, "parent", self.n)
        o = drsf_default_opts()
        o.max_batch = max_batch
        o.inputs_on_device = int(inputs_on_device)
        o.validate_forest = int(validate)
        o.profile = int(profile)
        o.delta_capacity = delta_capacity
        o.sweep_mode = sweep_mode
        o.rounds_queued = rounds_queued
        o.levels_queued = levels_queued
        o.reverse_mode = reverse_mode
        o.replacement_mode = replacement_mode
        o.small_graph_vertices = small_graph_vertices
        o.small_threads = small_threads
        o.validate_batches = int(validate_batches)
        o.launch_mode = launch_mode
        o.walk_limit = walk_limit
        if stream is not None:
            o.stream = stream
        self.allocator = allocator
        if allocator is not None:
            allocator.install(o)
        self.ctx = drsf_multi_create(self.G, self.n_off, row_ptr, col, parent, o)

    def _multi_args(self, edges, b_off, op):
        edges, b = _batch(edges, self.on_device)
        b_off = np.ascontiguousarray(b_off, dtype=np.int64)
        op = np.ascontiguousarray(op, dtype=np.int8)
        if len(b_off) != self.G + 1 or len(op) != self.G:
            raise DrsfError(DRSF_E_ARG, f"b_off needs {self.G + 1} entries and op {self.G}")
        if b_off[-1] > b:
            raise DrsfError(DRSF_E_ARG, f"b_off[G] = {b_off[-1]} but edges hold {b} pairs")
        return edges, b_off, op

    def apply_multi(self, edges, b_off, op) -> np.ndarray:
        """Per-graph status (DRSF_OK or DRSF_E_BATCH)."""
        edges, b_off, op = self._multi_args(edges, b_off, op)
        return drsf_multi_apply(self.ctx, edges, b_off, op)

    def apply_multi_async(self, edges, b_off, op) -> None:
        edges, b_off, op = self._multi_args(edges, b_off, op)
        self._pending_multi = edges
        drsf_multi_apply_async(self.ctx, edges, b_off, op)

    def wait_multi(self) -> np.ndarray:
        st = drsf_multi_wait(self.ctx, self.G)
        self._pending_multi = None
        return st

    def num_edges(self) -> np.ndarray:
        return drsf_multi_num_edges(self.ctx, self.G)

    def set_small_schedule(self, threads: int = 0, workgroups: int = 0) -> None:
        drsf_set_small_schedule(self.ctx, threads, workgroups)


# ---- serving ------------------------------------------------------------------

def _scheck(rc: int, srv):
    if rc != DRSF_OK:
        msg = load().drsf_server_error(srv) if srv else b""
        raise DrsfError(rc, msg.decode() if msg else "")


class Server:
    """Several graphs resident under a device memory budget, served by the
    library's scheduler thread (drsf_server_* in include/drsf.h)."""

    def __init__(self, budget_bytes: int, *, max_batch: int = 1 << 17, digests: bool = False,
                 serial: bool = False, coalesce: bool = False, sweep_mode: int = 0):
        o = drsf_default_opts()
        o.max_batch = max_batch
        o.sweep_mode = sweep_mode
        flags = ((DRSF_SERVER_DIGESTS if digests else 0) | (DRSF_SERVER_SERIAL if serial else 0) |
                 (DRSF_SERVER_COALESCE if coalesce else 0))
        out = ctypes.c_void_p()
        _scheck(load().drsf_server_create(int(budget_bytes), ctypes.byref(o), flags, ctypes.byref(out)),
                None)
        self.srv = out

    def admit(self, n: int, row_ptr, col, parent, arrive_ns: int = -1) -> int:
        row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int32)
        parent = np.ascontiguousarray(parent, dtype=np.int32)
        t = ctypes.c_int32()
        _scheck(load().drsf_server_admit(self.srv, n, _ptr(row_ptr), _ptr(col), _ptr(parent),
                                         int(arrive_ns), ctypes.byref(t)), self.srv)
        return t.value

    def submit(self, tenant: int, edges, op: int, arrive_ns: int = -1) -> int:
        edges = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)
        r = ctypes.c_int64()
        _scheck(load().drsf_server_submit(self.srv, tenant, _ptr(edges), edges.shape[0], op,
                                          int(arrive_ns), ctypes.byref(r)), self.srv)
        return r.value

    def release(self, tenant: int) -> None:
        _scheck(load().drsf_server_release(self.srv, tenant), self.srv)

    def start(self) -> None:
        _scheck(load().drsf_server_start(self.srv), self.srv)

    def wait_all(self) -> None:
        _scheck(load().drsf_server_wait_all(self.srv), self.srv)

    def result(self, req: int) -> dict:
        st = ctypes.c_int32()
        t = np.zeros(3, dtype=np.uint64)
        dg = np.zeros(2, dtype=np.uint64)
        _scheck(load().drsf_server_result(self.srv, req, ctypes.byref(st), t.ctypes.data,
                                          dg.ctypes.data), self.srv)
        return {"status": st.value, "t_arrive": int(t[0]), "t_start": int(t[1]), "t_done": int(t[2]),
                "digest": (int(dg[0]), int(dg[1]))}

    def batch(self, req: int) -> int:
        """Id of the first request of the device batch that carried req."""
        b = ctypes.c_int64()
        _scheck(load().drsf_server_batch(self.srv, req, ctypes.byref(b)), self.srv)
        return b.value

    def stats(self) -> dict:
        out = np.zeros(8, dtype=np.float64)
        _scheck(load().drsf_server_stats(self.srv, out.ctypes.data), self.srv)
        return {"completed": int(out[0]), "p50_ms": float(out[1]), "p99_ms": float(out[2]),
                "updates_per_s": float(out[3]), "peak_bytes": int(out[4]), "budget": int(out[5]),
                "service_p50_ms": float(out[6]), "service_p99_ms": float(out[7])}

    def tenant_state(self, tenant: int) -> int:
        return int(load().drsf_server_tenant_state(self.srv, tenant))

    def copy_out(self, tenant: int, n: int):
        """(parent, label) of a live tenant once its submitted requests are done."""
        p = np.empty(n, dtype=np.int32)
        lab = np.empty(n, dtype=np.int32)
        _scheck(load().drsf_server_copy_out(self.srv, tenant, p.ctypes.data, lab.ctypes.data), self.srv)
        return p, lab

    def close(self) -> None:
        if self.srv is not None:
            load().drsf_server_destroy(self.srv)
            self.srv = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
