"""Python binding of libsphview.so (ctypes).  Argument marshalling only: every
step of the SPH path runs in the library's HIP kernels.  torch provides device
memory (workspaces are uint8 tensors) and streams.

Function names are the C entry points without the ``sphv_`` prefix.  A missing
library raises immediately: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import inputs

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsphview.so")

# ------------------------------------------------------------ constants

OK, E_INVALID_ARG, E_DESCRIPTOR, E_WORKSPACE, E_ALIAS, E_STATE, E_HIP, E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
F_NONFINITE_INPUT, F_H_NOT_CONVERGED, F_H_CAP_HIT, F_QUEUE_OVERFLOW = 1, 2, 4, 8
F_NONFINITE_OUTPUT, F_GRID_TOO_SMALL, F_OUT_OF_BOX, F_LIST_MISMATCH = 16, 32, 64, 128
F64, F32, I64, I32 = 1, 2, 3, 4
IN, OUT, INOUT = 1, 2, 3
LAYOUT_SOA, LAYOUT_AOSOA, LAYOUT_DIRECT, LAYOUT_SORTED = 0, 1, 2, 3
PREC_FP64, PREC_FP32 = 0, 1
KERNEL_CUBIC, KERNEL_QUARTIC = 0, 1
DESC_RECORD_POINTERS = 1
LOOP_DENSITY, LOOP_FORCE = 0, 1

ROLES = ["user", "x", "y", "z", "vx", "vy", "vz", "vhx", "vhy", "vhz", "ax", "ay", "az", "m", "h", "rho",
         "omega", "u", "uh", "u_dt", "alpha", "v_sig", "wcount"]
ROLE = {name: i for i, name in enumerate(ROLES)}

EXPORTS = [
    "sphv_status_string", "sphv_version", "sphv_params_init", "sphv_state_bytes", "sphv_state_init",
    "sphv_begin_step", "sphv_read_state", "sphv_write_state", "sphv_cells_workspace_bytes", "sphv_cells_create",
    "sphv_cells_build", "sphv_cells_get_info", "sphv_cells_destroy", "sphv_view_workspace_bytes",
    "sphv_view_create", "sphv_aos_to_soa", "sphv_aos_to_soa_prefetch", "sphv_soa_to_aos", "sphv_view_field",
    "sphv_view_destroy",
    "sphv_sph_density", "sphv_sph_force", "sphv_step_reduce", "sphv_kick_drift", "sphv_graph_begin", "sphv_graph_end",
    "sphv_graph_launch", "sphv_graph_destroy", "sphv_autotune_candidates", "sphv_autotune_workspace_bytes",
    "sphv_autotune", "sphv_records_sort_workspace_bytes", "sphv_records_sort", "sphv_records_sort_static",
    "sphv_grid_for",
    "sphv_autotune_grid_workspace_bytes", "sphv_autotune_grid",
]


class Field(C.Structure):
    _fields_ = [("offset", C.c_uint64), ("role", C.c_uint32), ("dtype", C.c_uint16), ("access", C.c_uint16)]


class Descriptor(C.Structure):
    _fields_ = [("stride", C.c_uint64), ("n_fields", C.c_uint32), ("flags", C.c_uint32),
                ("fields", C.POINTER(Field))]


class Params(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("len", C.c_double * 3), ("cell", C.c_double * 3),
                ("inv_cell", C.c_double * 3), ("grid", C.c_int32 * 3), ("periodic", C.c_int32 * 3),
                ("gamma", C.c_double), ("eta", C.c_double), ("cfl", C.c_double), ("h_tol", C.c_double),
                ("headroom", C.c_double), ("max_iter", C.c_int32), ("kernel", C.c_int32),
                ("list_cap", C.c_int32), ("symmetric", C.c_int32)]


class State(C.Structure):
    _fields_ = [("flags", C.c_uint32), ("max_iters", C.c_int32), ("nstep", C.c_int64), ("dt", C.c_double),
                ("dt_prev", C.c_double), ("t", C.c_double), ("sums", C.c_double * 8),
                ("pairs_density", C.c_int64), ("pairs_force", C.c_int64), ("pair_evals_density", C.c_int64),
                ("pairs_total", C.c_int64), ("reserved", C.c_int64 * 3)]


class Layout(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("aosoa_width", C.c_uint32), ("tpi", C.c_uint32), ("masked", C.c_uint32)]


class CellsInfo(C.Structure):
    _fields_ = [("perm", C.c_void_p), ("cell_start", C.c_void_p), ("key", C.c_void_p), ("reach", C.c_void_p),
                ("n", C.c_int64), ("n_cells", C.c_int64), ("max_items", C.c_int64)]


class SphvError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {status_string(status)} ({status})")
        self.status = status


_LIB = None
VP = C.c_void_p


def lib():
    """Load libsphview.so; raises if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() (or python -m "
                          f"paper_2502_16517_amd._build) first; there is no non-HIP fallback")
    # torch ships its own HIP runtime under another file name: loaded first, it
    # also serves this library (one runtime per process); loaded after this
    # library, it would bring a second runtime, whose allocations the first
    # cannot use
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    sig = {
        "sphv_status_string": (C.c_char_p, [C.c_int32]),
        "sphv_version": (C.c_int32, []),
        "sphv_params_init": (C.c_int32, [C.POINTER(Params), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                         C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
        "sphv_state_bytes": (C.c_size_t, []),
        "sphv_state_init": (C.c_int32, [VP, VP]),
        "sphv_begin_step": (C.c_int32, [VP, VP]),
        "sphv_read_state": (C.c_int32, [VP, C.POINTER(State), VP]),
        "sphv_write_state": (C.c_int32, [VP, C.POINTER(State), VP]),
        "sphv_cells_workspace_bytes": (C.c_size_t, [C.c_int64, C.POINTER(Params)]),
        "sphv_cells_create": (C.c_int32, [C.POINTER(VP), C.c_int64, C.POINTER(Params), VP, C.c_size_t]),
        "sphv_cells_build": (C.c_int32, [VP, VP, C.POINTER(Descriptor), VP, VP]),
        "sphv_cells_get_info": (C.c_int32, [VP, C.POINTER(CellsInfo)]),
        "sphv_cells_destroy": (None, [VP]),
        "sphv_view_workspace_bytes": (C.c_size_t, [C.POINTER(Descriptor), C.c_int64, C.POINTER(Layout),
                                                   C.c_int32]),
        "sphv_view_create": (C.c_int32, [C.POINTER(VP), C.POINTER(Descriptor), C.c_int64, C.POINTER(Layout),
                                         C.c_int32, VP, VP, VP, C.c_size_t]),
        "sphv_aos_to_soa": (C.c_int32, [VP, VP, VP]),
        "sphv_aos_to_soa_prefetch": (C.c_int32, [VP, VP, VP]),
        "sphv_soa_to_aos": (C.c_int32, [VP, VP]),
        "sphv_view_field": (C.c_int32, [VP, C.c_uint32, C.POINTER(VP), C.POINTER(C.c_int32),
                                        C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
        "sphv_view_destroy": (None, [VP]),
        "sphv_sph_density": (C.c_int32, [VP, VP, C.POINTER(Params), VP, VP]),
        "sphv_sph_force": (C.c_int32, [VP, VP, C.POINTER(Params), VP, VP]),
        "sphv_step_reduce": (C.c_int32, [VP, C.POINTER(Params), VP, VP]),
        "sphv_kick_drift": (C.c_int32, [VP, C.POINTER(Descriptor), C.c_int64, C.POINTER(Params), VP, VP]),
        "sphv_graph_begin": (C.c_int32, [VP]),
        "sphv_graph_end": (C.c_int32, [VP, C.POINTER(VP)]),
        "sphv_graph_launch": (C.c_int32, [VP, VP]),
        "sphv_graph_destroy": (None, [VP]),
        "sphv_autotune_candidates": (C.c_int32, [C.POINTER(Layout), C.c_int32]),
        "sphv_autotune_workspace_bytes": (C.c_size_t, [C.POINTER(Descriptor), C.c_int64, C.c_int32,
                                                       C.POINTER(Layout), C.c_int32]),
        "sphv_autotune": (C.c_int32, [C.c_int32, VP, C.POINTER(Descriptor), VP, C.POINTER(Params), C.c_int32,
                                      C.POINTER(Layout), C.c_int32, C.c_int32, VP, C.c_size_t,
                                      C.POINTER(Layout), C.POINTER(C.c_float), VP]),
        "sphv_records_sort_workspace_bytes": (C.c_size_t, [C.c_uint32, C.c_int64]),
        "sphv_records_sort": (C.c_int32, [VP, VP, C.c_uint32, VP, C.c_size_t, VP]),
        "sphv_records_sort_static": (C.c_int32, [VP, VP, C.c_uint32, VP]),
        "sphv_grid_for": (C.c_int32, [C.POINTER(Params), C.c_double, C.c_int32, C.POINTER(C.c_int32)]),
        "sphv_autotune_grid_workspace_bytes": (C.c_size_t, [C.POINTER(Descriptor), C.POINTER(Descriptor),
                                                            C.c_int64, C.POINTER(Params), C.c_int32,
                                                            C.POINTER(Layout), C.POINTER(Layout),
                                                            C.POINTER(C.c_int32), C.c_int32]),
        "sphv_autotune_grid": (C.c_int32, [VP, C.POINTER(Descriptor), C.POINTER(Descriptor), C.c_int64,
                                           C.POINTER(Params), C.c_int32, C.POINTER(Layout), C.POINTER(Layout),
                                           C.POINTER(C.c_int32), C.c_int32, C.c_int32, VP, C.c_size_t,
                                           C.POINTER(C.c_int32), C.POINTER(C.c_float), VP]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = L
    return L


def status_string(s: int) -> str:
    return lib().sphv_status_string(int(s)).decode()


def _chk(s: int, what: str) -> None:
    if s != OK:
        raise SphvError(s, what)


def _ptr(x) -> int | None:
    """Device (or host) address of a torch tensor, or an int address."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream) -> int | None:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ------------------------------------------------------------ descriptors

def descriptor(fields, stride: int = inputs.STRIDE, flags: int = 0):
    """fields: iterable of (role name or None, offset bytes, dtype, access);
    flags: DESC_RECORD_POINTERS for records reached through an address list."""
    fl = list(fields)
    arr = (Field * max(1, len(fl)))()
    for k, (role, off, dt, acc) in enumerate(fl):
        arr[k].offset = off
        arr[k].role = ROLE[role] if role else 0
        arr[k].dtype = dt
        arr[k].access = acc
    d = Descriptor(stride, len(fl), flags, C.cast(arr, C.POINTER(Field)))
    d._keep = arr
    return d


def _rec_fields(spec):
    return [(name, inputs.SLOT[name] * 8, F64, acc) for name, acc in spec]


def _rec_descriptor(spec, flags=0):
    return descriptor(_rec_fields(spec), flags=flags)


DENSITY_FIELDS = [("x", IN), ("y", IN), ("z", IN), ("m", IN), ("h", INOUT), ("rho", OUT), ("omega", OUT),
                  ("wcount", OUT)]
FORCE_FIELDS = [("x", IN), ("y", IN), ("z", IN), ("vx", IN), ("vy", IN), ("vz", IN), ("m", IN), ("h", IN),
                ("rho", IN), ("omega", IN), ("u", IN), ("alpha", IN), ("ax", OUT), ("ay", OUT), ("az", OUT),
                ("u_dt", OUT), ("v_sig", OUT)]
KICK_FIELDS = [("x", INOUT), ("y", INOUT), ("z", INOUT), ("vx", INOUT), ("vy", INOUT), ("vz", INOUT),
               ("vhx", INOUT), ("vhy", INOUT), ("vhz", INOUT), ("ax", IN), ("ay", IN), ("az", IN),
               ("u", INOUT), ("uh", INOUT), ("u_dt", IN)]
CELLS_FIELDS = [("x", IN), ("y", IN), ("z", IN), ("h", IN)]
# one view over density and force: the union of both loops' members; h, rho and
# omega are written by the density loop and read by the force loop inside it
MERGED_FIELDS = [("x", IN), ("y", IN), ("z", IN), ("vx", IN), ("vy", IN), ("vz", IN), ("m", IN), ("h", INOUT),
                 ("rho", INOUT), ("omega", INOUT), ("wcount", OUT), ("u", IN), ("alpha", IN), ("ax", OUT),
                 ("ay", OUT), ("az", OUT), ("u_dt", OUT), ("v_sig", OUT)]


def density_descriptor(flags=0):
    return _rec_descriptor(DENSITY_FIELDS, flags)


def force_descriptor(flags=0):
    return _rec_descriptor(FORCE_FIELDS, flags)


def kick_descriptor(flags=0):
    return _rec_descriptor(KICK_FIELDS, flags)


def cells_descriptor(flags=0):
    return _rec_descriptor(CELLS_FIELDS, flags)


def merged_descriptor(flags=0):
    return _rec_descriptor(MERGED_FIELDS, flags)


def soa_descriptor(spec, n: int, base_slots=None):
    """Descriptor of a struct-of-arrays store: member k is an array of n doubles
    at byte offset slot_k * n * 8 (slot_k from the record layout)."""
    fl = []
    for name, acc in spec:
        slot = inputs.SLOT[name] if base_slots is None else base_slots[name]
        fl.append((name, slot * n * 8, F64, acc))
    return descriptor(fl, stride=8)


# ------------------------------------------------------------ params / layout

def params_init(lo, length, grid, periodic, **kw) -> Params:
    p = Params()
    lo_a = (C.c_double * 3)(*lo)
    le_a = (C.c_double * 3)(*length)
    g_a = (C.c_int32 * 3)(*grid)
    pe_a = (C.c_int32 * 3)(*periodic)
    _chk(lib().sphv_params_init(C.byref(p), lo_a, le_a, g_a, pe_a), "params_init")
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def layout(kind=LAYOUT_SOA, aosoa_width=0, tpi=0, masked=0) -> Layout:
    return Layout(kind, aosoa_width, tpi, masked)


# ------------------------------------------------------------ state

def state_bytes() -> int:
    return int(lib().sphv_state_bytes())


def state_init(state, stream=None):
    _chk(lib().sphv_state_init(_ptr(state), _stream(stream)), "state_init")


def begin_step(state, stream=None):
    _chk(lib().sphv_begin_step(_ptr(state), _stream(stream)), "begin_step")


def read_state(state, stream=None) -> State:
    s = State()
    _chk(lib().sphv_read_state(_ptr(state), C.byref(s), _stream(stream)), "read_state")
    return s


def write_state(state, s: State, stream=None):
    _chk(lib().sphv_write_state(_ptr(state), C.byref(s), _stream(stream)), "write_state")


# ------------------------------------------------------------ cells

def cells_workspace_bytes(n: int, p: Params) -> int:
    return int(lib().sphv_cells_workspace_bytes(n, C.byref(p)))


def cells_create(n: int, p: Params, ws, ws_bytes: int | None = None):
    h = VP()
    nb = ws_bytes if ws_bytes is not None else (ws.numel() if ws is not None else 0)
    _chk(lib().sphv_cells_create(C.byref(h), n, C.byref(p), _ptr(ws), nb), "cells_create")
    return h


def cells_build(cells, aos, d: Descriptor, state, stream=None):
    _chk(lib().sphv_cells_build(cells, _ptr(aos), C.byref(d), _ptr(state), _stream(stream)), "cells_build")


def cells_get_info(cells) -> CellsInfo:
    info = CellsInfo()
    _chk(lib().sphv_cells_get_info(cells, C.byref(info)), "cells_get_info")
    return info


def cells_destroy(cells):
    lib().sphv_cells_destroy(cells)


def records_sort_workspace_bytes(stride: int, n: int) -> int:
    return int(lib().sphv_records_sort_workspace_bytes(stride, n))


def records_sort(cells, aos, stride: int, ws, stream=None, ws_bytes: int | None = None):
    """Moves the records into the cells' sorted order (whole records)."""
    nb = ws_bytes if ws_bytes is not None else (ws.numel() if ws is not None else 0)
    _chk(lib().sphv_records_sort(cells, _ptr(aos), stride, _ptr(ws), nb, _stream(stream)), "records_sort")


# largest stride * n that sphv_records_sort_static takes (its fixed device array)
RECORDS_SORT_STATIC_MAX_BYTES = 96 << 20


def records_sort_static(cells, aos, stride: int, stream=None):
    """records_sort without a workspace: the library's fixed per-GPU array
    holds the copy (calls that overlap on one GPU race)."""
    _chk(lib().sphv_records_sort_static(cells, _ptr(aos), stride, _stream(stream)), "records_sort_static")


# ------------------------------------------------------------ views

def view_workspace_bytes(d: Descriptor, n: int, l: Layout, precision: int) -> int:
    return int(lib().sphv_view_workspace_bytes(C.byref(d), n, C.byref(l), precision))


def view_create(d: Descriptor, n: int, l: Layout, precision: int, aos, index, ws, ws_bytes: int | None = None):
    h = VP()
    nb = ws_bytes if ws_bytes is not None else (ws.numel() if ws is not None else 0)
    _chk(lib().sphv_view_create(C.byref(h), C.byref(d), n, C.byref(l), precision, _ptr(aos), _ptr(index),
                                _ptr(ws), nb), "view_create")
    return h


def aos_to_soa(view, cells=None, stream=None):
    _chk(lib().sphv_aos_to_soa(view, cells, _stream(stream)), "aos_to_soa")


def aos_to_soa_prefetch(view, cells=None, stream=None):
    """Gathers ahead the read-only members no open view writes (see the header)."""
    _chk(lib().sphv_aos_to_soa_prefetch(view, cells, _stream(stream)), "aos_to_soa_prefetch")


def soa_to_aos(view, stream=None):
    _chk(lib().sphv_soa_to_aos(view, _stream(stream)), "soa_to_aos")


def view_field(view, k: int):
    ptr, dt, bl, bb = VP(), C.c_int32(), C.c_uint64(), C.c_uint64()
    _chk(lib().sphv_view_field(view, k, C.byref(ptr), C.byref(dt), C.byref(bl), C.byref(bb)), "view_field")
    return ptr.value, dt.value, bl.value, bb.value


def view_destroy(view):
    lib().sphv_view_destroy(view)


def sph_density(view, cells, p: Params, state, stream=None):
    _chk(lib().sphv_sph_density(view, cells, C.byref(p), _ptr(state), _stream(stream)), "sph_density")


def sph_force(view, cells, p: Params, state, stream=None):
    _chk(lib().sphv_sph_force(view, cells, C.byref(p), _ptr(state), _stream(stream)), "sph_force")


def step_reduce(view, p: Params, state, stream=None):
    _chk(lib().sphv_step_reduce(view, C.byref(p), _ptr(state), _stream(stream)), "step_reduce")


def kick_drift(aos, d: Descriptor, n: int, p: Params, state, stream=None):
    _chk(lib().sphv_kick_drift(_ptr(aos), C.byref(d), n, C.byref(p), _ptr(state), _stream(stream)),
         "kick_drift")


# ------------------------------------------------------------ graphs

def graph_begin(stream):
    _chk(lib().sphv_graph_begin(_stream(stream)), "graph_begin")


def graph_end(stream):
    g = VP()
    _chk(lib().sphv_graph_end(_stream(stream), C.byref(g)), "graph_end")
    return g


def graph_launch(g, stream):
    _chk(lib().sphv_graph_launch(g, _stream(stream)), "graph_launch")


def graph_destroy(g):
    lib().sphv_graph_destroy(g)


# ------------------------------------------------------------ autotuner

def autotune_candidates() -> list:
    """The library's built-in candidate layouts."""
    k = int(lib().sphv_autotune_candidates(None, 0))
    arr = (Layout * k)()
    lib().sphv_autotune_candidates(arr, k)
    return [Layout(c.kind, c.aosoa_width, c.tpi, c.masked) for c in arr]


def _layout_array(cands):
    if cands is None:
        return None, 0
    arr = (Layout * len(cands))(*[Layout(c.kind, c.aosoa_width, c.tpi, c.masked) for c in cands])
    return arr, len(cands)


def autotune_workspace_bytes(d: Descriptor, n: int, precision: int, candidates=None) -> int:
    arr, k = _layout_array(candidates)
    return int(lib().sphv_autotune_workspace_bytes(C.byref(d), n, precision, arr, k))


def autotune(loop: int, aos, d: Descriptor, cells, p: Params, precision: int, ws, candidates=None, reps: int = 3,
             stream=None, ws_bytes: int | None = None):
    """Times every candidate layout for one loop; returns (best Layout, list of
    (Layout, median ms)) in candidate order."""
    cands = candidates if candidates is not None else autotune_candidates()
    arr, k = _layout_array(cands)
    ms = (C.c_float * k)()
    best = Layout()
    nb = ws_bytes if ws_bytes is not None else (ws.numel() if ws is not None else 0)
    _chk(lib().sphv_autotune(loop, _ptr(aos), C.byref(d), cells, C.byref(p), precision, arr, k, reps, _ptr(ws), nb,
                             C.byref(best), ms, _stream(stream)), "autotune")
    return best, [(c, float(ms[i])) for i, c in enumerate(cands)]


def grid_for(p: Params, h_ref: float, cells_per_support: int) -> tuple:
    """Cells per axis with cells_per_support cells across the support 2 h_ref."""
    g = (C.c_int32 * 3)()
    _chk(lib().sphv_grid_for(C.byref(p), h_ref, cells_per_support, g), "grid_for")
    return tuple(int(v) for v in g)


def _grid_array(grids):
    flat = [int(v) for g in grids for v in g]
    return (C.c_int32 * len(flat))(*flat), len(grids)


def autotune_grid_workspace_bytes(d_density: Descriptor, d_force: Descriptor, n: int, p: Params, precision: int,
                                  l_density: Layout, l_force: Layout, grids) -> int:
    arr, k = _grid_array(grids)
    return int(lib().sphv_autotune_grid_workspace_bytes(C.byref(d_density), C.byref(d_force), n, C.byref(p),
                                                        precision, C.byref(l_density), C.byref(l_force), arr, k))


def autotune_grid(aos, d_density: Descriptor, d_force: Descriptor, n: int, p: Params, precision: int,
                  l_density: Layout, l_force: Layout, grids, ws, reps: int = 3, stream=None,
                  ws_bytes: int | None = None):
    """Times cells_build + density + force on every grid; returns (index of the
    fastest, list of (grid, median ms))."""
    grids = [tuple(g) for g in grids]
    arr, k = _grid_array(grids)
    ms = (C.c_float * k)()
    best = C.c_int32(-1)
    nb = ws_bytes if ws_bytes is not None else (ws.numel() if ws is not None else 0)
    _chk(lib().sphv_autotune_grid(_ptr(aos), C.byref(d_density), C.byref(d_force), n, C.byref(p), precision,
                                  C.byref(l_density), C.byref(l_force), arr, k, reps, _ptr(ws), nb,
                                  C.byref(best), ms, _stream(stream)), "autotune_grid")
    return int(best.value), [(g, float(ms[i])) for i, g in enumerate(grids)]


def layout_name(l: Layout) -> str:
    kind = {LAYOUT_SOA: "soa", LAYOUT_AOSOA: f"aosoa{l.aosoa_width}", LAYOUT_DIRECT: "direct",
            LAYOUT_SORTED: "sorted"}[l.kind]
    return f"{kind}/tpi{l.tpi or 'auto'}/{'masked' if l.masked else 'branch'}"


# ------------------------------------------------------------ step driver

class Stepper:
    """Owns the device buffers of one particle set and runs whole SPH steps
    through the C-ABI: cells_build, the density view (gather, density, scatter),
    the force view (gather, force + dt + sums, scatter) and kick_drift.

    layout_density / layout_force: Layout of each view (SPHV_LAYOUT_DIRECT runs
    the loops on the records themselves, SPHV_LAYOUT_SORTED on records moved
    into cell order after each cells_build).  sort_records: move the records
    into cell order after each cells_build (implied by a SORTED layout).  aos
    may be an (n*256,) uint8 device tensor holding 256-byte records, or None to
    upload ``rec``.  record_ptrs: a device uint64 tensor of n record addresses
    (records reached through an address list, DESC_RECORD_POINTERS): every
    call then takes the list, and ``aos`` must be the buffer the records live
    in (records() reads them back in list order).  merged: one view over both loops (MERGED_FIELDS, FP64,
    layout_density), gathered before the density loop and scattered after the
    force loop, so the density's outputs never leave the view in between.
    """

    def __init__(self, rec: np.ndarray, params: Params, precision: int = PREC_FP64,
                 layout_density: Layout | None = None, layout_force: Layout | None = None,
                 device="cuda", aos=None, stream=None, sort_records: bool = False, merged: bool = False,
                 record_ptrs=None, overlap: bool = False):
        import torch
        self.torch = torch
        self.ptrs = record_ptrs
        if record_ptrs is not None:
            self.n = record_ptrs.numel()
        else:
            self.n = rec.shape[0] if rec is not None else aos.numel() // inputs.STRIDE
        self.p = params
        self.precision = precision
        self.merged = merged
        # overlap: the force view's read-only members are prefetched on a side
        # stream (default priority) while the density loop runs
        self.overlap = overlap and not merged
        self.side = torch.cuda.Stream() if self.overlap else None
        self.pref_ev = torch.cuda.Event() if self.overlap else None
        if merged and precision != PREC_FP64:
            raise ValueError("a merged view is FP64: the FP32 force loop stages its members as floats, which a "
                             "view stores only for members it does not write")
        self.ld = layout_density or layout()
        self.lf = self.ld if merged else (layout_force or layout())
        self.sort_always = sort_records
        self.sort_ws = None
        self.stream = stream
        self.device = device
        if aos is None:
            aos = torch.from_numpy(inputs.as_bytes(np.ascontiguousarray(rec))).to(device)
        self.aos = aos
        # what the calls take as the records: the buffer, or the address list
        self.rec_arg = aos if record_ptrs is None else record_ptrs
        fl = 0 if record_ptrs is None else DESC_RECORD_POINTERS
        u8 = dict(dtype=torch.uint8, device=device)
        self.state = torch.zeros(state_bytes(), **u8)
        self.d_cells = cells_descriptor(fl)
        self.d_dens = density_descriptor(fl)
        self.d_force = force_descriptor(fl)
        self.d_kick = kick_descriptor(fl)
        self.d_merged = merged_descriptor(fl)
        self.v_dens = self.v_force = self.cells = None
        self._make_cells()
        self.set_layouts(self.ld, self.lf)
        state_init(self.state, self.stream)

    def _make_cells(self):
        u8 = dict(dtype=self.torch.uint8, device=self.device)
        self.cells_ws = self.torch.empty(max(256, cells_workspace_bytes(self.n, self.p)), **u8)
        self.cells = cells_create(self.n, self.p, self.cells_ws)
        self.perm_ptr = cells_get_info(self.cells).perm

    @property
    def sorting(self) -> bool:
        return self.sort_always or LAYOUT_SORTED in (self.ld.kind, self.lf.kind)

    # the pieces of a step, in order
    def build(self):
        begin_step(self.state, self.stream)
        cells_build(self.cells, self.rec_arg, self.d_cells, self.state, self.stream)
        if self.sorting:
            self._sort_workspace()
            records_sort(self.cells, self.aos, inputs.STRIDE, self.sort_ws, self.stream)

    def _sort_workspace(self):
        if self.sort_ws is None:
            nb = records_sort_workspace_bytes(inputs.STRIDE, self.n)
            self.sort_ws = self.torch.empty(max(256, nb), dtype=self.torch.uint8, device=self.device)

    def _main(self):
        return self.stream if self.stream is not None else self.torch.cuda.current_stream()

    def prefetch(self):
        """With overlap (after the density view opened, so that the members it
        writes are left out): the force view's other read-only members are
        gathered on the side stream, concurrently with the density loop."""
        if not self.overlap:
            return
        ev = self.torch.cuda.Event()
        ev.record(self._main())
        self.side.wait_event(ev)
        aos_to_soa_prefetch(self.v_force, self.cells, self.side)
        self.pref_ev.record(self.side)

    def density(self):
        aos_to_soa(self.v_dens, self.cells, self.stream)
        self.prefetch()
        sph_density(self.v_dens, self.cells, self.p, self.state, self.stream)
        if not self.merged:
            soa_to_aos(self.v_dens, self.stream)

    def force(self):
        if self.overlap:
            self._main().wait_event(self.pref_ev)
        if not self.merged:
            aos_to_soa(self.v_force, self.cells, self.stream)
        sph_force(self.v_force, self.cells, self.p, self.state, self.stream)
        step_reduce(self.v_force, self.p, self.state, self.stream)
        soa_to_aos(self.v_force, self.stream)

    def kick(self):
        kick_drift(self.rec_arg, self.d_kick, self.n, self.p, self.state, self.stream)

    def step(self):
        self.build()
        self.density()
        self.force()
        self.kick()

    def read_state(self) -> State:
        return read_state(self.state, self.stream)

    def set_layouts(self, layout_density: Layout | None = None, layout_force: Layout | None = None):
        """Re-plans the views (no view may be open)."""
        u8 = dict(dtype=self.torch.uint8, device=self.device)
        if self.merged:
            lay = layout_density or layout_force
            if lay is not None:
                self._destroy_views()
                self.ld = self.lf = lay
                self.ws_dens = self.torch.empty(max(256, view_workspace_bytes(self.d_merged, self.n, lay,
                                                                              self.precision)), **u8)
                self.v_dens = self.v_force = view_create(self.d_merged, self.n, lay, self.precision, self.rec_arg,
                                                         self.perm_ptr, self.ws_dens)
            if self.sorting:
                self._sort_workspace()
            return
        if layout_density is not None:
            if self.v_dens:
                view_destroy(self.v_dens)
            self.v_dens = None
            self.ld = layout_density
            self.ws_dens = self.torch.empty(max(256, view_workspace_bytes(self.d_dens, self.n, self.ld,
                                                                          self.precision)), **u8)
            self.v_dens = view_create(self.d_dens, self.n, self.ld, self.precision, self.rec_arg, self.perm_ptr,
                                      self.ws_dens)
        if layout_force is not None:
            if self.v_force:
                view_destroy(self.v_force)
            self.v_force = None
            self.lf = layout_force
            self.ws_force = self.torch.empty(max(256, view_workspace_bytes(self.d_force, self.n, self.lf,
                                                                           self.precision)), **u8)
            self.v_force = view_create(self.d_force, self.n, self.lf, self.precision, self.rec_arg, self.perm_ptr,
                                       self.ws_force)
        if self.sorting:
            self._sort_workspace()      # allocated here, never inside a graph capture

    def set_grid(self, grid):
        """Re-plans cells and views for another grid (no view may be open)."""
        self._destroy_views()
        cells_destroy(self.cells)
        self.cells = None
        q = params_init(tuple(self.p.lo), tuple(self.p.len), tuple(int(g) for g in grid), tuple(self.p.periodic))
        for name in ("gamma", "eta", "cfl", "h_tol", "headroom", "max_iter", "kernel"):
            setattr(q, name, getattr(self.p, name))
        self.p = q
        self._make_cells()
        self.set_layouts(self.ld, self.lf)

    def autotune(self, candidates=None, reps: int = 3, cells_per_support=None, h_ref: float | None = None,
                 within: float | None = None):
        """Picks the density and the force layouts on the current records (run
        after at least one step, so the force inputs are valid) and re-plans
        both views with them.  With cells_per_support (e.g. (1, 2)) it first
        picks the grid among sphv_grid_for(h_ref, k) for those k, h_ref
        defaulting to the records' largest h, and rebuilds the cells on it.
        candidates: None (the built-in set), a list for both loops, or a dict
        with a list per loop ("density", "force"); earlier candidates win ties.
        within: None keeps the library's choice (the first candidate within
        1.5 % of the fastest); a fraction takes the first candidate within that
        fraction of the fastest instead.
        The density layout is chosen first; the force layouts are then timed
        after one density pass with it (the records hold that pass's results
        afterwards).  Returns {"density": (best, table), "force": ...,
        ["grid": ...]}.  Not for a merged view (the tuner times each loop on a
        view of its own)."""
        if self.merged:
            raise ValueError("autotune times each loop on its own view; use set_layouts on a merged Stepper")
        out = {}
        if cells_per_support:
            if h_ref is None:
                h_ref = float(self.records()[:, inputs.SLOT["h"]].max())
            grids = []
            for k in cells_per_support:
                g = grid_for(self.p, h_ref, int(k))
                if g not in grids:
                    grids.append(g)
            if tuple(self.p.grid) not in grids:
                grids.append(tuple(self.p.grid))
            ld = self.ld if self.ld.kind != LAYOUT_SORTED else layout()
            lf = self.lf if self.lf.kind != LAYOUT_SORTED else layout()
            nb = autotune_grid_workspace_bytes(self.d_dens, self.d_force, self.n, self.p, self.precision, ld, lf,
                                               grids)
            ws = self.torch.empty(max(256, nb), dtype=self.torch.uint8, device=self.device)
            best, table = autotune_grid(self.aos, self.d_dens, self.d_force, self.n, self.p, self.precision, ld, lf,
                                        grids, ws, reps, self.stream)
            del ws
            out["grid"] = (grids[best], table)
            if grids[best] != tuple(self.p.grid):
                self.set_grid(grids[best])
        self.build()
        for loop, d, key in ((LOOP_DENSITY, self.d_dens, "density"), (LOOP_FORCE, self.d_force, "force")):
            cands = candidates.get(key) if isinstance(candidates, dict) else candidates
            nb = autotune_workspace_bytes(d, self.n, self.precision, cands)
            ws = self.torch.empty(max(256, nb), dtype=self.torch.uint8, device=self.device)
            out[key] = autotune(loop, self.aos, d, self.cells, self.p, self.precision, ws, cands, reps,
                                self.stream)
            del ws
            if within is not None:
                table = out[key][1]
                lo = min(ms for _, ms in table)
                out[key] = (next(c for c, ms in table if ms <= (1.0 + within) * lo), table)
            if loop == LOOP_DENSITY:
                # the force loop reuses the density loop's cached candidate masks
                # when both use the same lanes per particle; the density trials
                # left the cache of their last candidate, so one density pass
                # with the chosen layout sets the state a step gives the force loop
                self.set_layouts(layout_density=out["density"][0])
                self.build()
                self.density()
        self.set_layouts(layout_force=out["force"][0])
        return out

    def records(self) -> np.ndarray:
        self.torch.cuda.synchronize()
        if self.ptrs is not None:
            buf = self.aos.cpu().numpy()
            slots = (self.ptrs.cpu().numpy().astype(np.int64) - self.aos.data_ptr()) // inputs.STRIDE
            return buf.view(np.float64).reshape(-1, inputs.NSLOT)[slots].copy()
        return self.aos.cpu().numpy().view(np.float64).reshape(self.n, inputs.NSLOT).copy()

    def cells_arrays(self):
        """perm, cell_start, key and the reach arrays (density reach, force
        window, cover of the force reach; host copies) of the last cells_build
        and force call."""
        import torch
        info = cells_get_info(self.cells)
        nc = info.n_cells
        ws = self.cells_ws
        base = ws.data_ptr()

        def view_i32(ptr, count):
            off = ptr - base
            return ws[off:off + 4 * count].view(torch.int32).cpu().numpy().copy()

        torch.cuda.synchronize()
        return (view_i32(info.perm, self.n), view_i32(info.cell_start, nc + 1), view_i32(info.key, self.n),
                view_i32(info.reach, 3 * nc))

    def _destroy_views(self):
        vd, vf = getattr(self, "v_dens", None), getattr(self, "v_force", None)
        if vd:
            view_destroy(vd)
        if vf and vf is not vd:
            view_destroy(vf)
        self.v_dens = self.v_force = None

    def close(self):
        self._destroy_views()
        if getattr(self, "cells", None):
            cells_destroy(self.cells)
        self.v_dens = self.v_force = self.cells = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# every physics member of a record: the state a persistent view keeps in SoA
# across steps (all of it read and written by some step of the loop)
STATE_FIELDS = [(name, INOUT) for name in ("x", "y", "z", "vx", "vy", "vz", "vhx", "vhy", "vhz", "ax", "ay", "az",
                                           "m", "h", "rho", "omega", "u", "uh", "u_dt", "alpha", "v_sig",
                                           "wcount")]


class PersistentStepper:
    """The particle state kept in SoA across loops and steps (the paper's
    future work: a larger member set held in SoA instead of converted per loop).

    One view over every physics member of the records (STATE_FIELDS, SoA,
    FP64 storage) is opened once, in the cell order of a first cells_build,
    and stays open: its storage is the state.  Each step runs, through the
    C-ABI, cells_build on the storage's own x, y, z, h; the density and force
    loops over views of the storage (default: loops directly on it through the
    cells' perm, so no member is copied); the step reduction; kick_drift on the
    storage.  The records are written only by flush() (the view's scatter, then
    a new gather) and close(); until then their physics members are temporarily
    invalid (paper Sec. 3.2) and the alias rule keeps other views off them.
    precision: FP64 or FP32 pair arithmetic (the storage stays FP64);
    layout_density / layout_force: layouts of the loop views over the storage
    (SPHV_LAYOUT_DIRECT: no copy; SoA / AoSoA: gathered from the storage in
    cell order each step)."""

    def __init__(self, rec: np.ndarray, params: Params, precision: int = PREC_FP64,
                 layout_density: Layout | None = None, layout_force: Layout | None = None, device="cuda",
                 aos=None, stream=None):
        import torch
        self.torch = torch
        self.n = rec.shape[0] if rec is not None else aos.numel() // inputs.STRIDE
        self.p = params
        self.precision = precision
        self.stream = stream
        self.device = device
        self.ld = layout_density or layout(LAYOUT_DIRECT)
        self.lf = layout_force or layout(LAYOUT_DIRECT)
        if aos is None:
            aos = torch.from_numpy(inputs.as_bytes(np.ascontiguousarray(rec))).to(device)
        self.aos = aos
        u8 = dict(dtype=torch.uint8, device=device)
        n = self.n
        self.state = torch.zeros(state_bytes(), **u8)
        state_init(self.state, stream)
        # the records' cells, once: the order the storage starts in
        self.cells_ws = torch.empty(max(256, cells_workspace_bytes(n, params)), **u8)
        self.cells = cells_create(n, params, self.cells_ws)
        cells_build(self.cells, self.aos, cells_descriptor(), self.state, stream)
        self.index = torch.empty(max(n, 1), dtype=torch.int32, device=device)
        if n:
            # the perm copied out of the cells workspace (every build rewrites it)
            off = cells_get_info(self.cells).perm - self.cells_ws.data_ptr()
            self.index.view(torch.uint8)[:4 * n].copy_(self.cells_ws[off:off + 4 * n])
        self.d_state = descriptor(_rec_fields(STATE_FIELDS))
        lay = layout(LAYOUT_SOA)
        self.ws_state = torch.empty(max(256, view_workspace_bytes(self.d_state, n, lay, PREC_FP64)), **u8)
        self.v_state = view_create(self.d_state, n, lay, PREC_FP64, self.aos, self.index, self.ws_state)
        aos_to_soa(self.v_state, None, stream)
        # the storage as a struct-of-arrays store: member k at its own array
        base = self.ws_state.data_ptr()
        self.base = base
        offs = {}
        for k, (name, _) in enumerate(STATE_FIELDS):
            ptr, dt, bl, bb = view_field(self.v_state, k) if n else (base + 8 * k, F64, 0, 0)
            offs[name] = ptr - base

        def store_desc(spec):
            return descriptor([(nm, offs[nm], F64, acc) for nm, acc in spec], stride=8)

        self.d_cells = store_desc(CELLS_FIELDS)
        self.d_dens = store_desc(DENSITY_FIELDS)
        self.d_force = store_desc(FORCE_FIELDS)
        self.d_kick = store_desc(KICK_FIELDS)
        self.perm_ptr = cells_get_info(self.cells).perm
        self.v_dens = self.v_force = None
        self._make_views()

    def _make_views(self):
        u8 = dict(dtype=self.torch.uint8, device=self.device)
        n = self.n
        self.ws_dens = self.torch.empty(max(256, view_workspace_bytes(self.d_dens, n, self.ld, self.precision)), **u8)
        self.v_dens = view_create(self.d_dens, n, self.ld, self.precision, self.base, self.perm_ptr, self.ws_dens)
        self.ws_force = self.torch.empty(max(256, view_workspace_bytes(self.d_force, n, self.lf, self.precision)),
                                         **u8)
        self.v_force = view_create(self.d_force, n, self.lf, self.precision, self.base, self.perm_ptr,
                                   self.ws_force)

    # the pieces of a step, in order
    def build(self):
        begin_step(self.state, self.stream)
        cells_build(self.cells, self.base, self.d_cells, self.state, self.stream)

    def density(self):
        aos_to_soa(self.v_dens, self.cells, self.stream)
        sph_density(self.v_dens, self.cells, self.p, self.state, self.stream)
        soa_to_aos(self.v_dens, self.stream)

    def force(self):
        aos_to_soa(self.v_force, self.cells, self.stream)
        sph_force(self.v_force, self.cells, self.p, self.state, self.stream)
        step_reduce(self.v_force, self.p, self.state, self.stream)
        soa_to_aos(self.v_force, self.stream)

    def kick(self):
        kick_drift(self.base, self.d_kick, self.n, self.p, self.state, self.stream)

    def step(self):
        self.build()
        self.density()
        self.force()
        self.kick()

    def read_state(self) -> State:
        return read_state(self.state, self.stream)

    def flush(self):
        """Writes the state back to the records (the view's scatter) and opens
        the view again (a new gather, same order): the records hold the
        current state afterwards."""
        soa_to_aos(self.v_state, self.stream)
        aos_to_soa(self.v_state, None, self.stream)

    def records(self) -> np.ndarray:
        self.flush()
        self.torch.cuda.synchronize()
        return self.aos.cpu().numpy().view(np.float64).reshape(self.n, inputs.NSLOT).copy()

    def close(self):
        """Writes the state back to the records and releases the views."""
        if getattr(self, "v_state", None):
            for v in (self.v_dens, self.v_force):
                if v:
                    view_destroy(v)
            soa_to_aos(self.v_state, self.stream)
            self.torch.cuda.synchronize()
            view_destroy(self.v_state)
            cells_destroy(self.cells)
        self.v_state = self.v_dens = self.v_force = self.cells = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def params_for(w, **kw) -> Params:
    """Params of a generated workload (inputs.Workload)."""
    p = params_init(w.lo, w.length, w.grid, w.periodic)
    p.eta = w.eta
    for k, v in kw.items():
        setattr(p, k, v)
    return p
