"""CPU oracle for the converted-view SPH hot path.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only users.  The product path never imports this
module, and nothing here imports the HIP library.

Two kinds of function live here:
  * exact definitions written with numpy (view conversions, binning and the
    stable sort, kick/drift, time step, conservation sums), and
  * thin ctypes calls into sph_oracle.c for the pair sums (density with the
    smoothing-length iteration, force), which are scalar double loops.

Inputs are record arrays from paper_2502_16517_amd.inputs (the shared seeded
generator, which holds no SPH arithmetic).
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

D = C.POINTER(C.c_double)
I64 = C.POINTER(C.c_int64)
I32 = C.POINTER(C.c_int32)


class Box(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("len", C.c_double * 3), ("periodic", C.c_int32 * 3)]


def box_of(lo, length, periodic) -> Box:
    b = Box()
    for d in range(3):
        b.lo[d] = float(lo[d])
        b.len[d] = float(length[d])
        b.periodic[d] = int(periodic[d])
    return b


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b  # noqa: WPS433
            _b.build()
        L = C.CDLL(path)
        for name in ("orc_w", "orc_dw", "orc_w5", "orc_dw5"):
            getattr(L, name).restype = C.c_double
            getattr(L, name).argtypes = [C.c_double]
        for name in ("orc_W", "orc_dWdr", "orc_dWdh"):
            getattr(L, name).restype = C.c_double
            getattr(L, name).argtypes = [C.c_int32, C.c_double, C.c_double]
        L.orc_density_at.restype = C.c_int
        L.orc_density_at.argtypes = [C.c_int64, D, D, D, D, C.POINTER(Box), C.c_int32, C.c_double,
                                     C.c_int64, I64, D, D, D, D, I64, C.c_int32, C.c_int32]
        L.orc_density.restype = C.c_int
        L.orc_density.argtypes = [C.c_int64, D, D, D, D, D, C.POINTER(Box), C.c_double, C.c_double,
                                  C.c_int32, C.c_int32, C.c_double, C.c_int64, I64,
                                  D, D, D, D, D, D, I64, I32, I32, C.c_int32, C.c_int32]
        L.orc_force.restype = C.c_int
        L.orc_force.argtypes = [C.c_int64] + [D] * 12 + [C.POINTER(Box), C.c_double, C.c_int32,
                                                         C.c_double, C.c_int64, I64] + [D] * 7 + \
                               [I64, C.c_int32, C.c_int32]
        L.orc_max_threads.restype = C.c_int
        _LIB = L
    return _LIB


def _d(a):
    return a.ctypes.data_as(D)


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ------------------------------------------------------------------ kernel

# kernel ids: 0 the cubic M4 spline, 1 the quartic M5 spline (both support 2h)
CUBIC, QUARTIC = 0, 1


def _kernel(kernel) -> int:
    k = int(kernel)
    if k not in (CUBIC, QUARTIC):
        raise ValueError(f"unknown kernel {kernel}")
    return k


def w(q: float, kernel: int = CUBIC) -> float:
    L = lib()
    return (L.orc_w5 if _kernel(kernel) == QUARTIC else L.orc_w)(float(q))


def dw(q: float, kernel: int = CUBIC) -> float:
    L = lib()
    return (L.orc_dw5 if _kernel(kernel) == QUARTIC else L.orc_dw)(float(q))


def W(r: float, h: float, kernel: int = CUBIC) -> float:
    return lib().orc_W(_kernel(kernel), float(r), float(h))


def dWdr(r: float, h: float, kernel: int = CUBIC) -> float:
    return lib().orc_dWdr(_kernel(kernel), float(r), float(h))


def dWdh(r: float, h: float, kernel: int = CUBIC) -> float:
    return lib().orc_dWdh(_kernel(kernel), float(r), float(h))


# --------------------------------------------------- view conversions (exact)

def gather(aos: np.ndarray, stride: int, fields, index=None) -> dict:
    """N o C (paper Sec. 4.2): for every field (offset, size) in A_in, the SoA
    array soa[p] = bytes of record index[p] at that offset.  Bit copies."""
    rec = aos.reshape(-1, stride)
    n = rec.shape[0] if index is None else len(index)
    idx = np.arange(n) if index is None else np.asarray(index)
    return {off: rec[idx, off:off + size].copy() for off, size in fields}


def scatter(aos: np.ndarray, stride: int, soa: dict, index=None) -> None:
    """C^T o W (paper Sec. 4.2): write back only the fields given (A_out)."""
    rec = aos.reshape(-1, stride)
    for off, arr in soa.items():
        idx = np.arange(arr.shape[0]) if index is None else np.asarray(index)
        rec[idx, off:off + arr.shape[1]] = arr


def cell_origin(keys, grid, lo, cell):
    """Lower corner of the cell with linear key (kz*ny + ky)*nx + kx, in double:
    lo_d + k_d * c_d, the product and the sum rounded separately."""
    keys = np.asarray(keys, dtype=np.int64)
    nx, ny, _ = grid
    k = [keys % nx, (keys // nx) % ny, keys // (nx * ny)]
    return [np.float64(lo[d]) + k[d].astype(np.float64) * np.float64(cell[d]) for d in range(3)]


def relative_f32(pos, keys, grid, lo, cell, axis):
    """FP32 view coordinate: float32(x - origin(cell)), nearest-even rounding."""
    o = cell_origin(keys, grid, lo, cell)[axis]
    return (np.asarray(pos, dtype=np.float64) - o).astype(np.float32)


# ---------------------------------------------------------- binning (exact)

def bin_keys(x, y, z, lo, inv_cell, grid):
    """k_d = clamp(floor((x_d - lo_d) * inv_c_d), 0, n_d - 1); key = (kz ny + ky) nx + kx.
    Non-finite coordinates go to key 0."""
    ks = []
    for v, l, ic, n in zip((x, y, z), lo, inv_cell, grid):
        t = np.floor((np.asarray(v, dtype=np.float64) - np.float64(l)) * np.float64(ic))
        t = np.where(np.isfinite(t), t, 0.0)
        ks.append(np.clip(t, 0, n - 1).astype(np.int64))
    nx, ny, _ = grid
    key = (ks[2] * ny + ks[1]) * nx + ks[0]
    bad = ~(np.isfinite(x) & np.isfinite(y) & np.isfinite(z))
    return np.where(bad, 0, key)


# Second level of the cells (a refinement of dense cells, as the paper's
# spacetree refines cells that hold many particles, Sec. 2.1): each cell is
# split into SUB^3 sub-cells, and inside a cell of more than DENSE particles
# the particles are ordered by the Morton (bit-interleaved) index of their
# sub-cell, so that consecutive runs of them are compact in space.
SUB_BITS = 4
DENSE = 64


def sub_keys(x, y, z, lo, inv_cell, grid):
    """Morton index of a particle's sub-cell inside its cell: along each axis
    t = (x - lo) * inv_cell (each step rounded, as for the key), k the cell
    index bin_keys takes (t floored and clamped to the grid), s =
    clamp(floor((t - k) * 2^SUB_BITS), 0, 2^SUB_BITS - 1); bit b of s_x, s_y,
    s_z goes to bit 3b, 3b+1, 3b+2 of the index.  Non-finite coordinates give 0."""
    n_sub = 1 << SUB_BITS
    s = []
    for v, l, ic, n in zip((x, y, z), lo, inv_cell, grid):
        t = (np.asarray(v, dtype=np.float64) - np.float64(l)) * np.float64(ic)
        ok = np.isfinite(t)
        t = np.where(ok, t, 0.0)
        k = np.clip(np.floor(t), 0, n - 1)
        q = np.floor((t - k) * np.float64(n_sub))
        s.append(np.clip(q, 0, n_sub - 1).astype(np.int64))
    code = np.zeros_like(s[0])
    for b in range(SUB_BITS):
        for d in range(3):
            code |= ((s[d] >> b) & 1) << (3 * b + d)
    bad = ~(np.isfinite(x) & np.isfinite(y) & np.isfinite(z))
    return np.where(bad, 0, code)


def sort_cells(keys, ncell, sub=None):
    """Order of the particles by cell, cell offsets.  Within a cell, particles
    keep their original index order (the stable sort by key); with sub given,
    inside cells of more than DENSE particles they are ordered by sub-cell
    index first, ties by original index."""
    keys = np.asarray(keys, dtype=np.int64)
    counts = np.bincount(keys, minlength=ncell)
    if sub is None:
        perm = np.argsort(keys, kind="stable").astype(np.int64)
    else:
        dense = counts[keys] > DENSE
        second = np.where(dense, np.asarray(sub, dtype=np.int64), 0)
        idx = np.arange(keys.shape[0], dtype=np.int64)
        perm = np.lexsort((idx, second, keys)).astype(np.int64)
    start = np.zeros(ncell + 1, dtype=np.int64)
    np.cumsum(counts, out=start[1:])
    return perm, start


# ---------------------------------------------------------- pair sums (C)

def density(x, y, z, m, h0, box: Box, eta, tol=1e-13, max_iter=16, brute=False,
            cell_hint=None, targets=None, nthreads=0, kernel=CUBIC):
    """Density with the smoothing-length iteration at the given targets."""
    x, y, z, m, h0 = map(_c64, (x, y, z, m, h0))
    n = x.shape[0]
    t = np.arange(n, dtype=np.int64) if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    nt = t.shape[0]
    if cell_hint is None:
        cell_hint = 2.0 * float(np.max(h0)) if n else 1.0
    out = {k: np.zeros(nt) for k in ("h", "rho", "omega", "wcount", "drho", "sdrho")}
    cnt = np.zeros(nt, dtype=np.int64)
    its = np.zeros(nt, dtype=np.int32)
    conv = np.zeros(nt, dtype=np.int32)
    rc = lib().orc_density(n, _d(x), _d(y), _d(z), _d(m), _d(h0), C.byref(box), eta, tol, max_iter,
                           int(brute), cell_hint, nt, t.ctypes.data_as(I64),
                           _d(out["h"]), _d(out["rho"]), _d(out["omega"]), _d(out["wcount"]),
                           _d(out["drho"]), _d(out["sdrho"]), cnt.ctypes.data_as(I64),
                           its.ctypes.data_as(I32), conv.ctypes.data_as(I32), nthreads, _kernel(kernel))
    if rc != 0:
        raise MemoryError("oracle density failed")
    out.update(count=cnt, iters=its, converged=conv)
    return out


def density_at(x, y, z, m, h_eval, box: Box, brute=False, cell_hint=None, targets=None, nthreads=0,
               kernel=CUBIC):
    """Density sums at fixed h (no iteration) at the given targets."""
    x, y, z, m = map(_c64, (x, y, z, m))
    n = x.shape[0]
    t = np.arange(n, dtype=np.int64) if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    he = _c64(np.broadcast_to(h_eval, t.shape))
    if cell_hint is None:
        cell_hint = 2.0 * float(np.max(he)) if len(he) else 1.0
    rho, drho, nsum = (np.zeros(t.shape[0]) for _ in range(3))
    cnt = np.zeros(t.shape[0], dtype=np.int64)
    rc = lib().orc_density_at(n, _d(x), _d(y), _d(z), _d(m), C.byref(box), int(brute), cell_hint,
                              t.shape[0], t.ctypes.data_as(I64), _d(he), _d(rho), _d(drho), _d(nsum),
                              cnt.ctypes.data_as(I64), nthreads, _kernel(kernel))
    if rc != 0:
        raise MemoryError("oracle density_at failed")
    return dict(rho=rho, drho=drho, nsum=nsum, count=cnt)


def force(x, y, z, vx, vy, vz, m, h, rho, omega, u, alpha, box: Box, gamma=5.0 / 3.0,
          brute=False, cell_hint=None, targets=None, nthreads=0, kernel=CUBIC):
    """Force (pressure with grad-h terms + signal-velocity viscosity) at targets."""
    arrs = list(map(_c64, (x, y, z, vx, vy, vz, m, h, rho, omega, u, alpha)))
    n = arrs[0].shape[0]
    t = np.arange(n, dtype=np.int64) if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    nt = t.shape[0]
    if cell_hint is None:
        cell_hint = 2.0 * float(np.median(arrs[7])) if n else 1.0
    out = {k: np.zeros(nt) for k in ("ax", "ay", "az", "udot", "vsig", "sa", "su")}
    cnt = np.zeros(nt, dtype=np.int64)
    rc = lib().orc_force(n, *[_d(a) for a in arrs], C.byref(box), gamma, int(brute), cell_hint,
                         nt, t.ctypes.data_as(I64), _d(out["ax"]), _d(out["ay"]), _d(out["az"]),
                         _d(out["udot"]), _d(out["vsig"]), _d(out["sa"]), _d(out["su"]),
                         cnt.ctypes.data_as(I64), nthreads, _kernel(kernel))
    if rc != 0:
        raise MemoryError("oracle force failed")
    out["count"] = cnt
    return out


def max_threads() -> int:
    return int(lib().orc_max_threads())


# ----------------------------------------------- time step, sums, kick/drift

def time_step(h, vsig, cfl):
    """dt = C_cfl * min_i h_i / v_sig,i (the division rounded per particle)."""
    return float(np.float64(cfl) * np.min(np.asarray(h, dtype=np.float64) / np.asarray(vsig, dtype=np.float64)))


def conservation_sums(m, vx, vy, vz, u, ax=None, ay=None, az=None, udot=None):
    """Long-double totals: P = sum m v, E = sum m (v^2/2 + u), and, when the
    accelerations are given, sum m a and dE/dt = sum m (v.a + du/dt)."""
    L = np.longdouble
    m, vx, vy, vz, u = (np.asarray(a, dtype=L) for a in (m, vx, vy, vz, u))
    out = [np.sum(m * vx), np.sum(m * vy), np.sum(m * vz),
           np.sum(m * (L(0.5) * (vx * vx + vy * vy + vz * vz) + u))]
    if ax is not None:
        ax, ay, az, udot = (np.asarray(a, dtype=L) for a in (ax, ay, az, udot))
        out += [np.sum(m * ax), np.sum(m * ay), np.sum(m * az),
                np.sum(m * (vx * ax + vy * ay + vz * az + udot))]
    return np.array(out, dtype=L)


def kick_drift(rec: np.ndarray, slot: dict, dt: float, dt_prev: float, first_step: bool,
               lo, length, periodic) -> None:
    """Kick-drift-kick leapfrog with prediction, in place on the records
    (paper Sec. 2.1 steps 3-5).  With a, du/dt evaluated at t_n:
      1. (not the first step) close the previous step:
         v = vh + a dt_prev/2,  u = uh + du/dt dt_prev/2
      2. open this step:   vh = v + a dt/2,  uh = u + du/dt dt/2
      3. drift:            x = wrap(x + vh dt)
      4. predict:          v = vh + a dt/2,  u = uh + du/dt dt/2
    Each product and sum is rounded on its own (numpy does not fuse)."""
    dt = np.float64(dt)
    half = np.float64(0.5) * dt
    half_prev = np.float64(0.5) * np.float64(dt_prev)
    ax = [rec[:, slot[k]] for k in ("ax", "ay", "az")]
    udot = rec[:, slot["u_dt"]]
    for d, (kv, kh, kx) in enumerate((("vx", "vhx", "x"), ("vy", "vhy", "y"), ("vz", "vhz", "z"))):
        v = rec[:, slot[kv]].copy()
        if not first_step:
            v = rec[:, slot[kh]] + ax[d] * half_prev
        vh = v + ax[d] * half
        xn = rec[:, slot[kx]] + vh * dt
        if periodic[d]:
            lo_d = np.float64(lo[d])
            L = np.float64(length[d])
            hi_d = lo_d + L
            xn = np.where(xn >= hi_d, xn - L, np.where(xn < lo_d, xn + L, xn))
        rec[:, slot[kx]] = xn
        rec[:, slot[kh]] = vh
        rec[:, slot[kv]] = vh + ax[d] * half
    u = rec[:, slot["u"]].copy()
    if not first_step:
        u = rec[:, slot["uh"]] + udot * half_prev
    uh = u + udot * half
    rec[:, slot["uh"]] = uh
    rec[:, slot["u"]] = uh + udot * half


# ---------------------------------------------------------- whole step

def step_fp64(rec: np.ndarray, slot: dict, box: Box, eta: float, cfl: float, gamma: float,
              tol: float = 1e-13, max_iter: int = 16, dt_prev: float = 0.0,
              first_step: bool = True, lo=None, length=None, periodic=None, nthreads=0,
              kernel: int = CUBIC):
    """One FP64 step on the records in place: density, force, dt, kick/drift.
    Returns a dict with dt, the pair counts and the per-particle outputs."""
    col = {k: rec[:, slot[k]] for k in slot}
    d = density(col["x"], col["y"], col["z"], col["m"], col["h"], box, eta, tol, max_iter,
                nthreads=nthreads, kernel=kernel)
    rec[:, slot["h"]] = d["h"]
    rec[:, slot["rho"]] = d["rho"]
    rec[:, slot["omega"]] = d["omega"]
    rec[:, slot["wcount"]] = d["wcount"]
    col = {k: rec[:, slot[k]] for k in slot}
    f = force(col["x"], col["y"], col["z"], col["vx"], col["vy"], col["vz"], col["m"], col["h"],
              col["rho"], col["omega"], col["u"], col["alpha"], box, gamma, nthreads=nthreads,
              kernel=kernel)
    rec[:, slot["ax"]] = f["ax"]
    rec[:, slot["ay"]] = f["ay"]
    rec[:, slot["az"]] = f["az"]
    rec[:, slot["u_dt"]] = f["udot"]
    rec[:, slot["v_sig"]] = f["vsig"]
    dt = time_step(d["h"], f["vsig"], cfl)
    sums = conservation_sums(col["m"], col["vx"], col["vy"], col["vz"], col["u"],
                             f["ax"], f["ay"], f["az"], f["udot"])
    kick_drift(rec, slot, dt, dt_prev, first_step, lo, length, periodic)
    return dict(dt=dt, density=d, force=f, sums=sums,
                pairs_density=int(d["count"].sum()), pairs_force=int(f["count"].sum()))
