"""Seeded synthetic particle sets in the 32-slot AoS record format.

This module is the one place that both the HIP path and the CPU oracle take
their inputs from.  It only lays out records and draws random numbers; it holds
none of the SPH arithmetic (no kernel, no density, no force).

Record layout (one particle = 32 slots of 8 bytes, stride 256 B).  The paper's
benchmark particle is a struct of a few up to hundreds of doubles mixing
physics and administration members (Sec. 2.2); this is a 32-slot instance of
that idea.  Slots 0..21 are physics members, 22..31 are "cold" administration
members that no SPH loop reads or writes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

STRIDE = 256
NSLOT = 32

# slot index of every named member (f64 unless listed in INT_SLOTS)
SLOT = {
    "x": 0, "y": 1, "z": 2,
    "vx": 3, "vy": 4, "vz": 5,
    "vhx": 6, "vhy": 7, "vhz": 8,
    "ax": 9, "ay": 10, "az": 11,
    "m": 12, "h": 13, "rho": 14, "omega": 15,
    "u": 16, "uh": 17, "u_dt": 18, "alpha": 19,
    "v_sig": 20, "wcount": 21,
    "id": 22, "cell_key": 23, "flags": 24, "h_iter": 25,
    "res0": 26, "res1": 27, "res2": 28, "res3": 29, "res4": 30, "res5": 31,
}
INT_SLOTS = ("id", "cell_key", "flags", "h_iter")
COLD_SLOTS = tuple(range(22, 32))

GAMMA = 5.0 / 3.0
ALPHA_VISC = 0.8
CFL = 0.3
# eta for 48 neighbours with support radius 2h:  (4 pi / 3) (2 eta)^3 = 48
ETA_48 = 0.5 * (36.0 / math.pi) ** (1.0 / 3.0)
ETA_LATTICE = 1.2


def new_records(n: int) -> np.ndarray:
    """Zeroed (n, 32) float64 array; one row is one 256-byte record."""
    return np.zeros((n, NSLOT), dtype=np.float64)


def as_bytes(rec: np.ndarray) -> np.ndarray:
    """The (n*256,) uint8 view of a record array (no copy)."""
    assert rec.dtype == np.float64 and rec.shape[1] == NSLOT and rec.flags.c_contiguous
    return rec.reshape(-1).view(np.uint8)


def int_slot(rec: np.ndarray, name: str) -> np.ndarray:
    """int64 view of an integer administration slot."""
    return rec.view(np.int64)[:, SLOT[name]]


def poison_cold(rec: np.ndarray, rng: np.random.Generator) -> None:
    """Fill the cold slots with arbitrary bit patterns, NaN payloads included."""
    bits = rng.integers(0, 2**63 - 1, size=(rec.shape[0], len(COLD_SLOTS)), dtype=np.int64)
    # a few quiet/signalling NaN payloads and infinities
    bits[:, 2] = np.int64(0x7FF8DEADBEEF0000) + np.arange(rec.shape[0], dtype=np.int64) % 4096
    bits[:, 3] = np.int64(0x7FF0000000000001)
    rec.view(np.int64)[:, list(COLD_SLOTS)] = bits
    int_slot(rec, "id")[:] = np.arange(rec.shape[0], dtype=np.int64)


@dataclass
class Workload:
    """A synthetic particle set plus the box and grid it is run on."""
    name: str
    rec: np.ndarray                      # (n, 32) float64 records
    lo: tuple                            # box lower corner
    length: tuple                        # box edge lengths
    periodic: tuple                      # per-axis periodicity (0/1)
    grid: tuple                          # cells per axis
    eta: float                           # target rho h^3 = m eta^3
    steps: int = 1
    notes: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.rec.shape[0]


def grid_for(length, h_ref: float, periodic, headroom: float = 1.1, min_cells: int = 3):
    """Cells per axis so that one cell spans at least 2*h_ref*headroom."""
    g = []
    for L, p in zip(length, periodic):
        n = int(math.floor(L / (2.0 * h_ref * headroom)))
        n = max(n, min_cells if p else 1)
        g.append(n)
    return tuple(g)


def _lattice(nx, ny, nz, s, origin=(0.0, 0.0, 0.0)):
    i = np.arange(nx, dtype=np.float64)
    j = np.arange(ny, dtype=np.float64)
    k = np.arange(nz, dtype=np.float64)
    Z, Y, X = np.meshgrid(k, j, i, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    return (pts + 0.5) * s + np.asarray(origin, dtype=np.float64)


def _fill_common(rec, pos, h, m, u, v=None, alpha=ALPHA_VISC):
    rec[:, SLOT["x"]] = pos[:, 0]
    rec[:, SLOT["y"]] = pos[:, 1]
    rec[:, SLOT["z"]] = pos[:, 2]
    if v is not None:
        rec[:, SLOT["vx"]] = v[:, 0]
        rec[:, SLOT["vy"]] = v[:, 1]
        rec[:, SLOT["vz"]] = v[:, 2]
    rec[:, SLOT["m"]] = m
    rec[:, SLOT["h"]] = h
    rec[:, SLOT["u"]] = u
    rec[:, SLOT["uh"]] = u
    rec[:, SLOT["alpha"]] = alpha
    # predicted-state slots start equal to the state itself
    rec[:, SLOT["vhx"]] = rec[:, SLOT["vx"]]
    rec[:, SLOT["vhy"]] = rec[:, SLOT["vy"]]
    rec[:, SLOT["vhz"]] = rec[:, SLOT["vz"]]


def _wrap(pos, lo, length):
    lo = np.asarray(lo)
    length = np.asarray(length)
    return lo + np.mod(pos - lo, length)


def lattice_box(n_side: int, seed: int, jitter: float = 0.1, u: float = 1.0,
                name: str | None = None, eta: float = ETA_LATTICE) -> Workload:
    """Jittered cubic lattice in the periodic unit box, equal masses, h = 1.2 s."""
    rng = np.random.Generator(np.random.PCG64(seed))
    s = 1.0 / n_side
    pos = _lattice(n_side, n_side, n_side, s)
    if jitter:
        pos = pos + rng.uniform(-jitter * s, jitter * s, size=pos.shape)
        pos = _wrap(pos, (0.0,) * 3, (1.0,) * 3)
    n = pos.shape[0]
    rec = new_records(n)
    _fill_common(rec, pos, h=1.2 * s, m=1.0 / n, u=u)
    poison_cold(rec, rng)
    lo, L, per = (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (1, 1, 1)
    return Workload(name or f"lattice{n_side}", rec, lo, L, per,
                    grid_for(L, 1.2 * s, per), eta)


def config1(seed: int = 16517 + 0) -> Workload:
    """16^3 jittered lattice (+-0.1 spacing), m = 1/N, h = 1.2 s, u = 1, v = 0."""
    w = lattice_box(16, seed, jitter=0.1, u=1.0, name="lattice16_fp64")
    return w


def two_state_tube(n_left: int, seed: int, jitter: float = 0.05,
                   fine_grid: bool = True, name: str | None = None) -> Workload:
    """Periodic box [0,2]x[0,1]^2: left half an n_left^3 lattice, right half an
    (n_left/2)^3 lattice, equal masses (density ratio 8), pressures 1 and 0.1."""
    assert n_left % 2 == 0
    rng = np.random.Generator(np.random.PCG64(seed))
    sl = 1.0 / n_left
    sr = 2.0 * sl
    pl = _lattice(n_left, n_left, n_left, sl)
    nr = n_left // 2
    pr = _lattice(nr, nr, nr, sr, origin=(1.0, 0.0, 0.0))
    pl = pl + rng.uniform(-jitter * sl, jitter * sl, size=pl.shape)
    pr = pr + rng.uniform(-jitter * sr, jitter * sr, size=pr.shape)
    pos = np.concatenate([pl, pr])
    lo, L, per = (0.0, 0.0, 0.0), (2.0, 1.0, 1.0), (1, 1, 1)
    pos = _wrap(pos, lo, L)
    n = pos.shape[0]
    m = 1.0 / pl.shape[0]                    # rho_left = 1
    h = np.concatenate([np.full(pl.shape[0], 1.2 * sl), np.full(pr.shape[0], 1.2 * sr)])
    # P = (gamma-1) rho u: left rho=1, P=1 -> u = 1.5 ; right rho=1/8, P=0.1 -> u = 1.2
    u = np.concatenate([np.full(pl.shape[0], 1.0 / ((GAMMA - 1.0) * 1.0)),
                        np.full(pr.shape[0], 0.1 / ((GAMMA - 1.0) * 0.125))])
    rec = new_records(n)
    _fill_common(rec, pos, h=h, m=m, u=u)
    poison_cold(rec, rng)
    h_ref = 1.2 * sl if fine_grid else 1.2 * sr
    return Workload(name or f"tube{n_left}", rec, lo, L, per, grid_for(L, h_ref, per),
                    ETA_LATTICE, steps=20)


def config2(seed: int = 16517 + 1, fine_grid: bool = True) -> Workload:
    """Two-state tube, 64^3 left block + 32^3 right block = 294,912 particles."""
    return two_state_tube(64, seed, fine_grid=fine_grid, name="tube64_fp64")


def kelvin_helmholtz(n_side: int, seed: int, name: str | None = None) -> Workload:
    """Unjittered n^3 lattice on the periodic unit box; density 2 in the band
    |y-0.5|<0.25 (by mass), 1 outside; vx = +-0.5, vy = 0.01 sin(4 pi x); P = 2.5."""
    rng = np.random.Generator(np.random.PCG64(seed))
    s = 1.0 / n_side
    pos = _lattice(n_side, n_side, n_side, s)
    n = pos.shape[0]
    band = np.abs(pos[:, 1] - 0.5) < 0.25
    rho = np.where(band, 2.0, 1.0)
    m = rho / n
    v = np.zeros_like(pos)
    v[:, 0] = np.where(band, 0.5, -0.5)
    v[:, 1] = 0.01 * np.sin(4.0 * math.pi * pos[:, 0])
    u = 2.5 / ((GAMMA - 1.0) * rho)
    rec = new_records(n)
    _fill_common(rec, pos, h=1.2 * s, m=m, u=u, v=v)
    poison_cold(rec, rng)
    lo, L, per = (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (1, 1, 1)
    return Workload(name or f"kh{n_side}", rec, lo, L, per, grid_for(L, 1.2 * s, per),
                    ETA_LATTICE, steps=1)


def config3(seed: int = 16517 + 2) -> Workload:
    return kelvin_helmholtz(128, seed, name="kh128")


def plummer(n: int, seed: int, a: float = 0.1, rmax: float = 1.0, cell: float = 0.02,
            name: str | None = None) -> Workload:
    """Plummer sphere sampled by inverting its mass profile, r = a / sqrt(U^(-2/3) - 1),
    rejecting r > rmax, in an open box [-1,1]^3.  m = 1/N, v = 0, u = 1.
    The starting h is eta (m / rho_Plummer(r))^(1/3)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty((0,), dtype=np.float64)
    while out.shape[0] < n:
        U = rng.uniform(0.0, 1.0, size=2 * n)
        U = U[U > 0.0]
        r = a / np.sqrt(U ** (-2.0 / 3.0) - 1.0)
        out = np.concatenate([out, r[r <= rmax]])
    r = out[:n]
    cth = rng.uniform(-1.0, 1.0, size=n)
    phi = rng.uniform(0.0, 2.0 * math.pi, size=n)
    sth = np.sqrt(1.0 - cth * cth)
    pos = np.stack([r * sth * np.cos(phi), r * sth * np.sin(phi), r * cth], axis=1)
    m = 1.0 / n
    mass_in = rmax ** 3 / (rmax ** 2 + a ** 2) ** 1.5      # untruncated mass inside rmax
    rho = (3.0 / (4.0 * math.pi * a ** 3)) * (1.0 + (r / a) ** 2) ** (-2.5) / mass_in
    h = ETA_48 * (m / rho) ** (1.0 / 3.0)
    rec = new_records(n)
    _fill_common(rec, pos, h=h, m=m, u=1.0)
    poison_cold(rec, rng)
    lo, L, per = (-1.0, -1.0, -1.0), (2.0, 2.0, 2.0), (0, 0, 0)
    g = int(round(2.0 / cell))
    return Workload(name or f"plummer{n}", rec, lo, L, per, (g, g, g), ETA_48)


def config4(seed: int = 16517 + 3) -> Workload:
    return plummer(1 << 20, seed, name="plummer1M")


def config5(seed: int = 16517 + 4) -> Workload:
    w = kelvin_helmholtz(256, seed, name="kh256")
    w.steps = 100
    return w


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}
