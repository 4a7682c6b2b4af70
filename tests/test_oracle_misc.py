"""Pins of the oracle's exact pieces: view conversions (the paper's Listing 5/6
worked example and the identities of Sec. 4.2), binning and the stable sort
against brute force, kick/drift against the closed form for constant
acceleration, the sums, and the seeded generators."""
import math

import numpy as np
import pytest
from scipy import stats

from paper_2502_16517_amd import inputs


# ------------------------------------------------------------- conversions

def test_worked_example_struct_a_b_unused(orc):
    """struct {double a, b, _unused}; loop a += b over the view (paper Sec. 6,
    worked example): A_in = {a, b}, A_out = {a}; the view holds 16 B per
    element; b and _unused are never written back."""
    rng = np.random.default_rng(0)
    n = 37
    rec = rng.standard_normal((n, 3))
    rec[:, 2] = np.frombuffer(np.full(n, 0x7FF8000000ABCDEF, dtype=np.uint64).tobytes(), dtype=np.float64)
    aos = rec.reshape(-1).view(np.uint8).copy()
    before = aos.copy()
    soa = orc.gather(aos, 24, [(0, 8), (8, 8)])
    assert sum(v.nbytes for v in soa.values()) == 16 * n
    a = soa[0].view(np.float64)[:, 0]
    b = soa[8].view(np.float64)[:, 0]
    a_new = (a + b).reshape(-1, 1).view(np.uint8)
    orc.scatter(aos, 24, {0: a_new})
    after = aos.reshape(n, 24)
    old = before.reshape(n, 24)
    assert np.array_equal(after[:, 8:24], old[:, 8:24])                 # b, _unused untouched
    expect = (rec[:, 0] + rec[:, 1])
    assert np.array_equal(after[:, 0:8].copy().view(np.float64)[:, 0], expect)


def test_gather_scatter_roundtrip_is_identity(orc):
    rng = np.random.default_rng(1)
    n, stride = 300, 256
    aos = rng.integers(0, 256, size=n * stride, dtype=np.uint8)
    perm = rng.permutation(n)
    fields = [(0, 8), (8, 8), (96, 8), (104, 8), (248, 8)]
    soa = orc.gather(aos, stride, fields, perm)
    out = rng.integers(0, 256, size=n * stride, dtype=np.uint8)
    keep = out.copy()
    orc.scatter(out, stride, soa, perm)
    R, K, A = out.reshape(n, stride), keep.reshape(n, stride), aos.reshape(n, stride)
    covered = np.zeros(stride, bool)
    for off, sz in fields:
        covered[off:off + sz] = True
    assert np.array_equal(R[:, covered], A[:, covered])                  # W o N = id on the view
    assert np.array_equal(R[:, ~covered], K[:, ~covered])                # nothing else written


def test_relative_f32_rounding(orc):
    x = np.array([0.123456789012345, 0.5, 0.999999999])
    keys = np.array([5, 24, 47])
    rel = orc.relative_f32(x, keys, (48, 1, 1), (0.0, 0, 0), (1 / 48, 1, 1), 0)
    expect = np.array([np.float32(x[i] - (0.0 + keys[i] * (1 / 48))) for i in range(3)])
    assert np.array_equal(rel, expect)
    assert np.all(np.abs(rel) <= 1 / 48 + 1e-7)


def test_relative_f32_hand_derived_3d(orc):
    """Cell-relative FP32 coordinates (Sec. 4.2, the AoS-to-SoA operator with a
    change of representation) worked by hand on a 4 x 5 x 6 grid over the box
    [-1, 1] x [0, 1] x [2, 5]: cells 0.5 x 0.2 x 0.5.
      (0.3, 0.65, 3.7):   k = (2, 3, 3), key = (3*5 + 3)*4 + 2 = 74,
                          corner (0, 0.6, 3.5), offsets (0.3, 0.05, 0.2);
      (-0.9, 0.99, 4.99): k = (0, 4, 5), key = (5*5 + 4)*4 + 0 = 116,
                          corner (-1, 0.8, 4.5), offsets (0.1, 0.19, 0.49).
    Every axis has a non-zero cell index in the first point, so a swapped key
    decoding or a cell-centre origin moves some offset by at least 0.1."""
    grid, lo, L = (4, 5, 6), (-1.0, 0.0, 2.0), (2.0, 1.0, 3.0)
    cell = tuple(l / g for l, g in zip(L, grid))
    inv = tuple(g / l for g, l in zip(grid, L))
    pts = np.array([[0.3, 0.65, 3.7], [-0.9, 0.99, 4.99]])
    keys = orc.bin_keys(pts[:, 0], pts[:, 1], pts[:, 2], lo, inv, grid)
    assert keys.tolist() == [74, 116]
    expect = np.array([[0.3, 0.05, 0.2], [0.1, 0.19, 0.49]])
    for axis in range(3):
        rel = orc.relative_f32(pts[:, axis], keys, grid, lo, cell, axis)
        assert rel.dtype == np.float32
        # the real offset, to within one float32 ulp plus the rounding of the inputs
        tol = np.spacing(expect[:, axis].astype(np.float32)).astype(np.float64) + 1e-15
        assert np.all(np.abs(rel.astype(np.float64) - expect[:, axis]) <= tol), (axis, rel)


@pytest.mark.parametrize("gen", ["config1", "tube", "config3"])
def test_relative_f32_inside_own_cell(orc, gen):
    """Every particle of the lattice, the two-state tube and the 128^3 shear
    layer: its offset from the corner of the cell bin_keys puts it in lies in
    [0, c) along each axis (the face rule: a coordinate whose scaled offset
    rounds onto the next face may sit a few ulp below it), both before and
    after the rounding to float."""
    w = {"config1": inputs.config1, "tube": lambda: inputs.two_state_tube(16, 7),
         "config3": inputs.config3}[gen]()
    S = inputs.SLOT
    cell = tuple(l / g for l, g in zip(w.length, w.grid))
    inv = tuple(g / l for g, l in zip(w.grid, w.length))
    pos = [w.rec[:, S[k]] for k in ("x", "y", "z")]
    keys = orc.bin_keys(*pos, w.lo, inv, w.grid)
    for axis in range(3):
        rel = orc.relative_f32(pos[axis], keys, w.grid, w.lo, cell, axis).astype(np.float64)
        c = cell[axis]
        slack = 8 * np.spacing(np.float64(w.lo[axis] + w.length[axis]))
        assert rel.min() >= -slack, (axis, rel.min())
        assert rel.max() <= np.float64(np.float32(c)), (axis, rel.max(), c)
        # occupancy of the whole cell span: offsets reach close to both faces
        assert rel.max() > 0.5 * c


# ------------------------------------------------------------ binning, sort

def test_binning_against_brute_force(orc):
    rng = np.random.default_rng(2)
    n = 2000
    lo, L, grid = (-1.0, 0.0, 2.0), (2.0, 1.0, 3.0), (7, 5, 9)
    x = rng.uniform(lo[0], lo[0] + L[0], n)
    y = rng.uniform(lo[1], lo[1] + L[1], n)
    z = rng.uniform(lo[2], lo[2] + L[2], n)
    x[:5] = [lo[0], lo[0] + L[0], -7.0, 99.0, lo[0] + 3 * L[0] / 7]    # faces and outside
    inv = tuple(g / l for g, l in zip(grid, L))
    keys = orc.bin_keys(x, y, z, lo, inv, grid)
    for i in range(n):
        k = []
        for v, l, ic, g in zip((x[i], y[i], z[i]), lo, inv, grid):
            t = math.floor((v - l) * ic)
            k.append(min(max(t, 0), g - 1))
        assert keys[i] == (k[2] * grid[1] + k[1]) * grid[0] + k[0]
    ncell = grid[0] * grid[1] * grid[2]
    perm, start = orc.sort_cells(keys, ncell)
    assert sorted(perm.tolist()) == list(range(n))
    # brute force stable sort: by key, then by original index
    expect = sorted(range(n), key=lambda i: (keys[i], i))
    assert perm.tolist() == expect
    for c in range(ncell):
        assert start[c + 1] - start[c] == int(np.sum(keys == c))


def test_nonfinite_positions_go_to_cell_zero(orc):
    x = np.array([0.5, np.nan, np.inf]); y = np.full(3, 0.5); z = np.full(3, 0.5)
    keys = orc.bin_keys(x, y, z, (0, 0, 0), (4, 4, 4), (4, 4, 4))
    assert keys[1] == 0 and keys[2] == 0 and keys[0] != 0


# ------------------------------------------------------------- kick / drift

def _rec(n, rng):
    r = inputs.new_records(n)
    S = inputs.SLOT
    for k in ("x", "y", "z"):
        r[:, S[k]] = rng.uniform(0.3, 0.7, n)
    for k in ("vx", "vy", "vz"):
        r[:, S[k]] = rng.normal(0, 0.01, n)
    r[:, S["u"]] = 1.0
    return r


def test_kick_drift_constant_acceleration_closed_form(orc):
    """KDK leapfrog is exact for constant acceleration: x(t) = x0 + v0 t + a t^2/2."""
    rng = np.random.default_rng(4)
    S = inputs.SLOT
    r = _rec(50, rng)
    a = rng.normal(0, 0.1, (50, 3))
    r[:, [S["ax"], S["ay"], S["az"]]] = a
    r[:, S["u_dt"]] = 0.25
    x0 = r[:, [S["x"], S["y"], S["z"]]].copy()
    v0 = r[:, [S["vx"], S["vy"], S["vz"]]].copy()
    dt, t = 1e-3, 0.0
    for step in range(40):
        orc.kick_drift(r, S, dt, dt, step == 0, (0, 0, 0), (1, 1, 1), (1, 1, 1))
        t += dt
    # positions after 40 drifts; velocities v are the predicted ones at t
    x = r[:, [S["x"], S["y"], S["z"]]]
    assert np.max(np.abs(x - (x0 + v0 * t + 0.5 * a * t * t))) < 1e-14
    v = r[:, [S["vx"], S["vy"], S["vz"]]]
    assert np.max(np.abs(v - (v0 + a * t))) < 1e-14
    assert abs(r[0, S["u"]] - (1.0 + 0.25 * t)) < 1e-14


def test_kick_drift_is_reversible(orc):
    rng = np.random.default_rng(5)
    S = inputs.SLOT
    r = _rec(40, rng)
    r[:, [S["ax"], S["ay"], S["az"]]] = rng.normal(0, 0.1, (40, 3))
    orig = r.copy()
    orc.kick_drift(r, S, 1e-3, 0.0, True, (0, 0, 0), (1, 1, 1), (1, 1, 1))
    # reverse: close with dt, then open with -dt (v is re-predicted with the same a)
    orc.kick_drift(r, S, -1e-3, 1e-3, False, (0, 0, 0), (1, 1, 1), (1, 1, 1))
    for k in ("x", "y", "z"):
        assert np.max(np.abs(r[:, S[k]] - orig[:, S[k]])) < 1e-15


def test_kick_drift_wraps_periodic(orc):
    S = inputs.SLOT
    r = inputs.new_records(2)
    r[:, S["x"]] = [0.999, 0.001]
    r[:, S["vx"]] = [1.0, -1.0]
    orc.kick_drift(r, S, 0.01, 0.0, True, (0, 0, 0), (1, 1, 1), (1, 1, 1))
    assert 0.0 <= r[0, S["x"]] < 1.0 and 0.0 <= r[1, S["x"]] < 1.0
    assert math.isclose(r[0, S["x"]], 0.009, abs_tol=1e-15)
    assert math.isclose(r[1, S["x"]], 0.991, abs_tol=1e-15)


def test_time_step_takes_the_smallest_ratio(orc):
    """dt = C min_i h_i / v_sig,i with unequal h and v_sig: the ratios are 0.1
    and 0.05, so dt = 0.3 * 0.05 = 0.015; the largest ratio would give 0.03,
    min h / max v_sig 0.025 and min h / min v_sig 0.03."""
    h = np.array([0.1, 0.2])
    vsig = np.array([1.0, 4.0])
    assert math.isclose(orc.time_step(h, vsig, 0.3), 0.015, rel_tol=1e-15)
    assert math.isclose(orc.time_step(h[::-1], vsig[::-1], 0.3), 0.015, rel_tol=1e-15)


def test_conservation_sums(orc):
    m = np.array([1.0, 2.0]); v = np.array([3.0, -1.5]); z = np.zeros(2); u = np.array([0.5, 0.25])
    s = orc.conservation_sums(m, v, z, z, u)
    assert s[0] == 0.0 and s[3] == 1 * (4.5 + 0.5) + 2 * (1.125 + 0.25)


# -------------------------------------------------------------- generators

def test_generators_are_deterministic():
    a = inputs.config1().rec
    b = inputs.config1().rec
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))


def test_config_sizes():
    w = inputs.two_state_tube(16, 1)
    assert w.n == 16 ** 3 + 8 ** 3
    w1 = inputs.config1()
    assert w1.n == 4096 and w1.grid == (6, 6, 6)


def test_plummer_radial_distribution():
    w = inputs.plummer(20000, 9)
    S = inputs.SLOT
    r = np.sqrt(w.rec[:, S["x"]] ** 2 + w.rec[:, S["y"]] ** 2 + w.rec[:, S["z"]] ** 2)
    a = 0.1
    M = lambda s: s ** 3 / (s ** 2 + a ** 2) ** 1.5
    cdf = lambda s: M(np.minimum(s, 1.0)) / M(1.0)
    res = stats.kstest(r, cdf)
    assert res.pvalue > 1e-3
    assert r.max() <= 1.0
    # isotropy: mean direction near zero
    assert abs(np.mean(w.rec[:, S["z"]] / r)) < 0.03


# ------------------------------------------------- second level of dense cells

def test_sub_keys_by_hand(orc):
    """Sub-cell codes computed by hand: a unit grid of 2 cells per axis on
    [0, 2)^3 (cell 1, 16 sub-cells of 1/16 per axis)."""
    assert orc.SUB_BITS == 4
    # x in cell 1 at 1 + 5/16 (sub 5 = 0101b), y at 3/16 (sub 3 = 0011b), z at
    # 1 + 15/16 + tiny (sub 15 = 1111b): bits interleave x0 y0 z0 x1 y1 z1 ...
    x, y, z = np.array([1 + 5 / 16]), np.array([3 / 16]), np.array([1 + 15 / 16 + 1e-9])
    code = int(orc.sub_keys(x, y, z, (0, 0, 0), (1, 1, 1), (2, 2, 2))[0])
    sx, sy, sz = 5, 3, 15
    expect = 0
    for b in range(4):
        expect |= ((sx >> b) & 1) << (3 * b)
        expect |= ((sy >> b) & 1) << (3 * b + 1)
        expect |= ((sz >> b) & 1) << (3 * b + 2)
    assert code == expect == 0b100_101_110_111   # z3 y3 x3 | z2 y2 x2 | z1 y1 x1 | z0 y0 x0
    # the corner of a cell is sub-cell 0; just below the next cell is all ones
    c0 = orc.sub_keys(np.array([1.0]), np.array([1.0]), np.array([0.0]), (0, 0, 0), (1, 1, 1), (2, 2, 2))
    c1 = orc.sub_keys(np.array([1 - 1e-12]), np.array([2 - 1e-12]), np.array([0.999999]), (0, 0, 0), (1, 1, 1),
                      (2, 2, 2))
    assert int(c0[0]) == 0 and int(c1[0]) == 4095
    # outside an open box: clamped into the edge sub-cell
    c2 = orc.sub_keys(np.array([-0.5]), np.array([2.5]), np.array([0.5]), (0, 0, 0), (1, 1, 1), (2, 2, 2))
    sx, sy, sz = 0, 15, 8
    e2 = 0
    for b in range(4):
        e2 |= ((sx >> b) & 1) << (3 * b) | ((sy >> b) & 1) << (3 * b + 1) | ((sz >> b) & 1) << (3 * b + 2)
    assert int(c2[0]) == e2


def test_dense_cells_ordered_by_sub_cell(orc):
    """Cells of more than 64 particles are ordered by sub-cell code, ties by
    index; other cells keep index order; a brute-force sort agrees, the cell
    offsets are those of the plain sort, and consecutive runs of 64 inside a
    dense cell are compact (a small box) while index order is not."""
    rng = np.random.default_rng(11)
    n = 6000
    grid, lo, L = (3, 3, 3), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0)
    inv = tuple(g / l for g, l in zip(grid, L))
    # most particles crowd into the centre cell, the rest spread thinly
    centre = rng.random(n) < 0.8
    x, y, z = (np.where(centre, rng.uniform(1 / 3, 2 / 3, n), rng.uniform(0, 1, n)) for _ in range(3))
    keys = orc.bin_keys(x, y, z, lo, inv, grid)
    sub = orc.sub_keys(x, y, z, lo, inv, grid)
    ncell = 27
    perm, start = orc.sort_cells(keys, ncell, sub)
    p0, s0 = orc.sort_cells(keys, ncell)
    assert np.array_equal(start, s0)
    counts = np.diff(start)
    expect = sorted(range(n), key=lambda i: (keys[i], sub[i] if counts[keys[i]] > 64 else 0, i))
    assert perm.tolist() == expect
    assert counts.max() > 64 and (counts[(counts > 0) & (counts <= 64)]).size > 0
    for c in range(ncell):
        seg = perm[start[c]:start[c + 1]]
        if counts[c] > 64:
            assert np.all(np.diff(sub[seg]) >= 0)
        else:
            assert np.array_equal(seg, np.sort(seg))
    c = int(np.argmax(counts))
    seg = perm[start[c]:start[c + 1]]
    ext = lambda ids: max(np.ptp(x[ids]), np.ptp(y[ids]), np.ptp(z[ids]))
    runs = [ext(seg[k:k + 64]) for k in range(0, len(seg) - 63, 64)]
    plain = [ext(np.sort(seg)[k:k + 64]) for k in range(0, len(seg) - 63, 64)]
    assert np.mean(runs) < 0.5 * np.mean(plain)
