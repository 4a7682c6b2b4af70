"""GPU parity of cells_build (bit-exact keys, stable sort, offsets) and of the
view conversions (bit-exact gather / scatter of exactly the view's members),
through the C-ABI, against the oracle's definitions."""
import numpy as np
import pytest

from paper_2502_16517_amd import inputs
from paper_2502_16517_amd import sphview as sv

from gpu_helpers import S, bits

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

WORKLOADS = {
    "lattice16": lambda: inputs.config1(),
    "tube16": lambda: inputs.two_state_tube(16, 7),
    "kh24": lambda: inputs.kelvin_helmholtz(24, 9),
    "plummer8k": lambda: inputs.plummer(8192, 5, cell=0.1),
    # 2^20 particles in cells of 0.02: thousands of cells of more than 64
    "plummer1M": lambda: inputs.config4(),
}


def _stepper(w, **kw):
    # the open Plummer box needs room for h to grow; lattices keep the default
    p = sv.params_for(w, headroom=1.6) if not any(w.periodic) else sv.params_for(w)
    return sv.Stepper(w.rec, p, **kw)


@pytest.mark.parametrize("name", list(WORKLOADS))
def test_cells_build_exact(orc, name):
    print(f"[cells] {name}", flush=True)
    w = WORKLOADS[name]()
    st = _stepper(w)
    st.build()
    perm, start, key, _ = st.cells_arrays()
    state = st.read_state()
    st.close()
    p = sv.params_for(w)
    c = w.rec
    ref_key = orc.bin_keys(c[:, S["x"]], c[:, S["y"]], c[:, S["z"]], w.lo, list(p.inv_cell), w.grid)
    ref_sub = orc.sub_keys(c[:, S["x"]], c[:, S["y"]], c[:, S["z"]], w.lo, list(p.inv_cell), w.grid)
    nc = w.grid[0] * w.grid[1] * w.grid[2]
    ref_perm, ref_start = orc.sort_cells(ref_key, nc, ref_sub)
    assert np.array_equal(key, ref_key)
    assert np.array_equal(start, ref_start)
    assert np.array_equal(perm, ref_perm)
    assert state.flags & ~sv.F_OUT_OF_BOX == 0


def _window_model(w, own):
    """Exact force window: R_f(A) = max(R(A), max{d : a cell B at Chebyshev
    distance d has own reach R(B) >= d}); and the cover G(A) = max{R(B) : B at
    Chebyshev distance d <= R(B)}, the largest own reach among the cells whose
    reach covers A."""
    g = tuple(int(v) for v in w.grid)
    R = own.reshape(g[2], g[1], g[0])
    Rg = int(R.max())
    out = R.copy()
    cover = R.copy()
    for dz in range(-Rg, Rg + 1):
        for dy in range(-Rg, Rg + 1):
            for dx in range(-Rg, Rg + 1):
                d = max(abs(dx), abs(dy), abs(dz))
                if d == 0:
                    continue
                sh = np.roll(R, shift=(-dz, -dy, -dx), axis=(0, 1, 2))   # sh[A] = R[A + offset]
                valid = np.ones_like(R, dtype=bool)
                for ax, off, per in ((2, dx, w.periodic[0]), (1, dy, w.periodic[1]), (0, dz, w.periodic[2])):
                    if not per:
                        idx = np.arange(R.shape[ax]) + off
                        shape = [1, 1, 1]
                        shape[ax] = -1
                        valid &= ((idx >= 0) & (idx < R.shape[ax])).reshape(shape)
                out = np.maximum(out, np.where(valid & (sh >= d), d, 0))
                cover = np.maximum(cover, np.where(valid & (sh >= d), sh, 0))
    return out.ravel(), Rg, cover.ravel()


def _own_force_reach(h, start, nc, cmin):
    own = np.zeros(nc, dtype=np.int64)
    for c in range(nc):
        if start[c + 1] > start[c]:
            # 2 h of the cell's largest h rounded up to float, as the kernel folds it
            H = 2.0 * h[start[c]:start[c + 1]].max()
            f = np.float32(H)
            if float(f) < H:
                f = np.nextafter(f, np.float32(np.inf))
            own[c] = max(1, int(np.ceil(float(f) * (1.0 + 1e-12) / cmin)))
    return own


@pytest.mark.parametrize("steps", [1, 6])
def test_force_window_is_exact(orc, steps):
    """The force loop's window of every cell holds each cell whose own force
    reach (from the converged h, no headroom) covers it, and for R_global <= 4
    on long periodic axes nothing more."""
    w = inputs.two_state_tube(24, 31)
    st = _stepper(w)
    for _ in range(steps):
        st.step()
    perm, start, _, reach = st.cells_arrays()
    rec = st.records()
    p = st.p
    st.close()
    nc = w.grid[0] * w.grid[1] * w.grid[2]
    rf = reach[nc:2 * nc]
    rs = reach[2 * nc:3 * nc]
    h = rec[perm, S["h"]]
    cmin = min(p.cell[0], p.cell[1], p.cell[2])
    own = _own_force_reach(h, start, nc, cmin)
    exact, Rg, cover = _window_model(w, own)
    assert (rf >= exact).all()
    if all(2 * Rg + 1 <= n for n in w.grid):
        assert np.array_equal(rs, cover)
    if Rg <= 4 and all(2 * Rg + 1 <= n for n in w.grid):
        assert np.array_equal(rf, exact)


def test_force_window_cover_open_box(orc):
    """A Plummer sphere in an open box, cells of 0.05: the halo's h spans many
    cells (global reach above 4), so every cell's window is the cover G, the
    largest own reach among the cells whose reach covers it."""
    w = inputs.plummer(65536, 5, cell=0.05)
    st = _stepper(w)
    for _ in range(2):
        st.step()
    perm, start, _, reach = st.cells_arrays()
    rec = st.records()
    p = st.p
    st.close()
    nc = w.grid[0] * w.grid[1] * w.grid[2]
    rf = reach[nc:2 * nc]
    rs = reach[2 * nc:3 * nc]
    h = rec[perm, S["h"]]
    own = _own_force_reach(h, start, nc, min(p.cell[0], p.cell[1], p.cell[2]))
    exact, Rg, cover = _window_model(w, own)
    assert Rg > 4
    assert np.array_equal(rs, cover)
    assert np.array_equal(rf, cover)
    assert (cover >= exact).all()
    # the particles' windows stay well inside +-R_global (the core's cells are
    # covered only by their neighbours' small reaches)
    key = np.repeat(np.arange(nc), np.diff(start))
    assert cover[key].mean() < 0.5 * Rg


def test_cells_flags_nonfinite(orc):
    w = inputs.config1()
    w.rec[5, S["x"]] = np.nan
    w.rec[9, S["h"]] = np.inf
    st = _stepper(w)
    st.build()
    perm, start, key, _ = st.cells_arrays()
    state = st.read_state()
    st.close()
    assert state.flags & sv.F_NONFINITE_INPUT
    assert key[5] == 0
    assert sorted(perm.tolist()) == list(range(w.n))


def _view_arrays(ws, view, n, fields, precision=sv.PREC_FP64):
    """Host copies of the view's member arrays (SoA layout)."""
    torch.cuda.synchronize()
    base = ws.data_ptr()
    out = []
    for k in range(len(fields)):
        ptr, dt, bl, bb = sv.view_field(view, k)
        size = 4 if dt in (sv.F32, sv.I32) else 8
        off = ptr - base
        out.append(ws[off:off + size * n].cpu().numpy().copy())
    return out


@pytest.mark.parametrize("precision", [sv.PREC_FP64, sv.PREC_FP32])
def test_gather_bit_exact(orc, precision):
    w = inputs.config1()
    st = _stepper(w, precision=precision)
    st.build()
    perm, _, key, _ = st.cells_arrays()
    sv.aos_to_soa(st.v_force, st.cells)
    got = _view_arrays(st.ws_force, st.v_force, w.n, sv.FORCE_FIELDS, precision)
    sv.soa_to_aos(st.v_force)
    st.close()
    aos = inputs.as_bytes(w.rec)
    p = sv.params_for(w)
    for (name, acc), g in zip(sv.FORCE_FIELDS, got):
        if acc == sv.OUT:
            continue
        off = S[name] * 8
        if precision == sv.PREC_FP64:
            ref = orc.gather(aos, 256, [(off, 8)], perm)[off].reshape(-1)
            assert np.array_equal(g, ref), name
        else:
            v = w.rec[perm, S[name]]
            if name in ("x", "y", "z"):
                ax = "xyz".index(name)
                ref = orc.relative_f32(v, key[perm], w.grid, w.lo, list(p.cell), ax)
            else:
                ref = v.astype(np.float32)
            assert np.array_equal(g.view(np.float32), ref), name


@pytest.mark.parametrize("lay", [sv.layout(sv.LAYOUT_SOA), sv.layout(sv.LAYOUT_AOSOA, 16),
                                 sv.layout(sv.LAYOUT_AOSOA, 64)])
def test_scatter_writes_only_a_out(orc, lay):
    """After gather + scatter with no loop in between, the records differ from
    the input only in A_out \\ A_in, which the view never initialised; every
    other byte, cold members with NaN payloads included, is unchanged."""
    w = inputs.config1()
    st = _stepper(w, layout_density=lay, layout_force=lay)
    st.build()
    before = st.records()
    sv.aos_to_soa(st.v_dens, st.cells)
    sv.soa_to_aos(st.v_dens)
    after = st.records()
    st.close()
    touched = [S[k] for k, acc in sv.DENSITY_FIELDS if acc == sv.OUT]
    keep = [k for k in range(inputs.NSLOT) if k not in touched]
    assert np.array_equal(bits(before[:, keep]), bits(after[:, keep]))
    # h is A_in and A_out: round trip is the identity (W o N = id)
    assert np.array_equal(bits(before[:, S["h"]]), bits(after[:, S["h"]]))


def test_worked_example_struct_on_gpu(orc):
    """struct {double a, b, _unused}, loop a += b over the view (paper Sec. 6
    worked example), container order as the index."""
    rng = np.random.default_rng(3)
    n = 1000
    rec = rng.standard_normal((n, 3))
    rec[:, 2] = np.frombuffer(np.full(n, 0x7FF4000000000ABC, dtype=np.uint64).tobytes(), dtype=np.float64)
    aos = torch.from_numpy(rec.reshape(-1).view(np.uint8).copy()).cuda()
    d = sv.descriptor([(None, 0, sv.F64, sv.INOUT), (None, 8, sv.F64, sv.IN)], stride=24)
    l = sv.layout()
    nb = sv.view_workspace_bytes(d, n, l, sv.PREC_FP64)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    v = sv.view_create(d, n, l, sv.PREC_FP64, aos, None, ws)
    sv.aos_to_soa(v)
    pa, _, _, _ = sv.view_field(v, 0)
    pb, _, _, _ = sv.view_field(v, 1)
    base = ws.data_ptr()
    a = ws[pa - base: pa - base + 8 * n].view(torch.float64)
    b = ws[pb - base: pb - base + 8 * n].view(torch.float64)
    a += b                                    # the loop body, on the view
    sv.soa_to_aos(v)
    sv.view_destroy(v)
    got = aos.cpu().numpy().view(np.float64).reshape(n, 3)
    assert np.array_equal(got[:, 0], rec[:, 0] + rec[:, 1])
    assert np.array_equal(bits(got[:, 1:]), bits(rec[:, 1:]))
    assert nb >= 16 * n


def test_out_only_members_do_not_leak(orc):
    """Poisoned A_out \\ A_in members (rho, omega, wcount) must not change any
    density result (paper Sec. 3.1: they need no preparation)."""
    w = inputs.config1()
    a = _run_density_records(w)
    rec = w.rec.copy()
    rec[:, S["rho"]] = np.nan
    rec[:, S["omega"]] = -1e300
    rec[:, S["wcount"]] = np.inf
    b = _run_density_records(w, rec)
    assert np.array_equal(bits(a), bits(b))


def _run_density_records(w, rec=None):
    from gpu_helpers import run_density
    out, state = run_density(w, rec=rec)
    assert state.flags == 0
    return out


@pytest.mark.parametrize("where", ["above", "below", "inside"])
def test_unwrapped_periodic_coordinate_is_flagged(orc, where):
    """A coordinate outside [lo, lo + len) on a periodic axis sets
    SPHV_F_OUT_OF_BOX (it is binned into an edge cell, whose window misses
    pairs across that face); wrapped records set no flag."""
    print(f"[cells] periodic face {where}", flush=True)
    w = inputs.config1()
    rec = w.rec.copy()
    if where == "above":
        rec[7, S["y"]] = np.nextafter(1.0, 2.0)          # just past the upper face
    elif where == "below":
        rec[7, S["z"]] = -1e-9                            # just below the lower face
    else:
        rec[7, S["x"]] = np.nextafter(1.0, 0.0)          # the last double inside
    st = sv.Stepper(rec, sv.params_for(w))
    st.build()
    state = st.read_state()
    st.close()
    if where == "inside":
        assert state.flags == 0
    else:
        assert state.flags & sv.F_OUT_OF_BOX
