"""GPU checks of records stored cell by cell (the particle sort that moves
whole records so that each cell's particles are one contiguous chunk, paper
Sec. 2.2 and Sec. 5.2) and of loops over them (SPHV_LAYOUT_SORTED):

- the move is a bit-exact permutation of whole records (cold members and NaN
  payloads included) and leaves the cells valid for the moved records;
- on one step, loops over sorted records give the same bits as the SoA view
  over the unsorted records (the particles of a cell keep their order);
- over several steps they follow the SoA run to rounding, and graph replay
  of a step that sorts equals the eager steps;
- the grid tuner returns one of its candidates and leaves the records as
  they were, and a Stepper on the chosen grid still matches the oracle.
"""
import numpy as np
import pytest

from paper_2502_16517_amd import inputs
from paper_2502_16517_amd import sphview as sv

from gpu_helpers import S, bits, check_density, check_force, oracle_density, oracle_force

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SORTED = sv.layout(sv.LAYOUT_SORTED)


def ids(rec):
    return inputs.int_slot(rec, "id").copy()


def in_id_order(rec):
    """Rows in the order of their id slot (the generators number particles 0..n-1)."""
    return rec[np.argsort(ids(rec), kind="stable")]


def test_records_sort_moves_whole_records(orc):
    w = inputs.two_state_tube(16, 31)
    print(f"[records_sort] n={w.n}", flush=True)
    st = sv.Stepper(w.rec, sv.params_for(w))
    st.build()
    perm, start, key, _ = st.cells_arrays()
    before = st.records()
    ws = torch.empty(sv.records_sort_workspace_bytes(inputs.STRIDE, st.n), dtype=torch.uint8, device="cuda")
    sv.records_sort(st.cells, st.aos, inputs.STRIDE, ws)
    after = st.records()
    assert np.array_equal(bits(after), bits(before[perm]))
    perm2, start2, key2, _ = st.cells_arrays()
    assert np.array_equal(perm2, np.arange(st.n, dtype=np.int32))
    assert np.array_equal(start2, start)
    assert np.array_equal(key2, key[perm])
    # a new build of the moved records finds the same cells in storage order
    st.build()
    perm3, start3, key3, _ = st.cells_arrays()
    assert np.array_equal(perm3, np.arange(st.n, dtype=np.int32))
    assert np.array_equal(start3, start) and np.array_equal(key3, key2)
    st.close()


def test_sorted_layout_needs_sorted_records(orc):
    w = inputs.two_state_tube(8, 32)
    st = sv.Stepper(w.rec, sv.params_for(w))
    st.build()
    ws = torch.empty(sv.view_workspace_bytes(st.d_dens, st.n, SORTED, sv.PREC_FP64) + 256, dtype=torch.uint8,
                     device="cuda")
    v = sv.view_create(st.d_dens, st.n, SORTED, sv.PREC_FP64, st.aos, st.perm_ptr, ws)
    sv.aos_to_soa(v, st.cells)
    with pytest.raises(sv.SphvError) as e:
        sv.sph_density(v, st.cells, st.p, st.state)
    assert e.value.status == sv.E_STATE
    sv.soa_to_aos(v)
    sv.view_destroy(v)
    st.close()


def _one_step(w, precision, lay, tol):
    p = sv.params_for(w)
    if tol is not None:
        p.h_tol = tol
    st = sv.Stepper(w.rec, p, precision, layout_density=lay, layout_force=lay)
    st.build()
    st.density()
    dens = st.records()
    st.force()
    out = st.records()
    state = st.read_state()
    st.close()
    return dens, out, state


@pytest.mark.parametrize("precision", [sv.PREC_FP64, sv.PREC_FP32])
def test_sorted_records_bit_identical_to_views(orc, precision):
    w = inputs.two_state_tube(16, 33)
    tol = 1e-6 if precision == sv.PREC_FP32 else None
    print(f"[sorted vs soa] prec={precision}", flush=True)
    for tpi, masked in ((0, 0), (2, 1)):
        # lanes per particle fix the summation order: compare like with like
        _, ref, sref = _one_step(w, precision, sv.layout(tpi=tpi, masked=masked), tol)
        _, out, s = _one_step(w, precision, sv.layout(sv.LAYOUT_SORTED, tpi=tpi, masked=masked), tol)
        assert s.flags == 0
        assert not np.array_equal(ids(out), ids(ref))      # the records did move
        diff = bits(in_id_order(out)) != bits(ref)
        assert not diff.any(), (tpi, masked, np.nonzero(diff.any(axis=0))[0], int(diff.any(axis=1).sum()))
        assert s.dt == sref.dt and tuple(s.sums) == tuple(sref.sums)
        assert s.pairs_density == sref.pairs_density and s.pairs_force == sref.pairs_force


def test_sorted_step_matches_oracle(orc):
    w = inputs.kelvin_helmholtz(24, 34)
    print(f"[sorted oracle] n={w.n}", flush=True)
    p = sv.params_for(w)
    st = sv.Stepper(w.rec, p, layout_density=SORTED, layout_force=SORTED)
    st.build()
    srt = st.records()                     # records in cell order, inputs unchanged
    assert np.array_equal(bits(in_id_order(srt)), bits(w.rec))
    st.density()
    dens = st.records()
    check_density(dens, oracle_density(orc, w, rec=srt), tol=1e-12)
    st.force()
    out = st.records()
    check_force(out, oracle_force(orc, w, dens), tol=1e-12, vsig_tol=1e-14)
    st.close()


def test_sorted_multistep_follows_views(orc):
    """After the first step the particles of a cell come in the order of the
    previous sort, so sums run in another order: equal to rounding."""
    w = inputs.two_state_tube(24, 35)
    runs = {}
    for name, lay, srt in (("soa", sv.layout(), False), ("sorted", SORTED, True),
                           ("soa_on_sorted", sv.layout(), True)):
        st = sv.Stepper(w.rec, sv.params_for(w), layout_density=lay, layout_force=lay, sort_records=srt)
        for _ in range(4):
            st.step()
        runs[name] = (in_id_order(st.records()), st.read_state())
        st.close()
    ref, sref = runs["soa"]
    for name in ("sorted", "soa_on_sorted"):
        r, s = runs[name]
        assert s.flags == 0 and s.nstep == 4
        assert np.array_equal(ids(r), ids(ref))
        assert abs(s.dt / sref.dt - 1) < 1e-10, name
        for k in ("x", "y", "z", "vx", "vy", "vz", "u", "h", "rho"):
            a, b = r[:, S[k]], ref[:, S[k]]
            scale = np.max(np.abs(b)) + 1e-300
            assert np.max(np.abs(a - b)) <= 1e-9 * scale, (name, k)
    # the sorted layout and the SoA view over sorted records sum in the same order
    assert np.array_equal(bits(runs["sorted"][0]), bits(runs["soa_on_sorted"][0]))


def test_graph_replay_with_record_sort(orc):
    w = inputs.two_state_tube(16, 36)
    s = torch.cuda.Stream()
    a = sv.Stepper(w.rec, sv.params_for(w), layout_density=SORTED, layout_force=SORTED, stream=s)
    for _ in range(3):
        a.step()
    ra, sta = a.records(), a.read_state()
    a.close()
    b = sv.Stepper(w.rec, sv.params_for(w), layout_density=SORTED, layout_force=SORTED, stream=s)
    torch.cuda.synchronize()
    sv.graph_begin(s)
    b.step()
    g = sv.graph_end(s)
    torch.cuda.synchronize()
    junk = torch.zeros(1 << 20, device="cuda")
    for _ in range(3):
        sv.graph_launch(g, s)
        junk.add_(1.0)
        torch.cuda.synchronize()
    rb, stb = b.records(), b.read_state()
    sv.graph_destroy(g)
    b.close()
    assert np.array_equal(bits(ra), bits(rb))
    assert sta.nstep == stb.nstep == 3 and sta.dt == stb.dt and tuple(sta.sums) == tuple(stb.sums)


def test_autotune_sorted_candidates_restore_records(orc):
    w = inputs.two_state_tube(16, 37)
    st = sv.Stepper(w.rec, sv.params_for(w))
    st.step()
    st.build()
    before = st.records()
    perm0, start0, key0, _ = st.cells_arrays()
    cands = [sv.layout(), SORTED, sv.layout(sv.LAYOUT_SORTED, tpi=4, masked=1)]
    u8 = dict(dtype=torch.uint8, device="cuda")
    for loop, d in ((sv.LOOP_DENSITY, st.d_dens), (sv.LOOP_FORCE, st.d_force)):
        ws = torch.empty(sv.autotune_workspace_bytes(d, st.n, sv.PREC_FP64, cands), **u8)
        best, table = sv.autotune(loop, st.aos, d, st.cells, st.p, sv.PREC_FP64, ws, cands, reps=2)
        assert all(ms > 0 for _, ms in table)
        assert np.array_equal(bits(st.records()), bits(before)), loop
        perm, start, key, _ = st.cells_arrays()
        assert np.array_equal(perm, perm0) and np.array_equal(key, key0) and np.array_equal(start, start0)
    # the cells still serve the unsorted records: a step on them matches a fresh run
    st.density()
    st.force()
    out = st.records()
    st.close()
    st2 = sv.Stepper(w.rec, sv.params_for(w))
    st2.step()
    st2.build()
    st2.density()
    st2.force()
    ref = st2.records()
    st2.close()
    assert np.array_equal(bits(out), bits(ref))


def test_grid_tuner(orc):
    """Cells per support k = 1 (sized by the right state's h, left cells hold
    ~150 particles) and k = 2 (the left state's h): the tuner times both,
    leaves the records alone, and the step on the chosen grid matches the
    oracle."""
    w = inputs.two_state_tube(16, 38)
    p = sv.params_for(w)
    st = sv.Stepper(w.rec, p)
    st.step()
    before = st.records()
    h_ref = float(w.rec[:, S["h"]].max())
    grids = [sv.grid_for(st.p, h_ref, 1), sv.grid_for(st.p, h_ref, 2)]
    assert grids[1] == tuple(w.grid)
    nb = sv.autotune_grid_workspace_bytes(st.d_dens, st.d_force, st.n, st.p, sv.PREC_FP64, st.ld, st.lf, grids)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    best, table = sv.autotune_grid(st.aos, st.d_dens, st.d_force, st.n, st.p, sv.PREC_FP64, st.ld, st.lf, grids,
                                   ws, reps=2)
    print(table, flush=True)
    assert best in (0, 1) and all(ms > 0 for _, ms in table)
    fastest = min(ms for _, ms in table)
    assert best == next(k for k, (_, ms) in enumerate(table) if ms <= fastest * np.float32(1.015))
    assert np.array_equal(bits(st.records()), bits(before))
    # through the Stepper: choose, rebuild on the grid, step, check
    res = st.autotune(candidates=[sv.layout(), sv.layout(tpi=2)], reps=2, cells_per_support=(1, 2), h_ref=h_ref)
    assert res["grid"][0] in grids and tuple(st.p.grid) == res["grid"][0]
    rec0 = st.records()
    st.build()
    st.density()
    dens = st.records()
    check_density(dens, oracle_density(orc, w, rec=rec0), tol=1e-12)
    st.force()
    check_force(st.records(), oracle_force(orc, w, dens), tol=1e-12, vsig_tol=1e-14)
    st.close()


def test_coarse_grid_matches_oracle(orc):
    """The cells-per-support = 1 grid of the two-state tube (27-cell stencil,
    dense left cells) gives the oracle's results too."""
    w = inputs.two_state_tube(16, 39, fine_grid=False)
    p = sv.params_for(w)
    st = sv.Stepper(w.rec, p)
    st.build()
    st.density()
    dens = st.records()
    check_density(dens, oracle_density(orc, w), tol=1e-12)
    st.force()
    check_force(st.records(), oracle_force(orc, w, dens), tol=1e-12, vsig_tol=1e-14)
    st.close()


def _steps_by_hand(aos, stride, n, p, steps):
    """cells_build, density and force views (SoA), reduction and kick_drift
    through the C ABI on records of any stride at any 8-byte aligned base."""
    u8 = dict(dtype=torch.uint8, device="cuda")
    fields = lambda spec: [(name, inputs.SLOT[name] * 8, sv.F64, acc) for name, acc in spec]
    dc, dd, df, dk = (sv.descriptor(fields(s), stride=stride) for s in
                      (sv.CELLS_FIELDS, sv.DENSITY_FIELDS, sv.FORCE_FIELDS, sv.KICK_FIELDS))
    state = torch.zeros(sv.state_bytes(), **u8)
    sv.state_init(state)
    cws = torch.empty(sv.cells_workspace_bytes(n, p), **u8)
    cells = sv.cells_create(n, p, cws)
    perm = sv.cells_get_info(cells).perm
    lay = sv.layout()
    views = []
    for d in (dd, df):
        ws = torch.empty(sv.view_workspace_bytes(d, n, lay, sv.PREC_FP64), **u8)
        views.append((sv.view_create(d, n, lay, sv.PREC_FP64, aos, perm, ws), ws))
    (vd, _), (vf, _) = views
    for _ in range(steps):
        sv.begin_step(state)
        sv.cells_build(cells, aos, dc, state)
        sv.aos_to_soa(vd, cells)
        sv.sph_density(vd, cells, p, state)
        sv.soa_to_aos(vd)
        sv.aos_to_soa(vf, cells)
        sv.sph_force(vf, cells, p, state)
        sv.step_reduce(vf, p, state)
        sv.soa_to_aos(vf)
        sv.kick_drift(aos, dk, n, p, state)
    st = sv.read_state(state)
    for v, _ in views:
        sv.view_destroy(v)
    sv.cells_destroy(cells)
    return st


def test_any_stride_and_alignment_bit_identical(orc):
    """Records whose stride (264 B) or base (8 B past a 16-B boundary) rule out
    the LDS staging of the conversions, kick and binning run the plain kernels:
    the same bits as the staged ones on 256-B records."""
    w = inputs.two_state_tube(16, 40)
    n = w.n
    p = sv.params_for(w)
    st = sv.Stepper(w.rec, p)
    for _ in range(2):
        st.step()
    ref, sref = st.records(), st.read_state()
    st.close()
    # stride 264: one extra slot holding a marker after every record
    wide = np.zeros((n, 33))
    wide[:, :32] = w.rec
    wide[:, 32] = np.arange(n) + 0.5
    buf = torch.from_numpy(wide.reshape(-1).view(np.uint8).copy()).cuda()
    s264 = _steps_by_hand(buf, 264, n, p, 2)
    got = buf.cpu().numpy().view(np.float64).reshape(n, 33)
    assert np.array_equal(bits(np.ascontiguousarray(got[:, :32])), bits(ref))
    assert np.array_equal(got[:, 32], np.arange(n) + 0.5)
    # stride 256 at a base 8 bytes past a 16-byte boundary
    raw = torch.zeros(n * 256 + 16, dtype=torch.uint8, device="cuda")
    aos = raw[8:8 + n * 256]
    assert aos.data_ptr() % 16 == 8
    aos.copy_(torch.from_numpy(inputs.as_bytes(np.ascontiguousarray(w.rec)).copy()).cuda())
    s8 = _steps_by_hand(aos, 256, n, p, 2)
    got8 = aos.cpu().numpy().view(np.float64).reshape(n, 32)
    assert np.array_equal(bits(got8), bits(ref))
    for s in (s264, s8):
        assert s.flags == sref.flags and s.nstep == 2
        assert s.dt == sref.dt and tuple(s.sums) == tuple(sref.sums)
