"""GPU parity of the list walks (sphv_params.list_cap > 0: per-particle
neighbour lists, one lane per particle) against the oracle, and the
invariances they promise: the view's layout does not change a bit; a list too
short for a particle (its window walked instead, the same candidates in the
same order) does not change a bit either; reruns are bit-identical."""
import numpy as np
import pytest

from paper_2502_16517_amd import inputs
from paper_2502_16517_amd import sphview as sv

from gpu_helpers import S, bits, check_density, check_force, oracle_density, oracle_force, run_density, \
    run_density_force

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CAP = 128

SMALL = {
    "lattice16": (lambda: inputs.config1(), {}),
    "tube16": (lambda: inputs.two_state_tube(16, 7), {}),
    "kh24": (lambda: inputs.kelvin_helmholtz(24, 9), {}),
    "plummer8k": (lambda: inputs.plummer(8192, 5, cell=0.1), {"headroom": 1.6}),
}


@pytest.mark.parametrize("name", list(SMALL))
def test_list_density_fp64_matches_oracle(orc, name):
    print(f"[list density fp64] {name}", flush=True)
    mk, pkw = SMALL[name]
    w = mk()
    out, state = run_density(w, list_cap=CAP, **pkw)
    assert state.flags & ~sv.F_OUT_OF_BOX == 0, state.flags
    ref = oracle_density(orc, w)
    worst = check_density(out, ref, tol=1e-12)
    print(worst)
    assert state.pairs_density == int(ref["count"].sum())
    assert state.max_iters == int(ref["iters"].max())
    keep = [k for k in range(inputs.NSLOT) if k not in (S["h"], S["rho"], S["omega"], S["wcount"])]
    assert np.array_equal(bits(out[:, keep]), bits(w.rec[:, keep]))


@pytest.mark.parametrize("name", list(SMALL))
def test_list_force_fp64_matches_oracle(orc, name):
    print(f"[list force fp64] {name}", flush=True)
    mk, pkw = SMALL[name]
    w = mk()
    dens, out, state = run_density_force(w, list_cap=CAP, **pkw)
    assert state.flags & ~sv.F_OUT_OF_BOX == 0, state.flags
    ref = oracle_force(orc, w, dens)
    worst = check_force(out, ref, tol=1e-12, vsig_tol=1e-14)
    print(worst)
    assert state.pairs_force == int(ref["count"].sum())
    dt = orc.time_step(dens[:, S["h"]], ref["vsig"], inputs.CFL)
    assert abs(state.dt / dt - 1) < 1e-14
    written = [S[k] for k in ("ax", "ay", "az", "u_dt", "v_sig")]
    keep = [k for k in range(inputs.NSLOT) if k not in written]
    assert np.array_equal(bits(out[:, keep]), bits(dens[:, keep]))


LAYOUTS = {
    "soa": sv.layout(sv.LAYOUT_SOA),
    "aosoa1": sv.layout(sv.LAYOUT_AOSOA, 1),
    "aosoa8": sv.layout(sv.LAYOUT_AOSOA, 8),
    "aosoa64": sv.layout(sv.LAYOUT_AOSOA, 64),
    "direct": sv.layout(sv.LAYOUT_DIRECT),
    "soa_masked_tpi4": sv.layout(sv.LAYOUT_SOA, masked=1, tpi=4),
}


@pytest.mark.parametrize("precision", [sv.PREC_FP64, sv.PREC_FP32])
def test_list_layouts_bit_identical(orc, precision):
    """The list walks read the view through its layout only: SoA, AoSoA and the
    records themselves give the same bits; tpi and masking do not apply."""
    w = inputs.two_state_tube(16, 11)
    tol = 1e-6 if precision == sv.PREC_FP32 else None
    res = {}
    for name, lay in LAYOUTS.items():
        print(f"[list layout] {name} prec={precision}", flush=True)
        _, out, state = run_density_force(w, precision=precision, lay=lay, tol=tol, list_cap=CAP)
        assert state.flags == 0
        res[name] = (out, state.dt, tuple(state.sums))
    ref = res["soa"]
    for name, (out, dt, sums) in res.items():
        assert np.array_equal(bits(out), bits(ref[0])), name
        assert dt == ref[1] and sums == ref[2], name


@pytest.mark.parametrize("precision", [sv.PREC_FP64, sv.PREC_FP32])
def test_short_lists_walk_the_window_bit_identical(orc, precision):
    """A list capacity below most particles' neighbour counts sends them to the
    window walk: the same candidates in the same order, so the same bits as
    with room for every list (and pair counts unchanged)."""
    w = inputs.two_state_tube(16, 7)
    tol = 1e-6 if precision == sv.PREC_FP32 else None
    outs = []
    for cap in (CAP, 24, 1):
        print(f"[list cap] {cap} prec={precision}", flush=True)
        dens, out, state = run_density_force(w, precision=precision, tol=tol, list_cap=cap)
        assert state.flags == 0
        outs.append((dens, out, state.pairs_density, state.pairs_force, state.pair_evals_density))
    for dens, out, pd, pf, pe in outs[1:]:
        assert np.array_equal(bits(dens), bits(outs[0][0]))
        assert np.array_equal(bits(out), bits(outs[0][1]))
        assert (pd, pf, pe) == outs[0][2:]


@pytest.mark.parametrize("precision", [sv.PREC_FP64, sv.PREC_FP32])
def test_dense_cells_lists_same_bits_as_window_walks(orc, precision):
    """A Plummer sphere whose core cells hold hundreds to thousands of
    particles: waves whose 64 particles share one dense cell build their lists
    from one walk of the shared window (candidates staged for the whole wave);
    the results are those of every particle walking its own window (a list
    capacity of one), bit for bit, with the same pair counts."""
    w = inputs.plummer(8192, 5, cell=0.1)
    tol = 1e-6 if precision == sv.PREC_FP32 else None
    outs = []
    for cap in (CAP, 1):
        print(f"[dense lists] cap {cap} prec={precision}", flush=True)
        dens, out, state = run_density_force(w, precision=precision, tol=tol, list_cap=cap, headroom=1.6)
        assert state.flags & ~sv.F_OUT_OF_BOX == 0, state.flags
        outs.append((dens, out, state.pairs_density, state.pairs_force, state.pair_evals_density))
    assert np.array_equal(bits(outs[1][0]), bits(outs[0][0]))
    assert np.array_equal(bits(outs[1][1]), bits(outs[0][1]))
    assert outs[1][2:] == outs[0][2:]


def _plummer_on_a_periodic_corner():
    """A Plummer sphere (radius 0.5) moved onto the corner of the periodic box
    [0, 2)^3: its dense core cells sit against all three periodic faces, so
    their windows wrap."""
    w = inputs.plummer(8192, 5, rmax=0.5, cell=0.1)
    rec = w.rec.copy()
    for k in ("x", "y", "z"):
        v = np.mod(rec[:, S[k]], 2.0)
        rec[:, S[k]] = np.where(v >= 2.0, v - 2.0, v)
    return inputs.Workload("plummer8k_periodic_corner", rec, (0.0, 0.0, 0.0), (2.0, 2.0, 2.0), (1, 1, 1),
                           (20, 20, 20), w.eta)


@pytest.mark.parametrize("precision", [sv.PREC_FP64, sv.PREC_FP32])
def test_dense_cells_across_periodic_faces(orc, precision):
    """Dense cells against periodic faces: the lists built by waves that share
    a dense cell (windows wrapping round the box) give the bits of every
    particle walking its own window, and (FP64) match the oracle."""
    w = _plummer_on_a_periodic_corner()
    tol = 1e-6 if precision == sv.PREC_FP32 else None
    outs = []
    for cap in (CAP, 1):
        print(f"[periodic dense lists] cap {cap} prec={precision}", flush=True)
        dens, out, state = run_density_force(w, precision=precision, tol=tol, list_cap=cap, headroom=1.6)
        assert state.flags == 0, state.flags
        outs.append((dens, out, state.pairs_density, state.pairs_force, state.pair_evals_density))
    assert np.array_equal(bits(outs[1][0]), bits(outs[0][0]))
    assert np.array_equal(bits(outs[1][1]), bits(outs[0][1]))
    assert outs[1][2:] == outs[0][2:]
    if precision == sv.PREC_FP64:
        dens, out = outs[0][0], outs[0][1]
        ref = oracle_density(orc, w)
        check_density(dens, ref, tol=1e-12)
        assert outs[0][2] == int(ref["count"].sum())
        fref = oracle_force(orc, w, dens)
        check_force(out, fref, tol=1e-12, vsig_tol=1e-14)
        assert outs[0][3] == int(fref["count"].sum())


def test_h_leaving_its_list_radius_matches_oracle(orc):
    """Starting h far below its converged value: h grows past the list radius
    (1 + 1/16 of the starting h) and those particles finish on the window walk;
    results still match the oracle from the same start."""
    w = inputs.config1()
    w.rec[:, S["h"]] *= 0.6
    out, state = run_density(w, list_cap=CAP)
    assert state.flags == 0, state.flags
    ref = oracle_density(orc, w)
    check_density(out, ref, tol=1e-12)
    assert state.pairs_density == int(ref["count"].sum())


@pytest.mark.parametrize("precision", [sv.PREC_FP64, sv.PREC_FP32])
def test_h_leaving_its_list_radius_same_bits_as_window(orc, precision):
    """Particles whose h outgrows the list radius hand their iteration over to
    the window walk mid-way; the window visits the list's candidates in the
    list's order, so the result has the bits of a run in which every particle
    walks its window from the first pass (a list too short for anyone)."""
    w = inputs.config1()
    w.rec[:, S["h"]] *= 0.6
    tol = 1e-6 if precision == sv.PREC_FP32 else None
    outs = []
    for cap in (CAP, 1):
        print(f"[list h leaving] cap={cap} prec={precision}", flush=True)
        dens, out, state = run_density_force(w, precision=precision, tol=tol, list_cap=cap)
        assert state.flags == 0, state.flags
        outs.append((dens, out, state.pairs_density, state.pair_evals_density, state.max_iters))
    assert np.array_equal(bits(outs[0][0]), bits(outs[1][0]))
    assert np.array_equal(bits(outs[0][1]), bits(outs[1][1]))
    assert outs[0][2:] == outs[1][2:]


def test_list_quartic_matches_oracle(orc):
    w = inputs.kelvin_helmholtz(24, 9)
    dens, out, state = run_density_force(w, list_cap=CAP, kernel=sv.KERNEL_QUARTIC)
    assert state.flags == 0
    check_density(dens, oracle_density(orc, w, kernel=sv.KERNEL_QUARTIC), tol=1e-12)
    check_force(out, oracle_force(orc, w, dens, kernel=sv.KERNEL_QUARTIC), tol=1e-12, vsig_tol=1e-14)


def test_list_fp32_within_budget(orc):
    w = inputs.kelvin_helmholtz(24, 9)
    dens, out, state = run_density_force(w, precision=sv.PREC_FP32, tol=1e-6, list_cap=CAP)
    assert state.flags == 0
    wd = check_density(dens, oracle_density(orc, w), tol=1e-5)
    wf = check_force(out, oracle_force(orc, w, dens), tol=1e-4, vsig_tol=1e-6)
    print("fp32 lists density", wd, "force", wf)


def test_list_matches_item_kernels_to_rounding(orc):
    """The list walks and the item kernels compute the same sums in different
    orders: equal to within the FP64 bound, pair counts exactly equal."""
    w = inputs.two_state_tube(16, 7)
    da, a, sa = run_density_force(w)
    db, b, sb = run_density_force(w, list_cap=CAP)
    assert (sa.pairs_density, sa.pairs_force) == (sb.pairs_density, sb.pairs_force)
    for k in ("h", "rho", "omega", "wcount"):
        assert np.max(np.abs(db[:, S[k]] / da[:, S[k]] - 1)) < 1e-12, k


def test_list_rerun_bit_identical(orc):
    w = inputs.kelvin_helmholtz(24, 9)
    _, a, sa = run_density_force(w, list_cap=CAP)
    _, b, sb = run_density_force(w, list_cap=CAP)
    assert np.array_equal(bits(a), bits(b))
    assert sa.dt == sb.dt and tuple(sa.sums) == tuple(sb.sums)


def test_list_graph_replay_matches_eager(orc):
    """Four steps with list walks replayed from one captured HIP graph give the
    bits of four eager steps (eager work and synchronisation between replays)."""
    w = inputs.two_state_tube(16, 5)
    p = sv.params_for(w, list_cap=CAP)
    sa = torch.cuda.Stream()
    a = sv.Stepper(w.rec, p, stream=sa)
    for _ in range(4):
        a.step()
    ra, sta = a.records(), a.read_state()
    a.close()
    sb = torch.cuda.Stream()
    b = sv.Stepper(w.rec, p, stream=sb)
    sv.graph_begin(sb)
    b.step()
    g = sv.graph_end(sb)
    torch.cuda.synchronize()
    junk = torch.zeros(1 << 20, device="cuda")
    for _ in range(4):
        sv.graph_launch(g, sb)
        junk.add_(1.0)
        torch.cuda.synchronize()
    rb, stb = b.records(), b.read_state()
    sv.graph_destroy(g)
    b.close()
    assert np.array_equal(bits(ra), bits(rb))
    assert sta.nstep == stb.nstep == 4
    assert sta.dt == stb.dt and tuple(sta.sums) == tuple(stb.sums)
