"""The state kept in SoA across loops and steps (PersistentStepper: one view
over every physics member, opened once; loops, step reduction and kick_drift
on its storage; records written only on request).  Every step is checked
against the oracle from that step's input; the run follows the per-loop
views to rounding; graph replay gives the eager bits; the records are not
touched between flushes."""
import numpy as np
import pytest

from paper_2502_16517_amd import inputs
from paper_2502_16517_amd import sphview as sv

from gpu_helpers import S, bits, check_density, check_force, cols, oracle_density, oracle_force

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _ids_order(rec):
    return rec[np.argsort(inputs.int_slot(rec, "id"), kind="stable")]


@pytest.mark.parametrize("list_cap", [0, 128])
@pytest.mark.parametrize("name", ["lattice16", "tube24"])
def test_persistent_steps_each_match_oracle(orc, name, list_cap):
    """Five steps; before each, the state is flushed to the records; the
    step's density and force outputs match the oracle run on that state, and
    its kick/drift matches the oracle's bit for bit."""
    # 24^3 + 12^3: room across y and z for h to grow over the steps
    w = inputs.config1() if name == "lattice16" else inputs.two_state_tube(24, 7)
    st = sv.PersistentStepper(w.rec, sv.params_for(w, list_cap=list_cap))
    box = orc.box_of(w.lo, w.length, w.periodic)
    before = st.records()
    for k in range(5):
        print(f"[persistent] {name} cap={list_cap} step {k}", flush=True)
        st.step()
        s = st.read_state()
        assert s.flags == 0, (k, s.flags)
        after = st.records()
        c = cols(before)
        rd = orc.density(c["x"], c["y"], c["z"], c["m"], c["h"], box, w.eta)
        check_density(after, rd, tol=1e-12)
        # the force from the step's own density results (as the step ran it)
        dens = before.copy()
        for f in ("h", "rho", "omega", "wcount"):
            dens[:, S[f]] = after[:, S[f]]
        rf = oracle_force(orc, w, dens)
        check_force(after, rf, tol=1e-12, vsig_tol=1e-14)
        # kick / drift from the step's density and force outputs: bit for bit
        kicked = dens.copy()
        for f in ("ax", "ay", "az", "u_dt", "v_sig"):
            kicked[:, S[f]] = after[:, S[f]]
        orc.kick_drift(kicked, S, s.dt, s.dt_prev, k == 0, w.lo, w.length, w.periodic)
        assert np.array_equal(bits(kicked), bits(after)), k
        before = after
    st.close()


def test_persistent_follows_views_to_rounding():
    """Ten steps kept in SoA against ten steps of per-loop views: the cells'
    stable sort orders a cell's particles by storage position, which differs
    after the first step, so sums run in another order: equal to rounding."""
    w = inputs.two_state_tube(24, 9)
    a = sv.Stepper(w.rec, sv.params_for(w))
    b = sv.PersistentStepper(w.rec, sv.params_for(w))
    for _ in range(10):
        a.step()
        b.step()
    ra, sa = _ids_order(a.records()), a.read_state()
    rb, sb = _ids_order(b.records()), b.read_state()
    a.close()
    b.close()
    assert sa.flags == sb.flags == 0 and sa.nstep == sb.nstep == 10
    assert abs(sb.dt / sa.dt - 1) < 1e-10
    for k in ("x", "y", "z", "vx", "vy", "vz", "u", "h", "rho"):
        scale = np.max(np.abs(ra[:, S[k]])) + 1e-300
        err = np.max(np.abs(rb[:, S[k]] - ra[:, S[k]])) / scale
        assert err <= 1e-9, (k, err)


def test_persistent_records_untouched_until_flush():
    """Between flushes the records keep what the last flush wrote (the state
    lives in the view); close() writes the final state."""
    w = inputs.config1()
    st = sv.PersistentStepper(w.rec, sv.params_for(w))
    torch.cuda.synchronize()
    first = st.aos.cpu().numpy().view(np.float64).reshape(w.n, inputs.NSLOT).copy()
    assert np.array_equal(bits(first), bits(w.rec))
    for _ in range(3):
        st.step()
    torch.cuda.synchronize()
    mid = st.aos.cpu().numpy().view(np.float64).reshape(w.n, inputs.NSLOT).copy()
    assert np.array_equal(bits(mid), bits(w.rec))
    s = st.read_state()
    last = st.records()
    assert not np.array_equal(bits(last), bits(w.rec))
    st.close()
    torch.cuda.synchronize()
    closed = st.aos.cpu().numpy().view(np.float64).reshape(w.n, inputs.NSLOT).copy()
    assert np.array_equal(bits(closed), bits(last))
    assert s.nstep == 3


@pytest.mark.parametrize("layout", ["direct", "soa"])
def test_persistent_graph_replay_matches_eager(layout):
    lay = sv.layout(sv.LAYOUT_DIRECT) if layout == "direct" else sv.layout(sv.LAYOUT_SOA)
    w = inputs.two_state_tube(16, 5)
    p = sv.params_for(w)
    sa = torch.cuda.Stream()
    a = sv.PersistentStepper(w.rec, p, layout_density=lay, layout_force=lay, stream=sa)
    for _ in range(4):
        a.step()
    ra, sta = a.records(), a.read_state()
    a.close()
    sb = torch.cuda.Stream()
    b = sv.PersistentStepper(w.rec, p, layout_density=lay, layout_force=lay, stream=sb)
    torch.cuda.synchronize()
    sv.graph_begin(sb)
    b.step()
    g = sv.graph_end(sb)
    junk = torch.zeros(1 << 16, device="cuda")
    for _ in range(4):
        sv.graph_launch(g, sb)
        junk.add_(1.0)
        torch.cuda.synchronize()
    rb, stb = b.records(), b.read_state()
    sv.graph_destroy(g)
    b.close()
    assert np.array_equal(bits(ra), bits(rb))
    assert sta.nstep == stb.nstep == 4 and sta.dt == stb.dt and tuple(sta.sums) == tuple(stb.sums)


def test_persistent_fp32_within_budget(orc):
    w = inputs.kelvin_helmholtz(24, 9)
    p = sv.params_for(w, h_tol=1e-6)
    st = sv.PersistentStepper(w.rec, p, sv.PREC_FP32)
    before = st.records()
    st.step()
    s = st.read_state()
    after = st.records()
    st.close()
    assert s.flags == 0
    check_density(after, oracle_density(orc, w, rec=before), tol=1e-5)
    dens = before.copy()
    for f in ("h", "rho", "omega", "wcount"):
        dens[:, S[f]] = after[:, S[f]]
    check_force(after, oracle_force(orc, w, dens), tol=1e-4, vsig_tol=1e-6)
