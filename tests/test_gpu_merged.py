"""One view over both pair loops (the persistent view the paper names as
future work, Sec. 8): gathered once before the density loop, the force loop
reading the density's h, rho and omega inside the view, scattered once after
the step reduction.  It must give the bits of the two-view step, and the FP32
form, whose force loop stages its members as floats, must refuse it."""
import numpy as np
import pytest

from paper_2502_16517_amd import inputs
from paper_2502_16517_amd import sphview as sv

from gpu_helpers import S, bits, check_density, check_force, oracle_density, oracle_force

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

LAYOUTS = {
    "soa": sv.layout(sv.LAYOUT_SOA),
    "aosoa8": sv.layout(sv.LAYOUT_AOSOA, 8),
    "aosoa8_masked": sv.layout(sv.LAYOUT_AOSOA, 8, masked=1),
    "aosoa64_tpi4": sv.layout(sv.LAYOUT_AOSOA, 64, tpi=4),
    "direct": sv.layout(sv.LAYOUT_DIRECT),
}


def _run(w, lay, merged, steps, kernel=sv.KERNEL_CUBIC):
    st = sv.Stepper(w.rec, sv.params_for(w, kernel=kernel), layout_density=lay, layout_force=lay, merged=merged)
    for _ in range(steps):
        st.step()
    out, state = st.records(), st.read_state()
    st.close()
    return out, state


@pytest.mark.parametrize("name", list(LAYOUTS))
def test_merged_view_bit_identical_to_two_views(name):
    print(f"[merged] {name}", flush=True)
    w = inputs.two_state_tube(16, 21)
    lay = LAYOUTS[name]
    a, sa = _run(w, lay, False, 3)
    b, sb = _run(w, lay, True, 3)
    # the small tube may report a coarse grid (a flag, not an error): both runs alike
    assert sa.flags == sb.flags
    assert np.array_equal(bits(a), bits(b))
    assert sa.dt == sb.dt and tuple(sa.sums) == tuple(sb.sums)
    assert sa.pairs_total == sb.pairs_total


def test_merged_view_quartic_bit_identical():
    w = inputs.kelvin_helmholtz(24, 4)
    lay = LAYOUTS["aosoa8"]
    a, sa = _run(w, lay, False, 2, sv.KERNEL_QUARTIC)
    b, sb = _run(w, lay, True, 2, sv.KERNEL_QUARTIC)
    assert np.array_equal(bits(a), bits(b)) and sa.dt == sb.dt


def test_merged_step_matches_oracle(orc):
    w = inputs.config1()
    st = sv.Stepper(w.rec, sv.params_for(w), layout_density=sv.layout(sv.LAYOUT_AOSOA, 8), merged=True)
    st.build()
    st.density()
    # inside the merged view the records do not hold the density's results
    # yet: its members are temporarily invalid until the scatter
    st.force()
    out = st.records()
    state = st.read_state()
    assert state.flags == 0, state.flags
    ref = oracle_density(orc, w)
    check_density(out, ref, tol=1e-12)
    check_force(out, oracle_force(orc, w, out), tol=1e-12, vsig_tol=1e-14)
    dt = orc.time_step(out[:, S["h"]], out[:, S["v_sig"]], inputs.CFL)
    assert abs(state.dt / dt - 1.0) < 1e-15
    st.kick()
    after = st.records()
    st.close()
    exp = out.copy()
    orc.kick_drift(exp, S, state.dt, 0.0, True, w.lo, w.length, w.periodic)
    assert np.array_equal(bits(exp), bits(after))


def test_merged_graph_replay_matches_eager():
    w = inputs.two_state_tube(16, 22)
    lay = LAYOUTS["aosoa8"]
    a, sta = _run(w, lay, True, 3)
    s = torch.cuda.Stream()
    b = sv.Stepper(w.rec, sv.params_for(w), layout_density=lay, merged=True, stream=s)
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
    assert np.array_equal(bits(a), bits(rb))
    assert sta.nstep == stb.nstep == 3 and sta.dt == stb.dt and tuple(sta.sums) == tuple(stb.sums)


def test_fp32_force_refuses_members_it_would_write():
    w = inputs.two_state_tube(16, 23)
    with pytest.raises(ValueError):
        sv.Stepper(w.rec, sv.params_for(w), sv.PREC_FP32, merged=True)
    # at the C level: an FP32 view over both loops serves the density loop (it
    # stages x, y, z, m, all read only) but the force loop refuses it (h, rho
    # and omega are written by the view, so it holds them as doubles)
    p = sv.params_for(w, h_tol=1e-6)
    st = sv.Stepper(w.rec, p, sv.PREC_FP32)
    st.build()
    d = sv.merged_descriptor()
    lay = sv.layout(sv.LAYOUT_SOA)
    ws = torch.empty(sv.view_workspace_bytes(d, w.n, lay, sv.PREC_FP32), dtype=torch.uint8, device="cuda")
    v = sv.view_create(d, w.n, lay, sv.PREC_FP32, st.aos, st.perm_ptr, ws)
    sv.aos_to_soa(v, st.cells)
    sv.sph_density(v, st.cells, p, st.state)
    with pytest.raises(sv.SphvError) as e:
        sv.sph_force(v, st.cells, p, st.state)
    assert e.value.status == sv.E_DESCRIPTOR
    sv.soa_to_aos(v)
    torch.cuda.synchronize()
    sv.view_destroy(v)
    st.close()


def test_merged_full_tube_bit_identical():
    """The 294,912-particle two-state tube in the benchmark's launch
    configuration (AoSoA 8): one merged step gives the two-view step's bits."""
    w = inputs.config2()
    lay = LAYOUTS["aosoa8"]
    a, sa = _run(w, lay, False, 1)
    b, sb = _run(w, lay, True, 1)
    assert sa.flags & ~sv.F_OUT_OF_BOX == 0
    assert np.array_equal(bits(a), bits(b))
    assert sa.dt == sb.dt and tuple(sa.sums) == tuple(sb.sums)
