"""GPU checks of the autotuner: it leaves the records bit-identical, reports a
median for every candidate, returns one of them, refuses to run under graph
capture, and the step with the chosen layouts matches the oracle."""
import numpy as np
import pytest

from paper_2502_16517_amd import inputs
from paper_2502_16517_amd import sphview as sv

from gpu_helpers import bits, check_density, check_force, oracle_density, oracle_force

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# a spread of the built-in candidates: every layout kind, several tile shapes
SUBSET = [sv.layout(sv.LAYOUT_SOA), sv.layout(sv.LAYOUT_SOA, tpi=1, masked=1),
          sv.layout(sv.LAYOUT_AOSOA, 8, tpi=2), sv.layout(sv.LAYOUT_AOSOA, 64, tpi=4, masked=1),
          sv.layout(sv.LAYOUT_DIRECT, tpi=8), sv.layout(sv.LAYOUT_DIRECT, masked=1)]


@pytest.mark.parametrize("precision", [sv.PREC_FP64, sv.PREC_FP32])
def test_autotune_leaves_records_and_picks_a_candidate(precision):
    w = inputs.two_state_tube(16, 21)
    p = sv.params_for(w)
    if precision == sv.PREC_FP32:
        p.h_tol = 1e-6
    st = sv.Stepper(w.rec, p, precision)
    st.step()                     # valid density outputs for the force loop
    st.build()
    before = st.records()
    u8 = dict(dtype=torch.uint8, device="cuda")
    for loop, d in ((sv.LOOP_DENSITY, st.d_dens), (sv.LOOP_FORCE, st.d_force)):
        ws = torch.empty(sv.autotune_workspace_bytes(d, st.n, precision, SUBSET), **u8)
        best, table = sv.autotune(loop, st.aos, d, st.cells, p, precision, ws, SUBSET, reps=3)
        after = st.records()
        assert np.array_equal(bits(before), bits(after)), loop
        assert len(table) == len(SUBSET)
        assert all(ms > 0 for _, ms in table)
        # the first candidate within 1.5 % of the fastest (timing noise)
        fastest = min(ms for _, ms in table)
        first = next(c for c, ms in table if ms <= fastest * np.float32(1.015))
        key = (best.kind, best.aosoa_width, best.tpi, best.masked)
        assert key == (first.kind, first.aosoa_width, first.tpi, first.masked)
    state = st.read_state()
    assert state.nstep == 1       # the trials used their own state block
    st.close()


def test_autotune_refuses_graph_capture():
    w = inputs.two_state_tube(16, 22)
    st = sv.Stepper(w.rec, sv.params_for(w))
    st.step()
    s = torch.cuda.Stream()
    ws = torch.empty(sv.autotune_workspace_bytes(st.d_dens, st.n, sv.PREC_FP64, SUBSET[:1]), dtype=torch.uint8,
                     device="cuda")
    torch.cuda.synchronize()
    sv.graph_begin(s)
    with pytest.raises(sv.SphvError) as e:
        sv.autotune(sv.LOOP_DENSITY, st.aos, st.d_dens, st.cells, st.p, sv.PREC_FP64, ws, SUBSET[:1], stream=s)
    status = e.value.status
    try:
        sv.graph_destroy(sv.graph_end(s))
    except sv.SphvError:
        pass
    assert status == sv.E_STATE
    st.close()


def test_step_with_tuned_layouts_matches_oracle(orc):
    w = inputs.two_state_tube(16, 23)
    p = sv.params_for(w)
    st = sv.Stepper(w.rec, p)
    st.step()
    res = st.autotune(candidates=SUBSET, reps=2)
    assert set(res) == {"density", "force"}
    rec0 = st.records()
    st.build()
    st.density()
    rec1 = st.records()
    ref_d = oracle_density(orc, w, rec=rec0)
    check_density(rec1, ref_d, tol=1e-12)
    st.force()
    rec2 = st.records()
    ref_f = oracle_force(orc, w, rec2)
    check_force(rec2, ref_f, tol=1e-12)
    st.close()
