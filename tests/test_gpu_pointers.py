"""Records reached through a list of their addresses (DESC_RECORD_POINTERS:
particles scattered in memory, held as a list of pointers, paper Sec. 5.1):
the cells, the views' gathers and scatters, both pair loops and kick_drift
read and write each record where the list says.  A step over records
scattered at shuffled slots of a larger buffer gives the bits of the step
over the same records stored contiguously, and matches the oracle; slots the
list does not name are never touched."""
import numpy as np
import pytest

from paper_2502_16517_amd import inputs
from paper_2502_16517_amd import sphview as sv

from gpu_helpers import S, bits, check_density, check_force, oracle_density, oracle_force

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _scattered(w, seed=5, spread=3, host=False):
    """The records at seeded, shuffled slots of a buffer `spread` times larger
    (the other slots hold NaN-payload junk), in device memory or in pinned host
    memory, and the device list of their addresses in particle order."""
    rng = np.random.default_rng(seed)
    n = w.n
    slots = rng.permutation(spread * n)[:n]
    buf = rng.integers(0, 2**63, size=(spread * n, inputs.NSLOT), dtype=np.uint64)
    buf.view(np.float64)[slots] = w.rec
    raw = torch.from_numpy(buf.view(np.uint8).reshape(-1).copy())
    dev = raw.pin_memory() if host else raw.cuda()
    ptrs = torch.from_numpy((dev.data_ptr() + slots.astype(np.uint64) * inputs.STRIDE).astype(np.uint64)
                            .view(np.int64)).cuda()
    return dev, ptrs, slots, buf


LAYOUTS = {"soa": sv.layout(sv.LAYOUT_SOA), "aosoa8": sv.layout(sv.LAYOUT_AOSOA, 8),
           "direct": sv.layout(sv.LAYOUT_DIRECT)}


@pytest.mark.parametrize("list_cap", [0, 128])
@pytest.mark.parametrize("name", list(LAYOUTS))
def test_pointer_records_give_contiguous_bits(orc, name, list_cap):
    print(f"[pointer records] {name} cap={list_cap}", flush=True)
    w = inputs.two_state_tube(24, 31)
    lay = LAYOUTS[name]
    p = sv.params_for(w, list_cap=list_cap)
    a = sv.Stepper(w.rec, p, layout_density=lay, layout_force=lay)
    dev, ptrs, slots, buf = _scattered(w)
    b = sv.Stepper(None, p, layout_density=lay, layout_force=lay, aos=dev, record_ptrs=ptrs)
    for _ in range(3):
        a.step()
        b.step()
    ra, sa = a.records(), a.read_state()
    rb, sb = b.records(), b.read_state()
    full = b.aos.cpu().numpy().view(np.uint64).reshape(-1, inputs.NSLOT)
    a.close()
    b.close()
    assert sa.flags == sb.flags == 0
    assert np.array_equal(bits(ra), bits(rb))
    assert sa.dt == sb.dt and tuple(sa.sums) == tuple(sb.sums) and sa.pairs_total == sb.pairs_total
    # the slots the list does not name keep their junk
    others = np.setdiff1d(np.arange(full.shape[0]), slots)
    assert np.array_equal(full[others], buf[others])


def test_pointer_records_in_pinned_host_memory(orc):
    """Records scattered through a pool in pinned host memory, reached by a
    device list of their addresses: three steps give the bits of the same
    records stored contiguously on the device."""
    w = inputs.two_state_tube(24, 31)
    p = sv.params_for(w)
    a = sv.Stepper(w.rec, p)
    host, ptrs, slots, buf = _scattered(w, seed=17, host=True)
    b = sv.Stepper(None, p, aos=host, record_ptrs=ptrs)
    for _ in range(3):
        a.step()
        b.step()
    ra, sa = a.records(), a.read_state()
    rb, sb = b.records(), b.read_state()
    a.close()
    b.close()
    assert sa.flags == sb.flags == 0
    assert np.array_equal(bits(ra), bits(rb))
    assert sa.dt == sb.dt and tuple(sa.sums) == tuple(sb.sums)


def test_pointer_records_step_matches_oracle(orc):
    w = inputs.config1()
    dev, ptrs, _, _ = _scattered(w, seed=9)
    st = sv.Stepper(None, sv.params_for(w), aos=dev, record_ptrs=ptrs)
    st.build()
    st.density()
    dens = st.records()
    st.force()
    out = st.records()
    state = st.read_state()
    st.close()
    assert state.flags == 0
    ref = oracle_density(orc, w)
    check_density(dens, ref, tol=1e-12)
    assert state.pairs_density == int(ref["count"].sum())
    rf = oracle_force(orc, w, dens)
    check_force(out, rf, tol=1e-12, vsig_tol=1e-14)
    assert state.pairs_force == int(rf["count"].sum())


def test_pointer_records_fp32(orc):
    w = inputs.kelvin_helmholtz(24, 9)
    dev, ptrs, _, _ = _scattered(w, seed=13)
    p = sv.params_for(w, h_tol=1e-6)
    a = sv.Stepper(w.rec, p, sv.PREC_FP32)
    b = sv.Stepper(None, p, sv.PREC_FP32, aos=dev, record_ptrs=ptrs)
    a.step()
    b.step()
    ra, rb = a.records(), b.records()
    a.close()
    b.close()
    assert np.array_equal(bits(ra), bits(rb))


def test_pointer_records_refuse_sorted_layout_and_tuner():
    w = inputs.config1()
    dev, ptrs, _, _ = _scattered(w)
    p = sv.params_for(w)
    with pytest.raises(sv.SphvError) as e:
        sv.Stepper(None, p, layout_density=sv.layout(sv.LAYOUT_SORTED), aos=dev, record_ptrs=ptrs)
    assert e.value.status == sv.E_UNSUPPORTED
    st = sv.Stepper(None, p, aos=dev, record_ptrs=ptrs)
    st.step()
    with pytest.raises(sv.SphvError) as e:
        st.autotune(reps=1)
    assert e.value.status == sv.E_UNSUPPORTED
    st.close()
