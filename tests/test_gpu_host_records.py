"""Records resident in host memory: pinned memory (allocated pinned, which the
device maps at the same address) serves every call that reads records, and a
step over it gives the bits of the step over device-resident records, with
views (which fetch each record once per loop) as with loops on the records;
pageable host memory, which the device cannot address, is refused on the host
before anything is enqueued."""
import numpy as np
import pytest

from paper_2502_16517_amd import inputs
from paper_2502_16517_amd import sphview as sv

from gpu_helpers import bits

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _records(w, where):
    raw = torch.from_numpy(inputs.as_bytes(np.ascontiguousarray(w.rec)))
    if where == "device":
        return raw.to("cuda")
    if where == "pinned":
        return raw.pin_memory()           # a new pinned allocation, the records copied in
    return raw.clone()                    # pageable


def _steps(w, where, lay, merged=False, steps=2, precision=sv.PREC_FP64):
    p = sv.params_for(w)
    if precision == sv.PREC_FP32:
        p.h_tol = 1e-6
    st = sv.Stepper(None, p, precision, layout_density=lay, layout_force=lay, aos=_records(w, where),
                    merged=merged)
    for _ in range(steps):
        st.step()
    out, state = st.records(), st.read_state()
    st.close()
    return out, state


@pytest.mark.parametrize("name,lay,merged", [
    ("soa", sv.layout(sv.LAYOUT_SOA), False),
    ("aosoa8", sv.layout(sv.LAYOUT_AOSOA, 8), False),
    ("direct", sv.layout(sv.LAYOUT_DIRECT), False),
    ("merged_aosoa8", sv.layout(sv.LAYOUT_AOSOA, 8), True),
])
def test_pinned_host_records_give_device_bits(name, lay, merged):
    print(f"[host records] {name}", flush=True)
    w = inputs.two_state_tube(16, 31)
    a, sa = _steps(w, "device", lay, merged)
    b, sb = _steps(w, "pinned", lay, merged)
    assert sa.flags == sb.flags
    assert np.array_equal(bits(a), bits(b))
    assert sa.dt == sb.dt and tuple(sa.sums) == tuple(sb.sums) and sa.pairs_total == sb.pairs_total


def test_pinned_host_records_fp32():
    """The FP32 form reads h and the reduction's inputs from the records (its
    views hold them as floats): over pinned records, the device bits."""
    w = inputs.two_state_tube(16, 34)
    lay = sv.layout(sv.LAYOUT_SOA)
    a, sa = _steps(w, "device", lay, precision=sv.PREC_FP32)
    b, sb = _steps(w, "pinned", lay, precision=sv.PREC_FP32)
    assert sa.flags == sb.flags
    assert np.array_equal(bits(a), bits(b))
    assert sa.dt == sb.dt and tuple(sa.sums) == tuple(sb.sums)


def test_pinned_host_records_sorted_and_tuned():
    """records_sort moves records in host memory, and the tuner's trials on
    sorted records move them there and back: the same bits as on the device
    (one candidate, so both runs choose alike)."""
    w = inputs.two_state_tube(16, 32)
    srt = sv.layout(sv.LAYOUT_SORTED)
    a, _ = _steps(w, "device", srt)
    b, _ = _steps(w, "pinned", srt)
    assert np.array_equal(bits(a), bits(b))

    def tuned(where):
        st = sv.Stepper(None, sv.params_for(w), aos=_records(w, where))
        st.step()
        st.autotune(candidates=[srt], reps=1)
        st.step()
        out = st.records()
        st.close()
        return out

    assert np.array_equal(bits(tuned("device")), bits(tuned("pinned")))


def test_pageable_host_records_refused():
    w = inputs.two_state_tube(8, 33)
    rec = _records(w, "pageable")
    st = sv.Stepper(None, sv.params_for(w), aos=rec)     # planning only: no device work yet
    with pytest.raises(sv.SphvError) as e:
        st.build()
    assert e.value.status == sv.E_INVALID_ARG
    with pytest.raises(sv.SphvError) as e:
        sv.kick_drift(rec, st.d_kick, st.n, st.p, st.state)
    assert e.value.status == sv.E_INVALID_ARG
    # a view over pageable records: refused at its first gather
    dev = sv.Stepper(w.rec, sv.params_for(w))
    dev.build()
    v = sv.view_create(st.d_dens, st.n, sv.layout(), sv.PREC_FP64, rec, dev.perm_ptr, dev.ws_dens)
    with pytest.raises(sv.SphvError) as e:
        sv.aos_to_soa(v, dev.cells)
    assert e.value.status == sv.E_INVALID_ARG
    sv.view_destroy(v)
    torch.cuda.synchronize()
    dev.close()
    st.close()
    # the records were never touched
    assert np.array_equal(bits(rec.numpy().view(np.float64).reshape(w.n, -1)), bits(w.rec))
