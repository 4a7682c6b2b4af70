"""sphv_records_sort_static (no allocation: the library's fixed per-GPU array
holds the sorted copy) against sphv_records_sort with a caller workspace, bit
for bit, on two calls in a row, the second on fewer records."""
from __future__ import annotations

import numpy as np
import pytest
import torch

from paper_2502_16517_amd import inputs
from paper_2502_16517_amd import sphview as sv

pytestmark = pytest.mark.gpu


def bits(a):
    return np.ascontiguousarray(a).view(np.uint64)


def _sorted_both_ways(w):
    """Records, perm and key after records_sort (workspace) and after
    records_sort_static, each on its own Stepper over the same records."""
    out = []
    for static in (False, True):
        st = sv.Stepper(w.rec, sv.params_for(w))
        st.build()
        if static:
            sv.records_sort_static(st.cells, st.aos, inputs.STRIDE)
        else:
            ws = torch.empty(sv.records_sort_workspace_bytes(inputs.STRIDE, st.n), dtype=torch.uint8,
                             device="cuda")
            sv.records_sort(st.cells, st.aos, inputs.STRIDE, ws)
        torch.cuda.synchronize()
        perm, start, key, _ = st.cells_arrays()
        out.append((st.records(), perm, start, key))
        st.close()
    return out


def test_records_sort_static_matches_workspace_form():
    # two calls in a row, the second with fewer records: the array keeps the
    # first call's bytes beyond the second's records, which must not leak in
    for w in (inputs.two_state_tube(16, 31), inputs.config1()):
        print(f"[records_sort_static] n={w.n}", flush=True)
        assert w.n * inputs.STRIDE <= sv.RECORDS_SORT_STATIC_MAX_BYTES
        (ra, pa, sa, ka), (rb, pb, sb, kb) = _sorted_both_ways(w)
        assert np.array_equal(bits(ra), bits(rb))
        assert np.array_equal(pa, pb) and np.array_equal(sa, sb) and np.array_equal(ka, kb)
        assert np.array_equal(pb, np.arange(w.n, dtype=np.int32))


def test_records_sort_static_then_step_matches():
    """A density + force step on records sorted by the static form gives the
    same bits as on records sorted with a workspace (the SORTED layout)."""
    w = inputs.config1()
    lay = sv.layout(sv.LAYOUT_SORTED)
    outs = []
    for static in (False, True):
        st = sv.Stepper(w.rec, sv.params_for(w), layout_density=lay, layout_force=lay)
        st.build()
        if static:
            sv.records_sort_static(st.cells, st.aos, inputs.STRIDE)
        else:
            ws = torch.empty(sv.records_sort_workspace_bytes(inputs.STRIDE, st.n), dtype=torch.uint8,
                             device="cuda")
            sv.records_sort(st.cells, st.aos, inputs.STRIDE, ws)
        st.density()
        st.force()
        outs.append(st.records())
        st.close()
    assert np.array_equal(bits(outs[0]), bits(outs[1]))


def test_records_sort_static_refuses_oversize():
    w = inputs.config1()
    p = sv.params_for(w)
    st = sv.Stepper(w.rec, p)
    st.build()
    # the cells were built for w.n records: a stride that pushes stride * n past
    # the maximum is refused before anything is enqueued
    big_stride = (sv.RECORDS_SORT_STATIC_MAX_BYTES // w.n + 4) // 4 * 4
    with pytest.raises(sv.SphvError) as e:
        sv.records_sort_static(st.cells, st.aos, big_stride)
    assert e.value.status == sv.E_WORKSPACE
    st.close()
