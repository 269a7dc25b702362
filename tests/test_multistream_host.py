"""Host logic of the multi-stream throughput mode: splitting a stream's
events into capped batches (no GPU)."""
import numpy as np
import pytest

from paper_2407_12119_amd import multistream, synth


def test_split_respects_caps_and_keeps_event_order():
    wl = synth.WORKLOADS["batch256"]
    events = synth.make_events(wl, 40, first=900)
    batches = multistream.split_events(events, hit_cap=20000, edge_cap=1 << 22, k_max=32)
    assert len(batches) > 1
    assert all(b.n_hits <= 20000 for b in batches)
    cat = synth.to_batch([b.event(i) for b in batches for i in range(b.n_events)])
    ref = synth.to_batch(events)
    for k in ("x", "y", "z", "plane", "event_offsets"):
        np.testing.assert_array_equal(getattr(cat, k), getattr(ref, k))


def test_edge_cap_bounds_the_hits_through_k_max():
    wl = synth.WORKLOADS["batch256"]
    events = synth.make_events(wl, 20, first=950)
    batches = multistream.split_events(events, hit_cap=1 << 20, edge_cap=32 * 10000, k_max=32)
    assert all(b.n_hits <= 10000 for b in batches)


def test_an_event_above_the_cap_is_refused():
    wl = synth.WORKLOADS["batch256"]
    ev = synth.make_events(wl, 1, first=0)
    with pytest.raises(ValueError):
        multistream.split_events(ev, hit_cap=10, edge_cap=1 << 22, k_max=32)
