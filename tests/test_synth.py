"""The synthetic event generator: geometry, truth and reproducibility."""
import numpy as np
import pytest

from paper_2407_12119_amd import synth


def test_event_reproducible_alone_and_in_batch():
    wl = synth.WORKLOADS["batch256"]
    alone = synth.make_event(wl.recipe, synth.event_rng(wl.index, 7))
    batch = synth.make_batch(wl, n_events=10)
    inb = batch.event(7)
    for f in ("x", "y", "z", "plane", "pid", "next_hit"):
        np.testing.assert_array_equal(getattr(alone, f), getattr(inb, f))


def test_sorted_by_plane_and_z_on_planes():
    wl = synth.WORKLOADS["batch256"]
    for ev in synth.make_events(wl, n_events=8):
        assert np.all(np.diff(ev.plane) >= 0)
        assert ev.plane.min(initial=0) >= 0 and ev.plane.max(initial=0) < synth.N_PLANES
        np.testing.assert_array_equal(ev.z, synth.PLANE_Z[ev.plane].astype(np.float32))


def test_acceptance_and_straight_tracks():
    """Every particle's hits lie on one straight line within the 0.01 mm smearing."""
    wl = synth.WORKLOADS["batch256"]
    ev = synth.make_events(wl, n_events=1, first=3)[0]
    r = np.hypot(ev.x.astype(np.float64), ev.y.astype(np.float64))
    assert np.all(r > synth.R_MIN - 0.1) and np.all(r < synth.R_MAX + 0.1)
    resid = []
    for p in np.unique(ev.pid[ev.pid >= 0]):
        m = ev.pid == p
        if m.sum() < 3:
            continue
        z = ev.z[m].astype(np.float64)
        for coord in (ev.x[m], ev.y[m]):
            A = np.stack([np.ones_like(z), z], 1)
            coef, *_ = np.linalg.lstsq(A, coord.astype(np.float64), rcond=None)
            resid.append(coord - A @ coef)
    resid = np.concatenate(resid)
    assert 0.005 < resid.std() < 0.012
    # one hit per plane per particle, planes increasing with z
    for p in np.unique(ev.pid[ev.pid >= 0]):
        pl = ev.plane[ev.pid == p]
        assert len(np.unique(pl)) == len(pl)


def test_noise_fraction_and_truth_links():
    wl = synth.WORKLOADS["batch256"]
    b = synth.make_batch(wl, n_events=16)
    n_noise = int((b.pid < 0).sum())
    n_sig = b.n_hits - n_noise
    assert abs(n_noise / n_sig - 0.05) < 0.01
    for e in range(b.n_events):
        ev = b.event(e)
        for i in range(ev.n):
            j = ev.next_hit[i]
            if j < 0:
                continue
            assert ev.pid[i] == ev.pid[j] >= 0 and ev.plane[j] > ev.plane[i]
            # no hit of the same particle in between
            same = (ev.pid == ev.pid[i]) & (ev.plane > ev.plane[i]) & (ev.plane < ev.plane[j])
            assert not same.any()


def test_single_event_size_and_empty_events():
    ev = synth.make_events(synth.WORKLOADS["single_event"])[0]
    assert 450 < ev.n < 700
    # Poisson(5) vertices: empty events occur in the 256-event batch
    b = synth.make_batch(synth.WORKLOADS["batch256"])
    sizes = np.diff(b.event_offsets)
    assert (sizes == 0).sum() >= 1
    assert 1200 < sizes.mean() < 2100


def test_params_layout_and_bounds():
    wl = synth.WORKLOADS["batch256"]
    p = synth.init_params(wl)
    assert p.dtype == np.float32 and p.shape[0] == synth.param_count(64, 4)
    v = synth.param_views(p, 64, 4)
    for name, (o, i) in synth.param_layout(64, 4):
        w, b = v[name]
        bound = 1 / np.sqrt(i)
        assert np.abs(w).max() <= bound and np.abs(b).max() <= bound
    np.testing.assert_array_equal(p, synth.init_params(wl))


@pytest.mark.parametrize("name", ["single_event", "batch256", "batch256_lowp", "train32", "batch1000_h128"])
def test_centred_bias_is_the_oracle_median(name):
    """The bias-centred variant's classifier bias equals the seeded bias minus
    the median float64 logit over the calibration event (pile-up recipe, seed
    words (998, 0)), rounded to float32."""
    import oracle
    wl = synth.WORKLOADS[name]
    calib = synth.make_event(synth.WORKLOADS["batch256"].recipe, synth._rng(998, 0))
    assert calib.n == 1516
    blob = synth.init_params(wl)
    out = oracle.pipeline(synth.to_batch([calib]), blob, wl.hidden, wl.iters, wl.radius, wl.k_max)
    med = float(np.median(out["logit"]))
    assert np.float32(float(blob[-1]) - med) == np.float32(synth.CENTRED_BIAS[name])
    centred = synth.centred_params(wl)
    assert centred[-1] == np.float32(synth.CENTRED_BIAS[name])
    np.testing.assert_array_equal(centred[:-1], blob[:-1])
