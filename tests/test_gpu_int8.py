"""GPU: the INT8 embedding (Sec. 7.4) against the float64 oracle's INT8 path.

Both sides take the same four per-tensor scales (the oracle's, from its own
calibration maxima), form the same INT8 codes of the weights (decided in
float32 on both sides), sum the integer products exactly and descale; the
differences left are float32 rounding of the descaled sums and, rarely, an
activation code decided on the other side of a rounding tie because the
float32 first layer differs from the float64 one in its last bit.  So:
  * at least 99% of hits agree to float32 rounding (1e-5 * max(1, |e|));
  * every hit stays within the effect of one flipped code of the second
    layer's input: sum_j |W3[c, j]| (s_x2 max|W2| + s_x3) per output c.
The GPU's own calibration must give the oracle's scales to float32 rounding
of the activation maxima (the weight scales exactly).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle                                           # noqa: E402
from paper_2407_12119_amd import synth, velo           # noqa: E402

pytestmark = pytest.mark.gpu


def _ctx(wl, batch):
    ctx = velo.Context(wl.hidden, wl.iters, oracle.d2max_f32(wl.radius), wl.k_max, wl.edge_logit_min, "fp32",
                       max_hits=max(batch.n_hits, 1), max_events=max(batch.n_events, 1),
                       max_event_hits=max(batch.max_event_hits(), 1))
    return ctx


def _flip_bound(blob, sc):
    o2 = 12 + 128 * 3 + 128
    w2 = blob[o2:o2 + 128 * 128].astype(np.float64)
    o3 = o2 + 128 * 128 + 128
    w3 = blob[o3:o3 + 4 * 128].astype(np.float64).reshape(4, 128)
    return np.abs(w3).sum(axis=1) * (float(sc[0]) * np.abs(w2).max() + float(sc[2]))


@pytest.mark.parametrize("weights", ["centred", "trained"])
def test_int8_embedding_matches_the_oracle(weights):
    wl = synth.WORKLOADS["batch256"]
    if weights == "trained":
        import os
        path = os.path.join(os.path.dirname(__file__), "golden", "trained_h64_n4.npy")
        if not os.path.exists(path):
            pytest.skip("trained weights not generated")
        blob = np.load(path)
        wl = synth.WORKLOADS["batch256_trained"]
    else:
        blob = synth.centred_params(wl)
    calib = synth.make_events(wl, 8, first=2000)
    sc = oracle.int8_scales(oracle.embed_amax(calib, blob), blob)
    batch = synth.make_batch(wl, n_events=6, first=40)
    print(f"\n[case] int8 embedding {weights} events={batch.n_events} hits={batch.n_hits} scales={sc}", flush=True)
    ctx = _ctx(wl, batch)
    ctx.set_params(torch.from_numpy(blob).cuda())
    hits = velo.DeviceHits.from_batch(batch)
    e32 = ctx.embed(hits).cpu().numpy()
    ctx.set_embed_int8(sc)
    e8 = ctx.embed(hits).cpu().numpy()
    bound = _flip_bound(blob, sc)
    close, worst = 0, 0.0
    for b in range(batch.n_events):
        ev = batch.event(b)
        o0 = int(batch.event_offsets[b])
        ref = oracle.embed_int8(ev.x, ev.y, ev.z, blob, sc)
        d = np.abs(e8[o0:o0 + ev.n] - ref)
        close += int(np.sum(np.all(d <= 1e-5 * np.maximum(1.0, np.abs(ref)), axis=1)))
        assert np.all(d <= bound[None, :]), (b, d.max(axis=0), bound)
        worst = max(worst, float(d.max()) if d.size else 0.0)
    frac = close / batch.n_hits
    q = np.abs(e8 - e32).max()
    print(f"  {frac:.5f} of hits within float32 rounding; worst |de| {worst:.3g} (bound {bound.max():.3g}); "
          f"INT8 vs float32 embedding: max |de| {q:.3g}", flush=True)
    assert frac >= 0.99
    # the fused path embeds with the same kernel
    g = ctx.infer(hits)
    ctx.check()
    ctx.set_embed_int8(None)
    np.testing.assert_array_equal(ctx.embed(hits).cpu().numpy(), e32)


def test_int8_calibration_matches_the_oracle():
    wl = synth.WORKLOADS["batch256"]
    blob = synth.centred_params(wl)
    calib_events = synth.make_events(wl, 8, first=2000)
    cb = synth.to_batch(calib_events)
    print(f"\n[case] int8 calibration events={cb.n_events} hits={cb.n_hits}", flush=True)
    ctx = _ctx(wl, cb)
    ctx.set_params(torch.from_numpy(blob).cuda())
    sc = ctx.calibrate_embed_int8(velo.DeviceHits.from_batch(cb))
    ref = oracle.int8_scales(oracle.embed_amax(calib_events, blob), blob)
    assert sc[1] == ref[1] and sc[3] == ref[3]
    np.testing.assert_allclose(sc, ref, rtol=1e-5)
    # set_params turns INT8 off again: the embedding is the float32 one
    batch = synth.make_batch(wl, n_events=2, first=50)
    hits = velo.DeviceHits.from_batch(batch)
    e_int8 = ctx.embed(hits).cpu().numpy()
    ctx.set_params(torch.from_numpy(blob).cuda())
    e_f32 = ctx.embed(hits).cpu().numpy()
    assert not np.array_equal(e_int8, e_f32)
    ev = batch.event(0)
    assert np.abs(e_f32[:ev.n] - oracle.embed(ev.x, ev.y, ev.z, blob)).max() <= 1e-5
    with pytest.raises(velo.VeloError):
        ctx.set_embed_int8([1.0, 0.0, 1.0, 1.0])
