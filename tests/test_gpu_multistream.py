"""GPU: the multi-stream throughput mode gives, batch for batch, the same
outputs as one context running the same batches one after the other (the
kernels are deterministic and every stream has its own context)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle                                                    # noqa: E402
from paper_2407_12119_amd import multistream, synth, velo       # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_streams_match_a_single_context(precision):
    wl = synth.WORKLOADS["batch256"]
    blob = synth.centred_params(wl)
    shares = [synth.make_events(wl, 10, first=1200 + 10 * s) for s in range(3)]
    print(f"\n[case] multistream {precision} streams=3 events=30", flush=True)
    ms = multistream.MultiStream(wl, blob, precision, shares, hit_cap=6000)
    assert all(len(b) > 1 for b in ms.batches)
    for _ in range(2):                     # twice: the second pass reuses the buffers
        ms.run()
    ms.synchronize()
    ref_ctx = velo.Context(wl.hidden, wl.iters, oracle.d2max_f32(wl.radius), wl.k_max, wl.edge_logit_min,
                           precision, max_hits=6000, max_events=16, max_event_hits=6000)
    ref_ctx.set_params(torch.from_numpy(blob).cuda())
    for s in range(3):
        for b, h, o in zip(ms.batches[s], ms.hits[s], ms.outs[s]):
            ref = velo.graph_to_host(ref_ctx.infer(h), b.n_hits)
            got = velo.graph_to_host(o, b.n_hits)
            for k in ("labels", "edge_offsets", "src", "dst", "logit"):
                np.testing.assert_array_equal(got[k], ref[k], err_msg=f"stream {s} {k}")
    ms.close()
