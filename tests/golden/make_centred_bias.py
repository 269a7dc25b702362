"""Write centred_bias.json: the classifier output bias that centres the edge
logits of the seeded random init on zero.

With the seeded random init every edge scores above 0.5, so the edge cut
(Sec. 5, overview) and the connected components (Sec. 7.3) would never be
exercised.  The "bias-centred" parameter variant therefore replaces the final
classifier bias b by b - median(logit) over one calibration event, so that
about half the edges are kept.  The median is taken from the float64 oracle
only.  Run:  python tests/golden/make_centred_bias.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle                                        # noqa: E402
from paper_2407_12119_amd import synth              # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "centred_bias.json")


def main():
    calib = synth.make_event(synth.WORKLOADS["batch256"].recipe, synth._rng(998, 0))
    batch = synth.to_batch([calib])
    res = {"calibration_event": "pile-up recipe, seed words (998, 0)", "n_hits": calib.n}
    for name in ("single_event", "batch256", "train32", "batch1000_h128"):
        wl = synth.WORKLOADS[name]
        blob = synth.init_params(wl)
        out = oracle.pipeline(batch, blob, wl.hidden, wl.iters, wl.radius, wl.k_max)
        med = float(np.median(out["logit"]))
        res[name] = {"median_logit": med, "centred_bias": float(np.float32(float(blob[-1]) - med)),
                     "n_edges": int(out["logit"].shape[0])}
        print(name, res[name], flush=True)
    with open(OUT, "w") as f:
        json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
