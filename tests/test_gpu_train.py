"""GPU: the training form (weighted BCE and the hand-written backward pass)
against the float64 oracle, whose own gradient is pinned by finite
differences in tests/test_oracle_grad.py.

Tolerances: the float32 backward differs from the float64 gradient by float32
rounding through n + 3 layers of MLPs and the message sums; per parameter
tensor the relative error of the gradient vector (2-norm) must stay below
1e-3, as must finite differences of the GPU forward on the largest entries.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle                                           # noqa: E402
from paper_2407_12119_amd import synth, velo           # noqa: E402

pytestmark = pytest.mark.gpu

GRAD_REL = 1e-3


def _setup(wl, batch, blob):
    print(f"\n[case] {wl.name} train events={batch.n_events} hits={batch.n_hits}", flush=True)
    ctx = velo.Context(wl.hidden, wl.iters, oracle.d2max_f32(wl.radius), wl.k_max, wl.edge_logit_min, "fp32",
                       max_hits=max(batch.n_hits, 1), max_events=max(batch.n_events, 1),
                       max_event_hits=max(batch.max_event_hits(), 1), training=True)
    params = torch.from_numpy(blob).cuda()
    ctx.set_params(params)
    hits = velo.DeviceHits.from_batch(batch)
    graph = ctx.build_graph(hits, ctx.embed(hits))
    return ctx, hits, graph, params


def _labels(batch, g):
    ys = []
    for b in range(batch.n_events):
        s, e = int(g["edge_offsets"][b]), int(g["edge_offsets"][b + 1])
        ys.append(synth.truth_labels(batch.event(b).next_hit, g["src"][s:e], g["dst"][s:e]))
    return np.concatenate(ys) if ys else np.zeros(0, np.uint8)


def _small_batch():
    wl = synth.WORKLOADS["train32"]
    return wl, synth.make_batch(synth.WORKLOADS["single_event"])


def test_train_forward_equals_inference():
    """The training forward (with checkpoints; the classifier as its own
    kernel) gives the inference logits to float32 rounding and is bitwise
    repeatable."""
    wl, batch = _small_batch()
    blob = synth.centred_params(wl)
    ctx, hits, graph, params = _setup(wl, batch, blob)
    ctx.gnn(hits, graph)
    z_inf = graph["edge_logit"].clone().cpu().numpy()
    ctx.train_forward(hits, graph, params, check=True)
    n = int(graph["n_edges"].cpu()[0])
    z_tr = graph["edge_logit"][:n].cpu().numpy()
    err = np.abs(z_tr - z_inf[:n]) / np.maximum(np.abs(z_inf[:n]), 1.0)
    assert err.max() <= 1e-5, err.max()
    ctx.train_forward(hits, graph, params, check=True)
    np.testing.assert_array_equal(graph["edge_logit"][:n].cpu().numpy(), z_tr)


def test_bce_matches_oracle():
    wl, batch = _small_batch()
    ctx, hits, graph, params = _setup(wl, batch, synth.centred_params(wl))
    rng = np.random.default_rng(1)
    z = rng.normal(0, 3, 5000).astype(np.float32)
    y = (rng.random(5000) < 0.2).astype(np.uint8)
    loss, dz = ctx.bce(torch.from_numpy(z).cuda(), torch.from_numpy(y).cuda(), 4.0, 5000)
    L_or, dz_or = oracle.bce(z.astype(np.float64), y, 4.0)
    assert float(loss.cpu()[0]) == pytest.approx(L_or, rel=1e-5)
    np.testing.assert_allclose(dz.cpu().numpy(), dz_or, rtol=1e-5, atol=1e-12)


@pytest.mark.parametrize("alpha,gamma", [(0.25, 2.0), (-1.0, 0.0), (0.6, 0.5)])
def test_focal_matches_oracle(alpha, gamma):
    """The sigmoid focal loss (Sec. 5.2) against the float64 oracle, on
    logits that include confident ones (|z| up to ~15)."""
    wl, batch = _small_batch()
    ctx, hits, graph, params = _setup(wl, batch, synth.centred_params(wl))
    rng = np.random.default_rng(2)
    z = rng.normal(0, 5, 7001).astype(np.float32)
    y = (rng.random(7001) < 0.3).astype(np.uint8)
    loss, dz = ctx.focal(torch.from_numpy(z).cuda(), torch.from_numpy(y).cuda(), alpha, gamma, 7001)
    L_or, dz_or = oracle.focal(z.astype(np.float64), y, alpha, gamma)
    assert float(loss.cpu()[0]) == pytest.approx(L_or, rel=1e-5)
    np.testing.assert_allclose(dz.cpu().numpy(), dz_or, rtol=1e-4, atol=1e-6 * np.abs(dz_or).max())
    # gamma = 0 without class weights is the plain cross-entropy
    if alpha < 0 and gamma == 0.0:
        lb, db = ctx.bce(torch.from_numpy(z).cuda(), torch.from_numpy(y).cuda(), 1.0, 7001)
        assert float(lb.cpu()[0]) == pytest.approx(float(loss.cpu()[0]), rel=1e-6)


def test_backward_matches_oracle_gradient():
    wl, batch = _small_batch()
    _check_gradient(wl, batch, synth.centred_params(wl))


def test_backward_matches_oracle_gradient_at_width_32():
    """H = 32 (the other width the training form takes), two steps."""
    wl = synth.dataclasses.replace(synth.WORKLOADS["train32"], hidden=32, iters=2)
    _check_gradient(wl, synth.make_batch(synth.WORKLOADS["single_event"]), synth.init_params(wl))


def test_backward_matches_oracle_gradient_on_six_training_events():
    """Six events of the 32-event training workload (about 280k edges): the
    weight-gradient pass splits the edge rows into 1,024 fixed chunks, so
    each chunk holds many 16-row tiles and the multi-tile loop (next-tile
    loads, the barrier between tiles) runs.  The reference is the sum of the
    float64 oracle's per-event gradients (events are independent and the
    objective sum(dlogit * z) adds over them)."""
    wl = synth.WORKLOADS["train32"]
    batch = synth.make_batch(wl, n_events=6)
    n_tiles = _check_gradient(wl, batch, synth.centred_params(wl))
    assert n_tiles / 1024 >= 8, n_tiles


def _check_gradient(wl, batch, blob):
    """Compare the GPU gradient of sum(dlogit * z) with the float64 oracle's
    on the GPU's graph; returns the number of 16-row edge tiles."""
    from concurrent.futures import ThreadPoolExecutor
    ctx, hits, graph, params = _setup(wl, batch, blob)
    ctx.train_forward(hits, graph, params, check=True)
    g = velo.graph_to_host(graph, batch.n_hits)
    rng = np.random.default_rng(2)
    dlogit = rng.normal(0, 1, g["n_edges"]).astype(np.float32)
    dp = ctx.train_backward(hits, params, torch.from_numpy(dlogit).cuda())
    ctx.check()
    dp = dp.cpu().numpy().astype(np.float64)
    eo = g["edge_offsets"]

    def one(b):
        ev = batch.event(b)
        s, e = int(eo[b]), int(eo[b + 1])
        return oracle.gnn_backward(ev.x, ev.y, ev.z, g["src"][s:e], g["dst"][s:e], blob, wl.hidden,
                                   wl.iters, dlogit[s:e].astype(np.float64))

    def oracle_grad(bl):
        nonlocal blob
        saved, blob = blob, bl
        try:
            with ThreadPoolExecutor(max_workers=min(8, max(batch.n_events, 1))) as ex:
                return sum(ex.map(one, range(batch.n_events)))
        finally:
            blob = saved

    def rel_errs(got, ref):
        vg, vr = synth.param_views(got, wl.hidden, wl.iters), synth.param_views(ref, wl.hidden, wl.iters)
        return {(name, j): np.linalg.norm(vg[name][j] - vr[name][j]) / max(np.linalg.norm(vr[name][j]), 1e-30)
                for name, _ in synth.param_layout(wl.hidden, wl.iters) if not name.startswith("emb")
                for j in (0, 1)}

    ref = oracle_grad(blob)
    assert np.all(dp[:12] == 0)
    for name, _ in synth.param_layout(wl.hidden, wl.iters):
        if name.startswith("emb"):
            assert all(np.all(v == 0) for v in synth.param_views(dp, wl.hidden, wl.iters)[name])
    errs = rel_errs(dp, ref)
    # The gradient is piecewise smooth: a hidden unit whose pre-activation
    # lies within float32 rounding of 0 takes either side of its ReLU (and
    # contributes a whole term, or none, to the weight gradients upstream).
    # A float32 layer output carries a relative rounding error of about
    # sqrt(K) u with K <= 3H inputs and u = 2^-24, i.e. about 2^-20.  How far
    # the float64 gradient itself moves when every parameter moves by a
    # random relative 2^-20 measures what any float32 evaluation can reach;
    # the GPU must stay within the larger of 1e-3 and twice the largest such
    # movement over three draws.
    rng_p = np.random.default_rng(11)
    sens = {k: 0.0 for k in errs}
    for _ in range(3):
        bl = (blob.astype(np.float64) * (1.0 + rng_p.uniform(-1.0, 1.0, blob.shape[0]) * 2.0 ** -20))
        bl = bl.astype(np.float32)
        bl[:12] = blob[:12]
        for k, v in rel_errs(oracle_grad(bl), ref).items():
            sens[k] = max(sens[k], v)
    tol = {k: max(GRAD_REL, 2 * sens[k]) for k in errs}
    worst = max(errs.values())
    print(f"  {g['n_edges']} edges, worst per-tensor relative gradient error {worst:.3g}; "
          f"{sum(t > GRAD_REL for t in tol.values())} tensors whose float32-rounding sensitivity exceeds "
          f"{GRAD_REL / 2:g}", flush=True)
    print("  " + ", ".join(f"{n}.{'wb'[j]} {e:.2g}/{tol[(n, j)]:.2g}" for (n, j), e in errs.items()), flush=True)
    bad = {k: (v, tol[k]) for k, v in errs.items() if v > tol[k]}
    assert not bad, bad
    return (g["n_edges"] + 15) // 16


def test_backward_against_finite_differences():
    """The GPU backward against central differences of L = sum dlogit * z.

    Differences of the float64 oracle forward (the method's definition) on the
    same graph for entries of every parameter tensor, and differences of the
    float32 GPU forward for the classifier's output layer, in which L is
    linear (exact differences; elsewhere float32 rounding noise of the forward
    is about 1e-3 of a difference quotient at usable step sizes).  A probe
    whose differences at h and h/2 disagree sits on a ReLU kink and is skipped.
    """
    wl = synth.dataclasses.replace(synth.WORKLOADS["train32"], iters=2)
    ev = synth.make_events(synth.WORKLOADS["single_event"])[0]
    keep = (ev.plane >= 9) & (ev.plane < 13)             # a small event: ~100 hits on four planes
    small = synth.Event(ev.x[keep], ev.y[keep], ev.z[keep], ev.plane[keep], ev.pid[keep],
                        np.full(int(keep.sum()), -1, np.int32))
    batch = synth.to_batch([small])
    blob = synth.init_params(wl)
    ctx, hits, graph, params = _setup(wl, batch, blob)
    g = velo.graph_to_host(graph, batch.n_hits)
    n = g["n_edges"]
    assert n > 20
    dl_np = np.random.default_rng(4).normal(0, 1, n).astype(np.float32)
    dl = torch.from_numpy(dl_np).cuda()
    ctx.train_forward(hits, graph, params)
    grad = ctx.train_backward(hits, params, dl).cpu().numpy()
    ev1 = batch.event(0)

    def L64(b):
        z = oracle.gnn_forward(ev1.x, ev1.y, ev1.z, g["src"], g["dst"], b, wl.hidden, wl.iters)
        return float(z @ dl_np.astype(np.float64))

    def L32(p):
        ctx.train_forward(hits, graph, p)
        return float((graph["edge_logit"][:n].double() * dl.double()).sum().cpu())

    lay = synth.param_layout(wl.hidden, wl.iters)
    offs, o = {}, 12
    for name, (r_, c_) in lay:
        offs[name] = (o, o + r_ * c_ + r_)
        o += r_ * c_ + r_
    picks = []
    for name, (a_, b_) in offs.items():
        if not name.startswith("emb"):
            picks += [a_ + int(k) for k in np.argsort(-np.abs(grad[a_:b_]))[:2]]

    L0 = L64(blob)

    def fd64(idx):
        """Central difference at the largest step whose left and right
        one-sided differences agree (no ReLU kink within the step)."""
        t = float(blob[idx])
        for k in range(8, 19):
            h = 2.0 ** -k * max(abs(t), 2.0 ** -4)
            bp, bm = blob.copy(), blob.copy()
            bp[idx] = np.float32(t + h)
            bm[idx] = np.float32(t - h)
            hp, hm = float(bp[idx]) - t, t - float(bm[idx])
            Lp, Lm = L64(bp), L64(bm)
            right, left = (Lp - L0) / hp, (L0 - Lm) / hm
            if abs(right - left) <= 1e-5 * max(abs(right), 1e-3):
                return (Lp - Lm) / (hp + hm)
        return None

    smooth = 0
    for idx in picks:
        f = fd64(idx)
        if f is None:
            continue
        smooth += 1
        assert f == pytest.approx(float(grad[idx]), rel=GRAD_REL, abs=1e-6 * np.abs(grad).max()), idx
    print(f"  {smooth} of {len(picks)} oracle-difference probes agree", flush=True)
    assert smooth >= len(picks) // 2

    # L is exactly linear in the classifier's output layer, so a large step
    # has no truncation error and keeps float32 rounding of the forward small
    a_, b_ = offs["cls1"]
    for idx in range(a_, b_, 7):
        t = float(blob[idx])
        h = 0.5
        pp, pm = params.clone(), params.clone()
        pp[idx] = t + h
        pm[idx] = t - h
        fd = (L32(pp) - L32(pm)) / (float(pp[idx].cpu()) - float(pm[idx].cpu()))
        assert fd == pytest.approx(float(grad[idx]), rel=GRAD_REL, abs=1e-6), idx


def test_backward_is_deterministic_and_descends():
    """Bitwise repeatable gradient; a small plain gradient step lowers the
    loss by the first-order prediction (Taylor: L(p - eta g) = L(p) -
    eta |g|^2 + O(eta^2)); and the Adam kernel applies the textbook update
    (Kingma and Ba, Algorithm 1) computed here in float64."""
    wl = synth.WORKLOADS["train32"]
    batch = synth.make_batch(wl, n_events=4)
    blob = synth.init_params(wl)
    ctx, hits, graph, params = _setup(wl, batch, blob)
    g = velo.graph_to_host(graph, batch.n_hits)
    n = g["n_edges"]
    y = _labels(batch, g)
    pw = float((y == 0).sum()) / max(float(y.sum()), 1.0)
    yt = torch.from_numpy(y).cuda()

    def loss_grad(p):
        ctx.train_forward(hits, graph, p)
        loss, dz = ctx.bce(graph["edge_logit"], yt, pw, n)
        return float(loss.cpu()[0]), ctx.train_backward(hits, p, dz).clone()

    L0, g1 = loss_grad(params)
    _, g2 = loss_grad(params)
    assert torch.equal(g1, g2)
    gn2 = float((g1.double() ** 2).sum())
    # a step whose predicted decrease is 0.1% of the loss: the second-order
    # term is then well below the first at these weights
    eta = 0.001 * L0 / gn2
    L1, _ = loss_grad(params - eta * g1)
    pred = eta * gn2
    print(f"  L {L0:.6f} -> {L1:.6f}: decrease {L0 - L1:.3e}, first-order {pred:.3e}", flush=True)
    assert L1 < L0
    assert abs((L0 - L1) - pred) <= 0.2 * pred

    # Adam: two steps against float64 arithmetic on the same gradients
    rng = np.random.default_rng(5)
    p = params.clone()
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    p64, m64, v64 = p.cpu().numpy().astype(np.float64), np.zeros(p.numel()), np.zeros(p.numel())
    lr, b1, b2, eps = 3e-3, 0.9, 0.999, 1e-8
    for step in (1, 2):
        gr = torch.from_numpy(rng.normal(0, 1e-2, p.numel()).astype(np.float32)).cuda()
        ctx.adam_step(p, gr, m, v, step, lr=lr, b1=b1, b2=b2, eps=eps)
        g64 = gr.cpu().numpy().astype(np.float64)
        m64 = b1 * m64 + (1 - b1) * g64
        v64 = b2 * v64 + (1 - b2) * g64 * g64
        p64 = p64 - lr * (m64 / (1 - b1 ** step)) / (np.sqrt(v64 / (1 - b2 ** step)) + eps)
        # float32 state: each update is exact to a few float32 roundings of lr
        np.testing.assert_allclose(p.cpu().numpy(), p64, rtol=0, atol=1e-6 + 1e-6 * np.abs(p64).max())
    ctx.check()


def test_autograd_function_gives_the_library_gradient():
    """loss.backward() through EdgeLogits and WeightedBCE equals the explicit
    forward / bce / backward calls, bitwise; a backward after another forward
    on the same context is refused."""
    from paper_2407_12119_amd import train
    wl = synth.WORKLOADS["train32"]
    batch = synth.make_batch(wl, n_events=3)
    blob = synth.init_params(wl)
    ctx, hits, graph, params = _setup(wl, batch, blob)
    g = velo.graph_to_host(graph, batch.n_hits)
    n = g["n_edges"]
    yt = torch.from_numpy(_labels(batch, g)).cuda()
    p = params.clone().requires_grad_(True)
    z = train.edge_logits(ctx, p, hits, graph, n)
    loss = train.weighted_bce(ctx, z, yt, 3.0)
    loss.backward()
    ctx.train_forward(hits, graph, params)
    loss2, dz = ctx.bce(graph["edge_logit"], yt, 3.0, n)
    g2 = ctx.train_backward(hits, params, dz)
    assert float(loss.detach()) == float(loss2.cpu()[0])
    assert torch.equal(p.grad, g2)
    z = train.edge_logits(ctx, p, hits, graph, n)
    ctx.train_forward(hits, graph, params)
    with pytest.raises(RuntimeError, match="checkpoints"):
        z.sum().backward()


def test_focal_autograd_gives_the_library_gradient():
    """loss.backward() through EdgeLogits and FocalLoss equals the explicit
    forward / focal / backward calls, bitwise."""
    from paper_2407_12119_amd import train
    wl = synth.WORKLOADS["train32"]
    batch = synth.make_batch(wl, n_events=2)
    blob = synth.init_params(wl)
    ctx, hits, graph, params = _setup(wl, batch, blob)
    g = velo.graph_to_host(graph, batch.n_hits)
    n = g["n_edges"]
    yt = torch.from_numpy(_labels(batch, g)).cuda()
    p = params.clone().requires_grad_(True)
    loss = train.focal_loss(ctx, train.edge_logits(ctx, p, hits, graph, n), yt, 0.25, 2.0)
    loss.backward()
    ctx.train_forward(hits, graph, params)
    loss2, dz = ctx.focal(graph["edge_logit"], yt, 0.25, 2.0, n)
    g2 = ctx.train_backward(hits, params, dz)
    assert float(loss) == float(loss2.cpu()[0])
    assert torch.equal(p.grad, g2)


def test_trainer_learns_edges_of_generated_events():
    """A few hundred Adam steps on generated events: the loss falls and the
    trained classifier separates true from fake edges on held-out events."""
    from paper_2407_12119_amd import train
    wl = synth.dataclasses.replace(synth.WORKLOADS["train32"], iters=4)
    batches = [synth.make_batch(wl, n_events=8, first=8 * i) for i in range(2)]
    params = torch.from_numpy(synth.init_params(wl)).cuda()
    tr = train.Trainer(wl, params, batches, lr=3e-3)
    first = float(tr.step().cpu())
    for _ in range(119):
        last = tr.step()
    last = float(last.cpu())
    tr.vctx.check()
    print(f"  loss {first:.4f} -> {last:.4f}", flush=True)
    assert last < 0.7 * first
    held = train.GraphBatch(tr.vctx, synth.make_batch(wl, n_events=4, first=100))
    tr.vctx.train_forward(held.hits, held.graph, tr.params)
    z = held.graph["edge_logit"][:held.n_edges].cpu().numpy()
    y = held.y.cpu().numpy().astype(bool)
    # the median true edge scores above the median fake edge
    assert np.median(z[y]) > np.median(z[~y])
    tr.close()
