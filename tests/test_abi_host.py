"""Host-side argument validation of the C ABI, without a GPU: every entry
point refuses a null context or a malformed argument before it touches the
device, with the status include/velognn.h documents."""
import ctypes as C

import pytest

from paper_2407_12119_amd import velo

ST = {"ok": velo.VELO_OK, "arg": velo.VELO_ERR_INVALID_ARG, "cap": velo.VELO_ERR_CAPACITY,
      "unsupported": velo.VELO_ERR_UNSUPPORTED}


def _cfg(**kw):
    c = dict(gnn_hidden=64, gnn_iters=4, d2_max=0.01, k_max=32, edge_logit_min=0.0, precision=velo.VELO_FP32,
             max_hits=1000, max_edges=32000, max_events=4, max_event_hits=600, training=0)
    c.update(kw)
    return velo._Config(**c)


@pytest.mark.parametrize("kw,status", [
    (dict(gnn_hidden=48), "unsupported"),
    (dict(gnn_hidden=128, precision=velo.VELO_FP32), "unsupported"),
    (dict(precision=9), "unsupported"),
    (dict(training=1, precision=velo.VELO_BF16), "unsupported"),
    (dict(gnn_iters=17), "arg"),
    (dict(gnn_iters=-1), "arg"),
    (dict(k_max=0), "arg"),
    (dict(k_max=65), "arg"),
    (dict(max_hits=-1), "arg"),
    (dict(max_events=-1), "arg"),
    (dict(max_event_hits=-1), "arg"),
    (dict(d2_max=float("nan")), "arg"),
    (dict(d2_max=-1.0), "arg"),
    (dict(max_edges=1 << 31), "unsupported"),
    (dict(max_hits=1 << 26, k_max=64), "unsupported"),
])
def test_create_refuses_bad_configs_on_the_host(kw, status):
    L = velo.lib()
    h = C.c_void_p()
    cfg = _cfg(**kw)
    assert L.velo_create(C.byref(cfg), C.byref(h)) == ST[status]
    assert not h.value


def test_create_refuses_null_pointers():
    L = velo.lib()
    h = C.c_void_p()
    assert L.velo_create(None, C.byref(h)) == ST["arg"]
    cfg = _cfg()
    assert L.velo_create(C.byref(cfg), None) == ST["arg"]


def test_every_entry_point_refuses_a_null_context():
    L = velo.lib()
    hits, out = velo._Hits(), velo._Outputs()
    hp, op = C.byref(hits), C.byref(out)
    calls = {
        "velo_set_params": (None, None, 0, None),
        "velo_calibrate": (None, hp, None),
        "velo_infer": (None, hp, op, None),
        "velo_embed": (None, hp, None, None),
        "velo_build_graph": (None, hp, None, op, None),
        "velo_build_graph_loop": (None, hp, None, op, None),
        "velo_gnn": (None, hp, op, None),
        "velo_components": (None, hp, op, None),
        "velo_components_sweep": (None, hp, op, None),
        "velo_set_timing": (None, 1),
        "velo_read_timing": (None, None, None),
        "velo_train_forward": (None, hp, op, None, None),
        "velo_bce": (None, None, None, 1.0, 0, None, None, None),
        "velo_focal": (None, None, None, 0.25, 2.0, 0, None, None, None),
        "velo_train_backward": (None, hp, None, None, None, None),
        "velo_adam_step": (None, None, None, None, None, 0, 1e-3, 0.9, 0.999, 1e-8, 1, None),
        "velo_autotune": (None, hp, op, None, None),
        "velo_set_tuning": (None, None),
        "velo_check": (None, None),
        "velo_set_embed_int8": (None, None),
        "velo_calibrate_embed_int8": (None, hp, None, None),
        "velo_set_triplet_params": (None, None, 0, 0.0, 0, None),
        "velo_embed_train_grad": (None, hp, None, None, 50, 1.5, 1.0, 2.0, None, None, None, None, None),
    }
    for name, args in calls.items():
        assert getattr(L, name)(*args) == ST["arg"], name
    assert L.velo_last_error(None) == b"null context"
    L.velo_destroy(None)           # safe on NULL


def test_noalloc_components_host_checks():
    """velo_components_noalloc refuses malformed arguments and sizes beyond
    its fixed working memory before any launch."""
    L = velo.lib()
    fake = 4096                     # never dereferenced: every call below is refused on the host
    out = velo._Outputs(fake, fake, fake, fake, fake, 100, fake)
    good = velo._Hits(2, 10, fake, fake, fake, fake, fake)
    assert L.velo_components_noalloc(None, C.byref(out), 0.0, 16, None) == ST["arg"]
    assert L.velo_components_noalloc(C.byref(good), None, 0.0, 16, None) == ST["arg"]
    assert L.velo_components_noalloc(C.byref(good), C.byref(out), 0.0, -1, None) == ST["arg"]
    bad = [velo._Hits(-1, 10, fake, fake, fake, fake, fake), velo._Hits(2, -5, fake, fake, fake, fake, fake),
           velo._Hits(0, 3, fake, fake, fake, fake, fake), velo._Hits(2, 10, None, fake, fake, fake, fake),
           velo._Hits(2, 10, fake, None, fake, fake, fake)]
    for h in bad:
        assert L.velo_components_noalloc(C.byref(h), C.byref(out), 0.0, 16, None) == ST["arg"]
    for o in (velo._Outputs(None, fake, fake, fake, fake, 100, fake), velo._Outputs(fake, fake, fake, fake, fake, 100, None),
              velo._Outputs(fake, fake, None, fake, fake, 100, fake), velo._Outputs(fake, fake, fake, fake, None, 100, fake),
              velo._Outputs(fake, fake, fake, fake, fake, -1, fake)):
        assert L.velo_components_noalloc(C.byref(good), C.byref(o), 0.0, 16, None) == ST["arg"]
    big = velo._Hits(2, (1 << 20) + 1, fake, fake, fake, fake, fake)
    assert L.velo_components_noalloc(C.byref(big), C.byref(out), 0.0, 16, None) == ST["cap"]
    many = velo._Hits((1 << 14) + 1, 10, fake, fake, fake, fake, fake)
    assert L.velo_components_noalloc(C.byref(many), C.byref(out), 0.0, 16, None) == ST["cap"]
    huge_cap = velo._Outputs(fake, fake, fake, fake, fake, 1 << 31, fake)
    assert L.velo_components_noalloc(C.byref(good), C.byref(huge_cap), 0.0, 16, None) == ST["unsupported"]


def test_parameter_counts_and_status_strings():
    L = velo.lib()
    assert L.velo_triplet_param_count(48) == -1
    assert L.velo_triplet_param_count(64) == 2 * (2 * 64 * 64 + 2 * 64 + 1)
    assert L.velo_param_count(64, -1) == -1
    for st in range(8):
        assert L.velo_status_str(st) and L.velo_status_str(st) != b"unknown status"
    assert L.velo_status_str(99) == b"unknown status"
