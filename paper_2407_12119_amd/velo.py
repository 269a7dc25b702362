"""Python binding of libvelognn.so (include/velognn.h): argument marshalling only.

Every step of the path runs in the library's HIP kernels; torch supplies device
memory and the current stream.  Loading fails loudly when the library is not
built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
from typing import Dict, Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
# VELO_LIB: another build of the library to load (the host-sanitizer test builds one)
LIB_PATH = os.environ.get("VELO_LIB") or os.path.join(_PKG, "libvelognn.so")

VELO_OK, VELO_ERR_INVALID_ARG, VELO_ERR_CAPACITY, VELO_ERR_OOM = 0, 1, 2, 3
VELO_ERR_DEVICE, VELO_ERR_UNSUPPORTED, VELO_ERR_INPUT, VELO_ERR_NOT_CALIBRATED = 4, 5, 6, 7
VELO_FP32, VELO_BF16, VELO_FP8, VELO_BF16X2 = 0, 1, 2, 3
PRECISIONS = {"fp32": VELO_FP32, "bf16": VELO_BF16, "fp8": VELO_FP8, "bf16x2": VELO_BF16X2}
N_PLANES, EMB_HIDDEN, EMB_DIM = 26, 128, 4

EXPORTS = ("velo_param_count", "velo_create", "velo_destroy", "velo_set_params", "velo_infer",
           "velo_embed", "velo_build_graph", "velo_gnn", "velo_components", "velo_check",
           "velo_status_str", "velo_last_error", "velo_set_timing", "velo_read_timing",
           "velo_train_forward", "velo_bce", "velo_train_backward", "velo_adam_step",
           "velo_graph_capture", "velo_graph_launch", "velo_graph_destroy", "velo_calibrate",
           "velo_autotune", "velo_embed_train_grad", "velo_focal", "velo_components_sweep",
           "velo_build_graph_loop", "velo_set_embed_int8", "velo_calibrate_embed_int8",
           "velo_triplet_param_count", "velo_set_triplet_params", "velo_triplets", "velo_components_noalloc", "velo_set_tuning")
# velo_autotune's candidate configurations (the table of include/velognn.h):
# MLP blocks per CU (0: by occupancy), MLP workgroup threads, k-NN / message
# blocks per CU, k-NN query hits per wavefront task, XCD-blocked mapping
AUTOTUNE_CANDIDATES = [
    {"mlp_per_cu": m, "mlp_block": b, "mem_per_cu": q, "knn_run": r, "xcd": x}
    for m, b, q, r, x in zip((0, 0, 1, 2, 0, 1, 0, 2), (512, 512, 512, 512, 256, 256, 1024, 1024),
                             (16, 16, 4, 8, 32, 32, 8, 16), (16, 16, 8, 32, 8, 32, 32, 8), (0, 1, 1, 1, 1, 0, 0, 1))]
STAGES = ("prepare", "embed", "knn", "compact", "lists", "node_enc", "edge_enc", "messages",
          "node_net", "edge_net", "edge_cls", "components", "bce", "bwd_mlp", "bwd_dw", "bwd_graph", "adam",
          "hit_proj", "emb_loss", "emb_bwd", "triplets")


class VeloError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(msg)
        self.status = status


class _Config(C.Structure):
    _fields_ = [("gnn_hidden", C.c_int32), ("gnn_iters", C.c_int32), ("d2_max", C.c_float),
                ("k_max", C.c_int32), ("edge_logit_min", C.c_float), ("precision", C.c_int32),
                ("max_hits", C.c_int64), ("max_edges", C.c_int64), ("max_events", C.c_int32),
                ("max_event_hits", C.c_int32), ("training", C.c_int32)]


class _Hits(C.Structure):
    _fields_ = [("n_events", C.c_int32), ("n_hits", C.c_int64), ("event_offsets", C.c_void_p),
                ("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p), ("plane", C.c_void_p)]


class _Outputs(C.Structure):
    _fields_ = [("labels", C.c_void_p), ("edge_offsets", C.c_void_p), ("edge_src", C.c_void_p),
                ("edge_dst", C.c_void_p), ("edge_logit", C.c_void_p), ("edge_capacity", C.c_int64),
                ("n_edges", C.c_void_p)]


class _TripletOutputs(C.Structure):
    _fields_ = [("art", C.c_void_p), ("art_offsets", C.c_void_p), ("art_logit", C.c_void_p),
                ("elb", C.c_void_p), ("elb_type", C.c_void_p), ("elb_offsets", C.c_void_p),
                ("elb_logit", C.c_void_p), ("capacity", C.c_int64), ("n_triplets", C.c_void_p),
                ("edge_seg", C.c_void_p), ("tracks", C.c_void_p), ("track_offsets", C.c_void_p),
                ("track_capacity", C.c_int64), ("n_tracks", C.c_void_p)]


_lib: Optional[C.CDLL] = None


def lib() -> C.CDLL:
    """Load libvelognn.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, st = C.c_void_p, C.c_int
        L.velo_param_count.argtypes = [C.c_int32, C.c_int32]
        L.velo_param_count.restype = C.c_int64
        L.velo_create.argtypes = [C.POINTER(_Config), C.POINTER(vp)]
        L.velo_create.restype = st
        L.velo_destroy.argtypes = [vp]
        L.velo_destroy.restype = None
        L.velo_set_params.argtypes = [vp, vp, C.c_int64, vp]
        L.velo_set_params.restype = st
        for name in ("velo_infer", "velo_gnn", "velo_components"):
            getattr(L, name).argtypes = [vp, C.POINTER(_Hits), C.POINTER(_Outputs), vp]
            getattr(L, name).restype = st
        L.velo_embed.argtypes = [vp, C.POINTER(_Hits), vp, vp]
        L.velo_embed.restype = st
        L.velo_build_graph.argtypes = [vp, C.POINTER(_Hits), vp, C.POINTER(_Outputs), vp]
        L.velo_build_graph.restype = st
        L.velo_check.argtypes = [vp, vp]
        L.velo_check.restype = st
        L.velo_status_str.argtypes = [st]
        L.velo_status_str.restype = C.c_char_p
        L.velo_last_error.argtypes = [vp]
        L.velo_last_error.restype = C.c_char_p
        L.velo_set_timing.argtypes = [vp, C.c_int32]
        L.velo_set_timing.restype = st
        L.velo_read_timing.argtypes = [vp, vp, vp]
        L.velo_read_timing.restype = st
        L.velo_train_forward.argtypes = [vp, C.POINTER(_Hits), C.POINTER(_Outputs), vp, vp]
        L.velo_train_forward.restype = st
        L.velo_bce.argtypes = [vp, vp, vp, C.c_float, C.c_int64, vp, vp, vp]
        L.velo_bce.restype = st
        L.velo_train_backward.argtypes = [vp, C.POINTER(_Hits), vp, vp, vp, vp]
        L.velo_train_backward.restype = st
        L.velo_adam_step.argtypes = [vp, vp, vp, vp, vp, C.c_int64, C.c_float, C.c_float, C.c_float, C.c_float,
                                     C.c_int32, vp]
        L.velo_adam_step.restype = st
        L.velo_graph_capture.argtypes = [vp, C.POINTER(_Hits), C.POINTER(_Outputs), vp, C.POINTER(vp)]
        L.velo_graph_capture.restype = st
        L.velo_graph_launch.argtypes = [vp, vp]
        L.velo_graph_launch.restype = st
        L.velo_graph_destroy.argtypes = [vp]
        L.velo_graph_destroy.restype = None
        L.velo_calibrate.argtypes = [vp, C.POINTER(_Hits), vp]
        L.velo_calibrate.restype = st
        L.velo_autotune.argtypes = [vp, C.POINTER(_Hits), C.POINTER(_Outputs), vp, vp]
        L.velo_autotune.restype = st
        L.velo_set_tuning.argtypes = [vp, vp]
        L.velo_set_tuning.restype = st
        L.velo_embed_train_grad.argtypes = [vp, C.POINTER(_Hits), C.POINTER(_EmbedTruth), vp, C.c_int32,
                                            C.c_float, C.c_float, C.c_float, vp, vp, vp, vp, vp]
        L.velo_embed_train_grad.restype = st
        L.velo_focal.argtypes = [vp, vp, vp, C.c_float, C.c_float, C.c_int64, vp, vp, vp]
        L.velo_focal.restype = st
        L.velo_components_noalloc.argtypes = [C.POINTER(_Hits), C.POINTER(_Outputs), C.c_float, C.c_int32, vp]
        L.velo_components_noalloc.restype = st
        L.velo_components_sweep.argtypes = [vp, C.POINTER(_Hits), C.POINTER(_Outputs), vp]
        L.velo_components_sweep.restype = st
        L.velo_build_graph_loop.argtypes = [vp, C.POINTER(_Hits), vp, C.POINTER(_Outputs), vp]
        L.velo_build_graph_loop.restype = st
        L.velo_set_embed_int8.argtypes = [vp, vp]
        L.velo_set_embed_int8.restype = st
        L.velo_calibrate_embed_int8.argtypes = [vp, C.POINTER(_Hits), vp, vp]
        L.velo_calibrate_embed_int8.restype = st
        L.velo_triplet_param_count.argtypes = [C.c_int32]
        L.velo_triplet_param_count.restype = C.c_int64
        L.velo_set_triplet_params.argtypes = [vp, vp, C.c_int64, C.c_float, C.c_int64, vp]
        L.velo_set_triplet_params.restype = st
        L.velo_triplets.argtypes = [vp, C.POINTER(_Hits), C.POINTER(_Outputs), C.POINTER(_TripletOutputs), vp]
        L.velo_triplets.restype = st
        _lib = L
    return _lib


def param_count(hidden: int, iters: int) -> int:
    return int(lib().velo_param_count(hidden, iters))


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


class _EmbedTruth(C.Structure):
    _fields_ = [("pid", C.c_void_p), ("query", C.c_void_p), ("rnd", C.c_void_p)]


@dataclasses.dataclass
class DeviceHits:
    """A batch of hits resident on the device (torch tensors)."""
    event_offsets: "object"     # int32 [B+1]
    x: "object"
    y: "object"
    z: "object"
    plane: "object"             # int32 [N]
    n_events: int
    n_hits: int
    max_event_hits: int

    @staticmethod
    def from_batch(batch, device="cuda") -> "DeviceHits":
        import torch
        t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(device)
        return DeviceHits(t(batch.event_offsets, np.int32), t(batch.x, np.float32), t(batch.y, np.float32),
                          t(batch.z, np.float32), t(batch.plane, np.int32), batch.n_events, batch.n_hits,
                          batch.max_event_hits())

    def c(self) -> _Hits:
        return _Hits(self.n_events, self.n_hits, _ptr(self.event_offsets), _ptr(self.x), _ptr(self.y),
                     _ptr(self.z), _ptr(self.plane))


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Context:
    """A library context: network shape, capacities and parameters."""

    def __init__(self, hidden: int, iters: int, d2_max: float, k_max: int = 32,
                 edge_logit_min: float = 0.0, precision: str = "fp32", max_hits: int = 1 << 20,
                 max_edges: Optional[int] = None, max_events: int = 1024, max_event_hits: int = 16384,
                 training: bool = False):
        self._lib = lib()
        self._train_gen = 0
        self.hidden, self.iters, self.k_max = hidden, iters, k_max
        if max_edges is None:
            max_edges = max(1, k_max * max_hits)
        self.cfg = _Config(hidden, iters, float(np.float32(d2_max)), k_max, float(edge_logit_min),
                           PRECISIONS[precision], max_hits, max_edges, max_events, max_event_hits,
                           1 if training else 0)
        h = C.c_void_p()
        st = self._lib.velo_create(C.byref(self.cfg), C.byref(h))
        if st != VELO_OK:
            raise VeloError(st, f"velo_create: {self._lib.velo_status_str(st).decode()}")
        self._h = h
        self.max_edges = max_edges

    def close(self):
        if getattr(self, "_h", None):
            self._lib.velo_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _raise(self, st: int, what: str):
        if st != VELO_OK:
            detail = self._lib.velo_last_error(self._h).decode()
            raise VeloError(st, f"{what}: {self._lib.velo_status_str(st).decode()} ({detail})")

    def set_params(self, params):
        """params: float32 device tensor with the blob layout of include/velognn.h."""
        self._params_ref = params
        self._raise(self._lib.velo_set_params(self._h, C.c_void_p(params.data_ptr()), params.numel(),
                                              _stream()), "velo_set_params")

    def set_timing(self, enable: bool):
        self._raise(self._lib.velo_set_timing(self._h, 1 if enable else 0), "velo_set_timing")

    def read_timing(self):
        """{stage: (milliseconds, launches)} since the last read (synchronises)."""
        ms = np.zeros(len(STAGES), np.float64)
        n = np.zeros(len(STAGES), np.int64)
        self._raise(self._lib.velo_read_timing(self._h, ms.ctypes.data, n.ctypes.data), "velo_read_timing")
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(STAGES)}

    def set_triplet_params(self, tparams, logit_min: float = 0.0, max_triplets: int = 1 << 20):
        """Enable the triplet stage with the two classifiers' parameters (a
        float32 device tensor); None disables it."""
        if tparams is None:
            self._raise(self._lib.velo_set_triplet_params(self._h, None, 0, 0.0, 0, _stream()),
                        "velo_set_triplet_params")
            return
        self._raise(self._lib.velo_set_triplet_params(self._h, _ptr(tparams), tparams.numel(), float(logit_min),
                                                      int(max_triplets), _stream()), "velo_set_triplet_params")
        self.max_triplets = int(max_triplets)

    def alloc_triplet_outputs(self, hits: DeviceHits, graph, capacity: int, track_capacity: int):
        import torch
        dev = hits.x.device
        B = hits.n_events
        return {"art": torch.empty(max(capacity, 1), 2, dtype=torch.int32, device=dev),
                "art_offsets": torch.empty(B + 1, dtype=torch.int32, device=dev),
                "art_logit": torch.empty(max(capacity, 1), dtype=torch.float32, device=dev),
                "elb": torch.empty(max(capacity, 1), 2, dtype=torch.int32, device=dev),
                "elb_type": torch.empty(max(capacity, 1), dtype=torch.int8, device=dev),
                "elb_offsets": torch.empty(B + 1, dtype=torch.int32, device=dev),
                "elb_logit": torch.empty(max(capacity, 1), dtype=torch.float32, device=dev),
                "capacity": int(capacity),
                "n_triplets": torch.zeros(2, dtype=torch.int32, device=dev),
                "edge_seg": torch.empty(max(int(graph["edge_capacity"]), 1), dtype=torch.int32, device=dev),
                "tracks": torch.empty(max(track_capacity, 1), 2, dtype=torch.int32, device=dev),
                "track_offsets": torch.empty(B + 1, dtype=torch.int32, device=dev),
                "track_capacity": int(track_capacity),
                "n_tracks": torch.zeros(1, dtype=torch.int32, device=dev)}

    def triplets(self, hits: DeviceHits, graph, out=None, capacity: Optional[int] = None,
                 track_capacity: Optional[int] = None, check: bool = True):
        """velo_triplets on the graph of the directly preceding gnn/infer call."""
        if out is None:
            cap = getattr(self, "max_triplets", 0) if capacity is None else capacity
            tcap = int(graph["edge_capacity"]) + cap if track_capacity is None else track_capacity
            out = self.alloc_triplet_outputs(hits, graph, cap, tcap)
        oc = self._out_c(graph)
        hc = hits.c()
        tc = _TripletOutputs(*[(_ptr(out[k]) if k not in ("capacity", "track_capacity") else out[k])
                               for k, _ in _TripletOutputs._fields_])
        self._raise(self._lib.velo_triplets(self._h, C.byref(hc), C.byref(oc), C.byref(tc), _stream()),
                    "velo_triplets")
        if check:
            self.check()
        out["graph_n_edges"] = graph["n_edges"]     # edge_seg holds this many entries
        return out

    def set_embed_int8(self, scales):
        """INT8 embedding with the four float32 scales {s_x2, s_w2, s_x3, s_w3}; None: off."""
        if scales is None:
            self._raise(self._lib.velo_set_embed_int8(self._h, None), "velo_set_embed_int8")
            return
        sc = (C.c_float * 4)(*[float(v) for v in scales])
        self._raise(self._lib.velo_set_embed_int8(self._h, C.cast(sc, C.c_void_p)), "velo_set_embed_int8")

    def calibrate_embed_int8(self, hits: DeviceHits):
        """Calibrate and enable the INT8 embedding on a batch; returns the four scales."""
        import numpy as np
        sc = (C.c_float * 4)()
        hc = hits.c()
        self._raise(self._lib.velo_calibrate_embed_int8(self._h, C.byref(hc), C.cast(sc, C.c_void_p), _stream()),
                    "velo_calibrate_embed_int8")
        return np.array(list(sc), np.float32)

    def calibrate(self, hits: DeviceHits, check: bool = True):
        """fp8: set the activation scales from a calibration batch."""
        hc = hits.c()
        self._raise(self._lib.velo_calibrate(self._h, C.byref(hc), _stream()), "velo_calibrate")
        if check:
            self.check()

    def autotune(self, hits: DeviceHits, out):
        """Pick launch parameters per stage by timing candidates on this batch."""
        oc = self._out_c(out)
        hc = hits.c()
        choice = np.zeros(len(STAGES), np.int32)
        self._raise(self._lib.velo_autotune(self._h, C.byref(hc), C.byref(oc), _stream(), choice.ctypes.data),
                    "velo_autotune")
        return {k: int(choice[i]) for i, k in enumerate(STAGES)}

    def set_tuning(self, choice=None):
        """Apply velo_autotune candidates: a {stage: index} dict (stages not
        named keep candidate 0), an int for every tuned stage, or None for
        the built-in launch parameters."""
        if choice is None:
            self._raise(self._lib.velo_set_tuning(self._h, None), "velo_set_tuning")
            return
        arr = np.zeros(len(STAGES), np.int32)
        if isinstance(choice, int):
            arr[:] = choice
        else:
            for k, v in choice.items():
                arr[STAGES.index(k)] = v
        self._raise(self._lib.velo_set_tuning(self._h, arr.ctypes.data), "velo_set_tuning")

    def check(self):
        self._raise(self._lib.velo_check(self._h, _stream()), "velo_check")

    # ---- output allocation ----
    def alloc_outputs(self, hits: DeviceHits, edge_capacity: Optional[int] = None) -> Dict[str, object]:
        import torch
        dev = hits.x.device
        cap = self.max_edges if edge_capacity is None else edge_capacity
        return {"labels": torch.empty(max(hits.n_hits, 1), dtype=torch.int32, device=dev),
                "edge_offsets": torch.empty(hits.n_events + 1, dtype=torch.int32, device=dev),
                "edge_src": torch.empty(max(cap, 1), dtype=torch.int32, device=dev),
                "edge_dst": torch.empty(max(cap, 1), dtype=torch.int32, device=dev),
                "edge_logit": torch.empty(max(cap, 1), dtype=torch.float32, device=dev),
                "n_edges": torch.zeros(1, dtype=torch.int32, device=dev),
                "edge_capacity": cap}

    @staticmethod
    def _out_c(o) -> _Outputs:
        return _Outputs(_ptr(o.get("labels")), _ptr(o.get("edge_offsets")), _ptr(o.get("edge_src")),
                        _ptr(o.get("edge_dst")), _ptr(o.get("edge_logit")), int(o["edge_capacity"]),
                        _ptr(o.get("n_edges")))

    # ---- calls ----
    def infer(self, hits: DeviceHits, out: Optional[Dict[str, object]] = None, check: bool = True):
        out = self.alloc_outputs(hits) if out is None else out
        oc = self._out_c(out)
        hc = hits.c()
        self._raise(self._lib.velo_infer(self._h, C.byref(hc), C.byref(oc), _stream()), "velo_infer")
        if check:
            self.check()
        return out

    def embed(self, hits: DeviceHits, check: bool = True):
        import torch
        emb = torch.empty((max(hits.n_hits, 1), EMB_DIM), dtype=torch.float32, device=hits.x.device)
        hc = hits.c()
        self._raise(self._lib.velo_embed(self._h, C.byref(hc), C.c_void_p(emb.data_ptr()), _stream()),
                    "velo_embed")
        if check:
            self.check()
        return emb[:hits.n_hits]

    def build_graph(self, hits: DeviceHits, emb, out=None, check: bool = True):
        out = self.alloc_outputs(hits) if out is None else out
        oc = self._out_c(out)
        hc = hits.c()
        self._raise(self._lib.velo_build_graph(self._h, C.byref(hc), C.c_void_p(emb.data_ptr()), C.byref(oc),
                                               _stream()), "velo_build_graph")
        if check:
            self.check()
        return out

    def build_graph_loop(self, hits: DeviceHits, emb, out=None, check: bool = True):
        """The paper's per-hit neighbour loop (Sec. 7.2): a comparison variant of build_graph."""
        out = self.alloc_outputs(hits) if out is None else out
        oc = self._out_c(out)
        hc = hits.c()
        self._raise(self._lib.velo_build_graph_loop(self._h, C.byref(hc), C.c_void_p(emb.data_ptr()), C.byref(oc),
                                                    _stream()), "velo_build_graph_loop")
        if check:
            self.check()
        return out

    def gnn(self, hits: DeviceHits, graph, check: bool = True):
        oc = self._out_c(graph)
        hc = hits.c()
        self._raise(self._lib.velo_gnn(self._h, C.byref(hc), C.byref(oc), _stream()), "velo_gnn")
        if check:
            self.check()
        return graph

    def components(self, hits: DeviceHits, graph, check: bool = True):
        oc = self._out_c(graph)
        hc = hits.c()
        self._raise(self._lib.velo_components(self._h, C.byref(hc), C.byref(oc), _stream()),
                    "velo_components")
        if check:
            self.check()
        return graph

    def components_sweep(self, hits: DeviceHits, graph, check: bool = True):
        """The paper's two plane sweeps (Sec. 7.3) into graph["labels"]: a comparison variant."""
        oc = self._out_c(graph)
        hc = hits.c()
        self._raise(self._lib.velo_components_sweep(self._h, C.byref(hc), C.byref(oc), _stream()),
                    "velo_components_sweep")
        if check:
            self.check()
        return graph


    # ---- graph capture ----
    def capture(self, hits: DeviceHits, out) -> "Graph":
        """Capture velo_infer on (hits, out) into a replayable HIP graph."""
        oc = self._out_c(out)
        hc = hits.c()
        g = C.c_void_p()
        self._raise(self._lib.velo_graph_capture(self._h, C.byref(hc), C.byref(oc), _stream(), C.byref(g)),
                    "velo_graph_capture")
        return Graph(self, g, hits, out)

    # ---- training form ----
    def train_forward(self, hits: DeviceHits, graph, params, check: bool = False):
        """Logits of `graph` under the float32 blob `params` (device); keeps checkpoints."""
        oc = self._out_c(graph)
        hc = hits.c()
        self._raise(self._lib.velo_train_forward(self._h, C.byref(hc), C.byref(oc), C.c_void_p(params.data_ptr()),
                                                 _stream()), "velo_train_forward")
        self._train_gen += 1          # the checkpoints now belong to this call
        if check:
            self.check()
        return graph

    def bce(self, logit, y, pos_weight: float, n: int):
        """(loss [1], dlogit [n]) device tensors of the weighted BCE on the first n logits."""
        import torch
        loss = torch.empty(1, dtype=torch.float32, device=logit.device)
        dz = torch.empty(max(n, 1), dtype=torch.float32, device=logit.device)
        self._raise(self._lib.velo_bce(self._h, C.c_void_p(logit.data_ptr()), C.c_void_p(y.data_ptr()),
                                       float(pos_weight), n, C.c_void_p(loss.data_ptr()), C.c_void_p(dz.data_ptr()),
                                       _stream()), "velo_bce")
        return loss, dz

    def focal(self, logit, y, alpha: float, gamma: float, n: int):
        """(loss [1], dlogit [n]) device tensors of the sigmoid focal loss on the first n logits."""
        import torch
        loss = torch.empty(1, dtype=torch.float32, device=logit.device)
        dz = torch.empty(max(n, 1), dtype=torch.float32, device=logit.device)
        self._raise(self._lib.velo_focal(self._h, C.c_void_p(logit.data_ptr()), C.c_void_p(y.data_ptr()),
                                         float(alpha), float(gamma), n, C.c_void_p(loss.data_ptr()),
                                         C.c_void_p(dz.data_ptr()), _stream()), "velo_focal")
        return loss, dz

    def train_backward(self, hits: DeviceHits, params, dlogit, dparams=None):
        import torch
        if dparams is None:
            dparams = torch.empty_like(params)
        hc = hits.c()
        self._raise(self._lib.velo_train_backward(self._h, C.byref(hc), C.c_void_p(params.data_ptr()),
                                                  C.c_void_p(dlogit.data_ptr()), C.c_void_p(dparams.data_ptr()),
                                                  _stream()), "velo_train_backward")
        return dparams

    def adam_step(self, params, grad, m, v, step: int, lr: float = 1e-3, b1: float = 0.9, b2: float = 0.999,
                  eps: float = 1e-8):
        self._raise(self._lib.velo_adam_step(self._h, C.c_void_p(params.data_ptr()), C.c_void_p(grad.data_ptr()),
                                             C.c_void_p(m.data_ptr()), C.c_void_p(v.data_ptr()), params.numel(),
                                             lr, b1, b2, eps, step, _stream()), "velo_adam_step")

    def embed_train_grad(self, hits: DeviceHits, pid, query, rnd, params, k_train: int = 50,
                         d2_train: float = 1.5, margin: float = 1.0, w_genuine: float = 2.0, dparams=None,
                         emb=None):
        """One embedding training step's loss and gradient (Sec. 5.1): returns
        (dparams, loss [3] = {L, genuine term, fake term}, counts [2] = {N_g, N_f});
        only the embedding entries of dparams are written.  pid int32, query
        uint8, rnd int32 (bits of a uint32 draw) device tensors over the hits."""
        import torch
        if dparams is None:
            dparams = torch.zeros_like(params)
        loss = torch.empty(3, dtype=torch.float32, device=params.device)
        counts = torch.empty(2, dtype=torch.int64, device=params.device)
        hc = hits.c()
        tr = _EmbedTruth(_ptr(pid), _ptr(query), _ptr(rnd))
        self._raise(self._lib.velo_embed_train_grad(self._h, C.byref(hc), C.byref(tr), _ptr(params), int(k_train),
                                                    float(d2_train), float(margin), float(w_genuine),
                                                    _ptr(dparams), _ptr(loss), _ptr(counts), _ptr(emb),
                                                    _stream()), "velo_embed_train_grad")
        return dparams, loss, counts


class Graph:
    """A captured velo_infer call; keeps its context and buffers alive."""

    def __init__(self, ctx: Context, handle, hits, out):
        self._ctx, self._g, self.hits, self.out = ctx, handle, hits, out

    def launch(self):
        self._ctx._raise(self._ctx._lib.velo_graph_launch(self._g, _stream()), "velo_graph_launch")

    def close(self):
        if getattr(self, "_g", None):
            self._ctx._lib.velo_graph_destroy(self._g)
            self._g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def components_noalloc(hits: DeviceHits, graph, edge_logit_min: float, max_event_hits: int) -> None:
    """velo_components_noalloc: components into graph["labels"] with no context
    and no device allocation (waits for the current stream; raises VeloError
    on a refused or invalid input)."""
    oc = Context._out_c(graph)
    hc = hits.c()
    st = lib().velo_components_noalloc(C.byref(hc), C.byref(oc), float(edge_logit_min), int(max_event_hits),
                                       _stream())
    if st != VELO_OK:
        raise VeloError(st, f"velo_components_noalloc: {lib().velo_status_str(st).decode()}")


def triplet_param_count(hidden: int) -> int:
    return int(lib().velo_triplet_param_count(hidden))


def triplets_to_host(t: Dict[str, object]) -> Dict[str, np.ndarray]:
    """Copy velo_triplets results to numpy (lists cut to their counts)."""
    na, ne = (int(v) for v in t["n_triplets"].cpu())
    nt = int(t["n_tracks"].cpu()[0])
    na, ne, nt = min(na, t["capacity"]), min(ne, t["capacity"]), min(nt, t["track_capacity"])
    E = t["edge_seg"].shape[0]
    if "graph_n_edges" in t:
        E = min(int(t["graph_n_edges"].cpu()[0]), E)
    return {"art": t["art"][:na].cpu().numpy(), "art_offsets": t["art_offsets"].cpu().numpy().astype(np.int64),
            "art_logit": t["art_logit"][:na].cpu().numpy(), "elb": t["elb"][:ne].cpu().numpy(),
            "elb_type": t["elb_type"][:ne].cpu().numpy(),
            "elb_offsets": t["elb_offsets"].cpu().numpy().astype(np.int64),
            "elb_logit": t["elb_logit"][:ne].cpu().numpy(), "edge_seg": t["edge_seg"][:E].cpu().numpy(),
            "tracks": t["tracks"][:nt].cpu().numpy(),
            "track_offsets": t["track_offsets"].cpu().numpy().astype(np.int64), "n_art": na, "n_elb": ne,
            "n_tracks": nt}


def graph_to_host(out: Dict[str, object], n_hits: Optional[int] = None) -> Dict[str, np.ndarray]:
    """Copy a result dictionary to numpy (edge arrays cut to n_edges)."""
    E = int(out["n_edges"].cpu()[0])
    E = min(E, int(out["edge_capacity"]))
    res = {"n_edges": E, "edge_offsets": out["edge_offsets"].cpu().numpy().astype(np.int64),
           "src": out["edge_src"][:E].cpu().numpy(), "dst": out["edge_dst"][:E].cpu().numpy(),
           "logit": out["edge_logit"][:E].cpu().numpy()}
    if n_hits is not None:
        res["labels"] = out["labels"][:n_hits].cpu().numpy()
    return res
