"""Python binding of libhgnn (the C-ABI in include/hgnn.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  PyTorch supplies device memory and the stream.  Importing this
module loads the library and fails loudly if it has not been built.

Also defines one ``torch.autograd.Function`` per GC layer and one for the
pooling + head, each backed by the library's hand-written adjoint kernels.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhgnn.so")

OK, EINVAL, ENOMEM, EDEVICE, EAGAIN, ESTATE = 0, -1, -2, -3, -4, -5
VALIDATE = 1
PREC_FP32, PREC_BF16 = 0, 1


class HgnnError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"hgnn error {code}: {msg}")
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [("num_layers", ctypes.c_int32), ("hidden", ctypes.c_int32),
                ("node_feat", ctypes.c_int32), ("edge_feat", ctypes.c_int32),
                ("max_degree", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("recompute", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("delta", ctypes.c_double), ("std_eps", ctypes.c_double)]


class CBatch(ctypes.Structure):
    _fields_ = [("num_graphs", ctypes.c_int32), ("num_nodes", ctypes.c_int32),
                ("num_edges", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("graph_ptr", ctypes.c_void_p), ("x", ctypes.c_void_p),
                ("edge_index", ctypes.c_void_p), ("edge_attr", ctypes.c_void_p),
                ("y", ctypes.c_void_p)]


class ServeConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("max_batch_nodes", ctypes.c_int32),
                ("max_batch_edges", ctypes.c_int32), ("max_batch_graphs", ctypes.c_int32),
                ("num_lanes", ctypes.c_int32), ("queue_capacity", ctypes.c_int32),
                ("use_graphs", ctypes.c_int32)]


class Heads(ctypes.Structure):
    _fields_ = [("graph_heads", ctypes.c_int32), ("node_heads", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2), ("graph_weights", ctypes.c_void_p),
                ("node_weights", ctypes.c_void_p)]


class StoreInfo(ctypes.Structure):
    _fields_ = [("num_batches", ctypes.c_int32), ("node_feat", ctypes.c_int32),
                ("edge_feat", ctypes.c_int32), ("has_y", ctypes.c_int32),
                ("max_graphs", ctypes.c_int32), ("max_nodes", ctypes.c_int32),
                ("max_edges", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("max_record_bytes", ctypes.c_int64)]


class ServeStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("batches", ctypes.c_int64), ("graph_replays", ctypes.c_int64),
                ("admission_waits", ctypes.c_int64), ("peak_inflight_bytes", ctypes.c_int64),
                ("lanes", ctypes.c_int64), ("lane_bytes", ctypes.c_int64)]


_P = ctypes.c_void_p
_I = ctypes.c_int32
_SIGS = {
    "hgnn_create": ([ctypes.POINTER(Config), _P, ctypes.c_uint64, _P, ctypes.POINTER(_P)], _I),
    "hgnn_init_params": ([_P, ctypes.c_uint64, _P], _I),
    "hgnn_op_generation": ([_P, ctypes.POINTER(ctypes.c_int64)], _I),
    "hgnn_create_multitask": ([ctypes.POINTER(Config), ctypes.POINTER(Heads),
                               ctypes.POINTER(_P)], _I),
    "hgnn_forward_multitask": ([_P, ctypes.POINTER(CBatch), _P, _P, _P, _P, _I, _P], _I),
    "hgnn_create_gc": ([ctypes.POINTER(Config), _I, ctypes.POINTER(Heads),
                        ctypes.POINTER(_P)], _I),
    "hgnn_param_views": ([_P, ctypes.POINTER(_P), ctypes.POINTER(_P)], _I),
    "hgnn_debug_fail_after": ([_P, _I], _I),
    "hgnn_destroy": ([_P], None),
    "hgnn_num_params": ([_P, ctypes.POINTER(ctypes.c_int64)], _I),
    "hgnn_set_params": ([_P, _P, _P], _I),
    "hgnn_get_params": ([_P, _P, _P], _I),
    "hgnn_get_grads": ([_P, _P, _P], _I),
    "hgnn_check": ([_P, _P], _I),
    "hgnn_forward": ([_P, ctypes.POINTER(CBatch), _P, _P, _I, _P], _I),
    "hgnn_backward": ([_P, _P, _P], _I),
    "hgnn_adam_step": ([_P, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                        ctypes.c_float, _P], _I),
    "hgnn_get_state": ([_P, _P, ctypes.POINTER(ctypes.c_size_t)], _I),
    "hgnn_set_state": ([_P, _P, ctypes.c_size_t], _I),
    "hgnn_op_prepare": ([_P, ctypes.POINTER(CBatch), _I, _P], _I),
    "hgnn_op_layer_forward": ([_P, _I, _P, _P, _P, _P], _I),
    "hgnn_op_layer_backward": ([_P, ctypes.c_int64, _I, _P, _P, _P, _P, _P, _P, _P], _I),
    "hgnn_op_head_forward": ([_P, _P, _P, _P, _P, _P, _P], _I),
    "hgnn_op_head_backward": ([_P, ctypes.c_int64, _P, _P, _P, _P, _P, _P, _P], _I),
    "hgnn_op_fetch": ([_P, _I, _I, _P, ctypes.c_size_t, _P], _I),
    "hgnn_serve_start": ([_P, ctypes.POINTER(ServeConfig)], _I),
    "hgnn_serve_submit": ([_P, ctypes.POINTER(CBatch), ctypes.POINTER(ctypes.c_uint64)], _I),
    "hgnn_serve_poll": ([_P, ctypes.c_uint64, _P, ctypes.POINTER(_I)], _I),
    "hgnn_serve_stats_get": ([_P, ctypes.POINTER(ServeStats)], _I),
    "hgnn_serve_stop": ([_P], _I),
    "hgnn_timer_start": ([_P, _I, _I], _I),
    "hgnn_timer_read": ([_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I)], _I),
    "hgnn_calib_copy": ([_P, _P, ctypes.c_int64, _P], _I),
    "hgnn_forward_noalloc": ([_P, ctypes.POINTER(CBatch), _P, _P, _I, _P], _I),
    "hgnn_noalloc_bytes": ([_P, _I, _I, _I, ctypes.POINTER(ctypes.c_int64)], _I),
    "hgnn_noalloc_max_bytes": ([], ctypes.c_int64),
    "hgnn_last_error": ([], ctypes.c_char_p),
    "hgnn_store_open": ([ctypes.c_char_p, _I, _I, ctypes.POINTER(_P)], _I),
    "hgnn_store_info_get": ([_P, _P], _I),
    "hgnn_store_next": ([_P, _P, ctypes.POINTER(CBatch), ctypes.POINTER(ctypes.c_int64)], _I),
    "hgnn_store_close": ([_P], _I),
}


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with "
                          "`python -m paper_2207_11333_amd.build` (no CPU fallback exists)")
    lib = ctypes.CDLL(path)
    for name, (args, res) in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib: Optional[ctypes.CDLL] = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        _lib = load_library()
    return _lib


def _check(rc: int):
    if rc != OK:
        raise HgnnError(rc, lib().hgnn_last_error().decode())


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


# ---------------------------------------------------------------------------
# batches on the device
# ---------------------------------------------------------------------------

class DeviceBatch:
    """A packed batch in device memory (Table 1 layout) plus its C struct."""

    def __init__(self, graph_ptr, x, edge_index, edge_attr=None, y=None, device="cuda"):
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt).to(device)
        self.graph_ptr = t(graph_ptr, torch.int32)
        self.x = t(x, torch.float32)
        self.edge_index = t(edge_index, torch.int32).reshape(2, -1).contiguous()
        self.edge_attr = None if edge_attr is None else t(edge_attr, torch.float32)
        self.y = None if y is None else t(y, torch.float32)
        self.num_graphs = int(self.graph_ptr.shape[0] - 1)
        self.num_nodes = int(self.x.shape[0])
        self.num_edges = int(self.edge_index.shape[1])

    @classmethod
    def from_host(cls, b, device="cuda"):
        return cls(b.graph_ptr, b.x, b.edge_index, b.edge_attr, b.y, device)

    def cstruct(self, with_y: bool = True) -> CBatch:
        return CBatch(self.num_graphs, self.num_nodes, self.num_edges, 0,
                      self.graph_ptr.data_ptr(), self.x.data_ptr(),
                      self.edge_index.data_ptr() if self.num_edges else None,
                      None if self.edge_attr is None else self.edge_attr.data_ptr(),
                      None if (self.y is None or not with_y) else self.y.data_ptr())


class StoreBatch:
    """A batch handed out by GraphStore.next(): device pointers owned by the
    store, valid for work enqueued on the stream until the next call."""

    def __init__(self, cb: CBatch, index: int):
        self._cb = cb
        self.index = index
        self.num_graphs, self.num_nodes, self.num_edges = cb.num_graphs, cb.num_nodes, cb.num_edges

    def cstruct(self, with_y: bool = True) -> CBatch:
        if with_y:
            return self._cb
        cb = CBatch.from_buffer_copy(self._cb)
        cb.y = None
        return cb


class GraphStore:
    """Reader of a packed graph store file (see graphstore.py): io_threads
    host threads read records into pinned buffers; next() returns the next
    batch on the device, its copy overlapped with the caller's compute."""

    def __init__(self, path: str, io_threads: int = 4, host_slots: int = 4):
        h = ctypes.c_void_p()
        _check(lib().hgnn_store_open(path.encode(), io_threads, host_slots, ctypes.byref(h)))
        self.handle = h
        info = StoreInfo()
        _check(lib().hgnn_store_info_get(self.handle, ctypes.byref(info)))
        self.info = {k: int(getattr(info, k)) for k, _ in StoreInfo._fields_}

    def next(self) -> StoreBatch:
        cb = CBatch()
        idx = ctypes.c_int64()
        _check(lib().hgnn_store_next(self.handle, _stream(), ctypes.byref(cb), ctypes.byref(idx)))
        return StoreBatch(cb, int(idx.value))

    def close(self):
        if self.handle:
            _check(lib().hgnn_store_close(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def host_cbatch(b):
    """C struct over host numpy arrays (for hgnn_serve_submit); keeps refs."""
    keep = [np.ascontiguousarray(b.graph_ptr, np.int32), np.ascontiguousarray(b.x, np.float32),
            np.ascontiguousarray(b.edge_index, np.int32)]
    ea = None if b.edge_attr is None else np.ascontiguousarray(b.edge_attr, np.float32)
    keep.append(ea)
    cb = CBatch(b.num_graphs, b.num_nodes, b.num_edges, 0,
                keep[0].ctypes.data, keep[1].ctypes.data,
                keep[2].ctypes.data if b.num_edges else None,
                None if ea is None else ea.ctypes.data, None)
    return cb, keep


# ---------------------------------------------------------------------------
# the context
# ---------------------------------------------------------------------------

KINDS = {"pna": 0, "sage": 1, "cgcnn": 2}


class _DeviceView:
    """A float32 [n] device vector owned by a context, exposed to torch through
    the CUDA array interface (torch.as_tensor(view, device="cuda") aliases it)."""

    def __init__(self, ptr: int, n: int, owner):
        self._owner = owner
        self.__cuda_array_interface__ = {"shape": (n,), "typestr": "<f4", "data": (ptr, False),
                                         "version": 2, "strides": None}

    def tensor(self) -> torch.Tensor:
        return torch.as_tensor(self, device="cuda")


class Model:
    """Owns an hgnn context: weights, gradients, AdamW state, workspaces."""

    def __init__(self, num_layers: int, hidden: int, node_feat: int = 9, edge_feat: int = 1,
                 max_degree: int = 4, precision: int = PREC_FP32, recompute: int = 0,
                 delta: float = 1.0, std_eps: float = 1e-5, graph_heads: int = 1,
                 node_heads: int = 0, graph_weights=None, node_weights=None,
                 kind: str = "pna", init_params=None, seed: int = 0):
        """graph_heads / node_heads > 1 / > 0 build a multitask model (several
        graph-level heads, node-level heads, weighted loss); kind "sage" or
        "cgcnn" selects the GraphSAGE or CGCNN layer kind (see the header).
        A single-head PNA model starts from init_params (packed [P]) or, when
        it is None, from the library's seeded initialisation (seed); the
        other kinds start at zero until set_params or init_params."""
        if kind not in KINDS:
            raise ValueError(f"kind must be one of {sorted(KINDS)}")
        self.kind = kind
        self.cfg = Config(num_layers, hidden, node_feat, edge_feat, max_degree, precision,
                          recompute, 0, delta, std_eps)
        h = ctypes.c_void_p()
        self.Tg, self.Tn = graph_heads, node_heads
        if kind != "pna":
            gw = None if graph_weights is None else np.asarray(graph_weights, np.float32)
            nw = None if node_weights is None else np.asarray(node_weights, np.float32)
            hd = Heads(graph_heads, node_heads, (ctypes.c_int32 * 2)(0, 0),
                       None if gw is None else gw.ctypes.data,
                       None if nw is None else nw.ctypes.data)
            _check(lib().hgnn_create_gc(ctypes.byref(self.cfg), KINDS[kind], ctypes.byref(hd),
                                        ctypes.byref(h)))
        elif graph_heads == 1 and node_heads == 0 and graph_weights is None:
            init = None
            if init_params is not None:
                init = torch.as_tensor(init_params, dtype=torch.float32).cuda().contiguous()
            _check(lib().hgnn_create(ctypes.byref(self.cfg), _ptr(init), seed, _stream(),
                                     ctypes.byref(h)))
            torch.cuda.current_stream().synchronize()
        else:
            gw = None if graph_weights is None else np.asarray(graph_weights, np.float32)
            nw = None if node_weights is None else np.asarray(node_weights, np.float32)
            hd = Heads(graph_heads, node_heads, (ctypes.c_int32 * 2)(0, 0),
                       None if gw is None else gw.ctypes.data,
                       None if nw is None else nw.ctypes.data)
            _check(lib().hgnn_create_multitask(ctypes.byref(self.cfg), ctypes.byref(hd),
                                               ctypes.byref(h)))
        self.handle = h
        n = ctypes.c_int64()
        _check(lib().hgnn_num_params(self.handle, ctypes.byref(n)))
        self.num_params = int(n.value)
        self.L, self.H, self.F0, self.Fe = num_layers, hidden, node_feat, edge_feat
        self._batch_keep = None

    # layout of the packed vector of a PNA model (mirrors the header's packing order)
    def layer_slices(self) -> List[slice]:
        out, off = [], 0
        H, Fe = self.H, self.Fe
        for l in range(self.L):
            F = self.F0 if l == 0 else H
            n = H * (2 * F + Fe) + H + H * (F + 12 * H) + H
            out.append(slice(off, off + n))
            off += n
        out.append(slice(off, off + H * H + 2 * H + 1))
        return out

    def close(self):
        if getattr(self, "handle", None):
            lib().hgnn_serve_stop(self.handle)
            lib().hgnn_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        if isinstance(params, _DeviceView):
            params = params.tensor()
        p = torch.as_tensor(params, dtype=torch.float32).cuda().contiguous()
        assert p.numel() == self.num_params
        _check(lib().hgnn_set_params(self.handle, _ptr(p), _stream()))
        torch.cuda.current_stream().synchronize()

    def params(self) -> torch.Tensor:
        out = torch.empty(self.num_params, dtype=torch.float32, device="cuda")
        _check(lib().hgnn_get_params(self.handle, _ptr(out), _stream()))
        return out

    def grads(self) -> torch.Tensor:
        out = torch.empty(self.num_params, dtype=torch.float32, device="cuda")
        _check(lib().hgnn_get_grads(self.handle, _ptr(out), _stream()))
        return out

    def param_views(self):
        """(params, grads): torch views of the context's own [P] vectors (no
        copy).  Writes to params reach the layers after set_params(params)."""
        p, g = _P(), _P()
        _check(lib().hgnn_param_views(self.handle, ctypes.byref(p), ctypes.byref(g)))
        return _DeviceView(p.value, self.num_params, self), _DeviceView(g.value, self.num_params, self)

    def init_params(self, seed: int):
        """The library's seeded initialisation (Xavier-uniform weights, U(+-0.1)
        biases from a SplitMix64 counter generator)."""
        _check(lib().hgnn_init_params(self.handle, seed, _stream()))
        torch.cuda.current_stream().synchronize()

    def generation(self) -> int:
        """Count of batches prepared so far (each forward prepares one)."""
        g = ctypes.c_int64()
        _check(lib().hgnn_op_generation(self.handle, ctypes.byref(g)))
        return int(g.value)

    def debug_fail_after(self, n: int):
        """Test hook: the n-th layer call from now fails as a launch would."""
        _check(lib().hgnn_debug_fail_after(self.handle, n))

    def check(self):
        _check(lib().hgnn_check(self.handle, _stream()))

    def forward(self, batch: DeviceBatch, pred: torch.Tensor, loss: Optional[torch.Tensor] = None,
                validate: bool = False, y_node: Optional[torch.Tensor] = None,
                pred_node: Optional[torch.Tensor] = None):
        """pred [B] (or [B, graph_heads]); a multitask model also takes the node
        targets y_node [N, node_heads] (kept until backward) and pred_node."""
        cb = batch.cstruct()
        self._batch_keep = batch
        self._ynode_keep = y_node
        flags = VALIDATE if validate else 0
        if self.Tn == 0 and y_node is None and pred_node is None:
            _check(lib().hgnn_forward(self.handle, ctypes.byref(cb), _ptr(pred), _ptr(loss),
                                      flags, _stream()))
        else:
            _check(lib().hgnn_forward_multitask(self.handle, ctypes.byref(cb), _ptr(y_node),
                                                _ptr(pred), _ptr(pred_node), _ptr(loss), flags,
                                                _stream()))

    def forward_noalloc(self, batch: DeviceBatch, pred: torch.Tensor,
                        loss: Optional[torch.Tensor] = None, validate: bool = False):
        """Inference forward whose workspace is the library's static device
        array (no allocation); leaves the training state alone."""
        cb = batch.cstruct()
        _check(lib().hgnn_forward_noalloc(self.handle, ctypes.byref(cb), _ptr(pred), _ptr(loss),
                                          VALIDATE if validate else 0, _stream()))

    def noalloc_bytes(self, num_graphs: int, num_nodes: int, num_edges: int) -> int:
        n = ctypes.c_int64()
        _check(lib().hgnn_noalloc_bytes(self.handle, num_graphs, num_nodes, num_edges,
                                        ctypes.byref(n)))
        return int(n.value)

    def backward(self, dpred: Optional[torch.Tensor] = None):
        _check(lib().hgnn_backward(self.handle, _ptr(dpred), _stream()))

    def adam_step(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
        _check(lib().hgnn_adam_step(self.handle, lr, beta1, beta2, eps, weight_decay, _stream()))

    def get_state(self) -> bytes:
        n = ctypes.c_size_t()
        _check(lib().hgnn_get_state(self.handle, None, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        _check(lib().hgnn_get_state(self.handle, buf, ctypes.byref(n)))
        return buf.raw

    def set_state(self, state: bytes):
        buf = ctypes.create_string_buffer(state, len(state))
        _check(lib().hgnn_set_state(self.handle, buf, len(state)))

    # -- per-op entries --
    def prepare(self, batch: DeviceBatch, validate: bool = False):
        cb = batch.cstruct()
        self._batch_keep = batch
        _check(lib().hgnn_op_prepare(self.handle, ctypes.byref(cb),
                                     VALIDATE if validate else 0, _stream()))

    def fetch(self, which: int, layer: int = 0, shape=None, dtype=torch.int32) -> torch.Tensor:
        out = torch.empty(shape, dtype=dtype, device="cuda")
        _check(lib().hgnn_op_fetch(self.handle, which, layer, _ptr(out),
                                   out.numel() * out.element_size(), _stream()))
        return out

    # -- measurement --
    SITES = {"message_gemm": 1, "aggregate": 2, "update_gemm": 3, "update_wgrad": 4,
             "agg_input_gemm": 5, "aggregate_bwd": 6, "input_gemm": 7, "message_wgrad": 8,
             "csr": 9}

    def timer_start(self, site: str, max_launches: int = 4096):
        _check(lib().hgnn_timer_start(self.handle, self.SITES[site], max_launches))

    def timer_read(self):
        ms = ctypes.c_double()
        n = ctypes.c_int32()
        _check(lib().hgnn_timer_read(self.handle, ctypes.byref(ms), ctypes.byref(n)))
        return float(ms.value), int(n.value)

    # -- serving --
    def serve_start(self, hbm_budget_bytes=16 << 30, max_batch_nodes=32768,
                    max_batch_edges=73728, max_batch_graphs=1024, num_lanes=2,
                    queue_capacity=4096, use_graphs=1):
        sc = ServeConfig(hbm_budget_bytes, max_batch_nodes, max_batch_edges, max_batch_graphs,
                         num_lanes, queue_capacity, use_graphs)
        _check(lib().hgnn_serve_start(self.handle, ctypes.byref(sc)))

    def serve_submit(self, b) -> int:
        cb, keep = host_cbatch(b)
        t = ctypes.c_uint64()
        rc = lib().hgnn_serve_submit(self.handle, ctypes.byref(cb), ctypes.byref(t))
        if rc == EAGAIN:
            return -1
        _check(rc)
        return int(t.value)

    def serve_poll(self, ticket: int, num_graphs: int):
        out = np.empty(num_graphs, np.float32)
        done = ctypes.c_int32()
        _check(lib().hgnn_serve_poll(self.handle, ticket, out.ctypes.data, ctypes.byref(done)))
        return out if done.value else None

    def serve_stats(self) -> dict:
        st = ServeStats()
        _check(lib().hgnn_serve_stats_get(self.handle, ctypes.byref(st)))
        return {k: int(getattr(st, k)) for k, _ in ServeStats._fields_}

    def serve_stop(self):
        _check(lib().hgnn_serve_stop(self.handle))


# ---------------------------------------------------------------------------
# autograd: one Function per GC layer, one for pooling + head
# ---------------------------------------------------------------------------

def calib_copy(src: torch.Tensor, dst: torch.Tensor):
    """Plain float4 copy kernel (known traffic) for counter calibration."""
    _check(lib().hgnn_calib_copy(_ptr(src), _ptr(dst), src.numel(), _stream()))


class PNALayerFunction(torch.autograd.Function):
    """h_out = PNA layer l (message, aggregation, scalers, update, ReLU)."""

    @staticmethod
    def forward(ctx, h_in, w_layer, model: Model, layer: int):
        h_in = h_in.contiguous()
        w_layer = w_layer.contiguous()
        h_out = torch.empty(h_in.shape[0], model.H, dtype=torch.float32, device=h_in.device)
        _check(lib().hgnn_op_layer_forward(model.handle, layer, _ptr(w_layer), _ptr(h_in),
                                           _ptr(h_out), _stream()))
        ctx.save_for_backward(h_in, w_layer, h_out)
        ctx.model, ctx.layer = model, layer
        # the context's stored messages, aggregates and CSR belong to this
        # batch; the library refuses the backward once another is prepared
        ctx.generation = model.generation()
        return h_out

    @staticmethod
    def backward(ctx, dh_out):
        h_in, w_layer, h_out = ctx.saved_tensors
        model = ctx.model
        dh_out = dh_out.contiguous()
        dh_in = torch.empty_like(h_in) if ctx.needs_input_grad[0] else None
        dw = torch.empty_like(w_layer)
        _check(lib().hgnn_op_layer_backward(model.handle, ctx.generation, ctx.layer,
                                            _ptr(w_layer), _ptr(h_in), _ptr(h_out),
                                            _ptr(dh_out), _ptr(dh_in), _ptr(dw), _stream()))
        return dh_in, dw, None, None


class PoolHeadFunction(torch.autograd.Function):
    """y = w2 ReLU(W1 mean_pool(h) + b1) + b2 per graph."""

    @staticmethod
    def forward(ctx, h, w_head, model: Model):
        h = h.contiguous()
        w_head = w_head.contiguous()
        pred = torch.empty(model._batch_keep.num_graphs, dtype=torch.float32, device=h.device)
        _check(lib().hgnn_op_head_forward(model.handle, _ptr(w_head), _ptr(h), None,
                                          _ptr(pred), None, _stream()))
        ctx.save_for_backward(h, w_head)
        ctx.model = model
        ctx.generation = model.generation()
        return pred

    @staticmethod
    def backward(ctx, dpred):
        h, w_head = ctx.saved_tensors
        dpred = dpred.contiguous()
        dh = torch.empty_like(h)
        dw = torch.empty_like(w_head)
        _check(lib().hgnn_op_head_backward(ctx.model.handle, ctx.generation, _ptr(w_head),
                                           _ptr(h), None, _ptr(dpred), _ptr(dh), _ptr(dw),
                                           _stream()))
        return dh, dw, None


class PNANet(torch.nn.Module):
    """GC stack + mean pooling + MLP head as autograd-visible parameters."""

    def __init__(self, model: Model, params):
        super().__init__()
        self.model = model
        p = torch.as_tensor(params, dtype=torch.float32).cuda()
        sl = model.layer_slices()
        self.layers = torch.nn.ParameterList(
            [torch.nn.Parameter(p[s].clone()) for s in sl[:-1]])
        self.head = torch.nn.Parameter(p[sl[-1]].clone())

    def packed_grad(self) -> torch.Tensor:
        return torch.cat([w.grad for w in self.layers] + [self.head.grad])

    def forward(self, batch: DeviceBatch, x: Optional[torch.Tensor] = None):
        self.model.prepare(batch)
        h = batch.x if x is None else x
        for l, w in enumerate(self.layers):
            h = PNALayerFunction.apply(h, w, self.model, l)
        return PoolHeadFunction.apply(h, self.head, self.model)


class ModelFunction(torch.autograd.Function):
    """pred = the whole model (any layer kind, one graph head) as a function of
    its packed parameter vector: the forward loads the parameters and runs
    hgnn_forward, the backward runs hgnn_backward with dpred and returns the
    packed gradient.  Lets torch optimisers drive GraphSAGE / CGCNN / PNA
    models through one parameter tensor."""

    @staticmethod
    def forward(ctx, params, model: Model, batch: DeviceBatch):
        if model.Tg != 1 or model.Tn != 0:
            raise ValueError("ModelFunction takes a model with one graph head and no node head")
        params = params.detach().contiguous()
        model.set_params(params)
        pred = torch.empty(batch.num_graphs, dtype=torch.float32, device=params.device)
        model.forward(batch, pred)
        ctx.model = model
        ctx.generation = model.generation()
        ctx.params = params
        return pred

    @staticmethod
    def backward(ctx, dpred):
        model = ctx.model
        # hgnn_backward differentiates the context's last forward
        if model.generation() != ctx.generation:
            raise HgnnError(EINVAL, "another forward ran on this model since this one: "
                                    "run the forward again before its backward")
        model.backward(dpred.contiguous())
        return model.grads(), None, None


class GCNet(torch.nn.Module):
    """One packed parameter tensor and the whole model of any layer kind
    (forward and backward through the library's fused entry points)."""

    def __init__(self, model: Model, params):
        super().__init__()
        self.model = model
        self.params = torch.nn.Parameter(torch.as_tensor(params, dtype=torch.float32).cuda().clone())

    def forward(self, batch: DeviceBatch):
        return ModelFunction.apply(self.params, self.model, batch)
