"""ctypes binding of libffbh (the C ABI in include/ffbh.h).

This module only marshals arguments: torch tensors supply device pointers and the current HIP stream,
and every step of the computation runs in the library's kernels.  If libffbh.so has not been built,
every entry point raises; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libffbh.so")
_lib = None

BH_OK, BH_EINVAL, BH_EWORKSPACE, BH_EDEVICE, BH_EDEGENERATE, BH_ESTATE = 0, -1, -2, -3, -4, -5
FLAG_NONFINITE, FLAG_COINCIDENT, FLAG_DEEP_LEAF, FLAG_STACK, FLAG_TREE, FLAG_OVERLAP = 1, 2, 4, 8, 16, 32
FP64, FP32_MIXED = 0, 1
PRECISIONS = {"fp64": FP64, "fp32_mixed": FP32_MIXED}


class bh_params(C.Structure):
    _fields_ = [("n", C.c_int64), ("batch", C.c_int32), ("leaf_size", C.c_int32),
                ("theta", C.c_double), ("precision", C.c_int32), ("tuning_id", C.c_int32),
                ("expansion", C.c_int32)]


class md_state(C.Structure):
    _fields_ = [("pos", C.c_void_p), ("vel", C.c_void_p), ("mom", C.c_void_p),
                ("omega", C.c_void_p), ("d_step", C.c_void_p)]


class md_params(C.Structure):
    _fields_ = [("dt", C.c_double), ("kT", C.c_double), ("gamma_t", C.c_double),
                ("gamma_r", C.c_double), ("mass", C.c_double), ("inertia", C.c_double),
                ("wca_eps", C.c_double), ("wca_sigma", C.c_double),
                ("box_lo", C.c_double * 3), ("box_hi", C.c_double * 3),
                ("d_hext", C.c_void_p), ("seed", C.c_uint64),
                ("sr_kind", C.c_int32), ("sr_cut", C.c_double)]


class BHError(RuntimeError):
    def __init__(self, fn: str, status: int):
        super().__init__(f"{fn}: {lib().bh_status_str(status).decode()} (status {status})")
        self.status = status


def lib():
    """Open libffbh.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first (__graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        P, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        L.bh_workspace_bytes.argtypes = [C.POINTER(bh_params), C.POINTER(C.c_size_t)]
        L.bh_num_tunings.restype = i32
        L.bh_create.argtypes = [C.POINTER(bh_params), P, C.c_size_t, C.POINTER(P)]
        L.bh_destroy.argtypes = [P]
        L.bh_handle_bytes.argtypes = []
        L.bh_handle_bytes.restype = C.c_size_t
        L.bh_init.argtypes = [P, C.c_size_t, C.POINTER(bh_params), P, C.c_size_t, P, C.POINTER(P)]
        L.bh_init.restype = i32
        L.bh_fini.argtypes = [P]
        L.bh_fini.restype = i32
        L.bh_build.argtypes = [P, P, P]
        L.bh_field.argtypes = [P, P, P, P, P, P]
        L.bh_field_backward.argtypes = [P, P, P, P, P, P, P, P, P]
        L.md_step.argtypes = [P, C.POINTER(md_state), C.POINTER(md_params), P]
        L.bh_check_status.argtypes = [P, P, C.POINTER(C.c_uint32)]
        L.bh_enable_counters.argtypes = [P, P, P]
        L.bh_num_nodes.argtypes = [P, P, C.POINTER(i64)]
        L.bh_export_tree.argtypes = [P] * 10
        L.bh_set_timing_events.argtypes = [P] * 5
        L.bh_set_timing_events.restype = i32
        L.bh_graph_capture_md.argtypes = [P, C.POINTER(md_state), C.POINTER(md_params), P, C.POINTER(P)]
        L.bh_graph_launch.argtypes = [P, P]
        L.bh_graph_destroy.argtypes = [P]
        for f in ("bh_graph_capture_md", "bh_graph_launch", "bh_graph_destroy"):
            getattr(L, f).restype = i32
        L.bh_morton_code.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32]
        L.bh_morton_code.restype = C.c_uint64
        L.bh_allpairs.argtypes = [i64, i32, i32, P, P, P, P, P, P, P]
        L.bh_allpairs.restype = i32
        L.bh_field_noalloc.argtypes = [C.POINTER(bh_params), P, P, P, P, P, P, P]
        L.bh_field_noalloc.restype = i32
        L.bh_status_str.argtypes = [i32]
        L.bh_status_str.restype = C.c_char_p
        for f in ("bh_workspace_bytes", "bh_create", "bh_destroy", "bh_build", "bh_field",
                  "bh_field_backward", "md_step", "bh_check_status", "bh_enable_counters",
                  "bh_num_nodes", "bh_export_tree"):
            getattr(L, f).restype = i32
        _lib = L
    return _lib


EXPORTED = ["bh_workspace_bytes", "bh_num_tunings", "bh_create", "bh_destroy", "bh_handle_bytes", "bh_init",
            "bh_fini", "bh_build", "bh_field",
            "bh_field_backward", "md_step", "bh_check_status", "bh_enable_counters", "bh_num_nodes",
            "bh_export_tree", "bh_set_timing_events", "bh_graph_capture_md", "bh_graph_launch",
            "bh_graph_destroy", "bh_allpairs", "bh_field_noalloc", "bh_morton_code", "bh_status_str"]


def _check(fn: str, st: int):
    if st != BH_OK:
        raise BHError(fn, st)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev64(t, shape=None, name="tensor"):
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float64 CUDA tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t


def make_params(n, batch=1, leaf_size=16, theta=0.5, precision="fp32_mixed", tuning_id=-1, expansion=1):
    """expansion 1: the paper's pseudo-particles; 2: plus each accepted cell's first moment (field only)."""
    return bh_params(int(n), int(batch), int(leaf_size), float(theta), PRECISIONS[precision],
                     int(tuning_id), int(expansion))


def workspace_bytes(params: bh_params) -> int:
    out = C.c_size_t(0)
    _check("bh_workspace_bytes", lib().bh_workspace_bytes(C.byref(params), C.byref(out)))
    return int(out.value)


class BarnesHut:
    """One handle: a batch of `batch` systems of `n` particles, fixed theta, leaf size, precision.

    Tensors are (batch, 3, n) float64 on the current CUDA (HIP) device; (3, n) is accepted for
    batch == 1 and results then come back as (3, n).
    """

    def __init__(self, n, batch=1, leaf_size=16, theta=0.5, precision="fp32_mixed", tuning_id=-1,
                 device=None, expansion=1, caller_memory=False):
        """caller_memory: the handle lives in host memory held here (bh_init) instead of the library's
        (bh_create); it then has no side stream."""
        self.params = make_params(n, batch, leaf_size, theta, precision, tuning_id, expansion)
        self.n, self.batch = int(n), int(batch)
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        nbytes = workspace_bytes(self.params)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        h = C.c_void_p()
        self._hmem = None
        with torch.cuda.device(self.device):
            if caller_memory:
                hb = int(lib().bh_handle_bytes())
                self._hmem = (C.c_char * (hb + 16))()
                addr = C.addressof(self._hmem)
                _check("bh_init", lib().bh_init(C.c_void_p(addr + (-addr) % 16), C.c_size_t(hb),
                                                C.byref(self.params), C.c_void_p(base + off), C.c_size_t(nbytes),
                                                _stream(), C.byref(h)))
            else:
                _check("bh_create", lib().bh_create(C.byref(self.params), C.c_void_p(base + off),
                                                    C.c_size_t(nbytes), C.byref(h)))
        self._h = h
        self._counters = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            if getattr(self, "_hmem", None) is not None:
                _lib.bh_fini(h)
            else:
                _lib.bh_destroy(h)
            self._h = None

    # -- shapes -----------------------------------------------------------------------------------
    def _as_batch(self, t, name):
        if t is None:
            return None, False
        if t.dim() == 2 and self.batch == 1:
            t = t.unsqueeze(0)
            squeeze = True
        else:
            squeeze = False
        return _dev64(t, (self.batch, 3, self.n), name), squeeze

    def _hext(self, hext):
        if hext is None:
            return None
        h = hext.reshape(self.batch, 3) if hext.numel() == 3 * self.batch else None
        if h is None and hext.numel() == 3:
            h = hext.reshape(1, 3).expand(self.batch, 3)
        return _dev64(h.contiguous(), (self.batch, 3), "hext")

    # -- entry points -----------------------------------------------------------------------------
    def build(self, pos):
        p, _ = self._as_batch(pos, "pos")
        _check("bh_build", lib().bh_build(self._h, _ptr(p), _stream()))
        self._pos = p  # keep alive until the stream has consumed it

    def field(self, mom, hext=None, energy=True):
        m, sq = self._as_batch(mom, "mom")
        he = self._hext(hext)
        H = torch.empty_like(m)
        E = torch.empty(self.batch, dtype=torch.float64, device=m.device) if energy else None
        _check("bh_field", lib().bh_field(self._h, _ptr(m), _ptr(he), _ptr(H), _ptr(E), _stream()))
        if sq:
            H = H[0]
        return (H, E) if energy else H

    def field_backward(self, mom, hext=None, gH=None, gE=None, want_dhext=False):
        m, sq = self._as_batch(mom, "mom")
        he = self._hext(hext)
        g, _ = self._as_batch(gH, "gH")
        ge = None if gE is None else _dev64(gE.reshape(self.batch).contiguous(), (self.batch,), "gE")
        dpos = torch.empty_like(m)
        dmom = torch.empty_like(m)
        dhext = torch.empty(self.batch, 3, dtype=torch.float64, device=m.device) if want_dhext else None
        _check("bh_field_backward", lib().bh_field_backward(
            self._h, _ptr(m), _ptr(he), _ptr(g), _ptr(ge), _ptr(dpos), _ptr(dmom), _ptr(dhext),
            _stream()))
        if sq:
            dpos, dmom = dpos[0], dmom[0]
        return (dpos, dmom, dhext) if want_dhext else (dpos, dmom)

    def enable_counters(self):
        """Record per-target far/near interaction counts on subsequent field calls."""
        nf = torch.zeros(self.batch, self.n, dtype=torch.int32, device=self.device)
        nr = torch.zeros(self.batch, self.n, dtype=torch.int32, device=self.device)
        _check("bh_enable_counters", lib().bh_enable_counters(self._h, _ptr(nf), _ptr(nr)))
        self._counters = (nf, nr)
        return self._counters

    def disable_counters(self):
        _check("bh_enable_counters", lib().bh_enable_counters(self._h, None, None))
        self._counters = None

    def set_raw_timing_events(self, events=None):
        """Record four raw hipEvent_t handles (forward start/stop, adjoint start/stop) around the
        traversal kernels; None disables."""
        ev = list(events) if events else [None] * 4
        self._events = events
        _check("bh_set_timing_events", lib().bh_set_timing_events(self._h, *ev))

    def check_status(self) -> int:
        """Device status flags since the last check (synchronises the stream)."""
        f = C.c_uint32(0)
        st = lib().bh_check_status(self._h, _stream(), C.byref(f))
        if st not in (BH_OK, BH_EDEGENERATE):
            raise BHError("bh_check_status", st)
        return int(f.value)

    def num_nodes(self) -> int:
        v = C.c_int64(0)
        _check("bh_num_nodes", lib().bh_num_nodes(self._h, _stream(), C.byref(v)))
        return int(v.value)

    def export_tree(self) -> dict:
        nn = self.num_nodes()
        dev = self.device
        i32 = dict(dtype=torch.int32, device=dev)
        out = dict(perm=torch.empty(self.batch * self.n, **i32), first=torch.empty(nn, **i32),
                   count=torch.empty(nn, **i32), level=torch.empty(nn, **i32),
                   nchild=torch.empty(nn, **i32), child=torch.empty(nn, **i32),
                   centroid=torch.empty(nn, 3, dtype=torch.float64, device=dev),
                   bbox=torch.empty(self.batch, 5, dtype=torch.float64, device=dev))
        _check("bh_export_tree", lib().bh_export_tree(
            self._h, _ptr(out["perm"]), _ptr(out["first"]), _ptr(out["count"]), _ptr(out["level"]),
            _ptr(out["nchild"]), _ptr(out["child"]), _ptr(out["centroid"]), _ptr(out["bbox"]),
            _stream()))
        torch.cuda.current_stream().synchronize()
        return {k: v.cpu().numpy() for k, v in out.items()}

    def _md_state(self, state):
        for k in ("pos", "vel", "mom", "omega"):
            self._as_batch(state[k], k)
        if not (state["step"].is_cuda and state["step"].dtype == torch.int64 and state["step"].numel() == 1):
            raise ValueError("step must be a one-element int64 CUDA tensor")
        return md_state(state["pos"].data_ptr(), state["vel"].data_ptr(), state["mom"].data_ptr(),
                        state["omega"].data_ptr(), state["step"].data_ptr())

    def capture_md_graph(self, state: dict, mdp: md_params, stream: "torch.cuda.Stream"):
        """Capture one md_step on `stream` (not the default stream) into a replayable graph."""
        st = self._md_state(state)
        g = C.c_void_p()
        _check("bh_graph_capture_md", lib().bh_graph_capture_md(self._h, C.byref(st), C.byref(mdp),
                                                                C.c_void_p(stream.cuda_stream), C.byref(g)))
        return MDGraph(g, self, state, mdp)

    def md_step(self, state: dict, mdp: md_params):
        """One MD step in place on state = {pos, vel, mom, omega: (B, 3, n) float64, step: int64[1]}."""
        for k in ("pos", "vel", "mom", "omega"):
            self._as_batch(state[k], k)
        if not (state["step"].is_cuda and state["step"].dtype == torch.int64 and state["step"].numel() == 1):
            raise ValueError("step must be a one-element int64 CUDA tensor")
        st = md_state(state["pos"].data_ptr(), state["vel"].data_ptr(), state["mom"].data_ptr(),
                      state["omega"].data_ptr(), state["step"].data_ptr())
        _check("md_step", lib().md_step(self._h, C.byref(st), C.byref(mdp), _stream()))


class MDGraph:
    """An instantiated HIP graph of one MD step; launch() replays it on a stream."""

    def __init__(self, g, owner, state, mdp):
        self._g = g
        self._keep = (owner, state, mdp)  # buffers the graph points into

    def launch(self, stream: "torch.cuda.Stream"):
        _check("bh_graph_launch", lib().bh_graph_launch(self._g, C.c_void_p(stream.cuda_stream)))

    def __del__(self):
        g = getattr(self, "_g", None)
        if g is not None and _lib is not None:
            _lib.bh_graph_destroy(g)
            self._g = None


def field_noalloc(pos, mom, hext=None, n=None, batch=1, leaf_size=16, theta=0.5, precision="fp32_mixed",
                  tuning_id=-1, expansion=1, out=None):
    """Build + field + energy through bh_field_noalloc (no handle, no workspace).

    pos, mom: (B, 3, n) or, for one system, (3, n) contiguous float64 CUDA tensors; hext (3,) or (B, 3)
    or None.  out: optional (H, E, flags) tensors to write into (H like pos, E (B,) float64, flags (1,)
    int32); fresh ones otherwise.  Returns (H, E, flags) with the batch dimension of the input."""
    squeeze = pos.dim() == 2
    P = pos.unsqueeze(0) if squeeze else pos
    M = mom.unsqueeze(0) if squeeze else mom
    B, _, nn = P.shape
    _dev64(P, (B, 3, nn), "pos")
    _dev64(M, (B, 3, nn), "mom")
    params = make_params(nn, B, leaf_size, theta, precision, tuning_id, expansion)
    he = None
    if hext is not None:
        h = hext.reshape(1, 3).expand(B, 3) if hext.numel() == 3 else hext.reshape(B, 3)
        he = _dev64(h.contiguous(), (B, 3), "hext")
    if out is None:
        H = torch.empty_like(P)
        E = torch.empty(B, dtype=torch.float64, device=P.device)
        F = torch.zeros(1, dtype=torch.int32, device=P.device)
    else:
        H, E, F = out
        H = H.unsqueeze(0) if H.dim() == 2 else H
        _dev64(H, (B, 3, nn), "H")
        _dev64(E, (B,), "E")
        if not (F.is_cuda and F.dtype == torch.int32 and F.numel() >= 1):
            raise ValueError("flags must be an int32 CUDA tensor")
    _check("bh_field_noalloc", lib().bh_field_noalloc(C.byref(params), _ptr(P), _ptr(M), _ptr(he), _ptr(H),
                                                      _ptr(E), _ptr(F), _stream()))
    return (H[0] if squeeze else H), E, F


def morton_code(qx: int, qy: int, qz: int) -> int:
    return int(lib().bh_morton_code(qx, qy, qz))


def allpairs(pos, mom, hext=None, precision="fp64", want_dEdr=False, want_E=False):
    """All-pairs field (and optionally energy gradient and energy) of one or a batch of systems.

    pos, mom: (3, n) or (B, 3, n) contiguous float64 CUDA tensors; hext: (3,) or (B, 3) or None.
    Returns (H, dEdr or None, E or None) with the batch dimension of the input."""
    squeeze = pos.dim() == 2
    P = pos.unsqueeze(0) if squeeze else pos
    M = mom.unsqueeze(0) if squeeze else mom
    B, _, n = P.shape
    _dev64(P, (B, 3, n), "pos")
    _dev64(M, (B, 3, n), "mom")
    he = None
    if hext is not None:
        he = _dev64(hext.reshape(B, 3).contiguous(), (B, 3), "hext")
    H = torch.empty_like(P)
    G = torch.empty_like(P) if want_dEdr else None
    E = torch.empty(B, dtype=torch.float64, device=P.device) if want_E else None
    _check("bh_allpairs", lib().bh_allpairs(int(n), int(B), PRECISIONS[precision], _ptr(P), _ptr(M), _ptr(he),
                                            _ptr(H), _ptr(G), _ptr(E), _stream()))
    if squeeze:
        H = H[0]
        G = None if G is None else G[0]
    return H, G, E
