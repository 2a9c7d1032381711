"""Python binding of libgsim (ctypes): argument marshalling only.

Every step of the simulation runs in the HIP kernels of ``libgsim.so``; this
module packs model descriptions, passes device pointers of torch tensors and the
current HIP stream, and turns status codes into exceptions.  Names follow the
C-ABI in ``include/gsim.h`` (``gsim_plan_create`` -> :class:`Plan`,
``gsim_rollout`` -> :meth:`Model.rollout`, ...).

Layouts: device states are SoA ``[3, n_particles]`` tensors; the helpers
:func:`soa` / :func:`aos` convert from / to numpy ``[n, 3]`` arrays.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
# GSIM_LIB selects another build of the same library (the sanitizer build of the host
# runtime, for instance); by default the in-tree libgsim.so.
LIB_PATH = os.environ.get("GSIM_LIB") or os.path.join(HERE, "libgsim.so")

GSIM_OK, GSIM_E_INVALID, GSIM_E_TOPOLOGY, GSIM_E_DEGENERATE = 0, -1, -2, -3
GSIM_E_WORKSPACE, GSIM_E_HIP, GSIM_E_NONFINITE, GSIM_E_UNSUPPORTED = -4, -5, -6, -7
EXEC_PLAIN, EXEC_GRAPH, EXEC_FUSED, EXEC_PERSIST = 0, 1, 2, 3
FLAG_NONFINITE, FLAG_INVERTED = 1, 2
TILE_DEFAULT = 256

ABI_SYMBOLS = ("gsim_last_error", "gsim_version", "gsim_plan_create", "gsim_plan_destroy", "gsim_plan_sizes",
               "gsim_plan_counts", "gsim_plan_colouring", "gsim_plan_tiles", "gsim_plan_codes", "gsim_plan_partials",
               "gsim_model_init", "gsim_model_destroy", "gsim_model_set_exec", "gsim_model_get_exec",
               "gsim_model_set_launch", "gsim_model_get_launch", "gsim_model_set_lanes", "gsim_model_get_lanes",
               "gsim_model_set_overlap",
               "gsim_step", "gsim_step_backward", "gsim_rollout", "gsim_rollout_backward",
               "gsim_loss_mse", "gsim_model_set_timing", "gsim_model_read_timing", "gsim_model_check",
               "gsim_controller_forward", "gsim_controller_backward",
               "gsim_rigid_sizes", "gsim_rigid_init", "gsim_rigid_destroy", "gsim_rigid_rollout", "gsim_rigid_loss",
               "gsim_rigid_rollout_backward",
               "gsim_raster_sizes", "gsim_raster_init", "gsim_raster_destroy", "gsim_raster_forward",
               "gsim_raster_forward_noalloc",
               "gsim_raster_backward",
               "gsim_engine_create", "gsim_engine_destroy", "gsim_engine_query_bytes", "gsim_engine_submit",
               "gsim_engine_tick", "gsim_engine_poll", "gsim_engine_stats", "gsim_engine_set_micro_steps",
               "gsim_engine_set_store_limit", "gsim_engine_prepare", "gsim_engine_submit_prepared",
               "gsim_prepared_destroy")
GSIM_F32, GSIM_F64 = 32, 64
KERNELS = ("element_fwd", "particle_fwd", "element_adj", "particle_adj", "fused_fwd", "fused_adj", "element_dual",
           "particle_dual")


class GsimError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("gsim error %d: %s" % (code, msg))
        self.code = code


class _Desc(C.Structure):
    _fields_ = [("dtype", C.c_int), ("n_bodies", C.c_int),
                ("n_particles", C.c_int64), ("n_tets", C.c_int64), ("n_tris", C.c_int64), ("n_hinges", C.c_int64),
                ("body_particle_off", C.c_void_p), ("body_tet_off", C.c_void_p), ("body_tri_off", C.c_void_p),
                ("body_hinge_off", C.c_void_p), ("rest_x", C.c_void_p), ("tet_idx", C.c_void_p),
                ("tri_idx", C.c_void_p), ("hinge_idx", C.c_void_p), ("pinned", C.c_void_p),
                ("gravity", C.c_void_p), ("dt", C.c_void_p), ("ground", C.c_void_p), ("contact_on", C.c_void_p),
                ("k_bend", C.c_void_p), ("air_on", C.c_void_p), ("tile_elems", C.c_int)]


class _State(C.Structure):
    _fields_ = [("x", C.c_void_p), ("v", C.c_void_p)]


class _Params(C.Structure):
    _fields_ = [("mu", C.c_void_p), ("lam", C.c_void_p), ("act", C.c_void_p), ("k_tri", C.c_void_p),
                ("mass", C.c_void_p), ("contact", C.c_void_p), ("hact", C.c_void_p), ("act_stride", C.c_int64),
                ("hact_stride", C.c_int64), ("air", C.c_void_p)]


class _RigidDesc(C.Structure):
    _fields_ = [("dtype", C.c_int), ("n_bodies", C.c_int), ("vert_off", C.c_void_p), ("verts", C.c_void_p),
                ("gravity", C.c_void_p), ("dt", C.c_void_p), ("ground", C.c_void_p), ("contact_on", C.c_void_p)]


class _RigidParams(C.Structure):
    _fields_ = [("mass", C.c_void_p), ("inertia", C.c_void_p), ("contact", C.c_void_p)]


class _RigidGrads(C.Structure):
    _fields_ = [("mass", C.c_void_p), ("inertia", C.c_void_p), ("contact", C.c_void_p)]


class _Camera(C.Structure):
    _fields_ = [("P", C.c_double * 12), ("sigma", C.c_double)]


class _Ctrl(C.Structure):
    _fields_ = [("n_signals", C.c_int), ("omega", C.c_double), ("dt", C.c_double), ("scale", C.c_double)]


class _Grads(C.Structure):
    _fields_ = [("mu", C.c_void_p), ("lam", C.c_void_p), ("k_tri", C.c_void_p), ("mass", C.c_void_p),
                ("contact", C.c_void_p), ("act", C.c_void_p), ("hact", C.c_void_p), ("act_stride", C.c_int64),
                ("hact_stride", C.c_int64)]


_lib = None


def load():
    """Loads libgsim.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libgsim.so is not built: run `python -m paper_2104_02646_amd.build`")
        lib = C.CDLL(LIB_PATH)
        lib.gsim_last_error.restype = C.c_char_p
        vp, ip = C.c_void_p, C.c_int
        lib.gsim_plan_create.argtypes = [C.POINTER(_Desc), C.POINTER(vp)]
        lib.gsim_plan_destroy.argtypes = [vp]
        lib.gsim_plan_sizes.argtypes = [vp, ip, ip, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]
        lib.gsim_plan_counts.argtypes = [vp] + [C.POINTER(C.c_int64)] * 4 + [C.POINTER(C.c_int)]
        lib.gsim_plan_colouring.argtypes = [vp, ip, vp, vp, ip, C.POINTER(ip)]
        lib.gsim_plan_tiles.argtypes = [vp, vp, C.POINTER(C.c_int64), vp, vp, vp, C.POINTER(C.c_int64)]
        lib.gsim_plan_codes.argtypes = [vp, ip, vp]
        lib.gsim_plan_partials.argtypes = [vp, vp, C.POINTER(C.c_int64), vp, C.POINTER(C.c_int64)]
        lib.gsim_model_init.argtypes = [vp, ip, ip, vp, C.c_size_t, vp, C.POINTER(vp)]
        lib.gsim_model_destroy.argtypes = [vp]
        lib.gsim_model_check.argtypes = [vp, vp, ip, vp]
        lib.gsim_model_set_exec.argtypes = [vp, ip, ip, ip]
        lib.gsim_model_get_exec.argtypes = [vp, C.POINTER(ip), C.POINTER(ip), C.POINTER(ip)]
        lib.gsim_model_set_launch.argtypes = [vp, ip, ip, ip]
        lib.gsim_model_get_launch.argtypes = [vp, ip, C.POINTER(ip), C.POINTER(ip)]
        lib.gsim_model_set_lanes.argtypes = [vp, ip]
        lib.gsim_model_get_lanes.argtypes = [vp, C.POINTER(ip)]
        lib.gsim_model_set_overlap.argtypes = [vp, vp, C.c_size_t]
        lib.gsim_step.argtypes = [vp, C.POINTER(_Params), _State, _State, ip, vp]
        lib.gsim_step_backward.argtypes = [vp, C.POINTER(_Params), _State, _State, _State, C.POINTER(_Grads), vp]
        lib.gsim_rollout.argtypes = [vp, C.POINTER(_Params), _State, ip, vp, _State, vp]
        lib.gsim_rollout_backward.argtypes = [vp, C.POINTER(_Params), vp, ip, vp, _State, _State, C.POINTER(_Grads), vp]
        lib.gsim_loss_mse.argtypes = [vp, _State, vp, vp, _State, vp]
        lib.gsim_model_set_timing.argtypes = [vp, ip]
        lib.gsim_model_read_timing.argtypes = [vp, ip, C.POINTER(C.c_int64), C.POINTER(C.c_double)]
        i64 = C.c_int64
        lib.gsim_controller_forward.argtypes = [ip, C.POINTER(_Ctrl), vp, i64, i64, i64, vp, vp]
        lib.gsim_controller_backward.argtypes = [ip, C.POINTER(_Ctrl), vp, vp, i64, i64, i64, vp, vp]
        RP, RG = C.POINTER(_RigidParams), C.POINTER(_RigidGrads)
        lib.gsim_rigid_sizes.argtypes = [C.POINTER(_RigidDesc), C.POINTER(C.c_size_t)]
        lib.gsim_rigid_init.argtypes = [C.POINTER(_RigidDesc), vp, C.c_size_t, vp, C.POINTER(vp)]
        lib.gsim_rigid_destroy.argtypes = [vp]
        lib.gsim_rigid_rollout.argtypes = [vp, RP, vp, ip, vp, vp]
        lib.gsim_rigid_loss.argtypes = [vp, vp, vp, vp, vp, vp]
        lib.gsim_rigid_rollout_backward.argtypes = [vp, RP, vp, ip, vp, vp, RG, vp]
        CP = C.POINTER(_Camera)
        lib.gsim_raster_sizes.argtypes = [ip, i64, i64, ip, ip, C.POINTER(C.c_size_t)]
        lib.gsim_raster_init.argtypes = [ip, i64, i64, vp, ip, ip, vp, C.c_size_t, vp, C.POINTER(vp)]
        lib.gsim_raster_destroy.argtypes = [vp]
        lib.gsim_raster_forward.argtypes = [vp, CP, vp, vp, vp]
        lib.gsim_raster_forward_noalloc.argtypes = [ip, C.c_int64, C.c_int64, vp, ip, ip, CP, vp, vp, vp]
        lib.gsim_raster_backward.argtypes = [vp, CP, vp, vp, vp, vp]
        _lib = lib
    return _lib


def _check(rc):
    if rc != GSIM_OK:
        raise GsimError(rc, load().gsim_last_error().decode())


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _device(device):
    d = torch.device(device)
    if d.type == "cuda" and d.index is None:
        d = torch.device("cuda", torch.cuda.current_device())
    return d


def _arg(t, name, dtype, device, numel, shape=None):
    """Device pointer of a caller tensor after checking what the library will assume of
    it: the model's dtype and device, contiguous storage, and at least ``numel``
    elements (exactly ``shape`` when given).  The library reads and writes through raw
    pointers, so a tensor of another dtype or size would be read past its end."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch.Tensor, got {type(t).__name__}")
    if t.dtype != dtype:
        raise TypeError(f"{name}: dtype {t.dtype}, the model computes in {dtype}")
    if t.device != device:
        raise ValueError(f"{name}: on {t.device}, the model is on {device}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: shape {tuple(t.shape)}, expected {tuple(shape)}")
    if t.numel() < numel:
        raise ValueError(f"{name}: {t.numel()} elements, at least {numel} needed")
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def soa(a, dtype=torch.float32, device="cuda"):
    """numpy [n, 3] -> device SoA tensor [3, n]."""
    return torch.as_tensor(np.ascontiguousarray(np.asarray(a, np.float64).T)).to(device=device, dtype=dtype).contiguous()


def aos(t):
    """device SoA tensor [3, n] -> numpy float64 [n, 3]."""
    return t.detach().double().cpu().numpy().T.copy()


# ----------------------------------------------------------------------------------
# Plan / Model
# ----------------------------------------------------------------------------------

# ----------------------------------------------------------------------------------
# Open-loop actuation controller (gsim_controller_*)
# ----------------------------------------------------------------------------------

def _ctrl_args(W, omega, dt, scale):
    if W.dim() != 2 or not W.is_contiguous() or W.dtype not in (torch.float32, torch.float64):
        raise ValueError("W must be a contiguous float32/float64 [n_signals, n] tensor")
    c = _Ctrl()
    c.n_signals, c.omega, c.dt, c.scale = W.shape[0], float(omega), float(dt), float(scale)
    return c, (GSIM_F32 if W.dtype == torch.float32 else GSIM_F64)


def controller_forward(W, omega, dt, n_steps, t0=0, scale=1.0, out=None, stream=None):
    """act[n_steps, n] = scale tanh(S W) for steps t0.. (rows feed the per-step
    actuation of a rollout)."""
    c, dt_code = _ctrl_args(W, omega, dt, scale)
    n = W.shape[1]
    act = torch.empty(int(n_steps), n, dtype=W.dtype, device=W.device) if out is None else out
    if act.shape != (int(n_steps), n) or act.dtype != W.dtype or not act.is_contiguous() or act.device != W.device:
        raise ValueError("out must be a contiguous [n_steps, n] tensor of W's dtype on W's device")
    _check(load().gsim_controller_forward(dt_code, C.byref(c), _ptr(W), n, int(t0), int(n_steps), _ptr(act),
                                          _stream(stream)))
    return act


def controller_backward(W, act_grad, omega, dt, t0=0, scale=1.0, W_grad=None, stream=None):
    """W_grad[n_signals, n] += d<act_grad, act>/dW (a new zeroed tensor if None)."""
    c, dt_code = _ctrl_args(W, omega, dt, scale)
    n = W.shape[1]
    if (act_grad.dim() != 2 or act_grad.shape[1] != n or act_grad.dtype != W.dtype or not act_grad.is_contiguous()
            or act_grad.device != W.device):
        raise ValueError("act_grad must be a contiguous [n_steps, n] tensor of W's dtype on W's device")
    gW = torch.zeros_like(W) if W_grad is None else W_grad
    if gW.shape != W.shape or gW.dtype != W.dtype or not gW.is_contiguous() or gW.device != W.device:
        raise ValueError("W_grad must be a contiguous tensor shaped like W, on W's device")
    _check(load().gsim_controller_backward(dt_code, C.byref(c), _ptr(W), _ptr(act_grad), n, int(t0),
                                           act_grad.shape[0], _ptr(gW), _stream(stream)))
    return gW


@dataclass
class Packed:
    """Host arrays of a packed multi-body description."""
    n_bodies: int
    poff: np.ndarray
    eoff: np.ndarray
    toff: np.ndarray
    hoff: np.ndarray
    X: np.ndarray
    tets: np.ndarray
    tris: np.ndarray
    hinges: np.ndarray
    pinned: np.ndarray
    gravity: np.ndarray
    dt: np.ndarray
    ground: np.ndarray
    contact_on: np.ndarray
    k_bend: np.ndarray
    air_on: np.ndarray


def pack(bodies) -> Packed:
    """Concatenates bodies (``workloads.Body``-like objects) into one model description;
    element indices become model-global."""
    poff = np.zeros(len(bodies) + 1, np.int64)
    eoff, toff, hoff = poff.copy(), poff.copy(), poff.copy()
    X, tets, tris, hinges, pinned = [], [], [], [], []
    for b, body in enumerate(bodies):
        p0 = poff[b]
        poff[b + 1] = p0 + body.np
        eoff[b + 1] = eoff[b] + body.ne
        toff[b + 1] = toff[b] + body.nt
        hoff[b + 1] = hoff[b] + body.nh
        X.append(np.asarray(body.X, np.float64))
        tets.append(np.asarray(body.tets, np.int64) + p0)
        tris.append(np.asarray(body.tris, np.int64) + p0)
        hinges.append(np.asarray(body.hinges, np.int64) + p0)
        pinned.append(np.asarray(body.pinned, np.uint8))
    cat = lambda a, shape, dt: np.ascontiguousarray(np.concatenate(a).astype(dt).reshape(shape))
    return Packed(len(bodies), poff, eoff, toff, hoff, cat(X, (-1, 3), np.float64), cat(tets, (-1, 4), np.int32),
                  cat(tris, (-1, 3), np.int32), cat(hinges, (-1, 4), np.int32), cat(pinned, (-1,), np.uint8),
                  np.ascontiguousarray([b.gravity for b in bodies], np.float64),
                  np.ascontiguousarray([b.dt for b in bodies], np.float64),
                  np.ascontiguousarray([b.plane for b in bodies], np.float64),
                  np.ascontiguousarray([1 if b.ground else 0 for b in bodies], np.uint8),
                  np.ascontiguousarray([b.kb for b in bodies], np.float64),
                  np.ascontiguousarray([1 if getattr(b, "air", False) else 0 for b in bodies], np.uint8))


class Plan:
    """``gsim_plan_create``: validated, oriented, precomputed host plan."""

    def __init__(self, bodies, dtype=torch.float32, tile_elems=0):
        lib = load()
        self.bodies = list(bodies)
        self.dtype = dtype
        self.tile_elems = int(tile_elems)
        pk = pack(self.bodies)
        self.packed = pk
        d = _Desc()
        d.dtype = GSIM_F64 if dtype == torch.float64 else GSIM_F32
        d.n_bodies = pk.n_bodies
        d.n_particles, d.n_tets, d.n_tris, d.n_hinges = len(pk.X), len(pk.tets), len(pk.tris), len(pk.hinges)
        a = lambda arr: arr.ctypes.data if arr is not None and arr.size else None
        d.body_particle_off = a(pk.poff)
        d.body_tet_off = a(pk.eoff) if len(pk.tets) else None
        d.body_tri_off = a(pk.toff) if len(pk.tris) else None
        d.body_hinge_off = a(pk.hoff) if len(pk.hinges) else None
        d.rest_x, d.tet_idx, d.tri_idx, d.hinge_idx = a(pk.X), a(pk.tets), a(pk.tris), a(pk.hinges)
        d.pinned, d.gravity, d.dt, d.ground = a(pk.pinned), a(pk.gravity), a(pk.dt), a(pk.ground)
        d.contact_on, d.k_bend = a(pk.contact_on), a(pk.k_bend)
        d.air_on = a(pk.air_on) if pk.air_on.any() else None
        d.tile_elems = self.tile_elems
        h = C.c_void_p()
        _check(lib.gsim_plan_create(C.byref(d), C.byref(h)))
        self._h = h
        self.np, self.ne, self.nt, self.nh, self.nb = d.n_particles, d.n_tets, d.n_tris, d.n_hinges, d.n_bodies
        self.any_air = bool(pk.air_on.any())

    def colouring(self, kind):
        """(order, bounds) of the colour-ordered element list of one kind (0 tet, 1 tri, 2 hinge)."""
        n = (self.ne, self.nt, self.nh)[kind]
        order = np.zeros(max(n, 1), np.int32)
        nb = C.c_int()
        _check(load().gsim_plan_colouring(self._h, kind, None, None, 0, C.byref(nb)))
        bounds = np.zeros(max(nb.value, 1), np.int32)
        _check(load().gsim_plan_colouring(self._h, kind, order.ctypes.data, bounds.ctypes.data, nb.value, C.byref(nb)))
        return order[:n], bounds[:nb.value]

    def tiles(self):
        """Element tiles of the two-pass path: (tiles [n, 5] = kind, body, first element,
        count, first tile particle; tile-particle index, run, partial slot arrays)."""
        nt, ntp = C.c_int64(), C.c_int64()
        _check(load().gsim_plan_tiles(self._h, None, C.byref(nt), None, None, None, C.byref(ntp)))
        tiles = np.zeros((max(nt.value, 1), 5), np.int64)
        tp, run, slot = (np.zeros(max(ntp.value, 1), np.int32) for _ in range(3))
        _check(load().gsim_plan_tiles(self._h, tiles.ctypes.data, C.byref(nt), tp.ctypes.data, run.ctypes.data,
                                      slot.ctypes.data, C.byref(ntp)))
        k = ntp.value
        return tiles[:nt.value], tp[:k], run[:k], slot[:k]

    def codes(self, kind):
        """Corner codes [corners, n] of one kind: tile-local particle | sorted position << 16."""
        n = (self.ne, self.nt, self.nh)[kind]
        nc = 3 if kind == 1 else 4
        out = np.zeros(max(nc * n, 1), np.uint32)
        _check(load().gsim_plan_codes(self._h, kind, out.ctypes.data))
        return out[:nc * n].reshape(nc, n)

    def partials(self):
        """(slice_base, degree, n_slots) of the sliced-ELL table of partials."""
        ns, nsl = C.c_int64(), C.c_int64()
        _check(load().gsim_plan_partials(self._h, None, C.byref(ns), None, C.byref(nsl)))
        base = np.zeros(max(ns.value, 1), np.int32)
        deg = np.zeros(self.np, np.int32)
        _check(load().gsim_plan_partials(self._h, base.ctypes.data, C.byref(ns), deg.ctypes.data, C.byref(nsl)))
        return base[:ns.value], deg, nsl.value
    def sizes(self, max_steps, ckpt_every):
        w, c, s = C.c_size_t(), C.c_size_t(), C.c_size_t()
        _check(load().gsim_plan_sizes(self._h, int(max_steps), int(ckpt_every), C.byref(w), C.byref(c), C.byref(s)))
        return w.value, c.value, s.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.gsim_plan_destroy(h)
            self._h = None


class Model:
    """``gsim_model_init`` over torch-allocated buffers, plus the per-call entry points."""

    def __init__(self, bodies, dtype=torch.float32, max_steps=100, ckpt_every=10, device="cuda", stream=None,
                 tile_elems=0, overlap=True):
        self.plan = Plan(bodies, dtype, tile_elems)
        self.dtype = dtype
        self.device = _device(device)
        self.max_steps, self.ckpt_every = int(max_steps), int(ckpt_every)
        ws, ck, seg = self.plan.sizes(max_steps, ckpt_every)
        self.bytes = {"workspace": ws, "ckpt": ck, "segment": seg}
        self.workspace = torch.empty(ws + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        self._ws_ptr = self.workspace.data_ptr() + off
        esz = 8 if dtype == torch.float64 else 4
        self.ckpt = torch.empty(max(ck // esz, 1), dtype=dtype, device=self.device)
        self.segment = torch.empty(max(seg // esz, 1), dtype=dtype, device=self.device)
        h = C.c_void_p()
        _check(load().gsim_model_init(self.plan._h, self.max_steps, self.ckpt_every, C.c_void_p(self._ws_ptr),
                                      ws, _stream(stream), C.byref(h)))
        self._h = h
        p = self.plan
        self.np, self.ne, self.nt, self.nh, self.nb = p.np, p.ne, p.nt, p.nh, p.nb
        self.segment2 = None
        self._overlap = False
        self.set_overlap(overlap)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.gsim_model_destroy(h)
            self._h = None

    # -- execution settings ---------------------------------------------------
    def set_exec(self, exec_mode=None, block=0, items=0):
        cur = self.get_exec()
        _check(load().gsim_model_set_exec(self._h, cur[0] if exec_mode is None else int(exec_mode), int(block), int(items)))

    def set_launch(self, pass_, block, items):
        """Launch shape of the element passes (pass_=0) or particle passes (pass_=1)."""
        _check(load().gsim_model_set_launch(self._h, int(pass_), int(block), int(items)))

    def get_launch(self, pass_):
        b, i = C.c_int(), C.c_int()
        _check(load().gsim_model_get_launch(self._h, int(pass_), C.byref(b), C.byref(i)))
        return b.value, i.value

    def set_lanes(self, lanes):
        """Launch lanes of the two-pass path (1..4, at most one per body; the bodies are
        split into that many concurrent groups of about equal work; default 2)."""
        _check(load().gsim_model_set_lanes(self._h, int(lanes)))

    def get_lanes(self):
        n = C.c_int()
        _check(load().gsim_model_get_lanes(self._h, C.byref(n)))
        return n.value

    def keeps_last_segment(self):
        """Whether the second segment buffer is in use (the library's rule: overlap on,
        plain, graph or persistent execution, no body with lift/drag), so that a
        checkpointed rollout leaves its last segment for the backward and that segment is
        not recomputed."""
        return self._overlap and not self.plan.any_air and self.get_exec()[0] in (EXEC_PLAIN, EXEC_GRAPH,
                                                                                   EXEC_PERSIST)

    def set_overlap(self, on=True):
        """Overlapped recompute in rollout_backward: a second segment buffer of
        max(ckpt_every - 1, 1) states lets the recompute of one checkpoint segment share
        launches with the adjoint steps of the next (results bitwise unchanged)."""
        if on:
            if self.segment2 is None:
                n = max(self.ckpt_every - 1, 1) * 6 * self.np
                self.segment2 = torch.empty(max(n, 1), dtype=self.dtype, device=self.device)
            t = self.segment2
            _check(load().gsim_model_set_overlap(self._h, C.c_void_p(t.data_ptr()), t.numel() * t.element_size()))
        else:  # the buffer is kept: launches already queued may still use it
            _check(load().gsim_model_set_overlap(self._h, None, 0))
        self._overlap = bool(on)

    def get_exec(self):
        e, b, i = C.c_int(), C.c_int(), C.c_int()
        _check(load().gsim_model_get_exec(self._h, C.byref(e), C.byref(b), C.byref(i)))
        return e.value, b.value, i.value

    def check(self, clear=False, stream=None):
        """``gsim_model_check``: per-body status flags (FLAG_NONFINITE, FLAG_INVERTED) as an
        int32 array; raises GsimError(GSIM_E_NONFINITE) when a body went non-finite
        (its .flags attribute holds the array)."""
        f = np.zeros(self.nb, np.int32)
        rc = load().gsim_model_check(self._h, f.ctypes.data, int(bool(clear)), _stream(stream))
        if rc:
            err = GsimError(rc, load().gsim_last_error().decode())
            err.flags = f
            raise err
        return f

    def set_timing(self, kernels=KERNELS):
        """Bracket every launch of the named kernels with HIP events (plain execution)."""
        mask = 0
        for k in kernels:
            mask |= 1 << KERNELS.index(k)
        _check(load().gsim_model_set_timing(self._h, mask))

    def read_timing(self):
        """{kernel: (launches, total_ms)} since the last read."""
        out = {}
        for i, k in enumerate(KERNELS):
            n, ms = C.c_int64(), C.c_double()
            _check(load().gsim_model_read_timing(self._h, i, C.byref(n), C.byref(ms)))
            out[k] = (n.value, ms.value)
        return out

    # -- tensors ----------------------------------------------------------------
    def empty_state(self):
        return (torch.empty(3, self.np, dtype=self.dtype, device=self.device),
                torch.empty(3, self.np, dtype=self.dtype, device=self.device))

    def params_from_bodies(self, bodies=None):
        """Device parameter tensors: mu, lam [ne], ktri [nt], mass [np], contact [nb, 4],
        and air [nb, 2] = (k_drag, k_lift) when a body has lift/drag."""
        bodies = self.plan.bodies if bodies is None else bodies
        t = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float64)).to(self.device, self.dtype)
        p = {"mass": t(np.concatenate([b.mass for b in bodies])),
             "contact": t([[b.ke, b.kd, b.kf, b.muf] for b in bodies])}
        if any(getattr(b, "air", False) for b in bodies):
            p["air"] = t([[b.kdrag, b.klift] if b.air else [0.0, 0.0] for b in bodies])
        if self.ne:
            p["mu"] = t(np.concatenate([b.mu for b in bodies if b.ne]))
            p["lam"] = t(np.concatenate([b.lam for b in bodies if b.ne]))
        if self.nt:
            p["ktri"] = t(np.concatenate([b.ktri for b in bodies if b.nt]))
        return p

    def zero_grads(self, which=("mu", "lam", "ktri", "mass", "contact"), steps=None):
        """Zeroed gradient buffers.  "act" and "hact" (tet and hinge actuation) are
        [ne] / [nh], or [steps, ne] / [steps, nh] for one gradient per step."""
        n = {"mu": self.ne, "lam": self.ne, "ktri": self.nt, "mass": self.np, "contact": 4 * self.nb,
             "act": self.ne, "hact": self.nh}
        g = {}
        for k in which:
            if n[k]:
                shape = (steps, n[k]) if steps is not None and k in ("act", "hact") else (n[k],)
                g[k] = torch.zeros(shape, dtype=self.dtype, device=self.device)
        if "contact" in g:
            g["contact"] = g["contact"].view(self.nb, 4)
        return g

    def _actuation(self, d, key, n_steps):
        """Pointer and step stride of an actuation tensor: [n] (the same for every
        step) or [steps, n] (row t for step t; at least n_steps rows)."""
        a = d.get(key) if d else None
        if a is None:
            return None, 0
        n = self.ne if key == "act" else self.nh
        if not isinstance(a, torch.Tensor) or a.dtype != self.dtype or a.device != self.device:
            raise TypeError(f"{key}: expected a {self.dtype} tensor on {self.device}")
        if a.dim() == 1:
            if a.shape[0] != n or a.stride(0) != 1:
                raise ValueError(f"{key}: expected a contiguous [{n}] tensor")
            return _ptr(a), 0
        if a.dim() != 2 or a.shape[1] != n or a.stride(1) != 1 or a.stride(0) < n:
            raise ValueError(f"{key}: expected [steps, {n}] with contiguous rows")
        if a.shape[0] < n_steps:
            raise ValueError(f"{key}: {a.shape[0]} rows for {n_steps} steps")
        return _ptr(a), a.stride(0)

    def _a(self, t, name, numel, shape=None):
        return _arg(t, name, self.dtype, self.device, numel, shape)

    def _sizes(self):
        return {"mu": self.ne, "lam": self.ne, "ktri": self.nt, "mass": self.np, "contact": 4 * self.nb,
                "air": 2 * self.nb}

    def _params(self, p, n_steps=1):
        s = _Params()
        n = self._sizes()
        a = lambda k: self._a(p.get(k), "params[%r]" % k, n[k])
        s.mu, s.lam, s.k_tri, s.mass, s.contact = a("mu"), a("lam"), a("ktri"), a("mass"), a("contact")
        s.act, s.act_stride = self._actuation(p, "act", n_steps)
        s.hact, s.hact_stride = self._actuation(p, "hact", n_steps)
        s.air = a("air")
        return s

    def _grads(self, g, n_steps=1):
        s = _Grads()
        if g:
            n = self._sizes()
            a = lambda k: self._a(g.get(k), "grads[%r]" % k, n[k])
            s.mu, s.lam, s.k_tri, s.mass, s.contact = a("mu"), a("lam"), a("ktri"), a("mass"), a("contact")
            s.act, s.act_stride = self._actuation(g, "act", n_steps)
            s.hact, s.hact_stride = self._actuation(g, "hact", n_steps)
        return s

    def _state(self, x, v, names=("x", "v")):
        s = _State()
        s.x = self._a(x, names[0], 3 * self.np, (3, self.np))
        s.v = self._a(v, names[1], 3 * self.np, (3, self.np))
        return s

    def _ck(self, ck):
        return self._a(ck, "ckpt", self.ckpt.numel())

    # -- entry points -------------------------------------------------------------
    def step(self, params, x, v, n_steps=1, out=None, stream=None):
        xo, vo = self.empty_state() if out is None else out
        _check(load().gsim_step(self._h, C.byref(self._params(params, n_steps)), self._state(x, v),
                                self._state(xo, vo, ("x_out", "v_out")), int(n_steps), _stream(stream)))
        return xo, vo

    def step_backward(self, params, x, v, xb_plus, vb_plus, grads=None, stream=None):
        xbm, vbm = self.empty_state()
        _check(load().gsim_step_backward(self._h, C.byref(self._params(params)), self._state(x, v),
                                         self._state(xb_plus, vb_plus, ("xb_plus", "vb_plus")), self._state(xbm, vbm),
                                         C.byref(self._grads(grads)), _stream(stream)))
        return xbm, vbm

    def new_checkpoints(self):
        """A checkpoint buffer of its own (for rollouts whose backward comes later)."""
        return torch.empty_like(self.ckpt)

    def rollout(self, params, x0, v0, n_steps, checkpoint=True, out=None, stream=None, ckpt=None):
        xo, vo = self.empty_state() if out is None else out
        ck = (self.ckpt if ckpt is None else ckpt) if checkpoint else None
        _check(load().gsim_rollout(self._h, C.byref(self._params(params, n_steps)), self._state(x0, v0, ("x0", "v0")),
                                   int(n_steps), self._ck(ck), self._state(xo, vo, ("x_out", "v_out")), _stream(stream)))
        return xo, vo

    def rollout_backward(self, params, n_steps, xb_final, vb_final, grads=None, out=None, stream=None, ckpt=None):
        xbi, vbi = self.empty_state() if out is None else out
        ck = self.ckpt if ckpt is None else ckpt
        _check(load().gsim_rollout_backward(self._h, C.byref(self._params(params, n_steps)), self._ck(ck), int(n_steps),
                                            _ptr(self.segment), self._state(xb_final, vb_final, ("xb_final", "vb_final")),
                                            self._state(xbi, vbi, ("xb_out", "vb_out")),
                                            C.byref(self._grads(grads, n_steps)), _stream(stream)))
        return xbi, vbi

    def loss_mse(self, x, target, seed=True, stream=None):
        loss = torch.empty(self.nb, dtype=self.dtype, device=self.device)
        xb, vb = self.empty_state() if seed else (None, None)
        _check(load().gsim_loss_mse(self._h, self._state(x, None), self._a(target, "target", 3 * self.np, (3, self.np)),
                                    _ptr(loss), self._state(xb, vb, ("xb", "vb")), _stream(stream)))
        return loss, xb, vb


# ----------------------------------------------------------------------------------
# Rigid bodies (gsim_rigid_*)
# ----------------------------------------------------------------------------------

class RigidModel:
    """A batch of rigid bodies (``workloads.RigidBody``-like) bound to a device
    workspace.  States are [n_bodies, 13] = x, quaternion (w first), v, omega;
    trajectories [(T + 1), n_bodies, 13]; parameters mass [nb], inertia [nb, 6],
    contact [nb, 4]."""

    def __init__(self, bodies, dtype=torch.float32, device="cuda"):
        lib = load()
        self.bodies = list(bodies)
        self.dtype, self.device = dtype, _device(device)
        self.nb = len(self.bodies)
        self.vert_off = np.zeros(self.nb + 1, np.int64)
        for i, b in enumerate(self.bodies):
            self.vert_off[i + 1] = self.vert_off[i] + len(b.verts)
        self.n_verts = int(self.vert_off[-1])
        self._verts = np.ascontiguousarray(np.concatenate([np.asarray(b.verts, np.float64) for b in self.bodies]))
        self._grav = np.ascontiguousarray([b.gravity for b in self.bodies], np.float64)
        self._dt = np.ascontiguousarray([b.dt for b in self.bodies], np.float64)
        self._plane = np.ascontiguousarray([b.plane for b in self.bodies], np.float64)
        self._on = np.ascontiguousarray([1 if b.ground else 0 for b in self.bodies], np.uint8)
        d = _RigidDesc()
        d.dtype = GSIM_F64 if dtype == torch.float64 else GSIM_F32
        d.n_bodies = self.nb
        d.vert_off, d.verts = self.vert_off.ctypes.data, self._verts.ctypes.data
        d.gravity, d.dt, d.ground, d.contact_on = (self._grav.ctypes.data, self._dt.ctypes.data,
                                                   self._plane.ctypes.data, self._on.ctypes.data)
        nbytes = C.c_size_t()
        _check(lib.gsim_rigid_sizes(C.byref(d), C.byref(nbytes)))
        self.workspace = torch.empty(max(int(nbytes.value), 256) + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        h = C.c_void_p()
        _check(lib.gsim_rigid_init(C.byref(d), C.c_void_p(self.workspace.data_ptr() + off), nbytes.value,
                                   _stream(None), C.byref(h)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.gsim_rigid_destroy(h)
            self._h = None

    def _t(self, a):
        return torch.as_tensor(np.ascontiguousarray(a, np.float64)).to(self.device, self.dtype)

    def params_from_bodies(self):
        return {"mass": self._t([b.mass for b in self.bodies]), "inertia": self._t([b.inertia for b in self.bodies]),
                "contact": self._t([b.contact() for b in self.bodies])}

    def initial_state(self):
        return self._t([b.s0 for b in self.bodies])

    def zero_grads(self):
        return {"mass": torch.zeros(self.nb, dtype=self.dtype, device=self.device),
                "inertia": torch.zeros(self.nb, 6, dtype=self.dtype, device=self.device),
                "contact": torch.zeros(self.nb, 4, dtype=self.dtype, device=self.device)}

    def _a(self, t, name, numel, shape=None):
        return _arg(t, name, self.dtype, self.device, numel, shape)

    def _params(self, p):
        s = _RigidParams()
        s.mass = self._a(p["mass"], "mass", self.nb)
        s.inertia = self._a(p["inertia"], "inertia", 6 * self.nb)
        s.contact = self._a(p["contact"], "contact", 4 * self.nb)
        return s

    def _traj(self, traj, n_steps):
        if traj is None or traj.dim() != 3 or traj.shape[0] < int(n_steps) + 1 or tuple(traj.shape[1:]) != (self.nb, 13):
            raise ValueError("traj must be a contiguous [n_steps + 1, n_bodies, 13] tensor")
        return self._a(traj, "traj", (int(n_steps) + 1) * self.nb * 13)

    def new_trajectory(self, n_steps):
        return torch.empty(int(n_steps) + 1, self.nb, 13, dtype=self.dtype, device=self.device)

    def rollout(self, params, s0, n_steps, traj=None, stream=None):
        traj = self.new_trajectory(n_steps) if traj is None else traj
        if traj.shape != (int(n_steps) + 1, self.nb, 13) or not traj.is_contiguous():
            raise ValueError("traj must be a contiguous [n_steps + 1, n_bodies, 13] tensor")
        _check(load().gsim_rigid_rollout(self._h, C.byref(self._params(params)),
                                         self._a(s0.contiguous(), "s0", 13 * self.nb, (self.nb, 13)), int(n_steps),
                                         self._traj(traj, n_steps), _stream(stream)))
        return traj

    def loss(self, state, target, stream=None):
        """(loss [nb], d loss / d state [nb, 13]) for world target vertices [n_verts, 3]."""
        loss = torch.empty(self.nb, dtype=self.dtype, device=self.device)
        sbar = torch.empty(self.nb, 13, dtype=self.dtype, device=self.device)
        _check(load().gsim_rigid_loss(self._h, self._a(state.contiguous(), "state", 13 * self.nb, (self.nb, 13)),
                                      self._a(target.contiguous(), "target", 3 * self.n_verts, (self.n_verts, 3)),
                                      _ptr(loss), _ptr(sbar), _stream(stream)))
        return loss, sbar

    def rollout_backward(self, params, traj, n_steps, sbar_final, grads=None, stream=None):
        """Adjoint of the initial state; parameter gradients accumulate into grads."""
        out = torch.empty(self.nb, 13, dtype=self.dtype, device=self.device)
        g = _RigidGrads()
        if grads:
            g.mass = self._a(grads.get("mass"), "grads['mass']", self.nb)
            g.inertia = self._a(grads.get("inertia"), "grads['inertia']", 6 * self.nb)
            g.contact = self._a(grads.get("contact"), "grads['contact']", 4 * self.nb)
        _check(load().gsim_rigid_rollout_backward(self._h, C.byref(self._params(params)), self._traj(traj, n_steps),
                                                  int(n_steps),
                                                  self._a(sbar_final.contiguous(), "sbar_final", 13 * self.nb,
                                                          (self.nb, 13)), _ptr(out), C.byref(g),
                                                  _stream(stream)))
        return out


# ----------------------------------------------------------------------------------
# Soft silhouette renderer (gsim_raster_*)
# ----------------------------------------------------------------------------------

class Renderer:
    """Soft silhouette of a triangle mesh (tris [nt, 3] over n_verts vertices) into a
    height x width image, for vertex positions given as SoA [3, n_verts] (a model's
    particle state)."""

    def __init__(self, tris, n_verts, height, width, dtype=torch.float32, device="cuda"):
        lib = load()
        self.tris = np.ascontiguousarray(np.asarray(tris, np.int32).reshape(-1, 3))
        self.nv, self.nt = int(n_verts), len(self.tris)
        self.H, self.W = int(height), int(width)
        self.dtype, self.device = dtype, _device(device)
        code = GSIM_F64 if dtype == torch.float64 else GSIM_F32
        nbytes = C.c_size_t()
        _check(lib.gsim_raster_sizes(code, self.nv, self.nt, self.H, self.W, C.byref(nbytes)))
        self.workspace = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        h = C.c_void_p()
        _check(lib.gsim_raster_init(code, self.nv, self.nt, self.tris.ctypes.data, self.H, self.W,
                                    C.c_void_p(self.workspace.data_ptr() + off), nbytes.value, _stream(None),
                                    C.byref(h)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.gsim_raster_destroy(h)
            self._h = None

    def _x(self, x):
        return _arg(x.contiguous(), "x", self.dtype, self.device, 3 * self.nv, (3, self.nv))

    @staticmethod
    def camera(P, sigma):
        c = _Camera()
        for k, v in enumerate(np.asarray(P, np.float64).ravel()):
            c.P[k] = float(v)
        c.sigma = float(sigma)
        return c

    def forward(self, x, P, sigma, stream=None):
        img = torch.empty(self.H, self.W, dtype=self.dtype, device=self.device)
        _check(load().gsim_raster_forward(self._h, C.byref(self.camera(P, sigma)), self._x(x), _ptr(img),
                                          _stream(stream)))
        return img

    def backward(self, x, P, sigma, image_bar, x_bar=None, stream=None):
        xb = torch.zeros(3, self.nv, dtype=self.dtype, device=self.device) if x_bar is None else x_bar
        _check(load().gsim_raster_backward(self._h, C.byref(self.camera(P, sigma)), self._x(x),
                                           _arg(image_bar.contiguous(), "image_bar", self.dtype, self.device,
                                                self.H * self.W, (self.H, self.W)),
                                           _arg(xb, "x_bar", self.dtype, self.device, 3 * self.nv, (3, self.nv)),
                                           _stream(stream)))
        return xb


RASTER_SCRATCH_BYTES = 32 << 20


def raster_forward_noalloc(tris, n_verts, height, width, x, P, sigma, out, stream=None):
    """``gsim_raster_forward_noalloc``: the renderer's forward with its scratch in the
    library's static device array (no renderer object, no workspace, nothing
    allocated).  tris: device int32 [nt, 3]; x: device SoA [3, n_verts]; out: device
    [height, width] of x's dtype (written)."""
    if x.dtype not in (torch.float32, torch.float64):
        raise TypeError("x must be float32 or float64")
    code = GSIM_F64 if x.dtype == torch.float64 else GSIM_F32
    nv, H, W = int(n_verts), int(height), int(width)
    tp = _arg(tris, "tris", torch.int32, x.device, 3 * tris.shape[0], (tris.shape[0], 3))
    xp = _arg(x, "x", x.dtype, x.device, 3 * nv, (3, nv))
    op = _arg(out, "out", x.dtype, x.device, H * W, (H, W))
    _check(load().gsim_raster_forward_noalloc(code, nv, int(tris.shape[0]), tp, H, W,
                                              C.byref(Renderer.camera(P, sigma)), xp, op, _stream(stream)))
    return out
