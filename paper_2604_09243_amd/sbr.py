"""ctypes binding of ``libsbr.so`` (the C ABI declared in ``include/sbr.h``).

Argument marshalling only: every step of the SBR path runs in the library's
HIP kernels.  torch supplies device memory (tensors are passed by
``data_ptr()``) and the stream (``torch.cuda.current_stream().cuda_stream``).
If the library is missing the import of this module fails: there is no CPU
fallback.
"""
import ctypes as C
import os
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsbr.so")

OK, ERR_INVALID_ARG, ERR_INVALID_MESH, ERR_SAMPLING, ERR_OOM, ERR_HIP, ERR_OVERFLOW, ERR_UNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6, -7
POL_H, POL_V = 0, 1
MODE_VECTOR, MODE_PAPER = 0, 1
MEM_HOST, MEM_DEVICE = 0, 1
BUILD_LBVH, BUILD_SAH, BUILD_PLOC = 0, 1, 2
REC_VALID, REC_TRAPPED, REC_BACK_LAST = 1, 2, 4
OPT_DROP_TRAPPED, OPT_PAPER_PATH, OPT_ALLOW_UNDERSAMPLING, OPT_SYNC, OPT_WAVEFRONT, OPT_NO_GRAPH = 1, 2, 4, 8, 16, 32
OPT_NO_MASK = 64
OPT_FP32_PATH = 128
OPT_FP64_TRAVERSE = 256
OPT_BVH4 = 512
OPT_PACKET = 1024
MAX_BOUNCES = 127

_vp = C.c_void_p
_d3 = C.c_double * 3


class BvhOpts(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("mem", C.c_int32), ("leaf_size", C.c_int32), ("builder", C.c_int32)]


class BvhInfo(C.Structure):
    _fields_ = [("n_tris", C.c_int64), ("n_live", C.c_int64), ("n_nodes", C.c_int64), ("depth", C.c_int32),
                ("eps", C.c_float), ("bbox", C.c_double * 6), ("device_bytes", C.c_int64), ("n_scenes", C.c_int32),
                ("reserved", C.c_int32)]


class BvhQuality(C.Structure):
    _fields_ = [("node_visits", C.c_double), ("tri_tests", C.c_double), ("leaves", C.c_int64),
                ("leaf_tris", C.c_int64), ("max_depth", C.c_int32), ("reserved", C.c_int32)]


class Rays(C.Structure):
    _fields_ = [("o", _vp), ("d", _vp), ("eH", _vp), ("eV", _vp)]


class Hits(C.Structure):
    _fields_ = [("n_bounce", _vp), ("tri_first", _vp), ("tri_last", _vp), ("flags", _vp), ("path", _vp),
                ("D", _vp), ("d_last", _vp), ("x_last", _vp), ("eH_last", _vp), ("eV_last", _vp),
                ("tri_path", _vp)]


class TraceOpts(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("flags", C.c_uint32), ("k_hat", _d3)]


class Stats(C.Structure):
    _fields_ = [("rays", C.c_int64), ("queries", C.c_int64), ("valid", C.c_int64), ("trapped", C.c_int64),
                ("hits", C.c_int64 * (MAX_BOUNCES + 1)), ("angles", C.c_int64), ("ms_trace", C.c_double),
                ("ms_po", C.c_double), ("ms_total", C.c_double), ("ms_bounce", C.c_double * (MAX_BOUNCES + 1)),
                ("queries_bounce", C.c_int64 * (MAX_BOUNCES + 1)), ("trav", C.c_int64 * 6),
                ("masked", C.c_int64), ("chunks", C.c_int64)]

    def as_dict(self):
        return dict(rays=self.rays, queries=self.queries, valid=self.valid, trapped=self.trapped,
                    hits=list(self.hits), angles=self.angles, ms_trace=self.ms_trace, ms_po=self.ms_po,
                    ms_total=self.ms_total, ms_bounce=list(self.ms_bounce),
                    queries_bounce=list(self.queries_bounce), trav=list(self.trav), masked=self.masked,
                    chunks=self.chunks)


class PoDesc(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("mode", C.c_int32), ("k_hat", _d3), ("theta_hat", _d3),
                ("phi_hat", _d3), ("dA", C.c_double)]


class Tune(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("schedule", C.c_int32), ("tile_w", C.c_int32),
                ("claim_tiles", C.c_int32), ("refill_min", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("chunk_log2", C.c_int32), ("reserved", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k not in ("struct_size", "reserved")}


def default_tune():
    t = Tune()
    _check(load_library().sbr_default_tune(C.byref(t)))
    return t


def make_tune(**kw):
    t = default_tune()
    for k, v in kw.items():
        setattr(t, k, int(v))
    return t


class Sweep(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("theta_deg", _vp), ("phi_deg", _vp), ("n_angles", C.c_int64),
                ("freqs_hz", _vp), ("n_freq", C.c_int32), ("max_bounces", C.c_int32), ("ds", C.c_double),
                ("samples_per_lambda", C.c_double), ("eta", C.c_double), ("mode", C.c_int32),
                ("flags", C.c_uint32), ("tune", C.POINTER(Tune))]


class BatchItem(C.Structure):
    _fields_ = [("scene", C.c_int32), ("n_freq", C.c_int32), ("freq_offset", C.c_int64),
                ("theta_deg", C.c_double), ("phi_deg", C.c_double), ("ds", C.c_double)]


class BatchDesc(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("items", C.POINTER(BatchItem)), ("n_items", C.c_int64),
                ("freqs_hz", _vp), ("n_freqs_total", C.c_int64), ("max_bounces", C.c_int32), ("mode", C.c_int32),
                ("flags", C.c_uint32), ("reserved", C.c_int32), ("samples_per_lambda", C.c_double),
                ("eta", C.c_double), ("tune", C.POINTER(Tune))]


class BatchInfo(C.Structure):
    _fields_ = [("n_items", C.c_int64), ("n_rows", C.c_int64), ("rays", C.c_int64), ("min_item_rays", C.c_int64),
                ("max_item_rays", C.c_int64), ("n_chunks", C.c_int32), ("graph_ready", C.c_int32),
                ("device_bytes", C.c_int64), ("tune", Tune)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "tune"}
        d["tune"] = self.tune.as_dict()
        return d


ACT_SILU, ACT_RELU = 0, 1


class MlpDesc(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("n_ff", C.c_int32), ("width", C.c_int32), ("depth", C.c_int32),
                ("act", C.c_int32), ("reserved", C.c_int32), ("ff_sigma", C.c_double), ("seed", C.c_uint64),
                ("lo", _d3), ("hi", _d3), ("out_scale", C.c_double)]


class MlpInfo(C.Structure):
    _fields_ = [("n_params", C.c_int64), ("n_ff", C.c_int32), ("width", C.c_int32), ("depth", C.c_int32),
                ("act", C.c_int32), ("out_scale", C.c_double), ("adam_steps", C.c_int64),
                ("flops_per_point", C.c_double)]


class TrainOpts(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("epochs", C.c_int32), ("batch", C.c_int32), ("reserved", C.c_int32),
                ("lr", C.c_double), ("lr_min", C.c_double), ("seed", C.c_uint64)]


class FillDesc(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("mode", C.c_int32), ("theta_deg", _vp), ("phi_deg", _vp),
                ("n_angles", C.c_int64), ("freqs_hz", _vp), ("n_freq", C.c_int32), ("tile_angles", C.c_int32),
                ("tile_freqs", C.c_int32), ("probes_per_tile", C.c_int32), ("probe_dir", _vp), ("probe_freq", _vp),
                ("max_bounces", C.c_int32), ("flags", C.c_uint32), ("ds", C.c_double), ("eta", C.c_double),
                ("tol_db", C.c_double), ("floor_db", C.c_double)]


class FillStats(C.Structure):
    _fields_ = [("tiles", C.c_int64), ("fallback_tiles", C.c_int64), ("points", C.c_int64),
                ("fallback_points", C.c_int64), ("probe_points", C.c_int64), ("ms_predict", C.c_double),
                ("ms_probe", C.c_double), ("ms_check", C.c_double), ("ms_fallback", C.c_double),
                ("ms_total", C.c_double), ("sbr_rays", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class AnglePlan(C.Structure):
    _fields_ = [("k_hat", _d3), ("theta_hat", _d3), ("phi_hat", _d3), ("uc", C.c_double), ("vc", C.c_double),
                ("s0", C.c_double), ("ds", C.c_double), ("nu", C.c_int64), ("nv", C.c_int64)]


# name -> (restype, argtypes); the full exported surface of include/sbr.h
SIGNATURES = {
    "sbr_version": (C.c_int, []),
    "sbr_last_error": (C.c_char_p, []),
    "sbr_create": (C.c_int, [C.POINTER(_vp), C.c_int, _vp]),
    "sbr_set_stream": (C.c_int, [_vp, _vp]),
    "sbr_synchronize": (C.c_int, [_vp]),
    "sbr_destroy": (None, [_vp]),
    "sbr_build_bvh": (C.c_int, [_vp, _vp, C.c_int64, _vp, C.c_int64, C.POINTER(BvhOpts), C.POINTER(_vp)]),
    "sbr_bvh_get_info": (C.c_int, [_vp, C.POINTER(BvhInfo)]),
    "sbr_bvh_validate": (C.c_int, [_vp]),
    "sbr_bvh_quality_of": (C.c_int, [_vp, C.POINTER(BvhQuality)]),
    "sbr_bvh_normals": (C.c_int, [_vp, _vp]),
    "sbr_free_bvh": (None, [_vp]),
    "sbr_trace": (C.c_int, [_vp, _vp, C.POINTER(Rays), C.c_int64, C.c_int, C.POINTER(TraceOpts),
                            C.POINTER(Hits), C.POINTER(Stats)]),
    "sbr_trace_noalloc": (C.c_int, [_vp, _vp, C.POINTER(Rays), C.c_int64, C.c_int, C.POINTER(TraceOpts),
                                    C.POINTER(Hits), C.POINTER(Stats)]),
    "sbr_po_integrate": (C.c_int, [_vp, _vp, C.POINTER(Hits), C.c_int64, C.POINTER(PoDesc), _vp, C.c_int, _vp]),
    "sbr_rcs_sweep": (C.c_int, [_vp, _vp, C.POINTER(Sweep), _vp, _vp, C.POINTER(Stats)]),
    "sbr_plan_angle": (C.c_int, [_vp, C.c_double, C.c_double, C.c_double, C.c_double, C.POINTER(AnglePlan)]),
    "sbr_default_tune": (C.c_int, [C.POINTER(Tune)]),
    "sbr_autotune": (C.c_int, [_vp, _vp, C.POINTER(Sweep), C.POINTER(Tune)]),
    "sbr_pack_scenes": (C.c_int, [_vp, C.POINTER(_vp), C.c_int, C.POINTER(_vp)]),
    "sbr_batch_create": (C.c_int, [_vp, _vp, C.POINTER(BatchDesc), C.POINTER(_vp)]),
    "sbr_batch_get_info": (C.c_int, [_vp, C.POINTER(BatchInfo)]),
    "sbr_batch_set_tune": (C.c_int, [_vp, C.POINTER(Tune)]),
    "sbr_batch_autotune": (C.c_int, [_vp, C.POINTER(Tune)]),
    "sbr_batch_run": (C.c_int, [_vp, _vp, _vp, C.POINTER(Stats)]),
    "sbr_batch_destroy": (None, [_vp]),
    "sbr_mlp_create": (C.c_int, [_vp, C.POINTER(MlpDesc), C.POINTER(_vp)]),
    "sbr_mlp_get_info": (C.c_int, [_vp, C.POINTER(MlpInfo)]),
    "sbr_mlp_get_params": (C.c_int, [_vp, _vp, C.c_int64]),
    "sbr_mlp_set_params": (C.c_int, [_vp, _vp, C.c_int64]),
    "sbr_mlp_get_features": (C.c_int, [_vp, _vp]),
    "sbr_mlp_set_scale": (C.c_int, [_vp, C.c_double]),
    "sbr_mlp_predict": (C.c_int, [_vp, _vp, C.c_int64, _vp]),
    "sbr_mlp_gradients": (C.c_int, [_vp, _vp, _vp, C.c_int64, _vp, C.POINTER(C.c_float)]),
    "sbr_mlp_train": (C.c_int, [_vp, _vp, _vp, C.c_int64, C.POINTER(TrainOpts), _vp]),
    "sbr_mlp_destroy": (None, [_vp]),
    "sbr_surrogate_fill": (C.c_int, [_vp, _vp, _vp, C.POINTER(FillDesc), _vp, _vp, _vp, C.POINTER(FillStats)]),
}

_lib = None


def load_library(path=LIB_PATH):
    """Loads the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libsbr.so not found at %s: build it with `python -m paper_2604_09243_amd.build` "
                           "(there is no CPU fallback)" % path)
    L = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


class SbrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("sbr status %d: %s" % (status, msg))
        self.status = status


def _check(rc):
    if rc != OK:
        raise SbrError(rc, load_library().sbr_last_error().decode())
    return rc


def plan_angle(bbox, theta_deg, phi_deg, ds, eta=0.1):
    """Host-only ray-grid plan of one angle (Eqs. L1-L3)."""
    bb = np.ascontiguousarray(bbox, dtype=np.float64)
    p = AnglePlan()
    _check(load_library().sbr_plan_angle(bb.ctypes.data, float(theta_deg), float(phi_deg), float(ds), float(eta),
                                         C.byref(p)))
    return dict(k_hat=np.array(p.k_hat), theta_hat=np.array(p.theta_hat), phi_hat=np.array(p.phi_hat),
                uc=p.uc, vc=p.vc, s0=p.s0, ds=p.ds, nu=p.nu, nv=p.nv)


def _torch():
    import torch
    return torch


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _dev_tensor(t, name, dtype, shape, device):
    """Checks that a tensor handed to the library as a device pointer lives
    on the context's GPU with the expected dtype and shape and is contiguous
    (a host tensor, a wrong dtype or a short array would be read out of
    bounds by the kernels).  ``shape`` entries of None match any size."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s: expected a torch tensor, got %s" % (name, type(t).__name__))
    if t.device.type != "cuda" or t.device.index != device:
        raise ValueError("%s: must be on cuda:%d, is on %s" % (name, device, t.device))
    if t.dtype != dtype:
        raise ValueError("%s: dtype must be %s, is %s" % (name, dtype, t.dtype))
    if t.dim() != len(shape) or any(w is not None and w != g for w, g in zip(shape, t.shape)):
        raise ValueError("%s: shape must be %s, is %s" % (name, tuple(shape), tuple(t.shape)))
    if not t.is_contiguous():
        raise ValueError("%s: must be contiguous" % name)
    return t


class BVH:
    def __init__(self, ctx, handle):
        self.ctx = ctx
        self.handle = handle
        info = BvhInfo()
        _check(load_library().sbr_bvh_get_info(handle, C.byref(info)))
        self.n_tris, self.n_live, self.n_nodes = info.n_tris, info.n_live, info.n_nodes
        self.depth, self.eps = info.depth, info.eps
        self.bbox = np.array(info.bbox)
        self.device_bytes = info.device_bytes
        self.n_scenes = info.n_scenes

    def quality(self):
        """Surface-area estimates of the traversal work (sbr_bvh_quality_of):
        dict of node_visits, tri_tests, leaves, leaf_tris, max_depth."""
        q = BvhQuality()
        _check(load_library().sbr_bvh_quality_of(self.handle, C.byref(q)))
        return {k: getattr(q, k) for k, _ in BvhQuality._fields_ if k != "reserved"}

    def validate(self):
        """Structural check of the node and triangle layout (sbr_bvh_validate);
        raises SbrError with the first violation."""
        _check(load_library().sbr_bvh_validate(self.handle))

    def normals(self):
        out = np.zeros((self.n_tris, 3), np.float32)
        _check(load_library().sbr_bvh_normals(self.handle, out.ctypes.data))
        return out

    def free(self):
        if self.handle:
            load_library().sbr_free_bvh(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Batch:
    """A planned batch (sbr_batch_create): ``run()`` replays its graph.

    ``row_offset[i]`` is the first output row of item i; rows of item i are
    its frequencies in order."""

    def __init__(self, ctx, scenes, handle, n_freq):
        self.ctx = ctx
        self.scenes = scenes  # the scene set must outlive the batch
        self.handle = handle
        self.row_offset = np.concatenate([[0], np.cumsum(n_freq)[:-1]]).astype(np.int64)
        self.n_freq = np.asarray(n_freq, np.int64)
        self._out = None

    def info(self):
        i = BatchInfo()
        _check(load_library().sbr_batch_get_info(self.handle, C.byref(i)))
        return i.as_dict()

    def set_tune(self, tune):
        _check(load_library().sbr_batch_set_tune(self.handle, C.byref(tune)))

    def autotune(self):
        t = Tune()
        _check(load_library().sbr_batch_autotune(self.handle, C.byref(t)))
        return t

    def run(self, stats=True, out=None):
        """Returns (A complex128 [n_rows, 2, 2], sigma_dbsm [n_rows, 2, 2],
        stats dict or None) as device tensors.  The output tensors are kept
        and reused by later calls (so the captured graph is replayed)."""
        torch = _torch()
        if out is None:
            if self._out is None:
                n = int(self.info()["n_rows"])
                dev = torch.device("cuda", self.ctx.device)
                self._out = (torch.empty(n, 2, 2, 2, dtype=torch.float64, device=dev),
                             torch.empty(n, 2, 2, dtype=torch.float64, device=dev))
            out = self._out
        A, S = out
        n = int(self.info()["n_rows"])
        _dev_tensor(A, "out A", torch.float64, (n, 2, 2, 2), self.ctx.device)
        if S is not None:
            _dev_tensor(S, "out sigma", torch.float64, (n, 2, 2), self.ctx.device)
        st = Stats() if stats else None
        _check(load_library().sbr_batch_run(self.handle, A.data_ptr(), S.data_ptr() if S is not None else None,
                                            C.byref(st) if stats else None))
        return torch.view_as_complex(A), S, (st.as_dict() if stats else None)

    def close(self):
        if getattr(self, "handle", None):
            load_library().sbr_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MLP:
    """The surrogate network (sbr_mlp_*).  Points are (theta_deg, phi_deg,
    f_hz) rows; fields are complex (A_HH, A_VV) pairs."""

    def __init__(self, ctx, handle):
        self.ctx = ctx
        self.handle = handle

    def info(self):
        i = MlpInfo()
        _check(load_library().sbr_mlp_get_info(self.handle, C.byref(i)))
        return {k: getattr(i, k) for k, _ in MlpInfo._fields_}

    def params(self):
        n = self.info()["n_params"]
        out = np.zeros(n, np.float32)
        _check(load_library().sbr_mlp_get_params(self.handle, out.ctypes.data, n))
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        _check(load_library().sbr_mlp_set_params(self.handle, p.ctypes.data, len(p)))

    def features(self):
        n = self.info()["n_ff"]
        out = np.zeros((n, 3), np.float32)
        _check(load_library().sbr_mlp_get_features(self.handle, out.ctypes.data))
        return out

    def set_scale(self, scale):
        _check(load_library().sbr_mlp_set_scale(self.handle, float(scale)))

    def _dev(self, x, dtype):
        torch = _torch()
        dev = torch.device("cuda", self.ctx.device)
        if isinstance(x, torch.Tensor):
            return x.to(dev, dtype).contiguous()
        return torch.from_numpy(np.ascontiguousarray(x)).to(dev, dtype).contiguous()

    def predict(self, pts):
        """pts [n, 3] -> complex128 device tensor [n, 2]."""
        torch = _torch()
        p = self._dev(pts, torch.float64)
        n = p.shape[0]
        _dev_tensor(p, "pts", torch.float64, (n, 3), self.ctx.device)
        A = torch.empty(n, 2, 2, dtype=torch.float64, device=p.device)
        _check(load_library().sbr_mlp_predict(self.handle, p.data_ptr(), n, A.data_ptr()))
        return torch.view_as_complex(A)

    def _targets(self, t):
        torch = _torch()
        if isinstance(t, torch.Tensor) and t.is_complex():
            t = torch.view_as_real(t.to(torch.complex128))
        elif not isinstance(t, torch.Tensor) and np.iscomplexobj(t):
            t = np.stack([np.real(t), np.imag(t)], axis=-1)
        return self._dev(t, torch.float64)

    def _check_pairs(self, p, t):
        """Points [n, 3] and targets of 4 reals per point (Re/Im of A_HH, A_VV)."""
        torch = _torch()
        n = p.shape[0]
        _dev_tensor(p, "pts", torch.float64, (n, 3), self.ctx.device)
        if t.numel() != 4 * n:
            raise ValueError("targets: need 4 reals per point (%d points), got %d values" % (n, t.numel()))
        _dev_tensor(t, "targets", torch.float64, tuple(t.shape), self.ctx.device)

    def gradients(self, pts, targets):
        """(grads float32 numpy [n_params], loss) for the points."""
        torch = _torch()
        p, t = self._dev(pts, torch.float64), self._targets(targets)
        self._check_pairs(p, t)
        g = torch.empty(self.info()["n_params"], dtype=torch.float32, device=p.device)
        loss = C.c_float()
        _check(load_library().sbr_mlp_gradients(self.handle, p.data_ptr(), t.data_ptr(), p.shape[0], g.data_ptr(),
                                                C.byref(loss)))
        return g.cpu().numpy(), loss.value

    def train(self, pts, targets, epochs, batch=1024, lr=1e-3, lr_min=1e-5, seed=0):
        """Adam training; returns the mean loss of every epoch."""
        torch = _torch()
        p, t = self._dev(pts, torch.float64), self._targets(targets)
        self._check_pairs(p, t)
        o = TrainOpts(C.sizeof(TrainOpts), int(epochs), int(batch), 0, float(lr), float(lr_min), int(seed))
        hist = np.zeros(int(epochs), np.float32)
        _check(load_library().sbr_mlp_train(self.handle, p.data_ptr(), t.data_ptr(), p.shape[0], C.byref(o),
                                            hist.ctypes.data))
        return hist

    def close(self):
        if getattr(self, "handle", None):
            load_library().sbr_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """An sbr_ctx on ``device`` enqueuing on torch's current stream."""

    def __init__(self, device=0, stream=None):
        torch = _torch()
        L = load_library()
        self.device = device
        torch.cuda.set_device(device)
        s = stream if stream is not None else torch.cuda.current_stream(device)
        self.stream = s
        h = C.c_void_p()
        _check(L.sbr_create(C.byref(h), int(device), C.c_void_p(s.cuda_stream)))
        self.handle = h
        self._batches = weakref.WeakSet()  # closed before the context
    def set_stream(self, stream):
        self.stream = stream
        _check(load_library().sbr_set_stream(self.handle, C.c_void_p(stream.cuda_stream)))

    def synchronize(self):
        _check(load_library().sbr_synchronize(self.handle))

    def close(self):
        if getattr(self, "handle", None):
            for b in list(getattr(self, "_batches", ())):
                b.close()
            load_library().sbr_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ build
    def build_bvh(self, V, T, leaf_size=0, builder=BUILD_LBVH):
        """V: [n_v, 3] float32, T: [n_t, 3] int32 (numpy host arrays or
        torch device tensors); leaf_size 1..4 (0 = library default);
        builder BUILD_LBVH (GPU), BUILD_SAH (host binned SAH) or BUILD_PLOC
        (GPU clustering by surface area)."""
        torch = _torch()
        opts = BvhOpts(C.sizeof(BvhOpts), MEM_HOST, int(leaf_size), int(builder))
        if isinstance(V, torch.Tensor):
            V = V.contiguous()
            T = T.contiguous()
            if V.dtype != torch.float32 or T.dtype != torch.int32:
                raise ValueError("build_bvh: V must be float32 and T int32")
            if V.dim() != 2 or V.shape[1] != 3 or T.dim() != 2 or T.shape[1] != 3:
                raise ValueError("build_bvh: V and T must be [n, 3]")
            if V.is_cuda != T.is_cuda or (V.is_cuda and (V.device.index != self.device or T.device.index != self.device)):
                raise ValueError("build_bvh: V and T must both be host tensors or both on cuda:%d" % self.device)
            opts.mem = MEM_DEVICE if V.is_cuda else MEM_HOST
            pv, pt, nv, nt = V.data_ptr(), T.data_ptr(), V.shape[0], T.shape[0]
            keep = (V, T)
        else:
            Vn = np.ascontiguousarray(V, dtype=np.float32).reshape(-1, 3)
            Tn = np.ascontiguousarray(T, dtype=np.int32).reshape(-1, 3)
            pv, pt, nv, nt = Vn.ctypes.data, Tn.ctypes.data, len(Vn), len(Tn)
            keep = (Vn, Tn)
        h = C.c_void_p()
        _check(load_library().sbr_build_bvh(self.handle, C.c_void_p(pv), nv, C.c_void_p(pt), nt, C.byref(opts),
                                            C.byref(h)))
        del keep
        return BVH(self, h)

    # ------------------------------------------------------------ trace
    _HIT_DTYPES = dict(n_bounce="int32", tri_first="int32", tri_last="int32", flags="int32", path="float64",
                       D="float64", d_last="float32", x_last="float32", eH_last="float32", eV_last="float32",
                       tri_path="int32")

    def trace(self, bvh, o, d, eH, eV, max_bounces, k_hat, flags=0, want_path=False, stats=False, out=None,
              noalloc=False):
        """Rays as [n, 3] float32 CUDA tensors; returns a dict of device
        tensors (the sbr_hits arrays) and, if ``stats``, the statistics.
        ``out``: caller-allocated result tensors (a dict with the sbr_hits
        names; absent names are skipped).  ``noalloc``: call
        sbr_trace_noalloc, which allocates nothing on the device."""
        torch = _torch()
        dev = torch.device("cuda", self.device)
        n = int(o.shape[0]) if hasattr(o, "shape") and len(o.shape) == 2 else -1
        for name, x in (("o", o), ("d", d), ("eH", eH), ("eV", eV)):
            _dev_tensor(x, name, torch.float32, (n, 3), self.device)
        if out is None:
            out = dict(n_bounce=torch.empty(n, dtype=torch.int32, device=dev),
                       tri_first=torch.empty(n, dtype=torch.int32, device=dev),
                       tri_last=torch.empty(n, dtype=torch.int32, device=dev),
                       flags=torch.empty(n, dtype=torch.int32, device=dev),
                       path=torch.empty(n, dtype=torch.float64, device=dev),
                       D=torch.empty(n, dtype=torch.float64, device=dev),
                       d_last=torch.empty(n, 3, dtype=torch.float32, device=dev),
                       x_last=torch.empty(n, 3, dtype=torch.float32, device=dev),
                       eH_last=torch.empty(n, 3, dtype=torch.float32, device=dev),
                       eV_last=torch.empty(n, 3, dtype=torch.float32, device=dev))
            if want_path:
                out["tri_path"] = torch.empty(n, max_bounces, dtype=torch.int32, device=dev)
        else:
            out = dict(out)
            for name, t in out.items():
                if name not in self._HIT_DTYPES:
                    raise ValueError("out: unknown result array %r" % name)
                shape = ((n, 3) if name in ("d_last", "x_last", "eH_last", "eV_last") else
                         (n, int(max_bounces)) if name == "tri_path" else (n,))
                _dev_tensor(t, name, getattr(torch, self._HIT_DTYPES[name]), shape, self.device)
        hits = self._hits(out)
        rays = Rays(o.data_ptr(), d.data_ptr(), eH.data_ptr(), eV.data_ptr())
        opts = TraceOpts(C.sizeof(TraceOpts), int(flags), _d3(*[float(x) for x in k_hat]))
        st = Stats() if stats else None
        fn = load_library().sbr_trace_noalloc if noalloc else load_library().sbr_trace
        _check(fn(self.handle, bvh.handle, C.byref(rays), n, int(max_bounces), C.byref(opts), C.byref(hits),
                  C.byref(st) if stats else None))
        if stats:
            out["stats"] = st.as_dict()
        return out

    @staticmethod
    def _hits(out):
        h = Hits()
        for name, _ in Hits._fields_:
            t = out.get(name)
            setattr(h, name, t.data_ptr() if t is not None else None)
        return h

    # ------------------------------------------------------------ PO
    def po_integrate(self, bvh, hits, mode, k_hat, theta_hat, phi_hat, dA, freqs):
        """PO sum over the valid rays of ``hits`` (a ``trace`` result).
        Returns a complex128 device tensor [n_freq, 2 receive, 2 transmit]."""
        torch = _torch()
        freqs = np.ascontiguousarray(np.atleast_1d(freqs), dtype=np.float64)
        nf = len(freqs)
        A = torch.empty(nf, 2, 2, 2, dtype=torch.float64, device=torch.device("cuda", self.device))
        desc = PoDesc(C.sizeof(PoDesc), int(mode), _d3(*map(float, k_hat)), _d3(*map(float, theta_hat)),
                      _d3(*map(float, phi_hat)), float(dA))
        n = int(hits["n_bounce"].shape[0])
        dtypes = dict(n_bounce=torch.int32, tri_first=torch.int32, tri_last=torch.int32, flags=torch.int32,
                      path=torch.float64, D=torch.float64, d_last=torch.float32, x_last=torch.float32,
                      eH_last=torch.float32, eV_last=torch.float32)
        for name, dt in dtypes.items():
            if hits.get(name) is not None:
                _dev_tensor(hits[name], name, dt, (n, 3) if name in ("d_last", "x_last", "eH_last", "eV_last")
                            else (n,), self.device)
        h = self._hits(hits)
        _check(load_library().sbr_po_integrate(self.handle, bvh.handle, C.byref(h), n, C.byref(desc),
                                               freqs.ctypes.data, nf, A.data_ptr()))
        return torch.view_as_complex(A)

    # ------------------------------------------------------------ sweep
    def autotune(self, bvh, theta_deg, phi_deg, freqs_hz, max_bounces=5, ds=0.0, samples_per_lambda=10.0, eta=0.1,
                 mode=MODE_VECTOR, flags=0):
        """Launch parameters for this BVH and sweep (sbr_autotune)."""
        th = np.ascontiguousarray(np.atleast_1d(theta_deg), dtype=np.float64)
        ph = np.ascontiguousarray(np.atleast_1d(phi_deg), dtype=np.float64)
        fr = np.ascontiguousarray(np.atleast_1d(freqs_hz), dtype=np.float64)
        sw = Sweep(C.sizeof(Sweep), th.ctypes.data, ph.ctypes.data, len(th), fr.ctypes.data, len(fr),
                   int(max_bounces), float(ds), float(samples_per_lambda), float(eta), int(mode), int(flags), None)
        t = Tune()
        _check(load_library().sbr_autotune(self.handle, bvh.handle, C.byref(sw), C.byref(t)))
        return t

    def rcs_sweep(self, bvh, theta_deg, phi_deg, freqs_hz, max_bounces=5, ds=0.0, samples_per_lambda=10.0,
                  eta=0.1, mode=MODE_VECTOR, flags=0, stats=True, out=None, tune=None):
        """Monostatic sweep.  Returns (A complex128 [n_angles, n_freq, 2, 2],
        sigma_dbsm float64 [n_angles, n_freq, 2, 2], stats dict or None), all
        device tensors; ``out`` may pass preallocated (A_real_view, sigma)."""
        torch = _torch()
        th = np.ascontiguousarray(np.atleast_1d(theta_deg), dtype=np.float64)
        ph = np.ascontiguousarray(np.atleast_1d(phi_deg), dtype=np.float64)
        fr = np.ascontiguousarray(np.atleast_1d(freqs_hz), dtype=np.float64)
        na, nf = len(th), len(fr)
        dev = torch.device("cuda", self.device)
        if out is None:
            A = torch.empty(na, nf, 2, 2, 2, dtype=torch.float64, device=dev)
            S = torch.empty(na, nf, 2, 2, dtype=torch.float64, device=dev)
        else:
            A, S = out
            _dev_tensor(A, "out A", torch.float64, (na, nf, 2, 2, 2), self.device)
            if S is not None:
                _dev_tensor(S, "out sigma", torch.float64, (na, nf, 2, 2), self.device)
        sw = Sweep(C.sizeof(Sweep), th.ctypes.data, ph.ctypes.data, na, fr.ctypes.data, nf, int(max_bounces),
                   float(ds), float(samples_per_lambda), float(eta), int(mode), int(flags),
                   C.pointer(tune) if tune is not None else None)
        st = Stats() if stats else None
        _check(load_library().sbr_rcs_sweep(self.handle, bvh.handle, C.byref(sw), A.data_ptr(),
                                            S.data_ptr() if S is not None else None,
                                            C.byref(st) if stats else None))
        return torch.view_as_complex(A), S, (st.as_dict() if stats else None)

    # ------------------------------------------------------------ batches
    def pack_scenes(self, bvhs):
        """One multi-scene set from several BVHs (sbr_pack_scenes)."""
        arr = (_vp * len(bvhs))(*[b.handle for b in bvhs])
        h = C.c_void_p()
        _check(load_library().sbr_pack_scenes(self.handle, arr, len(bvhs), C.byref(h)))
        return BVH(self, h)

    def batch(self, scenes, items, freqs_hz, max_bounces=6, samples_per_lambda=10.0, eta=0.1, mode=MODE_VECTOR,
              flags=0, tune=None):
        """Plans a batch.  ``items``: sequence of (scene, theta_deg, phi_deg,
        freq_offset, n_freq[, ds]) tuples; ``freqs_hz`` the frequency array
        the offsets index."""
        fr = np.ascontiguousarray(np.atleast_1d(freqs_hz), dtype=np.float64)
        arr = (BatchItem * len(items))()
        nf = []
        for i, it in enumerate(items):
            sc, th, ph, off, n = it[:5]
            ds = it[5] if len(it) > 5 else 0.0
            arr[i] = BatchItem(int(sc), int(n), int(off), float(th), float(ph), float(ds))
            nf.append(int(n))
        d = BatchDesc(C.sizeof(BatchDesc), arr, len(items), fr.ctypes.data, len(fr), int(max_bounces), int(mode),
                      int(flags), 0, float(samples_per_lambda), float(eta),
                      C.pointer(tune) if tune is not None else None)
        h = C.c_void_p()
        _check(load_library().sbr_batch_create(self.handle, scenes.handle, C.byref(d), C.byref(h)))
        b = Batch(self, scenes, h, nf)
        self._batches.add(b)
        return b

    # ------------------------------------------------------------ surrogate
    def mlp(self, lo, hi, out_scale=1.0, n_ff=64, width=256, depth=4, act=ACT_SILU, ff_sigma=4.0, seed=0):
        """A new surrogate network (sbr_mlp_create)."""
        d = MlpDesc(C.sizeof(MlpDesc), int(n_ff), int(width), int(depth), int(act), 0, float(ff_sigma), int(seed),
                    _d3(*map(float, lo)), _d3(*map(float, hi)), float(out_scale))
        h = C.c_void_p()
        _check(load_library().sbr_mlp_create(self.handle, C.byref(d), C.byref(h)))
        return MLP(self, h)

    def surrogate_fill(self, bvh, mlp, theta_deg, phi_deg, freqs_hz, tile_angles, tile_freqs, probe_dir,
                       probe_freq, ds, max_bounces=8, mode=MODE_VECTOR, flags=0, eta=0.1, tol_db=0.5,
                       floor_db=40.0):
        """Dense grid fill (sbr_surrogate_fill).  Returns (A complex128
        device [n_angles, n_freq, 2], tile_err [n_at, n_ft], fallback mask,
        stats dict)."""
        torch = _torch()
        th = np.ascontiguousarray(theta_deg, dtype=np.float64)
        ph = np.ascontiguousarray(phi_deg, dtype=np.float64)
        fr = np.ascontiguousarray(freqs_hz, dtype=np.float64)
        pdir = np.ascontiguousarray(probe_dir, dtype=np.float64).reshape(-1, 2)
        pfr = np.ascontiguousarray(probe_freq, dtype=np.float64).ravel()
        na, nf = len(th), len(fr)
        n_at = (na + tile_angles - 1) // tile_angles
        n_ft = (nf + tile_freqs - 1) // tile_freqs
        ppt = len(pfr) // n_ft
        d = FillDesc(C.sizeof(FillDesc), int(mode), th.ctypes.data, ph.ctypes.data, na, fr.ctypes.data, nf,
                     int(tile_angles), int(tile_freqs), int(ppt), pdir.ctypes.data, pfr.ctypes.data,
                     int(max_bounces), int(flags), float(ds), float(eta), float(tol_db), float(floor_db))
        A = torch.empty(na, nf, 2, 2, dtype=torch.float64, device=torch.device("cuda", self.device))
        err = np.zeros((n_at, n_ft), np.float64)
        fb = np.zeros((n_at, n_ft), np.uint8)
        st = FillStats()
        _check(load_library().sbr_surrogate_fill(self.handle, bvh.handle, mlp.handle, C.byref(d), A.data_ptr(),
                                                 err.ctypes.data, fb.ctypes.data, C.byref(st)))
        return torch.view_as_complex(A), err, fb, st.as_dict()
