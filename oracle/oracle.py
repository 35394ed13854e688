"""Python face of the CPU oracle (ctypes over ``liboracle.so``).

TEST INFRASTRUCTURE ONLY: the independent reference for the SBR path.  Only
``tests/``, the smoke check and the benchmark's CPU-baseline leg use it.

Functions and the paper passages they follow:
  frame / aperture / gen_rays  -- incidence frame and ray grid, Eqs. (L1)-(L3), Sec. 4
  Mesh.build_bvh               -- Algorithm 1 with the SAH cost equation (fast mode)
  trace                        -- Algorithm 2 (multi-bounce transport), Sec. 4
  po                           -- Eq. (po_sum) (PAPER) / Eqs. (em5)-(em6) per ray tube (VECTOR)
  sigma_dbsm                   -- sigma = 4 pi |A|^2, 10 log10 (Sec. 4)
"""
import ctypes as C
import os

import numpy as np

from .build import ensure_built

C0 = 299_792_458.0
F_VALID, F_TRAPPED, F_BACK_LAST, F_EDGE = 1, 2, 4, 8
MODE_VECTOR, MODE_PAPER = 0, 1
_USE_BVH, _DROP_TRAPPED, _PAPER_PATH, _EDGE_DIAG = 1, 2, 4, 8
_FP32_PATH = 16  # precision study only: path, D and phase in float32
_MT_ONLY = 32    # brute force without the hit rule's box test (to show what the rule refuses)

_dp = C.POINTER(C.c_double)
_fp = C.POINTER(C.c_float)
_ip = C.POINTER(C.c_int32)
_lp = C.POINTER(C.c_int64)


class _TraceOut(C.Structure):
    _fields_ = [("nb", _ip), ("tri_first", _ip), ("tri_last", _ip), ("flags", _ip),
                ("path", _dp), ("D", _dp), ("d_last", _fp), ("x_last", _fp),
                ("eH_last", _dp), ("eV_last", _dp), ("tri_path", _ip),
                ("counters", C.c_int64 * 4)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = ensure_built()
        L = C.CDLL(path)
        L.orc_mesh_new.restype = C.c_void_p
        L.orc_mesh_new.argtypes = [_fp, C.c_int64, _ip, C.c_int64, C.POINTER(C.c_int)]
        L.orc_mesh_free.argtypes = [C.c_void_p]
        L.orc_mesh_info.argtypes = [C.c_void_p, _dp, _fp, _lp, _lp, C.POINTER(C.c_int)]
        L.orc_mesh_normals.argtypes = [C.c_void_p, _fp]
        L.orc_mesh_leaf_boxes.argtypes = [C.c_void_p, _dp, C.c_int64]
        L.orc_mesh_leaf_boxes.restype = C.c_int64
        L.orc_mesh_build_bvh.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int]
        L.orc_frame.argtypes = [C.c_double, C.c_double, _dp, _dp, _dp]
        L.orc_aperture.argtypes = [_dp, C.c_double, C.c_double, C.c_double, C.c_double,
                                   _lp, _lp, _dp, _dp, _dp]
        L.orc_gen_rays.argtypes = [_dp, C.c_double, C.c_double, C.c_double, C.c_double, _fp, _fp]
        L.orc_trace.argtypes = [C.c_void_p, C.c_int64, _fp, _fp, _dp, _dp, _dp, C.c_int, C.c_int,
                                C.POINTER(_TraceOut)]
        L.orc_po.argtypes = [C.c_void_p, C.c_int64, _ip, _ip, _ip, _ip, _dp, _fp, _dp, _dp,
                             C.c_int, _dp, _dp, _dp, C.c_double, _dp, C.c_int, _dp]
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _ptr(a, t):
    return a.ctypes.data_as(t) if a is not None else None


def num_threads():
    return lib().orc_num_threads()


def set_num_threads(n):
    lib().orc_set_num_threads(int(n))


class Mesh:
    """Prepared mesh: float32 edges, float64-derived unit normals, bounding
    box and offset epsilon (1e-5 of the box diagonal)."""

    def __init__(self, V, T):
        self.V = np.ascontiguousarray(V, dtype=np.float32).reshape(-1, 3)
        self.T = np.ascontiguousarray(T, dtype=np.int32).reshape(-1, 3)
        st = C.c_int(0)
        self._h = lib().orc_mesh_new(_ptr(self.V, _fp), len(self.V), _ptr(self.T, _ip), len(self.T),
                                     C.byref(st))
        if not self._h:
            raise ValueError("invalid mesh (status %d)" % st.value)
        self.nt = len(self.T)
        self._info()

    def _info(self):
        bb = np.zeros(6)
        eps = C.c_float()
        nd, nn, dep = C.c_int64(), C.c_int64(), C.c_int()
        lib().orc_mesh_info(self._h, _ptr(bb, _dp), C.byref(eps), C.byref(nd), C.byref(nn), C.byref(dep))
        self.bbox = bb
        self.eps = np.float32(eps.value)
        self.n_degen = nd.value
        self.n_nodes = nn.value
        self.depth = dep.value

    @property
    def normals(self):
        out = np.zeros((self.nt, 3), np.float32)
        lib().orc_mesh_normals(self._h, _ptr(out, _fp))
        return out

    def leaf_boxes(self):
        """(n_leaves, 6) float64 boxes (lo, hi) of the BVH's leaves (for
        pricing traversal work only)."""
        n = lib().orc_mesh_leaf_boxes(self._h, None, 0)
        out = np.zeros((max(n, 1), 6))
        lib().orc_mesh_leaf_boxes(self._h, _ptr(out, _dp), n)
        return out[:n]

    def build_bvh(self, rule="sah", nleaf=4, nbins=16):
        """Algorithm 1: recursive split by the median centroid (``median``) or
        by the binned SAH cost (``sah``) until a leaf holds <= nleaf triangles."""
        lib().orc_mesh_build_bvh(self._h, 1 if rule == "sah" else 0, int(nleaf), int(nbins))
        self._info()
        return self

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_mesh_free(h)
            self._h = None


def frame(theta_deg, phi_deg):
    """(k, theta_hat, phi_hat) in float64; k = -r_hat is the wave direction."""
    k, th, ph = np.zeros(3), np.zeros(3), np.zeros(3)
    lib().orc_frame(float(theta_deg), float(phi_deg), _ptr(k, _dp), _ptr(th, _dp), _ptr(ph, _dp))
    return k, th, ph


def aperture(bbox, theta_deg, phi_deg, ds, eta=0.1):
    """Eqs. (L1)-(L3): (Nu, Nv, uc, vc, s0)."""
    bb = np.ascontiguousarray(bbox, dtype=np.float64)
    Nu, Nv = C.c_int64(), C.c_int64()
    uc, vc, s0 = C.c_double(), C.c_double(), C.c_double()
    lib().orc_aperture(_ptr(bb, _dp), float(theta_deg), float(phi_deg), float(ds), float(eta),
                       C.byref(Nu), C.byref(Nv), C.byref(uc), C.byref(vc), C.byref(s0))
    return Nu.value, Nv.value, uc.value, vc.value, s0.value


def gen_rays(bbox, theta_deg, phi_deg, ds, eta=0.1):
    """Orthographic ray bundle: origins (Nu*Nv, 3) float32 in ray order
    j*Nu + i, and the common float32 direction."""
    Nu, Nv, *_ = aperture(bbox, theta_deg, phi_deg, ds, eta)
    bb = np.ascontiguousarray(bbox, dtype=np.float64)
    o = np.zeros((Nu * Nv, 3), np.float32)
    d = np.zeros(3, np.float32)
    lib().orc_gen_rays(_ptr(bb, _dp), float(theta_deg), float(phi_deg), float(ds), float(eta),
                       _ptr(o, _fp), _ptr(d, _fp))
    return o, d, Nu, Nv


def trace(mesh, o, d, eH0, eV0, k, bmax, use_bvh=False, drop_trapped=False, paper_path=False,
          edge_diag=False, want_path=False, fp32_path=False, mt_only=False):
    """Algorithm 2 for every ray.  ``d`` may be one direction for all rays or
    one per ray.  Returns a dict of per-ray arrays and counters.
    ``fp32_path``: accumulate P and form D in float32 (the single-precision
    variant whose phase error Sec. 6 discusses; a study, not the method).
    ``mt_only``: brute force with the Moller-Trumbore conditions alone, without
    the hit rule's box test (a study of what the rule refuses)."""
    o = np.ascontiguousarray(o, dtype=np.float32).reshape(-1, 3)
    n = len(o)
    d = np.asarray(d, dtype=np.float32)
    if d.ndim == 1:
        d = np.broadcast_to(d, (n, 3))
    d = np.ascontiguousarray(d, dtype=np.float32)
    eH0 = np.ascontiguousarray(eH0, dtype=np.float64)
    eV0 = np.ascontiguousarray(eV0, dtype=np.float64)
    k = np.ascontiguousarray(k, dtype=np.float64)
    r = dict(nb=np.zeros(n, np.int32), tri_first=np.zeros(n, np.int32), tri_last=np.zeros(n, np.int32),
             flags=np.zeros(n, np.int32), path=np.zeros(n), D=np.zeros(n),
             d_last=np.zeros((n, 3), np.float32), x_last=np.zeros((n, 3), np.float32),
             eH_last=np.zeros((n, 3)), eV_last=np.zeros((n, 3)))
    if want_path:
        r["tri_path"] = np.zeros((n, bmax), np.int32)
    out = _TraceOut()
    for name, t in (("nb", _ip), ("tri_first", _ip), ("tri_last", _ip), ("flags", _ip), ("path", _dp),
                    ("D", _dp), ("d_last", _fp), ("x_last", _fp), ("eH_last", _dp), ("eV_last", _dp)):
        setattr(out, name, _ptr(r[name], t))
    out.tri_path = _ptr(r["tri_path"], _ip) if want_path else None
    opts = ((_USE_BVH if use_bvh else 0) | (_DROP_TRAPPED if drop_trapped else 0)
            | (_PAPER_PATH if paper_path else 0) | (_EDGE_DIAG if edge_diag else 0)
            | (_FP32_PATH if fp32_path else 0) | (_MT_ONLY if mt_only else 0))
    if mt_only and use_bvh:
        raise ValueError("mt_only is a brute-force study option")
    if use_bvh and mesh.n_nodes == 0:
        mesh.build_bvh()
    rc = lib().orc_trace(mesh._h, n, _ptr(o, _fp), _ptr(d, _fp), _ptr(eH0, _dp), _ptr(eV0, _dp),
                         _ptr(k, _dp), int(bmax), opts, C.byref(out))
    if rc != 0:
        raise ValueError("orc_trace failed (%d)" % rc)
    r["queries"], r["box_tests"], r["tri_tests"], r["edge_rays"] = (int(x) for x in out.counters)
    return r


def po(mesh, rec, mode, k, th_hat, ph_hat, dA, freqs, fp32_phase=False):
    """Ray-tube PO sum over the valid rays of ``rec`` (a ``trace`` result).
    Returns complex A of shape (n_freq, 2, 2), [f, receive, transmit] with
    polarisation index 0 = H (phi_hat), 1 = V (theta_hat).  ``fp32_phase``:
    the phase k D formed in float32 (precision study only)."""
    freqs = np.ascontiguousarray(np.atleast_1d(freqs), dtype=np.float64)
    nf = len(freqs)
    A = np.zeros(nf * 8)
    n = len(rec["nb"])
    k, th_hat, ph_hat = (np.ascontiguousarray(x, dtype=np.float64) for x in (k, th_hat, ph_hat))
    rc = lib().orc_po(mesh._h, n, _ptr(rec["nb"], _ip), _ptr(rec["tri_first"], _ip), _ptr(rec["tri_last"], _ip),
                      _ptr(rec["flags"], _ip), _ptr(rec["D"], _dp), _ptr(rec["d_last"], _fp),
                      _ptr(rec["eH_last"], _dp), _ptr(rec["eV_last"], _dp),
                      int(mode) | (_FP32_PATH if fp32_phase else 0),
                      _ptr(k, _dp), _ptr(th_hat, _dp), _ptr(ph_hat, _dp), float(dA),
                      _ptr(freqs, _dp), nf, _ptr(A, _dp))
    if rc != 0:
        raise ValueError("orc_po failed (%d)" % rc)
    A = A.reshape(nf, 2, 2, 2)
    return A[..., 0] + 1j * A[..., 1]


def sigma_dbsm(A):
    """sigma = 4 pi |A|^2 in m^2, expressed in dBsm (-400 dB for sigma = 0)."""
    s = 4.0 * np.pi * np.abs(np.asarray(A)) ** 2
    with np.errstate(divide="ignore"):
        return np.where(s > 0, 10.0 * np.log10(np.where(s > 0, s, 1.0)), -400.0)


def rcs_angle(mesh, theta_deg, phi_deg, freqs, samples_per_lambda=10.0, ds=None, eta=0.1, bmax=5,
              mode=MODE_VECTOR, use_bvh=False, drop_trapped=False, edge_diag=False, want_path=False,
              ray_subset=None, fp32_path=False):
    """One incidence angle end to end: ray grid at ds = lambda(f_max)/s (one
    trace serves every frequency), trace, PO sum.  ``ray_subset`` restricts
    the trace to the given ray indices (the PO sum then covers only them).
    ``fp32_path``: path, D and phase in float32 (precision study only)."""
    freqs = np.atleast_1d(np.asarray(freqs, dtype=np.float64))
    if ds is None:
        ds = C0 / float(freqs.max()) / samples_per_lambda
    k, th, ph = frame(theta_deg, phi_deg)
    o, d, Nu, Nv = gen_rays(mesh.bbox, theta_deg, phi_deg, ds, eta)
    ids = np.arange(len(o)) if ray_subset is None else np.asarray(ray_subset)
    rec = trace(mesh, o[ids], d, ph, th, k, bmax, use_bvh=use_bvh, drop_trapped=drop_trapped,
                edge_diag=edge_diag, want_path=want_path, fp32_path=fp32_path)
    A = po(mesh, rec, mode, k, th, ph, ds * ds, freqs, fp32_phase=fp32_path)
    rec.update(A=A, Nu=Nu, Nv=Nv, ds=ds, o=o[ids], d=d, k=k, th_hat=th, ph_hat=ph, ray_ids=ids)
    return rec
