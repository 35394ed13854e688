"""Batched uneven workload: many seeded scenes of different kinds and sizes,
each with its own incidence angles and frequency list.

Scene ``s`` (seeds 1..n) is built from ``numpy.random.default_rng(seed)``:
its kind cycles through sphere, plate, dihedral, trihedral and ellipsoid
assembly; its triangle count is log-uniform in [10k, 500k]; it has 16..256
incidence directions uniform over the sphere of directions and 1..32
frequencies uniform in [2, 18] GHz.  Sampling is lambda(f_max)/10 of the
scene and at most 6 bounces.  Geometry only: no SBR arithmetic here.
"""
from dataclasses import dataclass, field

import numpy as np

from . import meshes
from .meshes import _finish, _grid_quad, _lathe

KINDS = ("sphere", "plate", "dihedral", "trihedral", "assembly")


def _rotation(rng):
    """Uniform random rotation (QR of a Gaussian matrix, sign-fixed)."""
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def ellipsoid(axes, n_lat, n_lon, center=(0.0, 0.0, 0.0), rot=None, vbase=0):
    """Latitude-longitude ellipsoid with semi-axes ``axes`` (float64 arrays,
    not yet rounded): n_lat bands, n_lon segments, poles joined by fans."""
    alpha = np.linspace(0.0, np.pi, n_lat + 1)
    xs = np.cos(alpha)
    rs = np.sin(alpha)
    rs[0] = rs[-1] = 0.0
    V, T = _lathe(xs, rs, n_lon, vbase=vbase)
    V = V * np.asarray(axes, dtype=np.float64)
    if rot is not None:
        V = V @ np.asarray(rot).T
    return V + np.asarray(center, dtype=np.float64), T


def _rotated(V, T, rot):
    V = V.astype(np.float64) @ rot.T
    return _finish(V, T)


def scene_mesh(kind, n_tris, rng):
    """(V, T, description) of one scene of ``kind`` with about n_tris triangles."""
    if kind == "sphere":
        r = rng.uniform(0.2, 2.0)
        n_lat = max(8, int(round(np.sqrt(n_tris / 4.0))))
        V, T = ellipsoid((r, r, r), n_lat, 2 * n_lat)
        V, T = _finish(V, T)
        return V, T, "sphere r=%.3f" % r
    if kind == "plate":
        a, b = rng.uniform(0.3, 2.0, size=2)
        n = max(4, int(round(np.sqrt(n_tris / 2.0))))
        V, T = meshes.plate(a, b, n, n)
        V, T = _rotated(V, T, _rotation(rng))
        return V, T, "plate %.3fx%.3f" % (a, b)
    if kind == "dihedral":
        a, b = rng.uniform(0.3, 1.5, size=2)
        n = max(4, int(round(np.sqrt(n_tris / 4.0))))
        V, T = meshes.dihedral(a, b, n)
        V, T = _rotated(V, T, _rotation(rng))
        return V, T, "dihedral %.3fx%.3f" % (a, b)
    if kind == "trihedral":
        a = rng.uniform(0.3, 1.5)
        n = max(4, int(round(np.sqrt(n_tris / 6.0))))
        V, T = meshes.trihedral(a, n)
        V, T = _rotated(V, T, _rotation(rng))
        return V, T, "trihedral a=%.3f" % a
    if kind == "assembly":
        k = int(rng.integers(3, 9))
        per = n_tris / k
        n_lat = max(6, int(round(np.sqrt(per / 4.0))))
        Vs, Ts, base = [], [], 0
        for _ in range(k):
            ax = rng.uniform(0.1, 0.8, size=3)
            c = rng.uniform(-1.0, 1.0, size=3)
            V, T = ellipsoid(ax, n_lat, 2 * n_lat, center=c, rot=_rotation(rng), vbase=base)
            Vs.append(V)
            Ts.append(T)
            base += len(V)
        V, T = _finish(np.concatenate(Vs), np.concatenate(Ts))
        return V, T, "assembly of %d ellipsoids" % k
    raise ValueError(kind)


@dataclass
class Scene:
    seed: int
    kind: str
    desc: str
    V: np.ndarray
    T: np.ndarray
    theta_deg: np.ndarray
    phi_deg: np.ndarray
    freqs_hz: np.ndarray


@dataclass
class BatchWorkload:
    name: str
    scenes: list
    samples_per_lambda: float = 10.0
    max_bounces: int = 6
    eta: float = 0.1
    meta: dict = field(default_factory=dict)

    def freqs(self):
        """All scenes' frequency lists, concatenated in scene order."""
        return np.concatenate([s.freqs_hz for s in self.scenes])

    def items(self):
        """(scene, theta_deg, phi_deg, freq_offset, n_freq) per (scene, angle),
        scenes in order, angles in order; offsets index ``freqs()``."""
        out, off = [], 0
        for si, s in enumerate(self.scenes):
            nf = len(s.freqs_hz)
            for th, ph in zip(s.theta_deg, s.phi_deg):
                out.append((si, float(th), float(ph), off, nf))
            off += nf
        return out


def batch_case(n_scenes=64, seed0=1, tri_range=(10_000, 500_000), angle_range=(16, 256), nf_range=(1, 32),
               f_range=(2.0e9, 18.0e9), max_bounces=6):
    """The batched uneven sweep; smaller ranges give reduced variants."""
    scenes = []
    for i in range(n_scenes):
        seed = seed0 + i
        rng = np.random.default_rng(seed)
        kind = KINDS[i % len(KINDS)]
        lo, hi = np.log(tri_range[0]), np.log(tri_range[1])
        n_tris = int(round(np.exp(rng.uniform(lo, hi))))
        V, T, desc = scene_mesh(kind, n_tris, rng)
        na = int(rng.integers(angle_range[0], angle_range[1] + 1))
        u, v = rng.uniform(size=na), rng.uniform(size=na)
        theta = np.degrees(np.arccos(1.0 - 2.0 * u))
        phi = 360.0 * v
        nf = int(rng.integers(nf_range[0], nf_range[1] + 1))
        freqs = np.sort(rng.uniform(f_range[0], f_range[1], size=nf))
        scenes.append(Scene(seed, kind, desc, V, T, theta, phi, freqs))
    return BatchWorkload("batch_%d_scenes" % n_scenes, scenes, 10.0, max_bounces)
