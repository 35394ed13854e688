"""Workload descriptions (meshes + incidence angles + frequencies + sampling)
for the sphere, trihedral and aircraft cases, and seeded random ray sets.

Angles are in degrees: theta is the polar angle from +z and phi the azimuth;
an elevation ``el`` maps to ``theta = 90 - el``.
"""
from dataclasses import dataclass, field
import numpy as np

from . import meshes

C_LIGHT = 299_792_458.0


@dataclass
class Workload:
    name: str
    V: np.ndarray
    T: np.ndarray
    theta_deg: np.ndarray
    phi_deg: np.ndarray
    freqs_hz: np.ndarray
    samples_per_lambda: float
    max_bounces: int
    eta: float = 0.1
    meta: dict = field(default_factory=dict)

    @property
    def n_angles(self):
        return int(self.theta_deg.size)

    @property
    def ds(self):
        return C_LIGHT / float(np.max(self.freqs_hz)) / self.samples_per_lambda


def sphere_case(subdivisions=5):
    """PEC sphere r = 1 m (icosphere), 3 GHz, theta = phi = 0, lambda/10,
    at most 5 bounces."""
    V, T = meshes.icosphere(subdivisions, 1.0)
    return Workload("sphere_r1_3GHz", V, T, np.array([0.0]), np.array([0.0]),
                    np.array([3.0e9]), 10.0, 5)


def trihedral_case(n_phi=181, faces_n=16):
    """Square trihedral a = 1 m, 10 GHz, elevation 35.26 deg, azimuth
    0..90 deg in 0.5 deg steps (181 angles), lambda/10, at most 5 bounces."""
    V, T = meshes.trihedral(1.0, faces_n)
    phi = np.linspace(0.0, 90.0, n_phi)
    theta = np.full_like(phi, 90.0 - 35.26)
    return Workload("trihedral_a1_10GHz", V, T, theta, phi, np.array([10.0e9]), 10.0, 5)


def aircraft_case(n_phi=360, scale=1.0, seed=0):
    """Procedural aircraft, 10 GHz, elevation 0, azimuth 0..359 deg in 1 deg
    steps, lambda/8, at most 8 bounces."""
    V, T = meshes.aircraft(seed=seed, scale=scale)
    phi = np.arange(n_phi, dtype=np.float64) * (360.0 / n_phi)
    theta = np.full_like(phi, 90.0)
    return Workload("aircraft_10GHz", V, T, theta, phi, np.array([10.0e9]), 8.0, 8)


def random_rays(n, seed=0, box=1.5):
    """Random rays: origins uniform in [-box, box]^3, unit directions uniform
    on the sphere, float32.  Returns (o, d) of shape (n, 3)."""
    rng = np.random.default_rng(seed)
    o = rng.uniform(-box, box, size=(n, 3))
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return o.astype(np.float32), d.astype(np.float32)
