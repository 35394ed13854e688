"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package only builds geometry (triangle meshes), incidence-angle lists,
frequency lists and random ray sets.  It holds none of the SBR arithmetic
(no intersection, reflection, aperture or physical-optics code), so both the
CPU oracle and the HIP path can take their inputs from it without sharing any
of the method's computation.
"""
from .meshes import (icosphere, plate, duct, dihedral, trihedral, aircraft,
                     random_triangles, mesh_area)
from .workloads import (C_LIGHT, sphere_case, trihedral_case, aircraft_case,
                        random_rays, Workload)
from .batch import batch_case, BatchWorkload, Scene, ellipsoid

__all__ = ["icosphere", "plate", "duct", "dihedral", "trihedral", "aircraft",
           "random_triangles", "mesh_area", "C_LIGHT", "sphere_case",
           "trihedral_case", "aircraft_case", "random_rays", "Workload",
           "batch_case", "BatchWorkload", "Scene", "ellipsoid"]
