"""Seeded synthetic inputs shared by the GPU path's tests/bench and the oracle.

This package only draws catalogues (positions, host-halo masses, candidate
types, line-of-sight velocities) and names the workload configurations.  It
holds none of the estimator's arithmetic: no pair finding, mass assignment,
transforms, binning or finalisation live here.
"""
from .catalog import Catalog, make_catalog, nfw_radius, soneira_peebles
from .configs import CONFIGS, Workload, get_config

__all__ = ["Catalog", "make_catalog", "nfw_radius", "soneira_peebles",
           "CONFIGS", "Workload", "get_config"]
