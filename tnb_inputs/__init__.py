"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds graph geometry, cluster maps and instance draws only.  It
contains none of the method's arithmetic (no energies, no Boltzmann weights, no
contractions): both the CPU oracle and the HIP path take its output as plain
arrays.
"""
from .rng import splitmix64, uniform01
from .geometry import zephyr_graph, zephyr_cross_cells, king_lattice, chain_lattice
from .instances import (Instance, make_instance, random_couplings, planted_loops, planted_king, transform, transform_cells,
                        N_TRANSFORMS)

__all__ = ["splitmix64", "uniform01", "zephyr_graph", "zephyr_cross_cells",
           "king_lattice", "chain_lattice", "Instance", "make_instance",
           "random_couplings", "planted_loops", "planted_king", "transform", "transform_cells", "N_TRANSFORMS"]
