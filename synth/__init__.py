"""Seeded synthetic inputs for the four-phonon rate kernel (structures, harmonic modes,
fourth-order force constants).  Shared by the tests, the benchmark and both
implementations; it holds none of the scattering-rate arithmetic."""
from .crystal import Crystal, diamond, wurtzite_like, layered_rhombohedral, grid_points, flat_index, minus_index
from .fc4 import FC4, random_fc4, scaled
from .configs import Instance, small, medium, large, diamond_instance

__all__ = ["Crystal", "diamond", "wurtzite_like", "layered_rhombohedral", "grid_points",
           "flat_index", "minus_index", "FC4", "random_fc4", "scaled", "Instance", "small",
           "medium", "large", "diamond_instance"]
