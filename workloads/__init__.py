"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark.  Holds random-number streams and initial-condition recipes only."""
from .rng import Stream, splitmix64_reference
from .ics import (FIELDS, HaloSpec, default_halo, no_halo, outer_period, plummer, exp_disk, kepler_pair,
                  kepler_relative_position, batch_sizes, batch_mix, request_stream, make)

__all__ = ["Stream", "splitmix64_reference", "FIELDS", "HaloSpec", "default_halo", "no_halo", "outer_period", "plummer",
           "exp_disk", "kepler_pair", "kepler_relative_position", "batch_sizes", "batch_mix",
           "request_stream", "make"]
