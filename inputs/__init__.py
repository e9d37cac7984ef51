"""Seeded synthetic workloads shared by the oracle, the tests and the benchmark.

This package only builds inputs: lattice sizes, parameter sets, node flags,
initial phase fields and electrode-voltage schedules.  It contains none of the
scheme's arithmetic (no equilibria, no forces, no wetting rule, no solver), so
the CPU oracle and the HIP library can both be fed from it without sharing any
part of the method.
"""
from .presets import (  # noqa: F401
    FLUID, GROUND, NEUMANN, ELECTRODE0,
    Case, make_case, case_names, default_params, splitmix64, uniform01,
    voltage_schedule,
)
