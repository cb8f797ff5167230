"""Seeded synthetic snapshot streams shared by the oracle, the tests and the bench.

This package only *generates inputs*: it holds none of the compression method's
arithmetic. Every generator evaluates a closed-form field on a grid, either on the
host (torch CPU, float64) or on a device (torch CUDA), so the CPU oracle and the
HIP path can consume the very same rounded snapshots.
"""
from .generators import (  # noqa: F401
    StreamSpec,
    analytic_cp5_spec,
    plume_spec,
    stochastic_plume_spec,
    fourier_ensemble_specs,
    channel_spec,
    runge_spec,
    lowrank_manifold_spec,
    switched_term_spec,
    counter_normal,
    gate_init_params,
)
