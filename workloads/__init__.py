"""Seeded synthetic inputs for the reduced-MBF array solver.

This package draws random numbers and places points; it holds none of the
method's arithmetic (no Green's function, no fit, no fill, no solve).  Both the
CPU oracle and the GPU path take their inputs from here.
"""
from .synthetic import (  # noqa: F401
    Element,
    Workload,
    element,
    layout_disk,
    directions,
    harp_orders,
    workload,
    batched_layouts,
    CONFIG_NAMES,
)
