"""Seeded synthetic power-grid instances for the block-structured AC-OPF.

This package only draws data (topology, line parameters, generator data, load
scenarios).  It holds none of the optimisation method's arithmetic and is the
one module that both the CPU oracle and the GPU path read their inputs from.
"""
from .grid import (Network, Scenarios, Instance, make_network, make_scenarios,
                   make_instance, preset, PRESETS, dims, batch_instances, line_outages)

__all__ = ["Network", "Scenarios", "Instance", "make_network", "make_scenarios",
           "make_instance", "preset", "PRESETS", "dims", "batch_instances", "line_outages"]
