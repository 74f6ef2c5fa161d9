"""Seeded synthetic inputs for the componentwise OPF ADMM: feeders
(`opfgen.feeder`) and their componentwise linear model (`opfgen.model`).

Both the oracle and the GPU path consume these inputs; neither is imported
from here, and nothing here performs a step of the ADMM."""
from .feeder import (Feeder, by_name, make_13bus, make_123bus, make_2500bus, make_8500bus,
                     scenario_load_factors)
from .model import Instance, Component, build_instance, instance_from_flat, scenario_rhs, scenario_zip, with_rhs

__all__ = ["Feeder", "by_name", "make_13bus", "make_123bus", "make_2500bus", "make_8500bus",
           "scenario_load_factors", "Instance", "Component", "build_instance", "instance_from_flat",
           "scenario_rhs", "scenario_zip", "with_rhs"]
