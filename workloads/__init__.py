"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This package holds no arithmetic of the method (no energy, no network, no
estimator).  It only draws disorder instances and parameter vectors from seeds
and describes the workloads by their sizes, so that the GPU path and the CPU
oracle can be fed identical inputs.
"""
from .configs import ModelConfig, Workload, WORKLOADS, workload
from .instances import sk_instance, ea_instance, Instance
from .params import param_layout, num_params, init_params

__all__ = [
    "ModelConfig", "Workload", "WORKLOADS", "workload",
    "sk_instance", "ea_instance", "Instance",
    "param_layout", "num_params", "init_params",
]
