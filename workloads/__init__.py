"""Seeded synthetic workloads (inputs only, no method arithmetic)."""
from .synth import Workload, CONFIGS, CONFIG_ORDER, get, f32_round  # noqa: F401
