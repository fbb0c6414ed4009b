"""Seeded synthetic workloads shared by the oracle tests, the GPU tests and the bench."""
from .synthetic import (Workload, batching_set, large_shaped, make_items, make_queries,
                        mf_shaped, precision_shaped, tiny, PRESETS)

__all__ = ["Workload", "batching_set", "large_shaped", "make_items", "make_queries",
           "mf_shaped", "precision_shaped", "tiny", "PRESETS"]
