"""Seeded synthetic inputs shared by the oracle tests and the GPU library.

This package holds graph and partition generators only; it performs none of
the consensus method's arithmetic.
"""
from .configs import (Instance, sbm_small, lfr, gmm_knn, sbm_batch_specs,  # noqa: F401
                      served_pool_specs, served_instance,
                      sbm_batch_instance, random_instance)
