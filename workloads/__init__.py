"""Seeded synthetic biometric feature workloads.

The paper measures on face (IJB-C, LFW, ...) and fingerprint (PolyU, FVC,
CASIA) embeddings from a trained ResNet-18; none of those datasets or weights
are available, so these generators stand in for them with the same shapes:
L2-normalised FP32 vectors of 16..512 dimensions, clustered around identity
centres where the workload is an identification gallery.

This module holds no homomorphic-encryption arithmetic.  Both the GPU
library's tests/benchmarks and the CPU oracle take their inputs from here.
Every generator uses numpy's PCG64 (`default_rng(seed)`).
"""
from .features import (normalize, tiny_gallery, face_gallery, fingerprint_gallery,
                       mixed_batch, serving_galleries, poisson_arrivals)

__all__ = ["normalize", "tiny_gallery", "face_gallery", "fingerprint_gallery",
           "mixed_batch", "serving_galleries", "poisson_arrivals"]
