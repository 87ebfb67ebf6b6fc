"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This package generates images, covariances and request streams only.  It holds
none of the filter's arithmetic (no whitening, no sampling of terms, no
filtering), so the product path and the oracle can both be fed from it without
sharing any of the method's code.
"""

from .images import (  # noqa: F401
    voronoi_image, lab_like_image, feature_image, random_spd, workload,
    WORKLOADS, serving_requests, request_image,
)
