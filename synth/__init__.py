"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This package holds no part of the moment arithmetic: it only draws frames
(blob / noise / polygon content inside the inscribed disk) and request
streams from documented seeds, so that the GPU path and the CPU oracle see
bit-identical inputs.
"""
from .frames import (  # noqa: F401
    FrameSpec,
    make_frame,
    config_frame,
    batch_sides,
    request_stream,
    dedup_set,
)
