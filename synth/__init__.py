"""Seeded synthetic particle-image pairs shaped like the paper's channel-flow recordings.

The paper measures on backward-facing-step water-channel recordings (8-bit camera,
laser-sheet-lit seeding particles, Sec. 2.2) that are not available; these generators
stand in for them.  This package holds no step of the optical-flow method: it only
renders particle images and the displacement fields that move them.  Both the oracle
and the HIP path are fed from here, byte-identical.
"""
from .particles import (  # noqa: F401
    WORKLOADS,
    Workload,
    lamb_oseen,
    make_pair,
    render,
    workload,
    batch_items,
    stream_field,
    stream_frame,
    stream_frames,
    stream_frames_parallel,
    stream_particles,
    stream_scale,
    table1_pair,
)
