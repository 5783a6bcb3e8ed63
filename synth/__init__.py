"""Seeded synthetic workloads for the VR-banded RZF precoding path.

This module only draws inputs (channels, visibility regions, symbols,
regularisers). It contains none of the precoding arithmetic, so both the
FP64 oracle and the HIP path can consume its output without sharing any
method code.
"""
from .channels import (  # noqa: F401
    Drop,
    WORKLOADS,
    make_drop,
    make_multipath_drop,
    make_subarray_drop,
    mask_hulls,
    make_workload,
    qpsk,
    qam16,
)
