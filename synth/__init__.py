"""Seeded synthetic inputs shaped like the paper's workloads.

This package holds input generators only: random derivative-ratio matrices O, local
energies E and local-energy derivatives D, and the correlator-product-state parameter
layout that shapes them.  It contains none of the method's arithmetic (no overlap,
gradient, product or solve), so both the GPU path and the CPU oracle may use it.
"""
from .configs import (  # noqa: F401
    CONFIGS, dense_inputs, cps_inputs, cps_index_inputs, cps_stream_layout, cps_stream_batch, lm_derivatives,
    small_cps_inputs, batched_shapes, relative_shifts,
)
from .cps_layout import (  # noqa: F401
    Correlator, CpsLayout, hubbard_4x4_layout, hydrogen_4x4_layout, hubbard_8x8_plaquette_layout,
)
