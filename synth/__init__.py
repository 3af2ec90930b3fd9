"""Seeded synthetic ventral-descent event windows.

This package only draws inputs (event coordinates, timestamps, polarities)
from a forward model of a camera descending onto a flat textured plane. It
contains none of the estimator's arithmetic (no warp, no event image, no
contrast, no bound), so both the CPU oracle and the HIP path can consume the
same inputs without sharing code.
"""

from .ventral import (  # noqa: F401
    WindowSpec,
    Window,
    make_window,
    config_windows,
    config_specs,
    CONFIG_NAMES,
    pack_batch,
)
