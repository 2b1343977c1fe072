"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This package generates *inputs only*: analytic scenes, RGB-D frames rendered
from them by exact ray casting, camera trajectories, grid layouts and initial
parameter values.  It holds none of the reconstruction method's arithmetic
(no interpolation, decoding, rendering weights, losses or optimiser), so both
the HIP path and the FP64 oracle can consume what it produces without sharing
any of the code under test.
"""

from .scenes import SphereScene, RoomScene  # noqa: F401
from .frames import Frames, render_frames, sphere_frames, room_frames  # noqa: F401
from .layout import GridLayout, padded_layout, sequential_layout  # noqa: F401
from .params import (init_params, init_proposal, init_colour, MLP_SIZES, mlp_slices, MLP_NUMEL,  # noqa: F401
                     PROPOSAL_NUMEL, COLOUR_MLP_NUMEL)
from . import params  # noqa: F401
from . import configs  # noqa: F401
