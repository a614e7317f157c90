"""Seeded synthetic microphone-array recordings (signal synthesis only)."""
from .arrays import (ArrayRecording, make_recording, white_pair, random_signals,  # noqa: F401
                     circular_array, square_array, far_field_delays, fractional_delay,
                     fractional_delay_frames, pair_room, sphere_grid,
                     random_planar_array, batch_arrays)
