"""Seeded synthetic off-axis holograms (inputs only; shared by the tests,
the bench and the smoke check). Holds the forward model |S+R|^2 and the
workload recipes; none of the processing path's arithmetic."""
from .holograms import (  # noqa: F401
    BASE_SEED, config, make_frames, hg_closed_form, forward_hologram, tile_pool,
)
