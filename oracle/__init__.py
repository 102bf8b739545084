"""FP64 CPU oracle for the off-axis digital-holography hot path.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.
The GPU library never calls it and shares no code with it.
"""
from .holo_oracle import (  # noqa: F401
    DEG, w_max_rad, tilt_bins, radius_bins, ifft_size, mode_list, mode_count,
    window_origin, mask_bins, geometry, hermite_gauss_1d, spectrum_window, window_pixels,
    field_from_window, overlap, power_normalise, process_frame, process_batch, captured_power, goal_db,
    INT16_FULL, fields_to_int16,
)
from .transfer_metrics import METRICS, transfer_matrix, column_keys, transfer_metrics  # noqa: F401,E402
from .align_snap import field_moments, batch_moments, snap_centre_waist, snap_defocus_magnitude  # noqa: F401,E402
from .plane_snap import SNAP_FRAMES, plane_power, snap_tilt_plane  # noqa: F401,E402
from .basis import (  # noqa: F401,E402
    lg_modes, lg_function, hg_to_lg, lg_blocks, apply_lg_blocks, custom_transform, apply_basis,
)
from .sweep_avg import (  # noqa: F401,E402
    SEQUENTIAL, INTERLACED, SEQUENTIAL_SWEEP, FAST, SLOW, frame_index_map, at_wavelength, average_windows,
    process_sweep,
)
from .window_fit import max_window_radius  # noqa: F401,E402
from .batch_summary import (  # noqa: F401,E402
    PARAMETERS, plane_parameters, fourier_axes, fourier_plane, field_axes, summarise, batch_summary_fourier,
    batch_summary_field,
)
