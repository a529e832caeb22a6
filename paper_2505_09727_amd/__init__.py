"""ESP long-range electrostatics on AMD Instinct MI355X (gfx950).

The compute path is the HIP library libesp.so (C ABI in include/esp.h);
this package only marshals arguments to it (see esp.py). Importing the
package does not load the library; the first call does, and raises if it has
not been built (python -m paper_2505_09727_amd.build).
"""
from .esp import (  # noqa: F401
    EspError,
    Plan,
    Server,
    esp_influence_tables,
    esp_local_kernel,
    esp_plan_query,
    esp_version,
    esp_warm_tables,
    esp_window_coeffs,
    lib,
)
