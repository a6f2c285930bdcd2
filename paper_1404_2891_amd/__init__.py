"""MI355X (gfx950) non-Hermitian FEAST: the Cauchy-integral accelerator and the R-FEAST /
Bi-FEAST iterations of Tang, Kestyn and Polizzi, as a HIP library with a thin ctypes binding."""
from .binding import (MLP, Feast, FeastBatch, FeastError, autotune, m0_from_estimate, set_panel_rows, IterateResult, contour_inside, contour_nodes, empty_cm, multi_domain, partition_grid, rectangle, lib, library_path,  # noqa: F401
                      polygon, reduced_eig, to_device, workspace_size)
