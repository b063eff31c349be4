"""Seeded synthetic inputs for the collapse-time path.

This package makes the *inputs* that both the product path and the oracle
consume: Gaussian linear density fields with a CDM spectrum, the six
components of the Hessian of the smoothed potential at each smoothing radius
(the stand-in for the upstream Initialization + FFT stages, Sec. 3 of the
paper), the linear growth table D(a) on its grid of scale factors (Sec. 3),
and the knot grids of the collapse table (Sec. 3, table coordinates).

It holds none of the collapse method's arithmetic: no eigenvalues, no
collapse condition, no interpolation.  Random numbers are drawn with numpy's
PCG64 from an explicit seed; FFTs run with torch on whatever device the caller
names.
"""

from .cosmo import Cosmology, bbks_transfer, power_spectrum, sigma_tophat, sigma_gauss
from .fields import (HESSIAN_COMPONENTS, white_noise, hessian_slabs, hessian_radius,
                     grid_sigma_gauss, log_radii)
from .growth import growth_table
from .tables import table_knots, table_grid_hessians
from .configs import CONFIGS, config

__all__ = [
    "Cosmology", "bbks_transfer", "power_spectrum", "sigma_tophat", "sigma_gauss",
    "HESSIAN_COMPONENTS", "white_noise", "hessian_slabs", "hessian_radius",
    "grid_sigma_gauss", "log_radii", "growth_table", "table_knots",
    "table_grid_hessians", "CONFIGS", "config",
]
