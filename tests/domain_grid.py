"""A spectrum for multi-domain runs: eigenvalues inside the square region [-1, 1]^2 placed in the
cells of a 6 x 6 grid away from the cell edges (so that every tile edge, a cell edge, has a gap
around it), and the rest outside the region.  Inputs only: no part of the method's arithmetic."""
import numpy as np

import pencils

REGION = (-1.0, 1.0, -1.0, 1.0)
GRID = (6, 6)


def grid_spectrum(n, m_in, seed, margin=0.3):
    return pencils.grid_spectrum(np.random.default_rng(seed), n, m_in, REGION, GRID, margin)


def in_region(lam):
    x0, x1, y0, y1 = REGION
    return (lam.real > x0) & (lam.real < x1) & (lam.imag > y0) & (lam.imag < y1)
