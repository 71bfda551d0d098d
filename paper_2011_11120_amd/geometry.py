"""Irregular acquisition geometry: Voronoi areal weights of the spatial integral.

For an irregularly sampled integration surface the paper weights each
receiver by the area of its Voronoi cell (Theory section: receiver-dependent
scaling of the kernel columns; Discussion: irregular geometry).  Host-side
preprocessing: the weights feed `mdc_set_kernel`'s per-column weight vector.

The cell areas are computed by assigning every pixel of a fine raster of the
acquisition rectangle to its nearest trace (the definition of a Voronoi cell),
so the area is exact up to the pixels cut by cell boundaries.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree


def voronoi_areas(x, y, bounds=None, pixel=None) -> np.ndarray:
    """Area of each trace's Voronoi cell clipped to `bounds` = (x0, x1, y0, y1).

    bounds defaults to the points' bounding box grown by half the median
    nearest-neighbour spacing; pixel defaults to 1/40 of that spacing.
    """
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    pts = np.stack([x, y], axis=1)
    tree = cKDTree(pts)
    if x.size > 1:
        d, _ = tree.query(pts, k=2)
        spacing = float(np.median(d[:, 1]))
    else:
        spacing = 1.0
    if bounds is None:
        h = spacing / 2
        bounds = (x.min() - h, x.max() + h, y.min() - h, y.max() + h)
    if pixel is None:
        pixel = spacing / 40
    x0, x1, y0, y1 = bounds
    nxp = max(1, int(round((x1 - x0) / pixel)))
    nyp = max(1, int(round((y1 - y0) / pixel)))
    px = x0 + (np.arange(nxp) + 0.5) * (x1 - x0) / nxp
    py = y0 + (np.arange(nyp) + 0.5) * (y1 - y0) / nyp
    area = (x1 - x0) * (y1 - y0) / (nxp * nyp)
    counts = np.zeros(x.size, dtype=np.int64)
    for j0 in range(0, nyp, 256):  # rows of the raster in blocks
        gx, gy = np.meshgrid(px, py[j0:j0 + 256], indexing="ij")
        _, owner = tree.query(np.stack([gx.ravel(), gy.ravel()], axis=1))
        counts += np.bincount(owner, minlength=x.size)
    return counts * area
