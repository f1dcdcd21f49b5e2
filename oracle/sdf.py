"""Signed-distance-field lookups (the paper gives no grid semantics).

Reading: the grid is node-sampled, value[iy][ix] (2-D) or value[iz][iy][ix]
(3-D) holds the distance at origin + (ix, iy[, iz]) * cell.  A query is
mapped to u = (x - origin) / cell per axis, clamped to [0, G-1]; the cell
index is i = min(floor(u), G-2) and t = u - i; the value is the bilinear
(trilinear) interpolation of the cell's corner values.  Outside the grid
the clamp holds the boundary value, which keeps the field continuous.
Grid values are FP32 in memory and promoted to FP64 here.
"""
from __future__ import annotations

import numpy as np


def _axis(coord, origin, cell, g):
    u = (coord - origin) / cell
    u = np.clip(u, 0.0, g - 1.0)
    i = np.minimum(np.floor(u), g - 2).astype(np.int64)
    return i, u - i


def bilinear(grid, origin, cell, pts):
    """grid [gy,gx] float32; pts [..., 2] (x, y) -> interpolated values."""
    grid = np.asarray(grid, dtype=np.float64)
    gy, gx = grid.shape
    ix, tx = _axis(pts[..., 0], origin[0], cell, gx)
    iy, ty = _axis(pts[..., 1], origin[1], cell, gy)
    v00 = grid[iy, ix]
    v01 = grid[iy, ix + 1]
    v10 = grid[iy + 1, ix]
    v11 = grid[iy + 1, ix + 1]
    return ((1 - ty) * ((1 - tx) * v00 + tx * v01)
            + ty * ((1 - tx) * v10 + tx * v11))


def trilinear(grid, origin, cell, pts):
    """grid [gz,gy,gx] float32; pts [..., 3] (x, y, z) -> values."""
    grid = np.asarray(grid, dtype=np.float64)
    gz, gy, gx = grid.shape
    ix, tx = _axis(pts[..., 0], origin[0], cell, gx)
    iy, ty = _axis(pts[..., 1], origin[1], cell, gy)
    iz, tz = _axis(pts[..., 2], origin[2], cell, gz)
    out = 0.0
    for dz in (0, 1):
        wz = tz if dz else 1 - tz
        for dy in (0, 1):
            wy = ty if dy else 1 - ty
            for dx in (0, 1):
                wx = tx if dx else 1 - tx
                out = out + wz * wy * wx * grid[iz + dz, iy + dy, ix + dx]
    return out
