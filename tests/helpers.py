"""Test-side closed forms: affine element maps of the box meshes and the
analytic polynomial map of ``workloads.poly_map_mesh``."""
import numpy as np


def box_affine(ex, ey, ez, nxyz, lo, hi, r):
    """x = lo + (hi - lo) * (e + (r + 1)/2) / n per axis (box_mesh layout)."""
    e = np.array([ex, ey, ez], float)
    n = np.asarray(nxyz, float)
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    return lo + (hi - lo) * (e + (np.asarray(r) + 1.0) * 0.5) / n


def box_elem_ids(E, nxyz):
    nx, ny, nz = nxyz
    e = np.arange(E)
    return e % nx, (e // nx) % ny, e // (nx * ny)


def phi_np(x, y, z, amp=0.04):
    return (x + amp * (y * y - 0.5 * x * z + x * x * y),
            y + amp * (z * z * x - 0.3 * y * y + 0.5 * x * z),
            z + amp * (x * x - y * z * z + 0.2 * x * y))


def dphi_np(x, y, z, amp=0.04):
    """Jacobian of phi_np, rows = components, columns = d/dx, d/dy, d/dz."""
    return np.array([
        [1 + amp * (-0.5 * z + 2 * x * y), amp * (2 * y + x * x), amp * (-0.5 * x)],
        [amp * (z * z + 0.5 * z), 1 + amp * (-0.6 * y), amp * (2 * z * x + 0.5 * x)],
        [amp * (2 * x + 0.2 * y), amp * (-z * z + 0.2 * x), 1 + amp * (-2 * y * z)],
    ])
