"""Test-side closed forms: affine element maps of the box meshes and the
analytic polynomial map of ``workloads.poly_map_mesh``, and exact points on
the spiral element through a library interpolant."""
import numpy as np
import workloads as w


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


def box_surface(lo, hi, N=4):
    """GLL nodes on the 6 faces of an axis-aligned box: points (3, P),
    weights (P,) = tensor GLL weights x face Jacobian, outward normals (3, P).
    GLL quadrature of degree 2N-1 is exact for the low-degree fields of the
    interface tests."""
    import oracle
    z, wq = oracle.gll(N)
    pts, ws, ns = [], [], []
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    for ax in range(3):
        a, b = [d for d in range(3) if d != ax]
        ja, jb = 0.5 * (hi[a] - lo[a]), 0.5 * (hi[b] - lo[b])
        for side, val in ((-1.0, lo[ax]), (1.0, hi[ax])):
            for i in range(N + 1):
                for j in range(N + 1):
                    p = np.zeros(3)
                    p[ax] = val
                    p[a] = lo[a] + ja * (z[i] + 1)
                    p[b] = lo[b] + jb * (z[j] + 1)
                    nn = np.zeros(3)
                    nn[ax] = side
                    pts.append(p)
                    ws.append(wq[i] * wq[j] * ja * jb)
                    ns.append(nn)
    return np.array(pts).T, np.array(ws), np.array(ns).T


def spiral_exact_points(m, P, seed):
    """P points x^e(r_true), r_true uniform in [-1, 1]^3, on element 0 of
    mesh m, through scipy's barycentric Lagrange interpolation on the GLL
    nodes: the tensor interpolant evaluated by a library routine, independent
    of the oracle's basis and map.  Returns (points (P, 3), r_true (P, 3))."""
    from scipy.interpolate import BarycentricInterpolator
    N = m.N
    rng = np.random.default_rng(seed)
    rt = rng.uniform(-1, 1, (P, 3))
    B = BarycentricInterpolator(w.gll_points(N), np.eye(N + 1))
    L = [B(rt[:, d]) for d in range(3)]
    hd = m.host()
    pts = np.stack([np.einsum("pi,pj,pk,kji->p", L[0], L[1], L[2],
                              hd[c][:(N + 1) ** 3].reshape(N + 1, N + 1, N + 1))
                    for c in "xyz"], 1)
    return pts, rt
