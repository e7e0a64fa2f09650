"""Oracle for the interface-data steps around findpts_eval (test
infrastructure only: the test suite and bench.py's CPU baseline may use it).

Plain numpy in binary64, written from the paper:
* flux_correct -- Section 2.2 (Mass-Balance): the tentative boundary velocity
  u_hat on the boundary of a subdomain is corrected on the interpolated
  (interface) part by gamma times the unit normal, with gamma the negative
  boundary flux of u_hat divided by the interface area (Eqs. 2-3), so that
  the corrected boundary data carries zero net flux (Eq. 1).
* extrapolate -- Section 2: interface data extrapolated in time to order m
  from the last m values (constant time step), the standard m-th order
  extrapolation weights.
"""
import numpy as np

# m-th order extrapolation to t_{n+1} from values at t_n, t_{n-1}, ... (equal
# steps): the weights of the degree m-1 polynomial through the last m values
EXT_WEIGHTS = {1: (1.0,), 2: (2.0, -1.0), 3: (3.0, -3.0, 1.0)}


def flux_correct(w, n, iface, u):
    """w: (P,) surface quadrature weights (area elements); n: (3, P) unit
    outward normals; iface: (P,) bool, True on the interpolated part; u:
    (3, P) tentative velocity.  Returns (gamma, corrected u)."""
    w = np.asarray(w, dtype=np.float64)
    n = np.asarray(n, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    iface = np.asarray(iface, dtype=bool)
    flux = 0.0
    for p in range(w.shape[0]):
        flux += w[p] * (u[0, p] * n[0, p] + u[1, p] * n[1, p] + u[2, p] * n[2, p])
    area = 0.0
    for p in np.nonzero(iface)[0]:
        area += w[p] * (n[0, p] * n[0, p] + n[1, p] * n[1, p] + n[2, p] * n[2, p])
    gamma = -flux / area if area > 0.0 else 0.0
    out = u.copy()
    out[:, iface] += gamma * n[:, iface]
    return gamma, out


def extrapolate(hist, order):
    """hist: sequence of arrays, most recent first (at least `order`)."""
    wts = EXT_WEIGHTS[order]
    out = np.zeros_like(np.asarray(hist[0], dtype=np.float64))
    for q, c in enumerate(wts):
        out = out + c * np.asarray(hist[q], dtype=np.float64)
    return out
