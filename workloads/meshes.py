"""Seeded synthetic meshes, query points and fields (see the package docstring).

Every generator is deterministic: the geometry is closed-form and all random
draws come from ``numpy.random.default_rng(seed)`` (PCG64).  Tensors are
float64 (int32 for integer data) and can be built on any torch device; the
oracle receives host copies of exactly the arrays the GPU path receives.

Workloads (the paper's meshes are not available, so these stand in for them):

* ``cube_c1``: unit cube, 4x4x4 elements, N = 5, nodes moved by
  0.05 * sin(2 pi x) sin(2 pi y) sin(2 pi z) on all three coordinates.
* ``annulus_c2``: cylinder-in-box annulus rho in [0.5, 1], z in [0, 1],
  64 azimuthal x 16 radial x 16 axial = 16,384 elements, N = 7, nodes at
  exact polar positions.
* ``overlap_c3``: two overlapping sessions (a box with a square hole,
  19,360 elements, and an annulus, 8,000 elements, N = 7) with the exact
  distance to each session's own boundary as the nodal discriminator field.
  This reproduces the shape of the paper's strong-scaling case (Section 3.1:
  E = 20,000 at N = 7, interface points exchanged every Schwarz iteration).
* ``big_box_c5``: 100x50x40 = 200,000 perturbed box elements, N = 7.
"""

from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch


# --------------------------------------------------------------------------
# GLL positions used to place mesh nodes (numpy's Legendre routines).
# --------------------------------------------------------------------------
def gll_points(N: int) -> np.ndarray:
    """GLL points on [-1, 1]: the endpoints and the roots of P_N'."""
    if N < 1:
        raise ValueError("N must be >= 1")
    inner = np.polynomial.legendre.Legendre.basis(N).deriv().roots()
    pts = np.concatenate([[-1.0], np.sort(np.real(inner)), [1.0]])
    # symmetric placement so mirrored elements get mirrored nodes
    pts = 0.5 * (pts - pts[::-1])
    if N % 2 == 0:
        pts[N // 2] = 0.0
    return pts


@dataclass
class Mesh:
    """A mesh of E hexahedral elements of order N (coordinates per node)."""

    name: str
    N: int
    x: torch.Tensor  # (E, n1, n1, n1) float64, index [e, k, j, i]
    y: torch.Tensor
    z: torch.Tensor
    session: Optional[torch.Tensor] = None  # (E,) int32
    delta: Optional[torch.Tensor] = None  # (E, n1, n1, n1) float64

    @property
    def E(self) -> int:
        return int(self.x.shape[0])

    @property
    def n1(self) -> int:
        return self.N + 1

    def to(self, device) -> "Mesh":
        mv = lambda t: None if t is None else t.to(device)
        return Mesh(self.name, self.N, mv(self.x), mv(self.y), mv(self.z),
                    mv(self.session), mv(self.delta))

    def host(self) -> dict:
        """Contiguous host numpy copies (what the oracle receives)."""
        out = {"x": self.x.detach().cpu().contiguous().numpy(),
               "y": self.y.detach().cpu().contiguous().numpy(),
               "z": self.z.detach().cpu().contiguous().numpy()}
        out["session"] = (None if self.session is None else
                          self.session.detach().cpu().contiguous().numpy())
        out["delta"] = (None if self.delta is None else
                        self.delta.detach().cpu().contiguous().numpy())
        return out


def _nodes_1d(nel: int, lo: float, hi: float, N: int, device) -> torch.Tensor:
    """Node positions along one axis, shape (nel, n1).

    Written as lo + (hi - lo) * (e + (xi + 1) / 2) / nel so that the last node
    of element e and the first node of element e + 1 are bit-identical.
    """
    xi = torch.tensor(gll_points(N), dtype=torch.float64, device=device)
    e = torch.arange(nel, dtype=torch.float64, device=device)[:, None]
    return lo + (hi - lo) * ((e + (xi[None, :] + 1.0) * 0.5) / nel)


def _tensor_grid(ax, ay, az):
    """Broadcast 1-D node tables into (nz, ny, nx, n1, n1, n1) arrays."""
    nx, n1 = ax.shape
    ny, nz = ay.shape[0], az.shape[0]
    X = ax[None, None, :, None, None, :].expand(nz, ny, nx, n1, n1, n1)
    Y = ay[None, :, None, None, :, None].expand(nz, ny, nx, n1, n1, n1)
    Z = az[:, None, None, :, None, None].expand(nz, ny, nx, n1, n1, n1)
    return X, Y, Z


def box_mesh(nx, ny, nz, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), N=5,
             device="cpu", name="box") -> Mesh:
    """Affine box mesh; element id e = ex + nx*(ey + ny*ez)."""
    ax = _nodes_1d(nx, lo[0], hi[0], N, device)
    ay = _nodes_1d(ny, lo[1], hi[1], N, device)
    az = _nodes_1d(nz, lo[2], hi[2], N, device)
    X, Y, Z = _tensor_grid(ax, ay, az)
    E, n1 = nx * ny * nz, N + 1
    sh = (E, n1, n1, n1)
    return Mesh(name, N, X.reshape(sh).contiguous(), Y.reshape(sh).contiguous(),
                Z.reshape(sh).contiguous())


def _perturb(m: Mesh, amp: float, fx: float, fy: float, fz: float) -> Mesh:
    """X <- X + amp * sin(fx pi x) sin(fy pi y) sin(fz pi z) * (1, 1, 1)."""
    s = (torch.sin(fx * math.pi * m.x) * torch.sin(fy * math.pi * m.y)
         * torch.sin(fz * math.pi * m.z))
    return Mesh(m.name, m.N, m.x + amp * s, m.y + amp * s, m.z + amp * s,
                m.session, m.delta)


def cube_c1(device="cpu", perturb: float = 0.05) -> Mesh:
    """Unit cube, 4x4x4 elements of order 5, sine-perturbed nodes.

    The perturbation vanishes on the cube faces, so the domain stays the
    unit cube; det(I + 0.05 (1,1,1) grad(s)^T) >= 1 - 0.05*2*pi*sqrt(3) > 0,
    so every element map stays invertible.
    """
    m = box_mesh(4, 4, 4, N=5, device=device, name="cube_c1")
    return _perturb(m, perturb, 2.0, 2.0, 2.0) if perturb else m


def annulus_mesh(n_rho, n_theta, n_z, r0=0.5, r1=1.0, z0=0.0, z1=1.0, N=7,
                 device="cpu", name="annulus") -> Mesh:
    """Annular (cylinder-in-box) mesh with nodes at exact polar positions.

    Reference axes: r -> radius, s -> angle, t -> axial (right-handed, so
    the map has a positive Jacobian).  Element id e = er + n_rho*(eth +
    n_theta*ez).  The seam theta = 2 pi is written as theta = 0 so that the
    first and last azimuthal elements share bit-identical nodes.
    """
    ar = _nodes_1d(n_rho, r0, r1, N, device)
    xi = torch.tensor(gll_points(N), dtype=torch.float64, device=device)
    eth = torch.arange(n_theta, dtype=torch.float64, device=device)[:, None]
    u = torch.remainder(eth + (xi[None, :] + 1.0) * 0.5, float(n_theta))
    ath = (2.0 * math.pi) * (u / n_theta)
    az = _nodes_1d(n_z, z0, z1, N, device)
    R, TH, Z = _tensor_grid(ar, ath, az)
    E, n1 = n_rho * n_theta * n_z, N + 1
    sh = (E, n1, n1, n1)
    X = (R * torch.cos(TH)).reshape(sh).contiguous()
    Y = (R * torch.sin(TH)).reshape(sh).contiguous()
    return Mesh(name, N, X, Y, Z.reshape(sh).contiguous())


def annulus_c2(device="cpu") -> Mesh:
    """16,384 annular elements of order 7 (64 azimuthal x 16 radial x 16 axial)."""
    return annulus_mesh(16, 64, 16, 0.5, 1.0, 0.0, 1.0, N=7, device=device,
                        name="annulus_c2")


def big_box_c5(device="cpu") -> Mesh:
    """200,000 sine-perturbed elements of order 7 on [0,2]x[0,1]x[0,0.8].

    Amplitude 0.02 with frequencies (pi, 2 pi, 2.5 pi): 0.02*(1+2+2.5)*pi
    < 1, so every element map stays invertible; the perturbation vanishes on
    the domain faces.
    """
    m = box_mesh(100, 50, 40, (0.0, 0.0, 0.0), (2.0, 1.0, 0.8), N=7,
                 device=device, name="big_box_c5")
    return _perturb(m, 0.02, 1.0, 2.0, 2.5)


def spiral_element(N=15, turns=1.5, pitch=0.25, half=0.2, device="cpu") -> Mesh:
    """One element of order N shaped as a thick spiral sheet, a stand-in for
    the paper's N = 15 spiral (its geometry is not given).  Reference r runs
    along the spiral, s across the sheet, t along z: the node at (r, s, t)
    sits at angle th = turns * pi * (r + 1), radius 1 + pitch * th + half * s,
    height t / 2.  Successive turns are 2 pi pitch apart (1.57 by default),
    more than the sheet thickness 2 half (0.4), so the map is one-to-one,
    while a point between the sheets sees a local minimum of the distance on
    every turn it faces."""
    z = torch.tensor(gll_points(N), dtype=torch.float64, device=device)
    r = z[None, None, :].expand(N + 1, N + 1, N + 1)
    s_ = z[None, :, None].expand(N + 1, N + 1, N + 1)
    t = z[:, None, None].expand(N + 1, N + 1, N + 1)
    th = turns * math.pi * (r + 1.0)
    rad = 1.0 + pitch * th + half * s_
    X = (rad * torch.cos(th))[None].contiguous()
    Y = (rad * torch.sin(th))[None].contiguous()
    Zc = (0.5 * t)[None].contiguous()
    return Mesh("spiral", N, X, Y, Zc)


def poly_map_mesh(nx, ny, nz, N, amp=0.04, device="cpu", name="polymap"):
    """Box mesh pushed through a fixed polynomial map Phi (exact in Q_N).

    Phi has degree <= 2 in each variable, so for N >= 2 every element map is
    Phi composed with an axis-aligned affine map, a polynomial of degree <= N
    in each reference variable that the nodal basis reproduces exactly.
    Returns (mesh, phi) where phi(x, y, z) evaluates the map in closed form
    (the exact-recovery tests use phi to generate x* = x^e(r_true)).
    """
    if N < 2:
        raise ValueError("poly_map_mesh needs N >= 2")
    m = box_mesh(nx, ny, nz, N=N, device=device, name=name)

    def phi(x, y, z):
        return (x + amp * (y * y - 0.5 * x * z + x * x * y),
                y + amp * (z * z * x - 0.3 * y * y + 0.5 * x * z),
                z + amp * (x * x - y * z * z + 0.2 * x * y))

    X, Y, Z = phi(m.x, m.y, m.z)
    return Mesh(name, N, X.contiguous(), Y.contiguous(), Z.contiguous()), phi


# --------------------------------------------------------------------------
# Two overlapping sessions with the distance-to-own-boundary field.
# --------------------------------------------------------------------------
def _box_with_hole(device, N):
    """Box [-1.65,1.65]^2 x [0,1], 33x33x20 cells minus the 11x11 hole."""
    n, nzl = 33, 20
    full = box_mesh(n, n, nzl, (-1.65, -1.65, 0.0), (1.65, 1.65, 1.0), N=N,
                    device=device)
    ex = torch.arange(n).repeat(n * nzl)
    ey = torch.arange(n).repeat_interleave(n).repeat(nzl)
    keep = ~((ex >= 11) & (ex < 22) & (ey >= 11) & (ey < 22))
    keep = keep.to(full.x.device)
    return Mesh("box_hole", N, full.x[keep].contiguous(),
                full.y[keep].contiguous(), full.z[keep].contiguous())


def _delta_box(x, y, z):
    outer = torch.minimum(1.65 - x.abs(), 1.65 - y.abs())
    dx = torch.clamp(x.abs() - 0.55, min=0.0)
    dy = torch.clamp(y.abs() - 0.55, min=0.0)
    hole = torch.sqrt(dx * dx + dy * dy)
    walls = torch.minimum(z, 1.0 - z)
    return torch.minimum(torch.minimum(outer, hole), walls).clamp(min=0.0)


def _delta_annulus(x, y, z):
    rho = torch.sqrt(x * x + y * y)
    d = torch.minimum(rho - 0.5, 1.0 - rho)
    return torch.minimum(d, torch.minimum(z, 1.0 - z)).clamp(min=0.0)


def overlap_c3(device="cpu", N=7) -> Mesh:
    """Session 0: box with a square hole (19,360 elements); session 1: annulus
    rho in [0.5, 1] (8,000 elements).  delta = exact distance to the own
    session's boundary, sampled at the nodes."""
    b = _box_with_hole(device, N)
    a = annulus_mesh(8, 50, 20, 0.5, 1.0, 0.0, 1.0, N=N, device=device)
    x = torch.cat([b.x, a.x]).contiguous()
    y = torch.cat([b.y, a.y]).contiguous()
    z = torch.cat([b.z, a.z]).contiguous()
    sess = torch.cat([torch.zeros(b.E, dtype=torch.int32),
                      torch.ones(a.E, dtype=torch.int32)]).to(x.device)
    delta = torch.cat([_delta_box(b.x, b.y, b.z),
                       _delta_annulus(a.x, a.y, a.z)]).contiguous()
    return Mesh("overlap_c3", N, x, y, z, sess, delta)


# --------------------------------------------------------------------------
# Query points.
# --------------------------------------------------------------------------
def _t(a, device):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64,
                           device=device)


def queries_uniform_box(n, lo, hi, seed, device="cpu") -> torch.Tensor:
    rng = np.random.default_rng(seed)
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    return _t(lo + (hi - lo) * rng.random((n, 3)), device)


def queries_c1(n=10_000, seed=1, device="cpu") -> torch.Tensor:
    """n points uniform in [0, 1)^3, shape (n, 3), xyz interleaved."""
    return queries_uniform_box(n, (0, 0, 0), (1, 1, 1), seed, device)


def queries_c2(n_in=1_000_000, seed=2, device="cpu") -> torch.Tensor:
    """Annulus queries: n_in area-uniform in the annulus plus 1 % outside.

    Outside points: half in the hole rho in [0.4, 0.5), half in the box
    corners rho > 1 of [-1,1]^2 (both have z uniform in [0,1)), and 1 % of
    those beyond the box (z in [1.2, 1.5)).  The concatenation is shuffled.
    """
    rng = np.random.default_rng(seed)
    n_out = n_in // 100
    n_far = max(n_out // 100, 1)
    n_hole = (n_out - n_far) // 2
    n_corner = n_out - n_far - n_hole

    def polar(n, a2, b2):
        rho = np.sqrt(rng.uniform(a2, b2, n))
        th = rng.uniform(0.0, 2.0 * math.pi, n)
        return np.stack([rho * np.cos(th), rho * np.sin(th),
                         rng.random(n)], axis=1)

    pin = polar(n_in, 0.25, 1.0)
    phole = polar(n_hole, 0.16, 0.25)
    corners = []
    while sum(len(c) for c in corners) < n_corner:
        c = rng.uniform(-1.0, 1.0, (4 * n_corner + 16, 2))
        corners.append(c[(c * c).sum(1) > 1.0])
    c = np.concatenate(corners)[:n_corner]
    pcorner = np.concatenate([c, rng.random((n_corner, 1))], axis=1)
    pfar = np.stack([rng.uniform(-1, 1, n_far), rng.uniform(-1, 1, n_far),
                     rng.uniform(1.2, 1.5, n_far)], axis=1)
    allp = np.concatenate([pin, phole, pcorner, pfar])
    allp = allp[rng.permutation(len(allp))]
    return _t(allp, device)


def queries_c3(kind="faces", n=1_200_000, seed=3, device="cpu"):
    """Interface queries of the two-session case, with their session tags.

    kind="nodes" is not generated here: the interface GLL nodes are a
    subset of the mesh nodes, selected by ``c3_interface_nodes``.
    kind="faces": n points uniform on the interface surfaces, i.e. the four
    hole faces of the box session (x or y = +-0.55, tagged 0) and the outer
    cylinder rho = 1 of the annulus session (tagged 1), in proportion to
    their GLL node counts (880 : 1000 faces).
    Returns (points (n, 3), tags (n,) int32).
    """
    rng = np.random.default_rng(seed)
    n0 = int(round(n * 880 / 1880))
    n1 = n - n0
    side = rng.integers(0, 4, n0)
    u = rng.uniform(-0.55, 0.55, n0)
    zz = rng.random(n0)
    xb = np.where(side == 0, 0.55, np.where(side == 1, -0.55, u))
    yb = np.where(side == 2, 0.55, np.where(side == 3, -0.55, u))
    th = rng.uniform(0.0, 2.0 * math.pi, n1)
    pa = np.stack([np.cos(th), np.sin(th), rng.random(n1)], axis=1)
    pts = np.concatenate([np.stack([xb, yb, zz], axis=1), pa])
    tags = np.concatenate([np.zeros(n0, np.int32), np.ones(n1, np.int32)])
    perm = rng.permutation(n)
    return (_t(pts[perm], device),
            torch.as_tensor(tags[perm], dtype=torch.int32, device=device))


def queries_c5(n=20_000_000, seed=5, device="cpu") -> torch.Tensor:
    """Points clustered near 8 random interior spheres of the large box.

    Centres uniform in [0.2, 1.8] x [0.2, 0.8] x [0.2, 0.6] (the domain shrunk
    by 0.2), radii U(0.1, 0.3); each point is uniform on its sphere, moved
    along the normal by N(0, (0.5 h)^2) with h = 0.02 (points outside the
    domain are kept).  Shape (n, 3).
    """
    rng = np.random.default_rng(seed)
    cen = rng.uniform((0.2, 0.2, 0.2), (1.8, 0.8, 0.6), (8, 3))
    rad = rng.uniform(0.1, 0.3, 8)
    which = rng.integers(0, 8, n)
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    r = rad[which] + rng.normal(0.0, 0.5 * 0.02, n)
    return _t(cen[which] + r[:, None] * d, device)


def c3_interface_nodes(mesh: Mesh):
    """All GLL nodes of the two-session interface faces, tagged by session.

    Box session (tag 0): element faces lying on the hole boundary
    (|x| = 0.55 with |y| <= 0.55, or |y| = 0.55 with |x| <= 0.55).  Annulus
    session (tag 1): element faces on the outer cylinder rho = 1.  Faces are
    recognised from their node positions.  Returns (points (P, 3), tags (P,)).
    """
    N, eps = mesh.N, 1e-12
    X, Y, Z, S = mesh.x, mesh.y, mesh.z, mesh.session
    slices = [(Ellipsis, 0), (Ellipsis, N), (slice(None), slice(None), 0),
              (slice(None), slice(None), N), (slice(None), 0), (slice(None), N)]
    pts, tags = [], []
    for sl in slices:
        fx, fy, fz = X[sl], Y[sl], Z[sl]
        ax, ay = fx.abs(), fy.abs()
        on_x = ((ax - 0.55).abs() < eps).all(dim=(1, 2)) & (ay <= 0.55 + eps).all(dim=(1, 2))
        on_y = ((ay - 0.55).abs() < eps).all(dim=(1, 2)) & (ax <= 0.55 + eps).all(dim=(1, 2))
        rho = torch.sqrt(fx * fx + fy * fy)
        on_r = ((rho - 1.0).abs() < 1e-12).all(dim=(1, 2))
        for sel, tag in (((on_x | on_y) & (S == 0), 0), (on_r & (S == 1), 1)):
            P = torch.stack([fx[sel], fy[sel], fz[sel]], -1).reshape(-1, 3)
            pts.append(P)
            tags.append(torch.full((P.shape[0],), tag, dtype=torch.int32,
                                   device=P.device))
    return torch.cat(pts).contiguous(), torch.cat(tags).contiguous()


def gll_weights(N: int) -> np.ndarray:
    """GLL quadrature weights 2 / (N (N+1) P_N(x_i)^2) at gll_points(N)."""
    x = gll_points(N)
    pn = np.polynomial.legendre.legval(x, [0.0] * N + [1.0])
    return 2.0 / (N * (N + 1) * pn * pn)


def c3_interface_quadrature(mesh: Mesh):
    """The two-session interface of the overlap mesh as boundary quadrature
    data: points, session tags, unit normals pointing out of the owning
    session, and surface weights (tensor GLL weights times the face area / 4;
    the faces of each kind all have the same area: 0.1 x 0.05 on the hole,
    (2 pi / 50) x 0.05 on the cylinder).  Returns torch tensors
    (pts (P, 3), tags (P,), normals (3, P), weights (P,))."""
    N, eps = mesh.N, 1e-12
    X, Y, Z, S = mesh.x, mesh.y, mesh.z, mesh.session
    wq = torch.as_tensor(gll_weights(N), dtype=torch.float64, device=X.device)
    w2 = (wq[:, None] * wq[None, :]) / 4.0
    slices = [(Ellipsis, 0), (Ellipsis, N), (slice(None), slice(None), 0),
              (slice(None), slice(None), N), (slice(None), 0), (slice(None), N)]
    pts, tags, nrm, wts = [], [], [], []
    for sl in slices:
        fx, fy, fz = X[sl], Y[sl], Z[sl]
        ax, ay = fx.abs(), fy.abs()
        on_x = ((ax - 0.55).abs() < eps).all(dim=(1, 2)) & (ay <= 0.55 + eps).all(dim=(1, 2))
        on_y = ((ay - 0.55).abs() < eps).all(dim=(1, 2)) & (ax <= 0.55 + eps).all(dim=(1, 2))
        rho = torch.sqrt(fx * fx + fy * fy)
        on_r = ((rho - 1.0).abs() < 1e-12).all(dim=(1, 2))
        for sel, tag, kind in (((on_x & (S == 0)), 0, "x"), ((on_y & (S == 0)), 0, "y"),
                               ((on_r & (S == 1)), 1, "r")):
            if not bool(sel.any()):
                continue
            px, py, pz = fx[sel], fy[sel], fz[sel]
            P = torch.stack([px, py, pz], -1).reshape(-1, 3)
            if kind == "x":      # hole face: the box session lies away from the hole
                nv = torch.stack([-torch.sign(px), 0 * px, 0 * px], 0)
                area = 0.1 * 0.05
            elif kind == "y":
                nv = torch.stack([0 * py, -torch.sign(py), 0 * py], 0)
                area = 0.1 * 0.05
            else:                # outer cylinder of the annulus session
                r = torch.sqrt(px * px + py * py)
                nv = torch.stack([px / r, py / r, 0 * px], 0)
                area = (2.0 * math.pi / 50.0) * 0.05
            pts.append(P)
            tags.append(torch.full((P.shape[0],), tag, dtype=torch.int32, device=P.device))
            nrm.append(nv.reshape(3, -1))
            wts.append((area * w2).expand(px.shape).reshape(-1))
    return (torch.cat(pts).contiguous(), torch.cat(tags).contiguous(),
            torch.cat(nrm, dim=1).contiguous(), torch.cat(wts).contiguous())


# --------------------------------------------------------------------------
# Nodal fields.
# --------------------------------------------------------------------------
def _poly_eval(coef: np.ndarray, x, y, z):
    """Sum over a+b+c <= d of coef[a,b,c] x^a y^b z^c (Horner in z)."""
    d = coef.shape[0] - 1
    xp = [torch.ones_like(x)]
    yp = [torch.ones_like(y)]
    for _ in range(d):
        xp.append(xp[-1] * x)
        yp.append(yp[-1] * y)
    acc = torch.zeros_like(x)
    for a in range(d + 1):
        for b in range(d + 1 - a):
            cz = torch.full_like(z, float(coef[a, b, d - a - b]))
            for c in range(d - a - b - 1, -1, -1):
                cz = cz * z + float(coef[a, b, c])
            acc = acc + (xp[a] * yp[b]) * cz
    return acc


def poly_fields(mesh: Mesh, nf: int, degree: int = 7, seed: int = 0):
    """nf random polynomials of total degree <= degree in (x, y, z),
    coefficients U(-1, 1), sampled at the mesh nodes.  Returns a list of
    (E, n1, n1, n1) float64 tensors and the coefficient arrays."""
    rng = np.random.default_rng(seed)
    fields, coefs = [], []
    for _ in range(nf):
        c = np.zeros((degree + 1,) * 3)
        for a in range(degree + 1):
            for b in range(degree + 1 - a):
                for cc in range(degree + 1 - a - b):
                    c[a, b, cc] = rng.uniform(-1.0, 1.0)
        coefs.append(c)
        fields.append(_poly_eval(c, mesh.x, mesh.y, mesh.z).contiguous())
    return fields, coefs


def ref_poly_fields(mesh: Mesh, nf: int, seed: int = 0):
    """Fields that are, on each element, a random polynomial of degree <= N
    in each reference variable, sampled at the GLL nodes.

    Returns (fields, coef) with coef of shape (nf, E, n1, n1, n1): the
    monomial coefficients c[f, e, c, b, a] of r^a s^b t^c, so the exact
    value at (e, r, s, t) is sum c * r^a s^b t^c (used as a closed form by
    the interpolation tests).
    """
    rng = np.random.default_rng(seed)
    N, E, n1 = mesh.N, mesh.E, mesh.n1
    xi = gll_points(N)
    coef = rng.uniform(-1.0, 1.0, (nf, E, n1, n1, n1))
    P = np.vander(xi, n1, increasing=True)  # P[i, a] = xi_i^a
    # value[f,e,k,j,i] = sum_{c,b,a} coef[f,e,c,b,a] P[k,c] P[j,b] P[i,a]
    vals = np.einsum("fecba,kc,jb,ia->fekji", coef, P, P, P, optimize=True)
    dev = mesh.x.device
    return [torch.as_tensor(np.ascontiguousarray(v), device=dev) for v in vals], coef
