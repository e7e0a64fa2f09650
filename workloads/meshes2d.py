"""Seeded two-dimensional meshes and query points (quadrilateral spectral
elements of order N; node (i, j) of element e at index [e, j, i]).

* box2d_mesh: affine nx x ny grid of a rectangle, optionally sine-perturbed.
* annulus2d_mesh: ring rho in [r0, r1] with nodes at exact polar positions
  (r -> radius, s -> angle).
* poly_map_mesh2d: a box pushed through a fixed polynomial map of degree 2
  per coordinate (exact in Q_N for N >= 2), for exact-recovery tests.
* overlap2d: two sessions, a square with a square hole and a ring covering
  the hole's edge, with the exact distance to the own boundary (the 2D
  analogue of the two-session 3D case; the paper's Figs. 1 and 6 are of this
  overlapping kind).
* annulus2d_c6 + queries2d_c6: the 2D benchmark (16,384 ring elements of
  order 7, 10^6 area-uniform points plus 1 % outside).
"""
import math
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from .meshes import gll_points


@dataclass
class Mesh2:
    """A mesh of E quadrilateral elements of order N (coordinates per node)."""

    name: str
    N: int
    x: torch.Tensor  # (E, n1, n1) float64, index [e, j, i]
    y: torch.Tensor
    session: Optional[torch.Tensor] = None  # (E,) int32
    delta: Optional[torch.Tensor] = None  # (E, n1, n1) float64

    @property
    def E(self) -> int:
        return int(self.x.shape[0])

    def to(self, device) -> "Mesh2":
        mv = lambda t: None if t is None else t.to(device)
        return Mesh2(self.name, self.N, mv(self.x), mv(self.y), mv(self.session), mv(self.delta))

    def host(self) -> dict:
        cp = lambda t: None if t is None else t.detach().cpu().contiguous().numpy()
        return {"x": cp(self.x), "y": cp(self.y), "session": cp(self.session),
                "delta": cp(self.delta)}


def _nodes_1d(nel, lo, hi, N, device):
    xi = torch.tensor(gll_points(N), dtype=torch.float64, device=device)
    e = torch.arange(nel, dtype=torch.float64, device=device)[:, None]
    return lo + (hi - lo) * ((e + (xi[None, :] + 1.0) * 0.5) / nel)


def box2d_mesh(nx, ny, lo=(0.0, 0.0), hi=(1.0, 1.0), N=5, perturb=0.0, device="cpu",
               name="box2d") -> Mesh2:
    """Element id e = ex + nx ey.  perturb > 0 adds perturb * sin(2 pi x)
    sin(2 pi y) to both coordinates (relative to the unit square; invertible
    for perturb * 4 pi < 1 on unit-sized boxes)."""
    ax = _nodes_1d(nx, lo[0], hi[0], N, device)
    ay = _nodes_1d(ny, lo[1], hi[1], N, device)
    n1 = N + 1
    X = ax[None, :, None, :].expand(ny, nx, n1, n1).reshape(nx * ny, n1, n1)
    Y = ay[:, None, :, None].expand(ny, nx, n1, n1).reshape(nx * ny, n1, n1)
    if perturb:
        s = torch.sin(2 * math.pi * X) * torch.sin(2 * math.pi * Y)
        X, Y = X + perturb * s, Y + perturb * s
    return Mesh2(name, N, X.contiguous(), Y.contiguous())


def annulus2d_mesh(n_rho, n_theta, r0=0.5, r1=1.0, N=7, device="cpu", name="annulus2d") -> Mesh2:
    """Element id e = er + n_rho eth; the seam theta = 2 pi is written as 0."""
    ar = _nodes_1d(n_rho, r0, r1, N, device)
    xi = torch.tensor(gll_points(N), dtype=torch.float64, device=device)
    eth = torch.arange(n_theta, dtype=torch.float64, device=device)[:, None]
    u = torch.remainder(eth + (xi[None, :] + 1.0) * 0.5, float(n_theta))
    ath = (2.0 * math.pi) * (u / n_theta)
    n1 = N + 1
    R = ar[None, :, None, :].expand(n_theta, n_rho, n1, n1).reshape(-1, n1, n1)
    TH = ath[:, None, :, None].expand(n_theta, n_rho, n1, n1).reshape(-1, n1, n1)
    return Mesh2(name, N, (R * torch.cos(TH)).contiguous(), (R * torch.sin(TH)).contiguous())


def phi2(a, b, amp=0.04):
    """The fixed polynomial map of poly_map_mesh2d (degree 2 per coordinate)."""
    return a + amp * (a * a - b * b + a * b), b + amp * (2 * a * b - a * a + b)


def poly_map_mesh2d(nx, ny, N, amp=0.04, device="cpu", name="polymap2d"):
    """Unit-square box mesh with nodes moved by phi2 (one-to-one for
    amp <= 0.05 on [0, 1]^2).  Returns (mesh, phi2)."""
    m = box2d_mesh(nx, ny, N=N, device=device)
    X, Y = phi2(m.x, m.y, amp)
    return Mesh2(name, N, X.contiguous(), Y.contiguous()), phi2


def _delta_square_hole(x, y):
    outer = torch.minimum(1.65 - x.abs(), 1.65 - y.abs())
    dx = torch.clamp(x.abs() - 0.55, min=0.0)
    dy = torch.clamp(y.abs() - 0.55, min=0.0)
    return torch.minimum(outer, torch.sqrt(dx * dx + dy * dy)).clamp(min=0.0)


def _delta_ring(x, y):
    rho = torch.sqrt(x * x + y * y)
    return torch.minimum(rho - 0.5, 1.0 - rho).clamp(min=0.0)


def overlap2d(N=7, device="cpu") -> Mesh2:
    """Session 0: [-1.65, 1.65]^2 on a 33 x 33 grid minus the 11 x 11 hole
    [-0.55, 0.55]^2 (968 elements); session 1: ring rho in [0.5, 1] (8 x 50
    elements).  delta = exact distance to the own session's boundary."""
    n = 33
    full = box2d_mesh(n, n, (-1.65, -1.65), (1.65, 1.65), N=N, device=device)
    ex = torch.arange(n).repeat(n)
    ey = torch.arange(n).repeat_interleave(n)
    keep = (~((ex >= 11) & (ex < 22) & (ey >= 11) & (ey < 22))).to(full.x.device)
    bx, by = full.x[keep], full.y[keep]
    a = annulus2d_mesh(8, 50, 0.5, 1.0, N=N, device=device)
    x = torch.cat([bx, a.x]).contiguous()
    y = torch.cat([by, a.y]).contiguous()
    sess = torch.cat([torch.zeros(bx.shape[0], dtype=torch.int32),
                      torch.ones(a.E, dtype=torch.int32)]).to(x.device)
    delta = torch.cat([_delta_square_hole(bx, by), _delta_ring(a.x, a.y)]).contiguous()
    return Mesh2("overlap2d", N, x, y, sess, delta)


def annulus2d_c6(device="cpu") -> Mesh2:
    """16,384 ring elements of order 7 (256 azimuthal x 64 radial), rho in [0.5, 1]."""
    return annulus2d_mesh(64, 256, 0.5, 1.0, N=7, device=device, name="annulus2d_c6")


def queries2d_c6(n_in=1_000_000, seed=6, device="cpu") -> torch.Tensor:
    """n_in area-uniform points in the ring plus 1 % outside (half in the
    hole rho in [0.4, 0.5), half in the corners of [-1, 1]^2 beyond rho = 1),
    shuffled; shape (n, 2)."""
    rng = np.random.default_rng(seed)
    n_out = n_in // 100
    n_hole = n_out // 2

    def polar(n, a2, b2):
        rho = np.sqrt(rng.uniform(a2, b2, n))
        th = rng.uniform(0.0, 2.0 * math.pi, n)
        return np.stack([rho * np.cos(th), rho * np.sin(th)], axis=1)

    pin = polar(n_in, 0.25, 1.0)
    phole = polar(n_hole, 0.16, 0.25)
    n_corner = n_out - n_hole
    cs = []
    while sum(len(c) for c in cs) < n_corner:
        c = rng.uniform(-1.0, 1.0, (4 * n_corner + 16, 2))
        cs.append(c[(c * c).sum(1) > 1.0])
    pc = np.concatenate(cs)[:n_corner]
    allp = np.concatenate([pin, phole, pc])
    allp = allp[rng.permutation(len(allp))]
    return torch.as_tensor(np.ascontiguousarray(allp), dtype=torch.float64, device=device)
