"""Seeded serving workload: many resident meshes of different size and order,
and a stream of requests of log-uniform size arriving as a Poisson process.

Mesh i (seed 4): E_i = floor(exp U(ln e_min, ln e_max)) rounded to a near-
cubic element grid, N_i uniform in `orders`; even i is a unit cube with the
sine perturbation of the unit-cube workload, odd i an annulus (rho in
[0.5, 1], z in [0, 1], nodes at exact polar positions).  Each mesh carries
`nfields` random polynomial fields of total degree 7.

Request j (seed 40): mesh uniform, P = floor(exp U(ln p_min, ln p_max))
points uniform in the mesh's domain (area-uniform in the annulus), n_f
uniform in 1..nf_max distinct field ids, and an exponential gap of mean 1
before it (scale by 1 / rate for a Poisson stream of that rate).
"""
import math
from dataclasses import dataclass, field
from typing import List

import numpy as np
import torch

from .meshes import Mesh, _perturb, annulus_mesh, box_mesh, poly_fields


@dataclass
class ServedMesh:
    mesh: Mesh
    kind: str  # "box" or "annulus"
    fields: List[torch.Tensor] = field(default_factory=list)


def _box_dims(E):
    n = max(1, round(E ** (1.0 / 3.0)))
    return n, n, max(1, round(E / (n * n)))


def _annulus_dims(E):
    h = (math.pi * 0.75 / E) ** (1.0 / 3.0)  # annulus volume pi (1 - 0.25) * 1
    return max(1, round(0.5 / h)), max(4, round(2.0 * math.pi * 0.75 / h)), max(1, round(1.0 / h))


def serving_meshes(count=16, e_min=500, e_max=50_000, orders=(5, 7, 9), nfields=5, seed=4,
                   device="cpu") -> List[ServedMesh]:
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        E = int(math.exp(rng.uniform(math.log(e_min), math.log(e_max))))
        N = int(rng.choice(orders))
        if i % 2 == 0:
            nx, ny, nz = _box_dims(E)
            m = _perturb(box_mesh(nx, ny, nz, N=N, device=device, name=f"box{i}"),
                         0.05, 2.0, 2.0, 2.0)
            kind = "box"
        else:
            nr, nt, nz = _annulus_dims(E)
            m = annulus_mesh(nr, nt, nz, N=N, device=device, name=f"annulus{i}")
            kind = "annulus"
        f, _ = poly_fields(m, nfields, degree=7, seed=1000 * seed + i)
        out.append(ServedMesh(m, kind, f))
    return out


def serving_requests(n, nmesh, p_min=1_000, p_max=1_000_000, nf_max=5, seed=40):
    rng = np.random.default_rng(seed)
    reqs = []
    for _ in range(n):
        mesh = int(rng.integers(0, nmesh))
        P = int(math.exp(rng.uniform(math.log(p_min), math.log(p_max))))
        nf = int(rng.integers(1, nf_max + 1))
        fids = sorted(rng.choice(nf_max, nf, replace=False).tolist())
        reqs.append({"mesh": mesh, "P": P, "field_ids": fids, "gap": float(rng.exponential(1.0)),
                     "seed": int(rng.integers(0, 2 ** 31))})
    return reqs


def serving_points(kind, P, seed, device="cpu") -> torch.Tensor:
    """P points uniform in the domain of a served mesh, shape (P, 3)."""
    rng = np.random.default_rng(seed)
    if kind == "box":
        p = rng.random((P, 3))
    else:
        rho = np.sqrt(rng.uniform(0.25, 1.0, P))
        th = rng.uniform(0.0, 2.0 * math.pi, P)
        p = np.stack([rho * np.cos(th), rho * np.sin(th), rng.random(P)], 1)
    return torch.as_tensor(p, dtype=torch.float64).to(device).contiguous()
