"""Seeded synthetic inputs shared by the oracle-side tests and the GPU path.

This package builds meshes of curved hexahedral spectral elements, query
points and nodal fields.  It holds none of the point-location or
interpolation arithmetic: no Lagrange basis, no element map, no Newton
solve, no bounding box and no hash.  Mesh nodes sit at Gauss-Lobatto-Legendre
(GLL) positions obtained from numpy's Legendre routines; the oracle and the
HIP library each compute their own GLL nodes.

Node layout of every mesh coordinate array: shape (E, n1, n1, n1) in C order
with index [e, k, j, i], i.e. the r index i runs fastest and the flat index
of node (i, j, k) of element e is i + n1*(j + n1*(k + n1*e)), n1 = N + 1.
"""

from .meshes import (  # noqa: F401
    Mesh,
    gll_points,
    box_mesh,
    cube_c1,
    annulus_mesh,
    annulus_c2,
    overlap_c3,
    big_box_c5,
    poly_map_mesh,
    spiral_element,
    queries_uniform_box,
    queries_c1,
    queries_c2,
    queries_c3,
    queries_c5,
    c3_interface_nodes,
    c3_interface_quadrature,
    gll_weights,
    poly_fields,
    ref_poly_fields,
)
from .serving import (  # noqa: F401
    ServedMesh,
    serving_meshes,
    serving_requests,
    serving_points,
)
from .meshes2d import (  # noqa: F401
    Mesh2,
    box2d_mesh,
    annulus2d_mesh,
    poly_map_mesh2d,
    phi2,
    overlap2d,
    annulus2d_c6,
    queries2d_c6,
)
