"""MI355X (gfx950) findpts / findpts_eval: point location and interpolation on
curved hexahedral spectral-element meshes (Mittal, Dutta & Fischer,
Section 2.1), as hand-written HIP kernels behind a C ABI (include/findpts.h).

    from paper_1811_04891_amd import findpts as fp
    h = fp.findpts_setup(x, y, z, N)            # x, y, z: CUDA float64
    code, el, rst, dist2 = fp.findpts(h, pts)   # pts: (npts, 3)
    vals = fp.findpts_eval(h, code, el, rst, [u, v, w, p])
"""
from . import findpts  # noqa: F401
