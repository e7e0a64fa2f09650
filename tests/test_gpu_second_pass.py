"""GPU parity of long second passes.  An annulus is rotated about a skew
axis, so its elements' axis-aligned boxes overlap their neighbours widely
while the oriented boxes stay tight.  Points in thin shells just outside its
curved faces lie inside the oriented box of a boundary element (the box
holds the face's bulge) but outside the element, and inside the axis-aligned
boxes of neighbours whose oriented boxes miss them: the first pass leaves
them without an inside candidate and with a partial candidate set, and the
second pass solves the candidates the oriented boxes dropped.  With tens of
thousands of such points the second pass holds more pairs than the
one-wavefront-per-pair kernel takes (8,192), so at orders 4 and 7 the
order's matrix-core kernel runs it: binary64, and in mixed precision also
resuming the pairs the binary32 phase left unsolved or outside.  Orders 9
(matrix cores, one plane per lane) and 12 (the scalar kernel) run the same
long passes on their own kernels.  Checked against the CPU oracle under the
rules of the other parity tests."""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads as w
from parity import compare_locate

pytestmark = pytest.mark.gpu

TOL = 1e-12
PAIR_MAX = 8192  # largest second pass the one-wavefront-per-pair kernel takes


def _fp():
    from paper_1811_04891_amd import findpts as fp
    return fp


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


def _rotation(axis, angle):
    """Rotation matrix about a unit axis (Rodrigues' formula)."""
    k = np.asarray(axis, dtype=np.float64)
    k = k / np.linalg.norm(k)
    K = np.array([[0.0, -k[2], k[1]], [k[2], 0.0, -k[0]], [-k[1], k[0], 0.0]])
    return np.eye(3) + np.sin(angle) * K + (1.0 - np.cos(angle)) * (K @ K)


def _rotated_annulus(N, R):
    base = w.annulus_mesh(4, 32, 4, N=N)
    X = torch.stack([base.x, base.y, base.z], -1) @ torch.as_tensor(R.T)
    return w.Mesh("annulus_rot", N, X[..., 0].contiguous(), X[..., 1].contiguous(),
                  X[..., 2].contiguous())


def _shell_points(seed):
    """Ragged mix: 23,999 points with radius in [1, 1.004] (outside the outer
    face), 12,001 with radius in [0.497, 0.5] (inside the hole) and 8,003
    area-uniform in the annulus, z in [0.02, 0.98], shuffled."""
    rng = np.random.default_rng(seed)

    def ring(n, a, b):
        rho = rng.uniform(a, b, n)
        th = rng.uniform(0.0, 2.0 * np.pi, n)
        z = rng.uniform(0.02, 0.98, n)
        return np.stack([rho * np.cos(th), rho * np.sin(th), z], axis=1)

    inner = np.sqrt(rng.uniform(0.25, 1.0, 8003))
    th = rng.uniform(0.0, 2.0 * np.pi, 8003)
    body = np.stack([inner * np.cos(th), inner * np.sin(th), rng.uniform(0.02, 0.98, 8003)], 1)
    p = np.concatenate([ring(23999, 1.0, 1.004), ring(12001, 0.497, 0.5), body])
    return torch.as_tensor(np.ascontiguousarray(p[rng.permutation(len(p))]))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("N", [4, 7, 9, 12])
def test_long_second_pass(dev, N, prec):
    fp = _fp()
    precision = fp.FP_PREC_MIXED if prec == "mixed" else fp.FP_PREC_FP64
    _say(f"case: long second pass, rotated annulus 4x32x4 N={N}, {prec}")
    R = _rotation([1.0, 2.0, 0.5], 0.7)
    mesh = _rotated_annulus(N, R)
    pts = _shell_points(500 + N) @ torch.as_tensor(R.T)
    md = mesh.to(dev)
    h = fp.findpts_setup(md.x, md.y, md.z, N, tol=TOL, max_points=1 << 16,
                         precision=precision)
    code, el, rst, d2 = fp.findpts(h, pts.to(dev))
    torch.cuda.synchronize()
    pairs, _, npts, _, pairs1, _ = fp.findpts_stats(h, first_pass=True)
    second = pairs - pairs1
    _say(f"pairs {pairs}, first pass {pairs1}, second pass {second}")
    assert npts == len(pts)
    # at orders up to 7 the matrix-core kernel ran the second pass (above
    # them there is no pair kernel: the order's own kernel always runs it)
    assert second > PAIR_MAX
    g = (code.cpu().numpy(), el.cpu().numpy(), rst.cpu().numpy(), d2.cpu().numpy())
    om = oracle.OracleMesh.from_mesh(mesh, TOL)
    o = om.findpts(pts.numpy())
    _, hs = om.bbox()
    st = compare_locate(om, pts.numpy(), g, o, hs, TOL)
    _say(f"ok {st}")
    assert st["inside"] >= 8003
    h.free()
