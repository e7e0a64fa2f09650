"""Pins for the oracle's element boxes and hash grid (Section 2.1: hash
table, then elementwise bounding boxes).  Boxes: equal the node box on
affine elements, contain dense samples of curved elements (computed in
closed form), including a bulge that the node box alone misses.  Hash: the
candidate set equals the brute-force set {e : x* in box_e}."""
import numpy as np
import pytest

import oracle
import workloads as w
from helpers import box_affine, box_elem_ids, phi_np


def _margin(xe):
    he = max(float(xe[c].max() - xe[c].min()) for c in range(3))
    return 1e-8 * he + 1e-14 * max(float(np.abs(xe[c]).max()) for c in range(3)), he


def test_affine_box_is_node_box():
    m = w.box_mesh(3, 2, 2, lo=(-1, 0.5, 2), hi=(2, 1.5, 2.6), N=5)
    om = oracle.OracleMesh.from_mesh(m)
    b, h = om.bbox()
    hd = m.host()
    for e in range(m.E):
        xe = [hd[c][e] for c in "xyz"]
        mg, he = _margin(xe)
        assert h[e] == he
        for c in range(3):
            assert abs(b[e, 2 * c] - (xe[c].min() - mg)) <= 1e-14
            assert abs(b[e, 2 * c + 1] - (xe[c].max() + mg)) <= 1e-14


def test_curved_box_contains_dense_sample():
    n = (2, 2, 2)
    m, _ = w.poly_map_mesh(*n, N=3, amp=0.3)
    om = oracle.OracleMesh.from_mesh(m)
    b, _ = om.bbox()
    ex, ey, ez = box_elem_ids(m.E, n)
    g = np.linspace(-1, 1, 24)
    R = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    for e in range(m.E):
        a = box_affine(ex[e], ey[e], ez[e], n, (0, 0, 0), (1, 1, 1), R)
        X = np.stack(phi_np(a[:, 0], a[:, 1], a[:, 2], amp=0.3), 1)
        for c in range(3):
            assert X[:, c].min() >= b[e, 2 * c] and X[:, c].max() <= b[e, 2 * c + 1]


def test_bulge_missed_by_node_box_is_covered():
    """One element whose face bulges between GLL nodes: x = r + 0.2 (1 - s^2)
    (1 - t^2) on N = 2 (nodes at s, t in {-1, 0, 1}).  The max over nodes of x
    is 1.2 at r = 1, which the nodes attain; use a cubic-in-s bulge instead
    that peaks between nodes: x = r + 0.3 s (1 - s^2) (degree 3, N = 3)."""
    N = 3
    z, _ = oracle.gll(N)
    R, S, T = np.meshgrid(z, z, z, indexing="ij")
    X = (R + 0.3 * S * (1 - S * S)).transpose(2, 1, 0)  # [k, j, i]
    Y = S.transpose(2, 1, 0).copy()
    Z = T.transpose(2, 1, 0).copy()
    om = oracle.OracleMesh(X.ravel(), Y.ravel(), Z.ravel(), N)
    b, _ = om.bbox()
    s = np.linspace(-1, 1, 2001)
    true_max = 1 + np.max(0.3 * s * (1 - s * s))
    assert X.max() < true_max - 1e-3          # the node box misses the bulge
    assert b[0, 1] >= true_max                 # the Bernstein hull does not


@pytest.mark.parametrize("which", ["c1", "annulus", "sessions"])
def test_hash_candidates_equal_brute_force(which):
    rng = np.random.default_rng(7)
    sess = None
    if which == "c1":
        m = w.cube_c1()
        pts = rng.uniform(-0.05, 1.05, (3000, 3))
    elif which == "annulus":
        m = w.annulus_mesh(4, 16, 3, N=5)
        pts = np.concatenate([rng.uniform(-1.05, 1.05, (3000, 2)),
                              rng.uniform(-0.05, 1.05, (3000, 1))], 1)
    else:
        m = w.cube_c1()
        sess = np.arange(m.E) % 3
        m.session = __import__("torch").as_tensor(sess, dtype=__import__("torch").int32)
        pts = rng.uniform(0, 1, (2000, 3))
    om = oracle.OracleMesh.from_mesh(m)
    b, _ = om.bbox()
    for i, p in enumerate(pts):
        ps = -1 if sess is None else i % 3
        inb = np.all((p >= b[:, 0::2]) & (p <= b[:, 1::2]), axis=1)
        if sess is not None:
            inb &= sess != ps
        ref = np.nonzero(inb)[0]
        got = om.candidates(p, ps)
        assert np.array_equal(got, ref), (i, p, got, ref)
