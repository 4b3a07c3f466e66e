"""Pins of the oracle's transfer between grids of arbitrary axis-aligned cells
(locally refined, non-nested; the static sender -> receiver map of Sec. 2.3):
twin cells copy, a refined cell restricts to its parent's average, rectilinear
grids agree with the separately pinned rectilinear transfer, constants and
integrals are preserved, the map is adjoint to its reverse, a hand example."""
import numpy as np

import workload as W


def test_twin_cells_copy(orc):
    g = W.refined_box_grid((1.0, 0.5, 0.75), (5, 3, 4), (0.2, 0.7, 0.0, 0.5, 0.3, 0.8))
    src = np.random.default_rng(1).normal(size=g.shape[0])
    # (|c| src) / |c|: one rounding of a product and one of a quotient
    np.testing.assert_allclose(orc.box_remap(src, g, g), src, rtol=3e-16, atol=0)


def test_children_restrict_to_parent_average(orc):
    box, n = (1.0, 1.0, 1.0), (3, 2, 2)
    fine = W.refined_box_grid(box, n, (0.0, 1.0, 0.0, 1.0, 0.0, 1.0))      # every cell split in 8
    coarse = W.box_grid(box, n)
    src = np.random.default_rng(2).normal(size=fine.shape[0])
    got = orc.box_remap(src, fine, coarse)
    want = src.reshape(-1, 8).mean(axis=1)     # children follow their parent, in raster order
    np.testing.assert_allclose(got, want, rtol=1e-14, atol=1e-15)
    # and the other way: each child receives its parent's value
    back = orc.box_remap(want, coarse, fine)
    np.testing.assert_allclose(back, np.repeat(want, 8), rtol=1e-14)


def test_rectilinear_grids_agree_with_rectilinear_transfer(orc):
    box = (1.0, 0.8, 1.2)
    ns, nd = (7, 5, 6), (4, 6, 5)
    src = np.random.default_rng(3).normal(size=int(np.prod(ns)))
    got = orc.box_remap(src, W.box_grid(box, ns), W.box_grid(box, nd))
    nodes = lambda n: [np.linspace(0.0, box[a], n[a] + 1) for a in range(3)]
    want = orc.remap(src.reshape(ns[2], ns[1], ns[0]), nodes(ns), nodes(nd)).ravel()
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-14)


def _pair():
    box = (1.0, 1.0, 2.0)
    s = W.refined_box_grid(box, (6, 6, 12), (0.0, 1.0, 0.0, 1.0, 0.0, 0.5))         # refined bottom quarter
    r = W.refined_box_grid(box, (5, 4, 9), (0.3, 0.9, 0.1, 0.6, 0.4, 1.5), split=3)  # another refinement
    return box, s, r


def vol(b):
    return (b[:, 1] - b[:, 0]) * (b[:, 3] - b[:, 2]) * (b[:, 5] - b[:, 4])


def test_constant_and_integral(orc):
    box, s, r = _pair()
    np.testing.assert_allclose(orc.box_remap(np.full(s.shape[0], 2.5), s, r), 2.5, rtol=1e-13)
    src = np.random.default_rng(4).normal(size=s.shape[0])
    dst = orc.box_remap(src, s, r)
    assert abs((dst * vol(r)).sum() - (src * vol(s)).sum()) <= 1e-12 * (np.abs(src) * vol(s)).sum()


def test_adjoint_of_reverse_map(orc):
    box, s, r = _pair()
    rng = np.random.default_rng(5)
    a, b = rng.normal(size=s.shape[0]), rng.normal(size=r.shape[0])
    lhs = (vol(r) * orc.box_remap(a, s, r) * b).sum()
    rhs = (vol(s) * a * orc.box_remap(b, r, s)).sum()
    assert abs(lhs - rhs) <= 1e-12 * (np.abs(vol(s) * a).sum() * np.abs(b).max())


def test_hand_example():
    import oracle as orc
    s = np.array([[0.0, 0.5, 0, 1, 0, 1], [0.5, 1.0, 0, 1, 0, 1]], dtype=np.float64)
    r = np.array([[0.25, 0.75, 0, 1, 0, 1], [0.0, 1.0, 0.5, 1.0, 0.0, 0.25]], dtype=np.float64)
    got = orc.box_remap(np.array([2.0, 6.0]), s, r)
    # first: half of each sender; second: covers both halves equally
    np.testing.assert_allclose(got, [4.0, 4.0], rtol=1e-15)
    got = orc.box_remap(np.array([2.0, 6.0]), s, np.array([[0.4, 0.6, 0.2, 0.3, 0.0, 1.0]]))
    np.testing.assert_allclose(got, [4.0], rtol=1e-15)      # 0.1 of each
    got = orc.box_remap(np.array([2.0, 6.0]), s, np.array([[0.4, 0.9, 0.2, 0.3, 0.0, 1.0]]))
    np.testing.assert_allclose(got, [(0.1 * 2 + 0.4 * 6) / 0.5], rtol=1e-15)


def test_fast_generator_matches():
    a = W.refined_box_grid((1.0, 0.5, 0.75), (5, 3, 4), (0.2, 0.7, 0.0, 0.5, 0.3, 0.8), split=3)
    b = W.refined_box_grid_fast((1.0, 0.5, 0.75), (5, 3, 4), (0.2, 0.7, 0.0, 0.5, 0.3, 0.8), split=3)
    np.testing.assert_array_equal(a, b)
    # the cells tile the box
    v = (a[:, 1] - a[:, 0]) * (a[:, 3] - a[:, 2]) * (a[:, 5] - a[:, 4])
    assert abs(v.sum() - 0.375) < 1e-14
