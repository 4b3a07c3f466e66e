"""Pins of the oracle's grid-to-grid transfer between grids that need not be
nested (the sender -> receiver interpolation of Sec. 2.3): the receiver value
is the volume-weighted average of the sender cells it overlaps.

What pins it, independently of its own code:
  * identical grids give the twin-cell copy (the paper's example);
  * a nested pair equals the restriction of the coupling step (average of the
    children), itself pinned in test_oracle_grid;
  * constants are preserved and the integral is conserved, in both directions;
  * adjointness: sum_c |c| (R s)_c t_c = sum_f |f| s_f (R' t)_f for the maps R
    (sender -> receiver) and R' (receiver -> sender);
  * a 1-D piecewise-constant field: the receiver values are its exact interval
    averages, integrated here from the breakpoints with numpy;
  * non-uniform (rectilinear) grids with random node spacing.
"""
import numpy as np
import pytest


def uniform_nodes(n, box):
    return [np.linspace(0.0, box[a], n[a] + 1) for a in range(3)]


def random_nodes(rng, n, box):
    out = []
    for a in range(3):
        w = rng.uniform(0.3, 1.7, n[a])
        x = np.concatenate([[0.0], np.cumsum(w)])
        x = x / x[-1] * box[a]
        x[-1] = box[a]
        out.append(x)
    return out


def volumes(nodes):
    d = [np.diff(x) for x in nodes]
    return d[2][:, None, None] * d[1][None, :, None] * d[0][None, None, :]


def test_identical_grids_copy(orc):
    rng = np.random.default_rng(41)
    nodes = random_nodes(rng, (5, 4, 3), (1.0, 2.0, 0.5))
    s = rng.normal(size=(3, 4, 5))
    np.testing.assert_allclose(orc.remap(s, nodes, nodes), s, rtol=1e-15, atol=0)


@pytest.mark.parametrize("r", [1, 2, 4])
def test_nested_pair_is_restriction(orc, r):
    nb, box = (4, 3, 5), (1.0, 0.75, 1.25)
    nf = tuple(n * r for n in nb)
    rng = np.random.default_rng(42)
    q = rng.normal(size=(nf[2], nf[1], nf[0]))
    got = orc.remap(q, uniform_nodes(nf, box), uniform_nodes(nb, box))
    np.testing.assert_allclose(got.ravel(), orc.restrict(q, nb, r), rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("ns,nd", [((13, 7, 5), (5, 4, 3)), ((3, 5, 2), (11, 8, 7)), ((6, 1, 9), (4, 3, 2))])
def test_constants_and_integral(orc, ns, nd):
    rng = np.random.default_rng(43)
    box = (1.3, 0.7, 2.1)
    S, D = random_nodes(rng, ns, box), random_nodes(rng, nd, box)
    one = orc.remap(np.full((ns[2], ns[1], ns[0]), 3.25), S, D)
    np.testing.assert_allclose(one, 3.25, rtol=1e-14)
    s = rng.normal(size=(ns[2], ns[1], ns[0]))
    t = orc.remap(s, S, D)
    assert abs((t * volumes(D)).sum() - (s * volumes(S)).sum()) <= 1e-13 * (np.abs(s) * volumes(S)).sum()


def test_adjoint_of_the_reverse_map(orc):
    rng = np.random.default_rng(44)
    box = (1.0, 1.0, 1.0)
    ns, nd = (9, 6, 4), (4, 7, 5)
    S, D = random_nodes(rng, ns, box), random_nodes(rng, nd, box)
    s = rng.normal(size=(ns[2], ns[1], ns[0]))
    t = rng.normal(size=(nd[2], nd[1], nd[0]))
    lhs = (volumes(D) * orc.remap(s, S, D) * t).sum()
    rhs = (volumes(S) * s * orc.remap(t, D, S)).sum()
    assert abs(lhs - rhs) <= 1e-13 * (np.abs(volumes(D) * t).sum() * np.abs(s).max())


def test_piecewise_constant_interval_averages(orc):
    rng = np.random.default_rng(45)
    xs = np.sort(np.concatenate([[0.0, 1.0], rng.random(11)]))
    xd = np.sort(np.concatenate([[0.0, 1.0], rng.random(6)]))
    v = rng.normal(size=len(xs) - 1)
    unit = [np.array([0.0, 1.0]), np.array([0.0, 1.0])]
    got = orc.remap(v.reshape(1, 1, -1), [xs] + unit, [xd] + unit).ravel()
    ref = []
    for a, b in zip(xd[:-1], xd[1:]):
        lo, hi = np.clip(xs[:-1], a, b), np.clip(xs[1:], a, b)
        ref.append(float(((hi - lo) * v).sum() / (b - a)))
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-15)
