"""Pins of the oracle's grid-to-grid transfers (Fig. 1, Sec. 2.1, 2.3): restriction
fine -> bulk, bulk pressure gradient, trilinear lookup, conservative prolongation
bulk -> fine; checked against closed forms, invariants and numpy routines."""
import math

import numpy as np
import pytest

import workload as W


def restrict_np(q, nb, r):
    nx, ny, nz = nb
    return q.reshape(nz, r, ny, r, nx, r).mean(axis=(1, 3, 5)).ravel()


def centres(n, L):
    return (np.arange(n) + 0.5) * (L / n)


def test_restrict_constant_affine_and_numpy(orc):
    nb, r, box = (5, 3, 4), 4, (1.0, 0.6, 0.8)
    nf = tuple(n * r for n in nb)
    zc, yc, xc = np.meshgrid(centres(nf[2], box[2]), centres(nf[1], box[1]), centres(nf[0], box[0]), indexing="ij")
    const = np.full(zc.shape, 3.25)
    np.testing.assert_allclose(orc.restrict(const, nb, r), 3.25, rtol=1e-15)
    aff = 0.7 + 1.3 * xc - 2.1 * yc + 0.4 * zc
    Zb, Yb, Xb = np.meshgrid(centres(nb[2], box[2]), centres(nb[1], box[1]), centres(nb[0], box[0]), indexing="ij")
    np.testing.assert_allclose(orc.restrict(aff, nb, r), (0.7 + 1.3 * Xb - 2.1 * Yb + 0.4 * Zb).ravel(), rtol=0, atol=1e-14)
    rnd = np.random.default_rng(0).normal(size=zc.shape)
    np.testing.assert_allclose(orc.restrict(rnd, nb, r), restrict_np(rnd, nb, r), rtol=0, atol=1e-15)


def test_restrict_taylor_green_closed_form(orc):
    """Average of the point-sampled Taylor-Green field over the r^3 children.

    For offsets symmetric about the bulk centre, the mean of sin/cos(k(x_c+o))
    is sin/cos(k x_c) times S = mean_l cos(k o_l); with r = 4 the offsets are
    +-h_f/2, +-3h_f/2, so S = (cos(k h_f/2) + cos(3k h_f/2))/2.  The pressure's
    cos(2k .) factors carry S2 = (cos(k h_f) + cos(3k h_f))/2.
    """
    w = W.WORKLOADS["cube8_ngp_fp64"]
    g = w.grid
    u, v, ww, p = W.fine_fields(w)
    k = W.TG_K
    hf = 1.0 / g.nf[0]
    S = (math.cos(k * hf / 2) + math.cos(3 * k * hf / 2)) / 2
    S2 = (math.cos(k * hf) + math.cos(3 * k * hf)) / 2
    Z, Y, X = np.meshgrid(*(centres(n, 1.0) for n in (8, 8, 8)), indexing="ij")
    U = orc.restrict(u, g.nb, 4)
    np.testing.assert_allclose(U, (S ** 3 * np.sin(k * X) * np.cos(k * Y) * np.cos(k * Z)).ravel(), atol=1e-14)
    V = orc.restrict(v, g.nb, 4)
    np.testing.assert_allclose(V, (-(S ** 3) * np.cos(k * X) * np.sin(k * Y) * np.cos(k * Z)).ravel(), atol=1e-14)
    P = orc.restrict(p, g.nb, 4)
    ref = w.rho_f / 16 * (S2 * np.cos(2 * k * X) + S2 * np.cos(2 * k * Y)) * (S2 * np.cos(2 * k * Z) + 2)
    np.testing.assert_allclose(P, ref.ravel(), atol=1e-11)
    # conservation of the integral
    vf, vb = hf ** 3, (1 / 8) ** 3
    assert abs(orc.fsum_axis(U) * vb - orc.fsum_axis(u) * vf) < 1e-15


def test_gradient_affine_and_taylor_green(orc):
    nb, box = (6, 5, 7), (1.2, 1.0, 1.4)
    Z, Y, X = np.meshgrid(*(centres(nb[a], box[a]) for a in (2, 1, 0)), indexing="ij")
    P = (3.0 - 2.0 * X + 0.5 * Y + 4.0 * Z).ravel()
    G = orc.gradient(P, nb, box)
    np.testing.assert_allclose(G[0], -2.0, atol=1e-12)
    np.testing.assert_allclose(G[1], 0.5, atol=1e-12)
    np.testing.assert_allclose(G[2], 4.0, atol=1e-12)
    # interior central difference of cos(2k x): -sin(2k x) sin(2k h)/h
    k = 2 * math.pi
    n = 16
    Z, Y, X = np.meshgrid(*(centres(n, 1.0),) * 3, indexing="ij")
    P = (np.cos(2 * k * X) * np.cos(2 * k * Y)).ravel()
    G = orc.gradient(P, (n, n, n), (1.0, 1.0, 1.0)).reshape(3, n, n, n)
    h = 1.0 / n
    ref = -np.sin(2 * k * X) * math.sin(2 * k * h) / h * np.cos(2 * k * Y)
    np.testing.assert_allclose(G[0][:, :, 1:-1], ref[:, :, 1:-1], atol=1e-12)
    # one-sided at the wall
    Pc = P.reshape(n, n, n)
    np.testing.assert_allclose(G[0][:, :, 0], (Pc[:, :, 1] - Pc[:, :, 0]) / h, atol=1e-12)
    # a single cell along an axis has zero gradient
    G1 = orc.gradient(np.arange(4.0), (4, 1, 1), (1.0, 1.0, 1.0))
    assert np.all(G1[1] == 0) and np.all(G1[2] == 0)


def test_interp_nodes_affine_and_clamp(orc):
    n, box = (5, 4, 6), (1.0, 0.8, 1.2)
    rng = np.random.default_rng(1)
    q = rng.normal(size=(n[2], n[1], n[0]))
    # node values at cell centres
    pts = np.array([[centres(n[0], 1.0)[i], centres(n[1], 0.8)[j], centres(n[2], 1.2)[k]]
                    for i, j, k in [(0, 0, 0), (2, 1, 3), (4, 3, 5), (1, 2, 0)]])
    got = orc.interp(q, n, box, pts)
    np.testing.assert_allclose(got, [q[0, 0, 0], q[3, 1, 2], q[5, 3, 4], q[0, 2, 1]], atol=1e-14)
    # affine field exact between the first and last centres
    Z, Y, X = np.meshgrid(*(centres(n[a], box[a]) for a in (2, 1, 0)), indexing="ij")
    aff = 1.0 + 2.0 * X - 3.0 * Y + 0.5 * Z
    h = np.array(box) / np.array(n)
    pts = h / 2 + rng.random((300, 3)) * (np.array(box) - h)
    got = orc.interp(aff, n, box, pts)
    np.testing.assert_allclose(got, 1.0 + 2.0 * pts[:, 0] - 3.0 * pts[:, 1] + 0.5 * pts[:, 2], atol=1e-13)
    # zero gradient beyond the outermost centres
    p0 = np.array([[0.0, 0.3, 0.5], [h[0] / 2, 0.3, 0.5]])
    got = orc.interp(aff, n, box, p0)
    assert got[0] == pytest.approx(got[1], abs=1e-14)


@pytest.mark.parametrize("name", ["cube8_ngp_fp64"])
def test_interp_taylor_green_error_bound(orc, name):
    """Tensor-product linear interpolation error <= (h^2/8) sum_a max|d2f/dx_a^2|,
    i.e. (3/8) k^2 h_f^2 A for the Taylor-Green velocity, away from the walls."""
    w = W.WORKLOADS[name]
    u, v, _, _ = W.fine_fields(w)
    rng = np.random.default_rng(3)
    hf = 1.0 / w.grid.nf[0]
    pts = hf / 2 + rng.random((5000, 3)) * (1.0 - hf)
    ua, va, _, _ = W.fluid_analytic(w, pts[:, 0], pts[:, 1], pts[:, 2])
    bound = 3.0 / 8.0 * W.TG_K ** 2 * hf ** 2
    eu = np.abs(orc.interp(u, w.grid.nf, w.grid.box, pts) - ua).max()
    ev = np.abs(orc.interp(v, w.grid.nf, w.grid.box, pts) - va).max()
    assert eu <= bound and ev <= bound
    assert eu > bound / 20  # the bound is not vacuous


@pytest.mark.parametrize("nb,r", [((4, 3, 5), 4), ((3, 3, 2), 2), ((2, 5, 3), 1), ((1, 4, 2), 4)])
def test_prolong_restrict_identity_and_conservation(orc, nb, r):
    B = np.random.default_rng(6).normal(size=int(np.prod(nb)))
    Pf = orc.prolong(B, nb, r, conservative=True)
    np.testing.assert_allclose(restrict_np(Pf, nb, r), B, rtol=0, atol=1e-14)
    assert abs(Pf.sum() / r ** 3 - B.sum()) < 1e-12
    np.testing.assert_allclose(orc.prolong(np.full(B.shape, 2.5), nb, r), 2.5, atol=1e-14)


def test_prolong_twin_cells_is_copy(orc):
    """Identical grids (ratio 1): the transfer maps each cell to its twin (Sec. 2.3)."""
    nb = (4, 3, 5)
    B = np.random.default_rng(8).normal(size=60)
    np.testing.assert_allclose(orc.prolong(B, nb, 1, conservative=True), B, atol=1e-15)
    np.testing.assert_allclose(orc.prolong(B, nb, 1, conservative=False), B, atol=1e-15)


def test_prolong_affine_interior_and_plain_trilinear_smoothing(orc):
    nb, r = (6, 5, 7), 4
    Z, Y, X = np.meshgrid(*(np.arange(nb[a]) + 0.5 for a in (2, 1, 0)), indexing="ij")
    B = (0.5 + 1.5 * X - 0.25 * Y + 2.0 * Z).ravel()
    Pf = orc.prolong(B, nb, r, conservative=True).reshape(nb[2] * r, nb[1] * r, nb[0] * r)
    fz, fy, fx = np.meshgrid(*((np.arange(nb[a] * r) + 0.5) / r for a in (2, 1, 0)), indexing="ij")
    ref = 0.5 + 1.5 * fx - 0.25 * fy + 2.0 * fz
    sl = tuple(slice(r, -r) for _ in range(3))  # parents not touching a wall
    np.testing.assert_allclose(Pf[sl], ref[sl], atol=1e-13)
    # plain trilinear (no defect): R(P(B)) = (1/8, 3/4, 1/8) smoothing along each axis, interior
    Bn = np.random.default_rng(2).normal(size=(nb[2], nb[1], nb[0]))
    R = restrict_np(orc.prolong(Bn.ravel(), nb, r, conservative=False), nb, r).reshape(Bn.shape)
    S = Bn.copy()
    for ax in range(3):
        S = 0.125 * np.roll(S, 1, ax) + 0.75 * S + 0.125 * np.roll(S, -1, ax)
    np.testing.assert_allclose(R[1:-1, 1:-1, 1:-1], S[1:-1, 1:-1, 1:-1], atol=1e-14)


def test_prolong_at_matches_full(orc):
    nb, r = (4, 3, 5), 4
    B = np.random.default_rng(7).normal(size=60)
    full = orc.prolong(B, nb, r)
    idx = np.random.default_rng(1).integers(0, full.size, 300)
    np.testing.assert_allclose(orc.prolong_at(B, nb, r, idx), full[idx], atol=1e-15)
