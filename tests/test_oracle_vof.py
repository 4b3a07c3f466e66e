"""Pins of the oracle's two-fluid (VOF) drag: the fluid density and viscosity at
a particle follow the liquid volume fraction alpha there (the local-property
mixture of Sec. 2.5), alpha being the volume average of the phase indicator --
on the bulk grid, the restriction of the fine alpha -- interpolated
trilinearly to the particle.

What pins it, independently of its own code:
  * alpha = 1 and alpha = 0 reduce to the pinned single-fluid drag with fluid 1
    or fluid 2, bit for bit;
  * at any alpha it equals the single-fluid drag evaluated with the mixture
    properties computed here;
  * the viscous (Stokes) limit: F -> 0.96 * 3 pi mu(alpha) d |u_r| (the Di
    Felice constant 4.8^2 / 24), independent of the density;
  * an affine alpha field gives the affine value at interior particles
    (restriction and trilinear interpolation are exact for affine fields).
"""
import math

import numpy as np
import pytest

import workload as W

RHO1, MU1, RHO2, MU2 = 1000.0, 1.0e-3, 1.2, 1.8e-5


def _particles(n, seed):
    rng = np.random.default_rng(seed)
    uf = rng.normal(0, 0.2, (n, 3))
    up = rng.normal(0, 0.1, (n, 3))
    d = rng.uniform(0.002, 0.01, n)
    eps = rng.uniform(0.25, 1.0, n)
    return uf, up, d, eps


def test_pure_phases_are_single_fluid_drag(orc):
    uf, up, d, eps = _particles(500, 31)
    for a, (rho, mu) in ((1.0, (RHO1, MU1)), (0.0, (RHO2, MU2))):
        f, b, nc = orc.drag_vof(uf, up, d, eps, np.full(500, a), RHO1, MU1, RHO2, MU2, 0.3)
        f1, b1, nc1 = orc.drag(uf, up, d, eps, rho, mu, 0.3)
        np.testing.assert_array_equal(f, f1)
        np.testing.assert_array_equal(b, b1)
        assert nc == nc1


def test_mixture_properties(orc):
    n = 300
    uf, up, d, eps = _particles(n, 32)
    alpha = np.random.default_rng(33).uniform(0.0, 1.0, n)
    f, b, _ = orc.drag_vof(uf, up, d, eps, alpha, RHO1, MU1, RHO2, MU2, 0.3)
    for p in range(n):
        rho = RHO1 * alpha[p] + RHO2 * (1.0 - alpha[p])
        mu = MU1 * alpha[p] + MU2 * (1.0 - alpha[p])
        f1, b1, _ = orc.drag(uf[p:p + 1], up[p:p + 1], d[p:p + 1], eps[p:p + 1], rho, mu, 0.3)
        assert b[p] == pytest.approx(b1[0], rel=1e-14)
        np.testing.assert_allclose(f[p], f1[0], rtol=1e-14, atol=0)


@pytest.mark.parametrize("alpha", [1.0, 0.5, 0.01, 0.0])
def test_stokes_limit_follows_mixture_viscosity(orc, alpha):
    d, U = 0.004, 1e-9                      # Re ~ 1e-6 for every mixture here
    uf = np.array([[U, 0.0, 0.0]])
    f, _, _ = orc.drag_vof(uf, np.zeros((1, 3)), np.array([d]), np.array([1.0]), np.array([alpha]),
                           RHO1, MU1, RHO2, MU2, 0.0)
    mu = MU1 * alpha + MU2 * (1.0 - alpha)
    stokes = 3.0 * math.pi * mu * d * U * 4.8 ** 2 / 24.0
    assert f[0, 0] == pytest.approx(stokes, rel=2e-3)


def test_affine_alpha_is_exact_at_interior_particles(orc):
    w = W.small_workload(nb=(6, 5, 8), ratio=4, box=(1.0, 0.8, 1.6), n=3000, seed=34, precision="fp32")
    pos, d, vel = W.particles(w)
    fine = W.fine_fields(w)
    nf = w.grid.nf
    hz = w.grid.box[2] / nf[2]
    zc = (np.arange(nf[2]) + 0.5) * hz
    a0, a1 = 0.1, 0.5                       # alpha = a0 + a1 z stays inside [0, 1]
    alpha = np.broadcast_to((a0 + a1 * zc)[:, None, None], (nf[2], nf[1], nf[0])).copy()
    o = orc.step(pos, vel, d, fine, w.grid, cic=True, prec32=False, alpha=alpha, rho2=RHO2, mu2=MU2,
                 fine_out="none")
    hb = w.grid.box[2] / w.grid.nb[2]
    z = pos[:, 2].astype(np.float64)
    inner = (z > 0.5 * hb) & (z < w.grid.box[2] - 0.5 * hb)
    assert inner.sum() > 2000
    np.testing.assert_allclose(o["alpha_p"][inner], a0 + a1 * z[inner], rtol=0, atol=1e-13)
    zb = (np.arange(w.grid.nb[2]) + 0.5) * hb
    np.testing.assert_allclose(o["alpha"].reshape(w.grid.nb[::-1]), np.broadcast_to(
        (a0 + a1 * zb)[:, None, None], w.grid.nb[::-1]), rtol=0, atol=1e-14)
