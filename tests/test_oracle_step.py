"""Pins of the composed oracle step: conservation invariants (deposited volume,
equal and opposite momentum exchange, conservative prolongation) and the
explicit-Euler advection closed form."""
import math

import numpy as np
import pytest

import workload as W


def test_cube8_step_conservation(orc):
    w = W.WORKLOADS["cube8_ngp_fp64"]
    pos, d, vel = W.particles(w)
    o = orc.step(pos, vel, d, W.fine_fields(w), w.grid, cic=False, prec32=False)
    dg = o["diag"]
    assert abs(dg["V_dep"] - dg["V_tot"]) <= 1e-13 * dg["V_tot"]
    sabs = np.abs(o["drag"]).sum(axis=0)
    for a in range(3):
        assert abs(dg["S_b"][a] + dg["sum_Fp"][a]) <= 1e-12 * sabs[a]
        assert abs(dg["S_f"][a] - dg["S_b"][a]) <= 1e-12 * sabs[a]
    assert dg["E_f"] == pytest.approx(1.0 - dg["V_dep"], abs=1e-13)
    assert o["count"].sum() == w.n_particles
    assert 15 < o["count"].mean() < 25


def test_small_cic_step_conservation_and_bulk_source(orc):
    w = W.small_workload(nb=(6, 5, 4), ratio=4, n=4000, seed=12, precision="fp32")
    pos, d, vel = W.particles(w)
    fine = W.fine_fields(w)
    for src in ("fine", "bulk"):
        o = orc.step(pos, vel, d, fine, w.grid, cic=True, prec32=True, vel_source=src)
        dg = o["diag"]
        assert abs(dg["V_dep"] - dg["V_tot"]) <= 1e-13 * dg["V_tot"]
        sabs = np.abs(o["drag"]).sum(axis=0)
        for a in range(3):
            assert abs(dg["S_b"][a] + dg["sum_Fp"][a]) <= 1e-12 * sabs[a]
            assert abs(dg["S_f"][a] - dg["S_b"][a]) <= 1e-12 * sabs[a]


def test_advect_constant_force_closed_form(orc):
    """x_n = x_0 + n dt u_0 + dt^2 (F/m) n(n-1)/2 under a constant force."""
    box = (10.0, 10.0, 10.0)
    x0 = np.array([[5.0, 5.0, 5.0]])
    u0 = np.array([[0.1, -0.2, 0.05]])
    d = np.array([0.02])
    F = np.array([[1e-3, 2e-3, -1e-3]])
    rho_p, dt = 2500.0, 1e-2
    m = rho_p * math.pi * d[0] ** 3 / 6
    x, u = x0, u0
    for _ in range(50):
        x, u = orc.advect(x, u, d, F, rho_p, dt, box, prec32=False)
    n = 50
    np.testing.assert_allclose(x, x0 + n * dt * u0 + dt * dt * F / m * n * (n - 1) / 2, rtol=1e-12)
    np.testing.assert_allclose(u, u0 + n * dt * F / m, rtol=1e-12)


def test_advect_reflection(orc):
    box = (1.0, 1.0, 1.0)
    x, u = orc.advect(np.array([[0.01, 0.99, 0.5]]), np.array([[-2.0, 2.0, 0.0]]), np.array([0.02]),
                      np.zeros((1, 3)), 2500.0, 0.01, box, prec32=False)
    np.testing.assert_allclose(x, [[0.01, 0.99, 0.5]], atol=1e-15)
    np.testing.assert_allclose(u, [[2.0, -2.0, 0.0]], atol=1e-15)
