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


def test_advect_prec32_only_changes_wall_decisions(orc):
    """Away from the walls the binary32 mode computes the same FP64 values as the
    FP64 mode, bit for bit: the mode changes the wall test only."""
    rng = np.random.default_rng(7)
    n = 2000
    x = rng.uniform(0.1, 0.9, (n, 3)).astype(np.float32).astype(np.float64)
    u = rng.normal(0, 0.1, (n, 3)).astype(np.float32).astype(np.float64)
    d = rng.uniform(0.01, 0.04, n).astype(np.float32).astype(np.float64)
    F = rng.normal(0, 1e-3, (n, 3))
    a = orc.advect(x, u, d, F, 2500.0, 1e-4, (1.0, 1.0, 1.0), prec32=True)
    b = orc.advect(x, u, d, F, 2500.0, 1e-4, (1.0, 1.0, 1.0), prec32=False)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    m = 2500.0 * (np.pi * d * d * d / 6.0)
    np.testing.assert_array_equal(a[0], x + 1e-4 * u)
    np.testing.assert_array_equal(a[1], u + 1e-4 * F / m[:, None])


def test_advect_prec32_wall_decisions_by_hand():
    """Hand-computed binary32 wall tests (dt = 2^-13, L = 1, no force)."""
    import oracle as orc
    dt = 2.0 ** -13
    d = np.array([0.02])
    F = np.zeros((1, 3))
    box = (1.0, 1.0, 1.0)
    x0 = 1.0 - 2.0 ** -24                      # largest binary32 below 1
    # (a) x + dt u = 1 + 2^-24 exactly: the midpoint between 1 and the next
    # binary32 (1 + 2^-23); ties to even give 1.0, not above L: no reflection
    # in binary32 (position clamped to L, velocity kept); FP64 reflects to
    # 2 - (1 + 2^-24) = 1 - 2^-24 and flips the velocity.
    u = 2.0 ** -10
    x32, v32 = orc.advect(np.array([[x0, 0.5, 0.5]]), np.array([[u, 0.0, 0.0]]), d, F, 2500.0, dt, box, True)
    x64, v64 = orc.advect(np.array([[x0, 0.5, 0.5]]), np.array([[u, 0.0, 0.0]]), d, F, 2500.0, dt, box, False)
    assert x32[0, 0] == 1.0 and v32[0, 0] == u
    assert x64[0, 0] == 1.0 - 2.0 ** -24 and v64[0, 0] == -u
    # (b) x + dt u = 1 + 2^-24 + 2^-30: above the midpoint, rounds to 1 + 2^-23 > L:
    # both modes reflect to 2 - (1 + 2^-24 + 2^-30) and flip the velocity.
    u = 2.0 ** -10 + 2.0 ** -17
    for prec32 in (True, False):
        xb, vb = orc.advect(np.array([[x0, 0.5, 0.5]]), np.array([[u, 0.0, 0.0]]), d, F, 2500.0, dt, box, prec32)
        assert xb[0, 0] == 1.0 - 2.0 ** -24 - 2.0 ** -30 and vb[0, 0] == -u
    # (c) below zero: x = 2^-20, dt u = -2^-19, candidate -2^-20 (exact in binary32):
    # both modes mirror to +2^-20 and flip the velocity.
    u = -(2.0 ** -6)
    for prec32 in (True, False):
        xc, vc = orc.advect(np.array([[2.0 ** -20, 0.5, 0.5]]), np.array([[u, 0.0, 0.0]]), d, F, 2500.0, dt, box,
                            prec32)
        assert xc[0, 0] == 2.0 ** -20 and vc[0, 0] == 2.0 ** -6
    # (d) the other axes are untouched by x's wall, y and z move by dt u_y, dt u_z
    xd, vd = orc.advect(np.array([[x0, 0.25, 0.75]]), np.array([[2.0 ** -10, 2.0 ** -3, -(2.0 ** -3)]]), d, F,
                        2500.0, dt, box, True)
    assert xd[0, 1] == 0.25 + 2.0 ** -16 and xd[0, 2] == 0.75 - 2.0 ** -16
    assert vd[0, 1] == 2.0 ** -3 and vd[0, 2] == -(2.0 ** -3)


def test_advect_prec32_closed_form(orc):
    """The constant-force closed form also holds in the binary32 mode: its values
    are FP64, but the position it starts each step from is the binary32 state
    (rounded once per step: 50 roundings of 2^-24 relative at most)."""
    box = (10.0, 10.0, 10.0)
    x0 = np.array([[5.0, 5.0, 5.0]])
    u0 = np.array([[0.1, -0.2, 0.05]])
    d = np.array([0.02])
    F = np.array([[1e-3, 2e-3, -1e-3]])
    rho_p, dt = 2500.0, 1e-2
    m = rho_p * math.pi * d[0] ** 3 / 6
    x, u = x0, u0
    for _ in range(50):
        x, u = orc.advect(x, u, d, F, rho_p, dt, box, prec32=True)
    n = 50
    np.testing.assert_allclose(x, x0 + n * dt * u0 + dt * dt * F / m * n * (n - 1) / 2, rtol=50 * 2.0 ** -24)
    np.testing.assert_allclose(u, u0 + n * dt * F / m, rtol=1e-12)
