"""Pins of the oracle's semi-implicit split of the momentum source (the drag
counterpart of Eq. UFP treated semi-implicitly, Sec. 2.5): the deposited drag
coefficient K_c = (1/V_b) sum_p w_pc beta_p and the beta-weighted particle
velocity KU_c = (1/V_b) sum_p w_pc beta_p u_p.

What pins them, independently of their own code:
  * brute force with CIC weights written as tent functions (and NGP indicator
    vectors) on every cell;
  * the identity F_fpi = -K U0 + KU when every particle sees the same fluid
    velocity U0, against the separately pinned drag and force deposition;
  * the sums: sum_c K_c V_b = sum_p beta_p and sum_c KU_c V_b = sum_p beta_p u_p,
    and their conservation through the prolongation, in a composed step.
"""
import numpy as np
import pytest

import workload as W
from test_oracle_deposit import tent_weights_brute


@pytest.mark.parametrize("cic", [False, True])
def test_semi_deposit_brute_force(orc, cic):
    box, nb = (1.0, 0.75, 1.25), (3, 2, 4)
    rng = np.random.default_rng(21)
    n = 50
    pos = rng.random((n, 3)) * np.array(box)
    pos[:3] = [[0, 0, 0], [1.0, 0.75, 1.25], [0.5, 0.375, 0.625]]
    beta = rng.uniform(0.1, 2.0, n)
    vel = rng.normal(size=(n, 3))
    cell, _ = orc.bin_particles(pos, box, nb, False)
    perm, _, _ = orc.sort_cells(cell, int(np.prod(nb)))
    K, KU = orc.deposit_semi(pos, beta, vel, perm, box, nb, cic)
    vb = np.prod(np.array(box) / np.array(nb))
    nc = int(np.prod(nb))
    Kref = np.zeros(nc)
    KUref = np.zeros((3, nc))
    for p in range(n):
        wd = tent_weights_brute(pos[p], box, nb) if cic else np.eye(nc)[cell[p]]
        Kref += wd * beta[p] / vb
        KUref += np.outer(vel[p], wd) * beta[p] / vb
    np.testing.assert_allclose(K, Kref, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(KU, KUref, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("cic", [False, True])
def test_semi_split_reproduces_source_in_uniform_flow(orc, cic):
    """F_p = beta_p (U0 - u_p) for all p  =>  F_fpi,c = -K_c U0 + KU_c."""
    box, nb = (1.0, 1.0, 2.0), (4, 4, 8)
    rng = np.random.default_rng(22)
    n = 3000
    pos = rng.random((n, 3)) * np.array(box)
    vel = rng.normal(0.0, 0.1, (n, 3))
    d = rng.uniform(0.01, 0.04, n)
    cell, _ = orc.bin_particles(pos, box, nb, False)
    perm, _, _ = orc.sort_cells(cell, int(np.prod(nb)))
    eps_p = orc.gather_eps(pos, orc.deposit_volume(pos, d, perm, box, nb, cic), box, nb, cic)
    U0 = np.array([0.3, -0.1, 0.5])
    uf = np.broadcast_to(U0, (n, 3))
    force, beta, _ = orc.drag(uf, vel, d, eps_p, 1000.0, 1e-3, 0.3)
    Fc = orc.deposit_force(pos, force, perm, box, nb, cic)
    K, KU = orc.deposit_semi(pos, beta, vel, perm, box, nb, cic)
    for a in range(3):
        scale = np.abs(K * U0[a]).max() + np.abs(KU[a]).max()
        np.testing.assert_allclose(Fc[a], -K * U0[a] + KU[a], rtol=0, atol=1e-12 * scale)


def test_semi_sums_equal_particle_sums(orc):
    box, nb = (1.0, 0.6, 1.5), (5, 3, 6)
    rng = np.random.default_rng(23)
    n = 4000
    pos = rng.random((n, 3)) * np.array(box)
    pos[:8] = 0.0
    pos[8:16] = np.array(box)
    beta = rng.uniform(0.0, 3.0, n)
    vel = rng.normal(size=(n, 3))
    vb = np.prod(np.array(box) / np.array(nb))
    for cic in (False, True):
        cell, _ = orc.bin_particles(pos, box, nb, False)
        perm, _, _ = orc.sort_cells(cell, int(np.prod(nb)))
        K, KU = orc.deposit_semi(pos, beta, vel, perm, box, nb, cic)
        kp = orc.fsum_axis(beta)
        assert abs(orc.fsum_axis(K) * vb - kp) <= 1e-13 * kp
        for a in range(3):
            ref = orc.fsum_axis(beta * vel[:, a])
            assert abs(orc.fsum_axis(KU[a]) * vb - ref) <= 1e-12 * np.abs(beta * vel[:, a]).sum()
        assert (K >= 0).all()


def test_semi_step_conservation_and_split(orc):
    """Composed step: bulk and fine sums equal the particle sums, and with a
    given uniform fluid velocity the split reproduces the source exactly."""
    w = W.small_workload(nb=(6, 5, 4), ratio=4, n=4000, seed=24, precision="fp32")
    pos, d, vel = W.particles(w)
    fine = W.fine_fields(w)
    o = orc.step(pos, vel, d, fine, w.grid, cic=True, prec32=True, semi_implicit=True)
    dg = o["diag"]
    assert abs(dg["K_b"] - dg["K_p"]) <= 1e-13 * dg["K_p"]
    assert abs(dg["K_f"] - dg["K_b"]) <= 1e-12 * dg["K_p"]
    bu = np.abs(o["beta"][:, None] * vel).sum(axis=0)
    for a in range(3):
        assert abs(dg["KU_b"][a] - dg["KU_p"][a]) <= 1e-12 * bu[a]
        assert abs(dg["KU_f"][a] - dg["KU_b"][a]) <= 1e-12 * bu[a]
    U0 = np.array([0.2, 0.0, -0.4])
    g = orc.step(pos, vel, d, fine, w.grid, cic=True, prec32=True, semi_implicit=True,
                 vel_source="given", bulk_velocity=np.broadcast_to(U0, pos.shape), fine_out="none")
    for a in range(3):
        scale = np.abs(g["K"] * U0[a]).max() + np.abs(g["KU"][a]).max()
        np.testing.assert_allclose(g["F"][a], -g["K"] * U0[a] + g["KU"][a], rtol=0, atol=1e-12 * scale)
