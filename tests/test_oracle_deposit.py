"""Pins of the oracle's particle -> bulk deposition (solid fraction / porosity of
Table 1 and Sec. 2.4, momentum source F_fpi of Eq. UFP) and of its transpose,
the void fraction seen by a particle."""
import numpy as np
import pytest

import workload as W


def tent_weights_brute(x, box, nb):
    """CIC weights written as tent functions on every cell centre, brute force.

    w(c) = prod_a max(0, 1 - |x_a - xc_a| / h_a), summed over the real cells and
    the ghost centres one cell beyond each wall; a ghost's weight belongs to the
    wall cell it mirrors (zero-gradient fold).  Returns a dense [ncell] vector.
    """
    w = np.zeros(int(np.prod(nb)))
    h = [box[a] / nb[a] for a in range(3)]
    ax = []
    for a in range(3):
        wa = np.zeros(nb[a])
        for i in range(-1, nb[a] + 1):
            xc = (i + 0.5) * h[a]
            t = max(0.0, 1.0 - abs(x[a] - xc) / h[a])
            wa[min(max(i, 0), nb[a] - 1)] += t
        ax.append(wa)
    for k in range(nb[2]):
        for j in range(nb[1]):
            for i in range(nb[0]):
                w[i + nb[0] * (j + nb[1] * k)] = ax[0][i] * ax[1][j] * ax[2][k]
    return w


@pytest.mark.parametrize("nb", [(4, 3, 5), (1, 2, 3), (2, 1, 1)])
def test_cic_weights_brute_force(orc, nb):
    box = (1.0, 0.6, 1.5)
    rng = np.random.default_rng(11)
    pts = rng.random((60, 3)) * np.array(box)
    pts[:6] = [[0, 0, 0], [1.0, 0.6, 1.5], [0.5, 0.3, 0.75], [1e-9, 0.6 - 1e-9, 0.1], [0.25, 0.2, 0.3], [0.125, 0.1, 0.15]]
    for x in pts:
        cells, w = orc.weights(x, box, nb, cic=True)
        dense = np.zeros(int(np.prod(nb)))
        dense[cells] += w
        np.testing.assert_allclose(dense, tent_weights_brute(x, box, nb), rtol=0, atol=1e-14)
        assert abs(w.sum() - 1.0) < 1e-14
        assert len(set(cells.tolist())) == len(cells)


def test_cic_centre_and_face(orc):
    box, nb = (1.0, 1.0, 1.0), (4, 4, 4)
    h = 0.25
    # particle at an interior cell centre deposits everything there
    cells, w = orc.weights([1.5 * h, 2.5 * h, 1.5 * h], box, nb, cic=True)
    dense = dict(zip(cells.tolist(), w.tolist()))
    assert dense[1 + 4 * (2 + 4 * 1)] == pytest.approx(1.0, abs=1e-15)
    # on the centre of an interior face between cells x=1 and x=2: one half each
    cells, w = orc.weights([2 * h, 2.5 * h, 1.5 * h], box, nb, cic=True)
    nz = {c: v for c, v in zip(cells.tolist(), w.tolist()) if v > 1e-15}
    assert set(nz) == {1 + 4 * (2 + 4 * 1), 2 + 4 * (2 + 4 * 1)}
    assert all(v == pytest.approx(0.5, abs=1e-15) for v in nz.values())


def test_ngp_deposit_is_per_cell_sum(orc):
    w = W.WORKLOADS["cube8_ngp_fp64"]
    pos, d, _ = W.particles(w)
    cell, _ = orc.bin_particles(pos, w.grid.box, w.grid.nb, False)
    perm, _, _ = orc.sort_cells(cell, w.grid.n_bulk)
    phi = orc.deposit_volume(pos, d, perm, w.grid.box, w.grid.nb, cic=False)
    vb = 1.0 / 512
    ref = np.bincount(cell, weights=np.pi * d ** 3 / 6 / vb, minlength=512)
    np.testing.assert_allclose(phi, ref, rtol=1e-13, atol=0)


@pytest.mark.parametrize("cic", [False, True])
def test_deposited_volume_equals_particle_volume(orc, cic):
    w = W.small_workload(nb=(5, 4, 3), n=3000, seed=3)
    pos, d, _ = W.particles(w)
    pos[:10] = 0.0  # a few on the walls and corners
    pos[10:20] = np.array(w.grid.box)
    cell, _ = orc.bin_particles(pos, w.grid.box, w.grid.nb, False)
    perm, _, _ = orc.sort_cells(cell, w.grid.n_bulk)
    phi = orc.deposit_volume(pos, d, perm, w.grid.box, w.grid.nb, cic)
    vb = np.prod(np.array(w.grid.box) / np.array(w.grid.nb))
    vtot = orc.fsum_axis(np.pi * d ** 3 / 6)
    assert abs(orc.fsum_axis(phi) * vb - vtot) <= 1e-13 * vtot


def test_cic_deposit_brute_force(orc):
    box, nb = (1.0, 0.75, 1.25), (3, 2, 4)
    rng = np.random.default_rng(2)
    n = 40
    pos = rng.random((n, 3)) * np.array(box)
    d = rng.uniform(0.01, 0.05, n)
    cell, _ = orc.bin_particles(pos, box, nb, False)
    perm, _, _ = orc.sort_cells(cell, int(np.prod(nb)))
    phi = orc.deposit_volume(pos, d, perm, box, nb, cic=True)
    vb = np.prod(np.array(box) / np.array(nb))
    ref = sum(tent_weights_brute(pos[p], box, nb) * (np.pi * d[p] ** 3 / 6) for p in range(n)) / vb
    np.testing.assert_allclose(phi, ref, rtol=1e-13, atol=1e-16)


@pytest.mark.parametrize("cic", [False, True])
def test_force_deposit_equal_and_opposite(orc, cic):
    box, nb = (1.0, 1.0, 2.0), (4, 4, 8)
    rng = np.random.default_rng(9)
    n = 2000
    pos = rng.random((n, 3)) * np.array(box)
    f = rng.normal(size=(n, 3))
    cell, _ = orc.bin_particles(pos, box, nb, False)
    perm, _, _ = orc.sort_cells(cell, int(np.prod(nb)))
    fc = orc.deposit_force(pos, f, perm, box, nb, cic)
    vb = np.prod(np.array(box) / np.array(nb))
    for a in range(3):
        assert abs(orc.fsum_axis(fc[a]) * vb + orc.fsum_axis(f[:, a])) <= 1e-12 * np.abs(f[:, a]).sum()
    # brute force per cell
    ref = np.zeros((3, int(np.prod(nb))))
    for p in range(n):
        wd = tent_weights_brute(pos[p], box, nb) if cic else np.eye(int(np.prod(nb)))[cell[p]]
        ref -= np.outer(f[p], wd) / vb
    np.testing.assert_allclose(fc, ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("cic", [False, True])
def test_gather_eps_is_transpose(orc, cic):
    box, nb = (1.0, 0.5, 0.75), (4, 2, 3)
    rng = np.random.default_rng(4)
    pos = rng.random((50, 3)) * np.array(box)
    phi = rng.uniform(0, 0.7, int(np.prod(nb)))
    eps_p = orc.gather_eps(pos, phi, box, nb, cic)
    cell, _ = orc.bin_particles(pos, box, nb, False)
    for p in range(50):
        wd = tent_weights_brute(pos[p], box, nb) if cic else np.eye(int(np.prod(nb)))[cell[p]]
        assert eps_p[p] == pytest.approx(float(wd @ (1.0 - phi)), abs=1e-14)
