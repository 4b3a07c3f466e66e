"""GPU parity of the grid-to-grid transfer between non-nested grids (the sender ->
receiver interpolation of Sec. 2.3) against the FP64 oracle, through the C ABI.

e_max of a receiver cell: |g - o| / max(M_c, 1e-3 max M), with M the transfer of
|src| (the size of the terms the cell sums).  FP32 within 1e-4, FP64 within 1e-6.
All three kernels are covered: receiver rows from LDS-staged sender rows, tiles
of receiver rows finer than the sender (with and without four-cell stores),
and one thread per receiver cell for sender rows longer than the LDS buffer.
At the packed bed's full fine-grid size the transfer is compared on sampled
receiver cells (each one an oracle call on the sender cells it overlaps) and
checked for constants and the conserved integral.
"""
import numpy as np
import pytest

from parity_util import TOL_FP32_FIELD, TOL_FP64_FIELD, TOL_NAIVE, emax

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    import paper_1807_11834_amd as cpl
    return torch, cpl, oracle


def uniform_nodes(n, box):
    return [np.linspace(0.0, box[a], n[a] + 1) for a in range(3)]


def random_nodes(rng, n, box):
    out = []
    for a in range(3):
        x = np.concatenate([[0.0], np.cumsum(rng.uniform(0.3, 1.7, n[a]))])
        x = x / x[-1] * box[a]
        x[-1] = box[a]
        out.append(x)
    return out


def volumes(nodes):
    d = [np.diff(x) for x in nodes]
    return d[2][:, None, None] * d[1][None, :, None] * d[0][None, None, :]


CASES = [
    # (sender cells, receiver cells, box, spacing, precision, fields)
    ((40, 36, 28), (15, 13, 11), (1.0, 0.9, 0.7), "uniform", "fp32w", 1),
    ((7, 5, 6), (23, 19, 17), (1.0, 1.0, 1.2), "uniform", "fp32w", 3),
    ((17, 13, 11), (9, 14, 6), (0.8, 1.3, 0.6), "random", "fp64", 2),
    ((32, 24, 20), (8, 6, 5), (1.0, 0.75, 0.625), "uniform", "fp32n", 1),
    ((1, 30, 2), (1, 7, 5), (0.1, 1.0, 0.3), "random", "fp32w", 1),
    ((61, 3, 47), (29, 5, 13), (1.0, 0.1, 0.8), "random", "fp32w", 1),
    # receiver finer in y and z with rows a multiple of 4 long: the tile kernel's
    # four-cell stores; with random spacing some receiver rows overlap more
    # than 2 x 2 sender rows (the table's overflow path)
    ((6, 9, 8), (16, 11, 10), (1.0, 0.8, 0.6), "random", "fp32w", 2),
    ((5, 4, 3), (12, 8, 8), (1.0, 1.0, 1.0), "uniform", "fp64", 1),
    # single cells
    ((1, 1, 1), (1, 1, 1), (0.5, 0.25, 2.0), "uniform", "fp32w", 2),
    ((1, 1, 1), (3, 2, 5), (0.5, 0.25, 2.0), "random", "fp64", 1),
    ((4, 7, 3), (1, 1, 1), (0.5, 0.25, 2.0), "random", "fp32w", 1),
    # sender rows longer than the LDS row buffer: the per-cell kernel
    ((20000, 2, 1), (7, 3, 2), (1.0, 0.2, 0.1), "random", "fp32w", 1),
    ((9000, 1, 2), (13, 1, 1), (1.0, 0.1, 0.1), "uniform", "fp64", 1),
    # Kahan-compensated FP32 sums in each kernel: rows, tile, per-cell
    ((40, 36, 28), (15, 13, 11), (1.0, 0.9, 0.7), "random", "fp32k", 2),
    ((6, 9, 8), (16, 11, 10), (1.0, 0.8, 0.6), "random", "fp32k", 2),
    ((20000, 2, 1), (7, 3, 2), (1.0, 0.2, 0.1), "random", "fp32k", 1),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-{c[1]}-{c[3]}-{c[4]}-f{c[5]}" for c in CASES])
def test_remap_parity(env, case):
    torch, cpl, oracle = env
    ns, nd, box, spacing, prec, nf = case
    rng = np.random.default_rng(500 + CASES.index(case))
    S = uniform_nodes(ns, box) if spacing == "uniform" else random_nodes(rng, ns, box)
    D = uniform_nodes(nd, box) if spacing == "uniform" else random_nodes(rng, nd, box)
    precision = {"fp32w": cpl.COUPLE_FP32_WIDE, "fp32k": cpl.COUPLE_FP32_KAHAN, "fp32n": cpl.COUPLE_FP32_NAIVE, "fp64": cpl.COUPLE_FP64}[prec]
    src = rng.normal(1.0, 2.0, (nf, ns[2], ns[1], ns[0]))
    print(f"case remap {case}", flush=True)
    r = cpl.Remap(S, D, precision=precision)
    try:
        src_d = torch.from_numpy(src).to(r.dtype).cuda()
        got = r.apply(src_d).cpu().numpy().astype(np.float64)
        nnz_axis, nnz = r.info()
    finally:
        r.close()
    assert nnz == int(np.prod(nnz_axis))
    src_used = src_d.double().cpu().numpy()        # the values the kernel read
    tol = TOL_FP64_FIELD if prec == "fp64" else (TOL_NAIVE if prec == "fp32n" else TOL_FP32_FIELD)
    for f in range(nf):
        ref = oracle.remap(src_used[f], S, D)
        mag = oracle.remap(np.abs(src_used[f]), S, D)
        e, det = emax(got[f].ravel(), ref.ravel(), mag.ravel(), detail=True)
        assert e <= tol, f"field {f}: e_max {e:.3e} > {tol}; worst {det}"
        # integral conserved by the GPU's own output
        tot = (src_used[f] * volumes(S)).sum()
        scale = (np.abs(src_used[f]) * volumes(S)).sum()
        assert abs((got[f] * volumes(D)).sum() - tot) <= (1e-6 if prec != "fp64" else 1e-12) * scale


def test_remap_identical_grids_copy_bitwise(env):
    torch, cpl, _ = env
    rng = np.random.default_rng(510)
    N = random_nodes(rng, (37, 21, 9), (1.0, 0.5, 0.25))
    r = cpl.Remap(N, N)
    try:
        x = torch.from_numpy(rng.normal(size=(9, 21, 37)).astype(np.float32)).cuda()
        y = r.apply(x)
        torch.cuda.synchronize()
        assert torch.equal(x, y)
    finally:
        r.close()


def test_remap_nested_equals_coupling_restriction(env):
    """A nested pair (ratio 4) reproduces the coupling step's restricted velocity."""
    torch, cpl, _ = env
    import workload as W
    from parity_util import cfg_for, run_gpu
    w = W.small_workload(nb=(9, 7, 5), ratio=4, box=(0.9, 0.7, 0.5), n=500, seed=511, precision="fp32")
    pos, d, vel = W.particles(w)
    fine = W.fine_fields(w)
    g = run_gpu(cpl, torch, cfg_for(cpl, w, 500), pos, vel, d, fine)
    r = cpl.Remap(uniform_nodes(w.grid.nf, w.grid.box), uniform_nodes(w.grid.nb, w.grid.box))
    try:
        U = r.apply(torch.from_numpy(np.stack(fine[:3])).cuda()).cpu().numpy()
    finally:
        r.close()
    Ug = g["bulk_U"].reshape(U.shape)
    scale = np.abs(Ug).max()
    np.testing.assert_allclose(U, Ug, rtol=0, atol=1e-6 * scale)


def _sample_oracle(oracle, src_d, S, D, cells):
    """Receiver cells `cells` [(i, j, k)], each from an oracle call on the sender
    block it overlaps."""
    out = []
    for (i, j, k) in cells:
        sl, sn, dn = [], [], []
        for a, idx in enumerate((i, j, k)):
            lo, hi = D[a][idx], D[a][idx + 1]
            j0 = int(np.searchsorted(S[a], lo, side="right") - 1)
            j1 = int(np.searchsorted(S[a], hi, side="left"))
            j0 = max(j0, 0)
            sl.append(slice(j0, j1))
            sn.append(S[a][j0:j1 + 1])
            dn.append(np.array([lo, hi]))
        block = src_d[sl[2], sl[1], sl[0]].double().cpu().numpy()
        # the block's end nodes extend beyond the receiver cell: clip them so both
        # grids span the same interval (the overlaps are unchanged)
        for a in range(3):
            sn[a] = sn[a].copy()
            sn[a][0], sn[a][-1] = dn[a][0], dn[a][1]
        out.append(float(oracle.remap(block, sn, dn).ravel()[0]))
    return np.array(out)


def test_remap_bed_fine_grid_full_size_sampled(env):
    """The bed's fine grid (512 x 512 x 1024 over 1 x 1 x 2) to a non-nested
    192 x 192 x 384 grid and back, FP32 Kahan: sampled cells against the oracle,
    constants, and the integral."""
    torch, cpl, oracle = env
    box = (1.0, 1.0, 2.0)
    nf, nc = (512, 512, 1024), (192, 192, 384)
    F, Cn = uniform_nodes(nf, box), uniform_nodes(nc, box)
    print("case remap bed full size", flush=True)
    g = torch.Generator(device="cuda").manual_seed(512)
    src = torch.rand((nf[2], nf[1], nf[0]), generator=g, device="cuda", dtype=torch.float32) - 0.25
    rng = np.random.default_rng(512)
    down = cpl.Remap(F, Cn)
    up = cpl.Remap(Cn, F)
    try:
        c = down.apply(src)
        cells = [(int(rng.integers(nc[0])), int(rng.integers(nc[1])), int(rng.integers(nc[2]))) for _ in range(200)]
        cells += [(0, 0, 0), (nc[0] - 1, nc[1] - 1, nc[2] - 1), (nc[0] - 1, 0, nc[2] // 2)]
        ref = _sample_oracle(oracle, src, F, Cn, cells)
        gotc = np.array([float(c[k, j, i]) for (i, j, k) in cells])
        assert np.abs(gotc - ref).max() <= 1e-5 * max(np.abs(ref).max(), 1.0)
        # integral (FP64 sums of the FP32 fields)
        vf = np.prod([box[a] / nf[a] for a in range(3)])
        vc = np.prod([box[a] / nc[a] for a in range(3)])
        tot = float(src.double().sum()) * vf
        scale = float(src.double().abs().sum()) * vf
        assert abs(float(c.double().sum()) * vc - tot) <= 1e-6 * scale
        # back to the fine grid: sampled fine cells, integral
        fb = up.apply(c)
        fcells = [(int(rng.integers(nf[0])), int(rng.integers(nf[1])), int(rng.integers(nf[2]))) for _ in range(200)]
        ref_f = _sample_oracle(oracle, c, Cn, F, fcells)
        got_f = np.array([float(fb[k, j, i]) for (i, j, k) in fcells])
        assert np.abs(got_f - ref_f).max() <= 1e-5 * max(np.abs(ref_f).max(), 1.0)
        assert abs(float(fb.double().sum()) * vf - float(c.double().sum()) * vc) <= 1e-6 * scale
        # constants
        one = down.apply(torch.full_like(src, 0.375))
        assert float((one - 0.375).abs().max()) <= 4e-7
        del one, fb, c
    finally:
        down.close()
        up.close()
    del src
    torch.cuda.empty_cache()
