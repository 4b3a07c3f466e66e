"""GPU parity of the transfer between grids of arbitrary axis-aligned cells
(include/couple_boxmap.h) against the oracle's brute-force box overlaps:
locally refined grids in both directions, the three precisions, many-term rows,
twin cells, a receiver outside the sender grid, and a bed-sized pair (a locally
refined 96^2 x 192 grid and the 128^2 x 256 bulk grid) on sampled receivers."""
import numpy as np
import pytest

import workload as W
from parity_util import TOL_FP32_FIELD, TOL_FP64_FIELD, emax

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    import paper_1807_11834_amd as cpl
    return torch, cpl, oracle


def _fields(nf, n, seed):
    rng = np.random.default_rng(seed)
    f = rng.normal(size=(nf, n))
    f[0] += 3.0                     # one field far from zero, one of mixed sign
    return f


def _check(torch, cpl, oracle, s, r, prec, nf=3, seed=0, label=""):
    src = _fields(nf, s.shape[0], seed)
    m = cpl.BoxMap(s, r, precision=prec)
    try:
        dt = m.dtype
        S = torch.from_numpy(src).to("cuda:0", dt).contiguous()
        D = m.apply(S)
        torch.cuda.synchronize()
        got = D.cpu().numpy().astype(np.float64)
        nnz, mr = m.info()
    finally:
        m.close()
    ref = np.stack([oracle.box_remap(src[k].astype(np.float32 if prec != cpl.COUPLE_FP64 else np.float64), s, r)
                    for k in range(nf)])
    # scale of each receiver value: the weighted average of |src| (the sum may cancel)
    mag = np.stack([oracle.box_remap(np.abs(src[k]), s, r) for k in range(nf)])
    tol = TOL_FP64_FIELD if prec == cpl.COUPLE_FP64 else (1e-3 if prec == cpl.COUPLE_FP32_NAIVE else TOL_FP32_FIELD)
    e = max(emax(got[k], ref[k], mag[k]) for k in range(nf))
    print(f"{label} prec {prec}: nnz {nnz}, longest row {mr}, e_max {e:.2e}", flush=True)
    assert e <= tol, (label, e)
    return e


def test_refined_pairs_all_precisions(env):
    torch, cpl, oracle = env
    box = (1.0, 1.0, 2.0)
    s = W.refined_box_grid(box, (6, 6, 12), (0.0, 1.0, 0.0, 1.0, 0.0, 0.5))
    r = W.refined_box_grid(box, (5, 4, 9), (0.3, 0.9, 0.1, 0.6, 0.4, 1.5), split=3)
    for prec in (cpl.COUPLE_FP32_WIDE, cpl.COUPLE_FP32_KAHAN, cpl.COUPLE_FP32_NAIVE, cpl.COUPLE_FP64):
        _check(torch, cpl, oracle, s, r, prec, label="refined s->r")
        _check(torch, cpl, oracle, r, s, prec, seed=1, label="refined r->s")


def test_many_term_rows_and_single_cells(env):
    torch, cpl, oracle = env
    box = (1.0, 1.0, 1.0)
    fine = W.refined_box_grid(box, (9, 8, 7), (0.0, 0.5, 0.0, 1.0, 0.0, 1.0), split=4)   # up to 64 children
    one = W.box_grid(box, (1, 1, 1))
    coarse = W.box_grid(box, (2, 3, 1))
    _check(torch, cpl, oracle, fine, one, cpl.COUPLE_FP32_WIDE, nf=5, label="fine->one cell")
    _check(torch, cpl, oracle, fine, coarse, cpl.COUPLE_FP32_WIDE, nf=5, label="fine->coarse")
    _check(torch, cpl, oracle, one, fine, cpl.COUPLE_FP64, nf=1, label="one cell->fine")


def test_twin_cells_and_outside_receiver(env):
    torch, cpl, oracle = env
    g = W.refined_box_grid((1.0, 0.5, 0.75), (5, 3, 4), (0.2, 0.7, 0.0, 0.5, 0.3, 0.8))
    src = _fields(2, g.shape[0], 3).astype(np.float32)
    m = cpl.BoxMap(g, g, precision=cpl.COUPLE_FP32_WIDE)
    got = m.apply(torch.from_numpy(src).cuda()).cpu().numpy()
    m.close()
    np.testing.assert_allclose(got, src, rtol=2e-7)
    # a receiver cell outside the sender grid receives 0; one straddling its edge the overlap's average
    r = np.array([[2.0, 3.0, 0.0, 0.5, 0.0, 0.75], [0.8, 1.2, 0.0, 0.5, 0.0, 0.75]])
    m = cpl.BoxMap(g, r, precision=cpl.COUPLE_FP64)
    got = m.apply(torch.from_numpy(src.astype(np.float64)).cuda()).cpu().numpy()
    m.close()
    assert got[0, 0] == 0.0 and got[1, 0] == 0.0
    o = oracle.box_remap(src[0].astype(np.float64), g, r[1:2])
    np.testing.assert_allclose(got[0, 1], o[0], rtol=1e-12)


def test_bed_sized_pair_sampled(env):
    """A locally refined grid over the bed's box (96 x 96 x 192 base cells, the
    bottom quarter split 2:1: 4.9M cells) and the bulk grid (128 x 128 x 256):
    fine -> bulk for four fields and bulk -> fine for four, each on 400 sampled
    receivers against the oracle."""
    torch, cpl, oracle = env
    box = (1.0, 1.0, 2.0)
    f = W.refined_box_grid_fast(box, (96, 96, 192), (0.0, 1.0, 0.0, 1.0, 0.0, 0.5))
    b = W.box_grid(box, (128, 128, 256))
    rng = np.random.default_rng(9)
    for s, r, label in ((f, b, "refined fine -> bulk"), (b, f, "bulk -> refined fine")):
        print(f"case boxmap {label}: {s.shape[0]} -> {r.shape[0]} cells", flush=True)
        src = rng.normal(size=(4, s.shape[0])).astype(np.float32)
        m = cpl.BoxMap(s, r, precision=cpl.COUPLE_FP32_WIDE)
        try:
            D = m.apply(torch.from_numpy(src).cuda())
            torch.cuda.synchronize()
            idx = rng.choice(r.shape[0], 400, replace=False)
            got = D[:, torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.float64)
            nnz, mr = m.info()
        finally:
            m.close()
        ref = np.stack([oracle.box_remap(src[k], s, r[idx]) for k in range(4)])
        mag = np.stack([oracle.box_remap(np.abs(src[k]), s, r[idx]) for k in range(4)])
        e = max(emax(got[k], ref[k], mag[k]) for k in range(4))
        print(f"{label}: nnz {nnz}, longest row {mr}, e_max {e:.2e}", flush=True)
        assert e <= TOL_FP32_FIELD
