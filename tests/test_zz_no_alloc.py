"""The coupling step without allocation (couple_step_noalloc, include/couple.h)
against couple_step on the same inputs: every output equal bit for bit (the same
kernels), on two calls in a row, the second with fewer particles, fewer bulk
cells and another precision; the scratch limit and the unsupported surrogate
source are rejected before any launch."""
import numpy as np
import pytest

import workload as W
from parity_util import cfg_for, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1807_11834_amd as cpl
    return torch, cpl


def _inputs(torch, w, cfg, dev="cuda:0"):
    pos, d, vel = W.particles(w)
    dt = cfg.dtype
    fine = [to_dev(f, torch, dev, dt) for f in W.fine_fields(w)]
    return {"n": pos.shape[0], "pos": to_dev(pos, torch, dev, dt), "vel": to_dev(vel, torch, dev, dt),
            "diam": to_dev(d, torch, dev, dt), "fine_u": fine[0], "fine_v": fine[1], "fine_w": fine[2],
            "fine_p": fine[3]}


def _both(torch, cpl, cfg, inp):
    """Outputs of couple_step (a handle) and of couple_step_noalloc on copies of
    the same inputs (advection updates pos and vel in place)."""
    n = inp["n"]
    ref = cpl.alloc_outputs(cfg, n, device="cuda:0")
    got = cpl.alloc_outputs(cfg, n, device="cuda:0")
    for o in (ref, got):
        for t in o.values():
            if t is not None:
                t.fill_(-7)              # stale values must all be overwritten
    a = {k: (v.clone() if hasattr(v, "clone") else v) for k, v in inp.items()}
    b = {k: (v.clone() if hasattr(v, "clone") else v) for k, v in inp.items()}
    h = cpl.couple_init(cfg)
    try:
        cpl.couple_step(h, a, ref)
        torch.cuda.synchronize()
    finally:
        cpl.couple_free(h)
    cpl.couple_step_noalloc(cfg, b, got)
    torch.cuda.synchronize()
    return a, ref, b, got


def _assert_same(torch, a, ref, b, got, label):
    for k, t in ref.items():
        if t is None:
            continue
        assert torch.equal(t, got[k]), f"{label}: output {k} differs"
    for k in ("pos", "vel"):
        assert torch.equal(a[k], b[k]), f"{label}: advected {k} differs"


def test_noalloc_matches_couple_step_twice(env):
    torch, cpl = env
    # first call: 60,000 particles, 24 x 20 x 16 bulk cells, FP32, CIC, advection
    w1 = W.small_workload(nb=(24, 20, 16), ratio=4, box=(1.2, 1.0, 0.8), n=60000, seed=901, precision="fp32")
    c1 = cfg_for(cpl, w1, 60000, advect=1, dt=1e-4)
    print("case noalloc 1: n=60000 nb=(24, 20, 16) fp32 cic advect", flush=True)
    _assert_same(torch, *_both(torch, cpl, c1, _inputs(torch, w1, c1)), "call 1")
    # second call, smaller: 3001 particles, 7 x 5 x 6 bulk cells, FP64, NGP, bulk velocity
    w2 = W.small_workload(nb=(7, 5, 6), ratio=2, box=(0.7, 0.5, 0.6), n=3001, seed=902, precision="fp64",
                          deposit="ngp")
    c2 = cfg_for(cpl, w2, 3001, vel_source=cpl.COUPLE_VEL_BULK)
    print("case noalloc 2: n=3001 nb=(7, 5, 6) fp64 ngp bulk", flush=True)
    _assert_same(torch, *_both(torch, cpl, c2, _inputs(torch, w2, c2)), "call 2")


def test_noalloc_semi_implicit_and_two_fluid(env):
    torch, cpl = env
    w = W.small_workload(nb=(10, 9, 8), ratio=4, box=(1.0, 0.9, 0.8), n=20000, seed=903, precision="fp32")
    c = cfg_for(cpl, w, 20000)
    c.semi_implicit, c.vof = 1, 1
    inp = _inputs(torch, w, c)
    inp["fine_alpha"] = to_dev(W.fine_alpha(w), torch, "cuda:0", c.dtype)
    print("case noalloc semi-implicit + two-fluid", flush=True)
    _assert_same(torch, *_both(torch, cpl, c, inp), "semi + vof")


def test_noalloc_rejections(env):
    torch, cpl = env
    # 4M particles need ~190 MB of scratch: more than the static array
    big = cpl.Config(nb=(8, 8, 8), ratio=1, max_particles=4_000_000)
    n = 4_000_000
    dev = "cuda:0"
    inp = {"n": n, "pos": torch.zeros(n, 3, device=dev), "vel": torch.zeros(n, 3, device=dev),
           "diam": torch.zeros(n, device=dev)}
    f = torch.zeros(big.n_fine, device=dev)
    inp.update(fine_u=f, fine_v=f, fine_w=f, fine_p=f)
    out = cpl.alloc_outputs(big, n, device=dev)
    out["drag"].fill_(5.0)
    with pytest.raises(cpl.CoupleError) as ei:
        cpl.couple_step_noalloc(big, inp, out)
    assert ei.value.code == cpl.COUPLE_ECAPACITY and "scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert bool((out["drag"] == 5.0).all())           # nothing was launched
    mlp = cpl.Config(nb=(8, 8, 8), ratio=1, vel_source=cpl.COUPLE_VEL_MLP, max_particles=10)
    with pytest.raises(cpl.CoupleError) as ei:
        small = {**inp, "n": 10, "pos": inp["pos"][:10], "vel": inp["vel"][:10], "diam": inp["diam"][:10]}
        cpl.couple_step_noalloc(mlp, small, cpl.alloc_outputs(mlp, 10, device=dev))
    assert ei.value.code == cpl.COUPLE_EINVAL and "MLP" in str(ei.value)
