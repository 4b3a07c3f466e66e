"""The surrogate trained on the GPU by the library's own kernels, and what it
gains over the method without it (bulk trilinear interpolation), measured against
the fine-grid lookup on held-out particles."""
import json
import os
import time

import numpy as np
import pytest

import workload as W
from parity_util import cfg_for, to_dev, results_dir

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TRAIN_STEPS = int(os.environ.get("SURROGATE_TEST_STEPS", "3000"))


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1807_11834_amd as cpl
    from paper_1807_11834_amd import surrogate as S
    return torch, cpl, S


def _rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _velocities(torch, cpl, cfg, pos, vel, d, fine, vel_source, mlp=None, tol=1e30):
    c = cpl.Config(**{**cfg.__dict__, "vel_source": vel_source, "advect": 0, "mlp_tol": tol})
    h = cpl.Coupler(c)
    if mlp is not None:
        cpl.couple_set_mlp(h.h, mlp.m)
    out = h.step(pos, vel, d, fine, uf=True)
    torch.cuda.synchronize()
    uf = out["uf"].cpu().numpy()
    dg = cpl.diag_dict(out["diag"])
    h.close()
    return uf, dg


def test_training_gain_cube64(env):
    """Pairs from the 64^3 / 256^3 Taylor-Green workload (20,000 particles from
    each of its 100 advected steps), training on the GPU (batch 65,536, Adam lr
    1e-3), validation on fresh particles (seed 101): the surrogate must reach
    1e-3 relative L2 error against the fine lookup and beat bulk interpolation
    (5.7e-3) by a wide margin."""
    torch, cpl, S = env
    dev = "cuda:0"
    w = W.WORKLOADS["cube64_cic"]
    pos, d, vel = W.particles(w)
    n = pos.shape[0]
    cfg = cfg_for(cpl, w, n)
    fine = W.fine_fields_torch(w, dev, torch.float32)
    P, V, D = to_dev(pos, torch, dev), to_dev(vel, torch, dev), to_dev(d, torch, dev)
    t0 = time.perf_counter()
    pool = S.PairPool(w.steps * 20000)
    S.collect(pool, cfg, P, V, D, fine, steps=w.steps, per_step=20000, seed=3)
    t_pairs = time.perf_counter() - t0
    print(f"pairs: {pool.n} in {t_pairs:.1f} s", flush=True)
    mlp = cpl.Mlp(65536)
    mlp.set_params(S.he_uniform(0))
    feat, resid = pool.view()
    mlp.fit_norm(feat, resid)
    t0 = time.perf_counter()
    hist = S.train(mlp, feat, resid, steps=TRAIN_STEPS, batch=65536, seed=3, log_every=500,
                   log=lambda s: print(s, flush=True))
    t_train = time.perf_counter() - t0
    print(f"training: {TRAIN_STEPS} steps in {t_train:.1f} s ({1e3 * t_train / TRAIN_STEPS:.2f} ms/step)", flush=True)
    del pool, feat, resid
    # held-out particles
    pv, dv, vv = W.particles(w, seed=101)
    Pv, Vv, Dv = to_dev(pv, torch, dev), to_dev(vv, torch, dev), to_dev(dv, torch, dev)
    uF, _ = _velocities(torch, cpl, cfg, Pv, Vv, Dv, fine, cpl.COUPLE_VEL_FINE)
    uB, _ = _velocities(torch, cpl, cfg, Pv, Vv, Dv, fine, cpl.COUPLE_VEL_BULK)
    uM, dm = _velocities(torch, cpl, cfg, Pv, Vv, Dv, fine, cpl.COUPLE_VEL_MLP, mlp)
    uMF, dmf = _velocities(torch, cpl, cfg, Pv, Vv, Dv, fine, cpl.COUPLE_VEL_MLP, mlp, tol=1e-3)
    e_bulk, e_mlp, e_mlp_fb = _rel(uB, uF), _rel(uM, uF), _rel(uMF, uF)
    sampled = float(np.sqrt(dm["mlp_err2"] / dm["mlp_ref2"]))
    rec = {"workload": "cube64_cic validation seed 101 (2M particles)", "train_steps": TRAIN_STEPS,
           "batch": 65536, "pairs": int(w.steps * 20000), "train_s": t_train, "pairs_s": t_pairs,
           "loss_first_last": [hist[0][1], hist[-1][1]], "rel_err_bulk": e_bulk, "rel_err_mlp": e_mlp,
           "rel_err_mlp_with_fallback": e_mlp_fb, "sampled_rel_err": sampled,
           "fallback_particles": dmf["n_fallback"], "n": int(pv.shape[0])}
    print(json.dumps(rec), flush=True)
    os.makedirs(results_dir(), exist_ok=True)
    with open(os.path.join(results_dir(), "surrogate_gain_cube64.json"), "w") as f:
        json.dump(rec, f, indent=1)
    mlp.close()
    assert hist[-1][1] < hist[0][1] / 20
    assert e_mlp <= 1e-3 and e_mlp < e_bulk / 3
    assert e_mlp_fb <= e_mlp + 1e-12
