"""FP64 CPU oracle of the dual-grid coupling exchange -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and its
Python binding) never imports, links or calls anything here, and nothing here
imports the product package.

The per-stage definitions live in ``couple_oracle.c`` (plain C, FP64), built into
``liboracle.so`` by ``build()``; this module loads it with ctypes and composes the
stages in the order of one coupling step (Fig. 1, Sec. 2.1-2.2):

    bin -> volume deposition -> restriction (+ pressure gradient) -> fluid value
    at particles -> drag -> momentum-source deposition (+ optional semi-implicit
    split K, KU) -> prolongation -> conservation sums (-> explicit Euler advection)

The learned surrogate's oracle is in :mod:`oracle.mlp`.

Parity status: every stage is pinned by closed forms, invariants or brute force in
``tests/test_oracle_*.py``; none is "parity unpinned".
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "couple_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force=True):
    """Compile the C oracle with gcc (plain FP64, no fast-math, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"])
        os.replace(_LIB + ".tmp", _LIB)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        P = C.c_void_p
        I64 = C.c_int64
        I = C.c_int
        D = C.c_double
        L.orc_bin.argtypes = [I64, P, P, P, I, P]
        L.orc_bin.restype = I64
        L.orc_sort.argtypes = [I64, P, I64, P, P, P]
        L.orc_sort.restype = None
        L.orc_weights.argtypes = [P, P, P, I, I, P, P]
        L.orc_weights.restype = I
        L.orc_deposit_volume.argtypes = [I64, P, P, P, P, P, I, I, P]
        L.orc_deposit_force.argtypes = [I64, P, P, P, P, P, I, I, P]
        L.orc_deposit_semi.argtypes = [I64, P, P, P, P, P, P, I, I, P, P]
        L.orc_gather_eps.argtypes = [I64, P, P, P, P, I, I, P]
        L.orc_restrict.argtypes = [P, P, I, P]
        L.orc_gradient.argtypes = [P, P, P, P]
        L.orc_interp.argtypes = [P, P, P, I64, P, I, P]
        L.orc_drag.argtypes = [I64, P, P, P, P, D, D, D, P, P]
        L.orc_drag.restype = I64
        L.orc_drag_vof.argtypes = [I64, P, P, P, P, P, D, D, D, D, D, P, P]
        L.orc_drag_vof.restype = I64
        L.orc_prolong.argtypes = [P, P, I, I, P]
        L.orc_prolong_at.argtypes = [P, P, I, I, I64, P, P]
        L.orc_advect.argtypes = [I64, P, P, P, P, D, D, P, I]
        L.orc_particle_volumes.argtypes = [I64, P, P]
        L.orc_remap.argtypes = [P, P, P, P, P, P]
        L.orc_box_remap.argtypes = [I64, P, I64, P, P, P]
        L.orc_box_remap.restype = None
        L.orc_set_threads.argtypes = [I]
        L.orc_set_threads.restype = None
        L.orc_get_threads.argtypes = []
        L.orc_get_threads.restype = I
        for name in ("orc_deposit_volume", "orc_deposit_force", "orc_deposit_semi", "orc_gather_eps", "orc_restrict",
                     "orc_gradient", "orc_interp", "orc_prolong", "orc_prolong_at", "orc_advect",
                     "orc_particle_volumes", "orc_remap"):
            getattr(L, name).restype = None
        L.orc_set_threads(1)    # one thread unless asked (set_threads)
        _lib = L
    return _lib


def set_threads(k):
    """Threads of the oracle's independent-iteration loops (the canonical-order
    sums are always serial; results do not depend on k).  Returns the previous
    setting."""
    prev = lib().orc_get_threads()
    lib().orc_set_threads(int(k))
    return prev


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32x3(nb):
    return np.asarray(nb, dtype=np.int32)


# ---------------------------------------------------------------------------
# Stage wrappers (numpy in, numpy out)
# ---------------------------------------------------------------------------

def bin_particles(pos, box, nb, prec32):
    """Containing bulk cell per particle; returns (cell int32[n], n_outside)."""
    pos = _f64(pos).reshape(-1, 3)
    cell = np.empty(pos.shape[0], dtype=np.int32)
    nout = lib().orc_bin(pos.shape[0], _p(pos), _p(_f64(box)), _p(_i32x3(nb)), int(prec32), _p(cell))
    return cell, int(nout)


def sort_cells(cell, ncell):
    """Canonical (cell, id) order: (perm, count, start)."""
    cell = np.ascontiguousarray(cell, dtype=np.int32)
    n = cell.shape[0]
    perm = np.empty(n, dtype=np.int32)
    count = np.empty(ncell, dtype=np.int32)
    start = np.empty(ncell + 1, dtype=np.int32)
    lib().orc_sort(n, _p(cell), ncell, _p(perm), _p(count), _p(start))
    return perm, count, start


def weights(x, box, nb, cic, prec32=False):
    """(cells int64[m], w float64[m]) of one particle at position x."""
    x = _f64(x).reshape(3)
    cells = np.empty(8, dtype=np.int64)
    w = np.empty(8, dtype=np.float64)
    m = lib().orc_weights(_p(x), _p(_f64(box)), _p(_i32x3(nb)), int(cic), int(prec32), _p(cells), _p(w))
    return cells[:m].copy(), w[:m].copy()


def deposit_volume(pos, diam, perm, box, nb, cic, prec32=False):
    pos = _f64(pos).reshape(-1, 3)
    phi = np.empty(int(np.prod(nb)), dtype=np.float64)
    lib().orc_deposit_volume(pos.shape[0], _p(pos), _p(_f64(diam)), _p(np.ascontiguousarray(perm, np.int32)),
                             _p(_f64(box)), _p(_i32x3(nb)), int(cic), int(prec32), _p(phi))
    return phi


def deposit_force(pos, force, perm, box, nb, cic, prec32=False):
    pos = _f64(pos).reshape(-1, 3)
    fc = np.empty(3 * int(np.prod(nb)), dtype=np.float64)
    lib().orc_deposit_force(pos.shape[0], _p(pos), _p(_f64(force).reshape(-1, 3)),
                            _p(np.ascontiguousarray(perm, np.int32)), _p(_f64(box)), _p(_i32x3(nb)),
                            int(cic), int(prec32), _p(fc))
    return fc.reshape(3, -1)


def deposit_semi(pos, beta, vel, perm, box, nb, cic, prec32=False):
    """Semi-implicit source fields: (K [ncell], KU [3, ncell])."""
    pos = _f64(pos).reshape(-1, 3)
    nc = int(np.prod(nb))
    K = np.empty(nc, dtype=np.float64)
    KU = np.empty(3 * nc, dtype=np.float64)
    lib().orc_deposit_semi(pos.shape[0], _p(pos), _p(_f64(beta)), _p(_f64(vel).reshape(-1, 3)),
                           _p(np.ascontiguousarray(perm, np.int32)), _p(_f64(box)), _p(_i32x3(nb)),
                           int(cic), int(prec32), _p(K), _p(KU))
    return K, KU.reshape(3, -1)


def gather_eps(pos, phi, box, nb, cic, prec32=False):
    pos = _f64(pos).reshape(-1, 3)
    out = np.empty(pos.shape[0], dtype=np.float64)
    lib().orc_gather_eps(pos.shape[0], _p(pos), _p(_f64(phi)), _p(_f64(box)), _p(_i32x3(nb)),
                         int(cic), int(prec32), _p(out))
    return out


def restrict(qf, nb, r):
    qf = _f64(qf)
    out = np.empty(int(np.prod(nb)), dtype=np.float64)
    lib().orc_restrict(_p(qf), _p(_i32x3(nb)), int(r), _p(out))
    return out


def gradient(P, nb, box):
    out = np.empty(3 * int(np.prod(nb)), dtype=np.float64)
    lib().orc_gradient(_p(_f64(P)), _p(_i32x3(nb)), _p(_f64(box)), _p(out))
    return out.reshape(3, -1)


def interp(q, n, box, pos, prec32=False):
    pos = _f64(pos).reshape(-1, 3)
    out = np.empty(pos.shape[0], dtype=np.float64)
    lib().orc_interp(_p(_f64(q)), _p(_i32x3(n)), _p(_f64(box)), pos.shape[0], _p(pos), int(prec32), _p(out))
    return out


def drag(uf, up, diam, eps_p, rho_f, mu_f, eps_min):
    """(force [n,3], beta [n], n_clamped)."""
    uf = _f64(uf).reshape(-1, 3)
    n = uf.shape[0]
    force = np.empty((n, 3), dtype=np.float64)
    beta = np.empty(n, dtype=np.float64)
    nc = lib().orc_drag(n, _p(uf), _p(_f64(up).reshape(-1, 3)), _p(_f64(diam)), _p(_f64(eps_p)),
                        float(rho_f), float(mu_f), float(eps_min), _p(force), _p(beta))
    return force, beta, int(nc)


def drag_vof(uf, up, diam, eps_p, alpha_p, rho1, mu1, rho2, mu2, eps_min):
    """Two-fluid drag: (force [n,3], beta [n], n_clamped) with the density and
    viscosity at each particle mixed by its liquid fraction alpha_p."""
    uf = _f64(uf).reshape(-1, 3)
    n = uf.shape[0]
    force = np.empty((n, 3), dtype=np.float64)
    beta = np.empty(n, dtype=np.float64)
    nc = lib().orc_drag_vof(n, _p(uf), _p(_f64(up).reshape(-1, 3)), _p(_f64(diam)), _p(_f64(eps_p)),
                            _p(_f64(alpha_p)), float(rho1), float(mu1), float(rho2), float(mu2), float(eps_min),
                            _p(force), _p(beta))
    return force, beta, int(nc)


def prolong(B, nb, r, conservative=True):
    out = np.empty(int(np.prod(nb)) * r ** 3, dtype=np.float64)
    lib().orc_prolong(_p(_f64(B)), _p(_i32x3(nb)), int(r), int(conservative), _p(out))
    return out


def prolong_at(B, nb, r, fidx, conservative=True):
    fidx = np.ascontiguousarray(fidx, dtype=np.int64)
    out = np.empty(fidx.shape[0], dtype=np.float64)
    lib().orc_prolong_at(_p(_f64(B)), _p(_i32x3(nb)), int(r), int(conservative), fidx.shape[0], _p(fidx), _p(out))
    return out


def advect(pos, vel, diam, force, rho_p, dt, box, prec32=False):
    """Return (new_pos, new_vel) as float64 arrays (inputs untouched)."""
    pos = _f64(pos).reshape(-1, 3).copy()
    vel = _f64(vel).reshape(-1, 3).copy()
    lib().orc_advect(pos.shape[0], _p(pos), _p(vel), _p(_f64(diam)), _p(_f64(force).reshape(-1, 3)),
                     float(rho_p), float(dt), _p(_f64(box)), int(prec32))
    return pos, vel


def remap(src, src_nodes, dst_nodes):
    """Volume-weighted transfer of a cell field between two rectilinear grids over
    the same box.  ``src_nodes`` / ``dst_nodes`` are three 1-D arrays of node
    coordinates (x, y, z); ``src`` is (nz, ny, nx) of the sender grid.  Returns
    the receiver field (nz, ny, nx)."""
    ns = np.array([len(a) - 1 for a in src_nodes], dtype=np.int32)
    nd = np.array([len(a) - 1 for a in dst_nodes], dtype=np.int32)
    sn = np.concatenate([_f64(a) for a in src_nodes])
    dn = np.concatenate([_f64(a) for a in dst_nodes])
    src = _f64(src).reshape(-1)
    assert src.shape[0] == int(np.prod(ns))
    out = np.empty(int(np.prod(nd)), dtype=np.float64)
    lib().orc_remap(_p(ns), _p(sn), _p(nd), _p(dn), _p(src), _p(out))
    return out.reshape(nd[2], nd[1], nd[0])


def box_remap(src, sender_boxes, receiver_boxes):
    """Volume-weighted transfer between two grids of axis-aligned cells (each
    grid an [n, 6] array of boxes x0, x1, y0, y1, z0, z1): receiver value =
    sum over overlapping sender cells of |overlap| * value / |receiver cell|."""
    sb = _f64(sender_boxes).reshape(-1, 6)
    rb = _f64(receiver_boxes).reshape(-1, 6)
    src = _f64(src).reshape(-1)
    assert src.shape[0] == sb.shape[0]
    out = np.empty(rb.shape[0], dtype=np.float64)
    lib().orc_box_remap(sb.shape[0], _p(sb), rb.shape[0], _p(rb), _p(src), _p(out))
    return out


def particle_volumes(diam):
    diam = _f64(diam)
    out = np.empty(diam.shape[0], dtype=np.float64)
    lib().orc_particle_volumes(diam.shape[0], _p(diam), _p(out))
    return out


# ---------------------------------------------------------------------------
# One coupling step
# ---------------------------------------------------------------------------

def fsum_axis(a):
    """Correctly rounded sum of a 1-D array (math.fsum)."""
    return math.fsum(np.asarray(a, dtype=np.float64).ravel().tolist())


def restrict_all(fine, grid):
    """Restricted U, P, bulk gradient G and the magnitude scales of one fine field set."""
    nb, r, box = tuple(grid.nb), int(grid.ratio), tuple(float(b) for b in grid.box)
    U = np.stack([restrict(f, nb, r) for f in fine[:3]])
    P = restrict(fine[3], nb, r)
    G = gradient(P, nb, box)
    U_mag = np.stack([restrict(np.abs(np.asarray(f, dtype=np.float64)), nb, r) for f in fine[:3]])
    P_mag = restrict(np.abs(np.asarray(fine[3], dtype=np.float64)), nb, r)
    return {"U": U, "P": P, "G": G, "U_mag": U_mag, "P_mag": P_mag}


def step(pos, vel, diam, fine, grid, rho_f=1000.0, mu_f=1e-3, rho_p=2500.0, eps_min=0.3,
         cic=True, prec32=True, vel_source="fine", advect_dt=None, fine_out="full",
         fine_sample=None, bulk_velocity=None, restricted=None, semi_implicit=False, alpha=None, rho2=None,
         mu2=None):
    """One coupling step in FP64.

    ``fine`` is (u, v, w, p), each (nfz, nfy, nfx).  ``vel_source`` is "fine"
    (trilinear lookup on the fine grid) or "bulk" (trilinear on the restricted
    bulk velocity) or "given" (``bulk_velocity`` is the fluid velocity [n,3] at
    the particles, e.g. a surrogate's prediction).  ``fine_out`` is "full" (all
    fine cells), "sample" (only the flat indices ``fine_sample``) or "none".
    ``restricted`` reuses the output of :func:`restrict_all` for the same fine
    fields (the restriction does not depend on the particles).  ``semi_implicit``
    adds the semi-implicit source fields K, KU (bulk and prolonged) and their sums.
    ``alpha`` (fine liquid volume fraction, (nfz, nfy, nfx)) turns on the
    two-fluid drag: alpha is restricted to the bulk grid, interpolated
    trilinearly to each particle, and mixes (rho_f, mu_f) with (rho2, mu2).
    Returns a dict of numpy arrays and the diagnostics.
    """
    box = tuple(float(b) for b in grid.box)
    nb = tuple(int(n) for n in grid.nb)
    r = int(grid.ratio)
    nf = tuple(n * r for n in nb)
    ncell = nb[0] * nb[1] * nb[2]
    vb = (box[0] / nb[0]) * (box[1] / nb[1]) * (box[2] / nb[2])
    vf = vb / r ** 3
    pos = _f64(pos).reshape(-1, 3)
    vel = _f64(vel).reshape(-1, 3)
    diam = _f64(diam)
    n = pos.shape[0]
    out = {}
    cell, nout = bin_particles(pos, box, nb, prec32)
    perm, count, start = sort_cells(cell, ncell)
    out.update(cell=cell, perm=perm, count=count, start=start)
    phi = deposit_volume(pos, diam, perm, box, nb, cic, prec32)
    out["phi"] = phi
    rr = restricted if restricted is not None else restrict_all(fine, grid)
    out.update(rr)   # U, P, G and the magnitude scales used by the parity metric
    U = rr["U"]
    eps_p = gather_eps(pos, phi, box, nb, cic, prec32)
    if vel_source == "fine":
        uf = np.stack([interp(f, nf, box, pos, prec32) for f in fine[:3]], axis=1)
    elif vel_source == "bulk":
        uf = np.stack([interp(U[a], nb, box, pos, prec32) for a in range(3)], axis=1)
    elif vel_source == "given":
        uf = _f64(bulk_velocity).reshape(-1, 3)
    else:
        raise ValueError(vel_source)
    if alpha is None:
        force, beta, nclamp = drag(uf, vel, diam, eps_p, rho_f, mu_f, eps_min)
    else:
        alpha_b = restrict(alpha, nb, r)
        alpha_p = interp(alpha_b, nb, box, pos, prec32)
        force, beta, nclamp = drag_vof(uf, vel, diam, eps_p, alpha_p, rho_f, mu_f, rho2, mu2, eps_min)
        out.update(alpha=alpha_b, alpha_p=alpha_p)
    out.update(eps_p=eps_p, uf=uf, drag=force, beta=beta)
    Fc = deposit_force(pos, force, perm, box, nb, cic, prec32)
    out["F"] = Fc
    # magnitude of the deposited terms, (1/V_b) sum_p w_pc |F_p|: the scale of
    # the summation error of F_fpi (used by the parity metric, not by the method)
    fmag = np.zeros_like(force)
    fmag[:, 0] = np.sqrt((force ** 2).sum(axis=1))
    out["F_mag"] = -deposit_force(pos, fmag, perm, box, nb, cic, prec32)[0]
    eps_b = 1.0 - phi
    fields = [eps_b, Fc[0], Fc[1], Fc[2]]
    if fine_out == "full":
        fo = [prolong(B, nb, r, True) for B in fields]
        out["fine_eps"], out["fine_F"] = fo[0], np.stack(fo[1:])
    elif fine_out == "sample":
        fo = [prolong_at(B, nb, r, fine_sample, True) for B in fields]
        out["fine_eps"], out["fine_F"] = fo[0], np.stack(fo[1:])
    if semi_implicit:
        K, KU = deposit_semi(pos, beta, vel, perm, box, nb, cic, prec32)
        out["K"], out["KU"] = K, KU
        # (1/V_b) sum_p w_pc beta_p |u_p|: the scale of the summation error of KU
        out["KU_mag"] = deposit_semi(pos, beta * np.sqrt((vel ** 2).sum(axis=1)), np.ones_like(vel), perm,
                                     box, nb, cic, prec32)[1][0]
        sf = [K, KU[0], KU[1], KU[2]]
        if fine_out == "full":
            fo = [prolong(B, nb, r, True) for B in sf]
            out["fine_K"], out["fine_KU"] = fo[0], np.stack(fo[1:])
        elif fine_out == "sample":
            fo = [prolong_at(B, nb, r, fine_sample, True) for B in sf]
            out["fine_K"], out["fine_KU"] = fo[0], np.stack(fo[1:])
    vp = particle_volumes(diam)
    diag = {
        "V_tot": fsum_axis(vp),
        "V_dep": fsum_axis(phi) * vb,
        "sum_Fp": [fsum_axis(force[:, a]) for a in range(3)],
        "S_b": [fsum_axis(Fc[a]) * vb for a in range(3)],
        "n_clamped": nclamp,
        "n_outside": nout,
        "max_phi": float(phi.max()) if ncell else 0.0,
    }
    if fine_out == "full":
        diag["S_f"] = [fsum_axis(out["fine_F"][a]) * vf for a in range(3)]
        diag["E_f"] = fsum_axis(out["fine_eps"]) * vf
    if semi_implicit:
        diag["K_p"] = fsum_axis(beta)
        diag["KU_p"] = [fsum_axis(beta * vel[:, a]) for a in range(3)]
        diag["K_b"] = fsum_axis(out["K"]) * vb
        diag["KU_b"] = [fsum_axis(out["KU"][a]) * vb for a in range(3)]
        if fine_out == "full":
            diag["K_f"] = fsum_axis(out["fine_K"]) * vf
            diag["KU_f"] = [fsum_axis(out["fine_KU"][a]) * vf for a in range(3)]
    out["diag"] = diag
    if advect_dt is not None:
        out["pos_new"], out["vel_new"] = advect(pos, vel, diam, force, rho_p, advect_dt, box, prec32)
    return out
