"""CPU checks of the C ABI: the library loads, exports every entry point that
the headers under include/ declare, its structs have the
headers' layout, and argument validation rejects bad calls before any device
work."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("couple.h", "couple_mlp.h", "couple_remap.h",
                                                       "couple_boxmap.h", "couple_hbmref.h")]
LIB = os.path.join(ROOT, "paper_1807_11834_amd", "libcouple.so")


def declared_functions():
    text = "".join(open(h).read() for h in HEADERS)
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(couple_[a-z_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    assert declared_functions() == sorted([
        "couple_free", "couple_init", "couple_last_error", "couple_step", "couple_timing_begin", "couple_timing_end",
        "couple_step_noalloc",
        "couple_mlp_init", "couple_mlp_free", "couple_mlp_last_error", "couple_mlp_set_params",
        "couple_mlp_set_norm", "couple_mlp_fit_norm", "couple_mlp_get_state", "couple_mlp_set_state",
        "couple_mlp_forward", "couple_mlp_grads", "couple_mlp_adam", "couple_mlp_train_step",
        "couple_mlp_features", "couple_set_mlp",
        "couple_remap_init", "couple_remap_apply", "couple_remap_info", "couple_remap_free", "couple_remap_last_error",
        "couple_boxmap_init", "couple_boxmap_apply", "couple_boxmap_info", "couple_boxmap_free",
        "couple_boxmap_last_error",
        "couple_part_init", "couple_part_step", "couple_part_comm_matrix", "couple_part_free",
        "couple_part_last_error", "couple_hbmref"])


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("libcouple.so not built")
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing


def test_struct_layout_matches_header(tmp_path):
    import paper_1807_11834_amd as cpl
    import ctypes as C
    src = tmp_path / "layout.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "couple_mlp.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(couple_config), offsetof(couple_config, rho_f),
         offsetof(couple_config, deposit), offsetof(couple_config, dt), offsetof(couple_config, max_particles),
         offsetof(couple_config, mlp_tol), offsetof(couple_config, mlp_period), offsetof(couple_config, semi_implicit));
  printf("%zu %zu %zu %zu %zu\\n", sizeof(couple_inputs), offsetof(couple_inputs, uf_given), offsetof(couple_inputs, step),
         offsetof(couple_inputs, fine_alpha), offsetof(couple_config, mu_f2));
  printf("%zu %zu %zu %zu %zu\\n", sizeof(couple_outputs), offsetof(couple_outputs, diag), offsetof(couple_outputs, uf),
         offsetof(couple_outputs, fine_KU), offsetof(couple_outputs, bulk_alpha));
  printf("%zu %zu %zu\\n", sizeof(couple_mlp_config), offsetof(couple_mlp_config, lr), offsetof(couple_mlp_config, eps));
  printf("%d %d %d %d\\n", COUPLE_DIAG_LEN, COUPLE_VEL_MLP, COUPLE_MLP_NFEAT, COUPLE_MLP_NPARAM);
  printf("%lld\\n", (long long)COUPLE_NOALLOC_SCRATCH_BYTES);
  return 0; }
""")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    lines = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    a = [int(x) for x in lines[0].split()]
    K = cpl._Config
    assert a == [C.sizeof(K), K.rho_f.offset, K.deposit.offset, K.dt.offset, K.max_particles.offset,
                 K.mlp_tol.offset, K.mlp_period.offset, K.semi_implicit.offset]
    b = [int(x) for x in lines[1].split()]
    assert b == [C.sizeof(cpl._Inputs), cpl._Inputs.uf_given.offset, cpl._Inputs.step.offset,
                 cpl._Inputs.fine_alpha.offset, cpl._Config.mu_f2.offset]
    c = [int(x) for x in lines[2].split()]
    assert c == [C.sizeof(cpl._Outputs), cpl._Outputs.diag.offset, cpl._Outputs.uf.offset,
                 cpl._Outputs.fine_KU.offset, cpl._Outputs.bulk_alpha.offset]
    d = [int(x) for x in lines[3].split()]
    assert d == [C.sizeof(cpl._MlpConfig), cpl._MlpConfig.lr.offset, cpl._MlpConfig.eps.offset]
    e = [int(x) for x in lines[4].split()]
    assert e == [cpl.DIAG_LEN, cpl.COUPLE_VEL_MLP, cpl.MLP_NFEAT, cpl.MLP_NPARAM]
    assert int(lines[5]) == cpl.NOALLOC_SCRATCH_BYTES


def test_noalloc_rejects_invalid_config_without_a_gpu():
    """The no-alloc step validates its configuration before touching the device."""
    import ctypes as C
    import paper_1807_11834_amd as cpl
    c = cpl.Config(ratio=3).to_c()
    i, o = cpl._Inputs(), cpl._Outputs()
    assert cpl._lib.couple_step_noalloc(C.byref(c), C.byref(i), C.byref(o), None) == cpl.COUPLE_EINVAL
    assert "couple_step_noalloc: ratio" in cpl.couple_last_error(None)
    assert cpl._lib.couple_step_noalloc(None, C.byref(i), C.byref(o), None) == cpl.COUPLE_EINVAL


BAD = [
    dict(box=(0.0, 1.0, 1.0)), dict(box=(1.0, float("nan"), 1.0)), dict(nb=(0, 4, 4)), dict(ratio=3),
    dict(rho_f=-1.0), dict(mu_f=0.0), dict(eps_min=1.0), dict(deposit=2), dict(precision=7),
    dict(vel_source=9), dict(advect=2), dict(advect=1, dt=float("inf")), dict(max_particles=-5),
    dict(nb=(2048, 2048, 1024)), dict(nb=(40000, 2, 2)),
    dict(vel_source=3, precision=0), dict(vel_source=3, mlp_period=0), dict(vel_source=3, mlp_tol=-1.0),
    dict(vel_source=3, mlp_tol=float("nan")), dict(semi_implicit=2), dict(semi_implicit=-1),
    dict(vof=2), dict(vof=1, rho_f2=0.0), dict(vof=1, mu_f2=float("inf")),
]


@pytest.mark.parametrize("kw", BAD)
def test_init_rejects_invalid_config(kw):
    import paper_1807_11834_amd as cpl
    cfg = cpl.Config(**{"max_particles": 10, **kw})
    with pytest.raises(cpl.CoupleError) as ei:
        cpl.couple_init(cfg)
    assert ei.value.code == cpl.COUPLE_EINVAL
    assert "couple_init" in str(ei.value)


def test_null_handle_and_free_null():
    import paper_1807_11834_amd as cpl
    import ctypes as C
    assert cpl._lib.couple_free(None) == cpl.COUPLE_OK
    i, o = cpl._Inputs(), cpl._Outputs()
    assert cpl._lib.couple_step(None, C.byref(i), C.byref(o), None) == cpl.COUPLE_EINVAL


@pytest.mark.parametrize("kw", [dict(max_batch=16), dict(max_batch=1 << 26), dict(lr=0.0), dict(beta1=1.0),
                                dict(beta2=-0.1), dict(eps=0.0)])
def test_mlp_init_rejects_invalid_config(kw):
    import paper_1807_11834_amd as cpl
    args = {"max_batch": 1024, **kw}
    with pytest.raises(cpl.CoupleError) as ei:
        cpl.couple_mlp_init(**args)
    assert ei.value.code == cpl.COUPLE_EINVAL
    assert "couple_mlp_init" in str(ei.value)


def test_mlp_null_handles():
    import paper_1807_11834_amd as cpl
    L = cpl._lib
    assert L.couple_mlp_free(None) == cpl.COUPLE_OK
    assert L.couple_mlp_set_params(None, None) == cpl.COUPLE_EINVAL
    assert L.couple_mlp_forward(None, None, 0, None, None) == cpl.COUPLE_EINVAL
    assert L.couple_mlp_train_step(None, None, None, 0, None, 0, None, None) == cpl.COUPLE_EINVAL
    assert L.couple_set_mlp(None, None) == cpl.COUPLE_EINVAL
    assert L.couple_mlp_features(None, 0, None, None, None, None, None, None, None, 0, None, None, None,
                                 None) == cpl.COUPLE_EINVAL


def _nodes(n, box=(1.0, 1.0, 1.0)):
    import numpy as np
    return [np.linspace(0.0, box[a], n[a] + 1) for a in range(3)]


@pytest.mark.parametrize("case", ["zero_cells", "not_increasing", "nan", "box_mismatch", "precision"])
def test_remap_init_rejects_invalid_grids(case):
    import numpy as np
    import paper_1807_11834_amd as cpl
    src, dst, prec = _nodes((4, 3, 2)), _nodes((2, 2, 2)), cpl.COUPLE_FP32_WIDE
    if case == "zero_cells":
        dst[1] = np.array([0.0])
    elif case == "not_increasing":
        src[0] = np.array([0.0, 0.5, 0.5, 0.75, 1.0])
    elif case == "nan":
        src[2] = np.array([0.0, float("nan"), 1.0])
    elif case == "box_mismatch":
        dst[2] = np.array([0.0, 0.5, 1.1])
    else:
        prec = 9
    with pytest.raises(cpl.CoupleError) as ei:
        cpl.Remap(src, dst, precision=prec)
    assert ei.value.code == cpl.COUPLE_EINVAL
    assert "couple_remap_init" in str(ei.value)


def test_remap_null_handles():
    import paper_1807_11834_amd as cpl
    L = cpl._lib
    assert L.couple_remap_free(None) == cpl.COUPLE_OK
    assert L.couple_remap_apply(None, None, None, 1, None) == cpl.COUPLE_EINVAL
    assert L.couple_remap_info(None, None, None) == cpl.COUPLE_EINVAL


@pytest.mark.parametrize("case", ["ns0", "nan", "inverted", "precision", "null"])
def test_boxmap_init_rejects_invalid_grids(case):
    import numpy as np
    import paper_1807_11834_amd as cpl
    good = np.array([[0.0, 1.0, 0.0, 1.0, 0.0, 1.0]])
    s, r, prec = good.copy(), good.copy(), cpl.COUPLE_FP32_WIDE
    if case == "ns0":
        s = np.zeros((0, 6))
    elif case == "nan":
        r[0, 3] = float("nan")
    elif case == "inverted":
        s[0, 4], s[0, 5] = 1.0, 0.5
    elif case == "precision":
        prec = 7
    if case == "null":
        import ctypes as C
        h = C.c_void_p()
        assert cpl._lib.couple_boxmap_init(1, None, 1, None, 1, C.byref(h)) == cpl.COUPLE_EINVAL
        return
    with pytest.raises(cpl.CoupleError) as ei:
        cpl.BoxMap(s, r, precision=prec)
    assert ei.value.code == cpl.COUPLE_EINVAL
    assert "couple_boxmap_init" in str(ei.value)


def test_boxmap_null_handles():
    import paper_1807_11834_amd as cpl
    L = cpl._lib
    assert L.couple_boxmap_free(None) == cpl.COUPLE_OK
    assert L.couple_boxmap_apply(None, None, None, 1, None) == cpl.COUPLE_EINVAL


PART_BAD = [
    (dict(), 0, "nparts"), (dict(nb=(4, 4, 4)), 5, "nparts"), (dict(), 65, "nparts"),
    (dict(vel_source=2), 2, "vel_source"), (dict(vel_source=3, precision=1), 2, "vel_source"),
    (dict(vof=1), 2, "two-fluid"), (dict(box=(1.0, 1.0, 3.0), nb=(4, 4, 4)), 2, "power of two"),
]


@pytest.mark.parametrize("kw,nparts,msg", PART_BAD)
def test_part_init_rejects_unsupported_configs(kw, nparts, msg):
    """The partitioned step refuses what it does not cover before allocating."""
    import paper_1807_11834_amd as cpl
    cfg = cpl.Config(**{"max_particles": 10, "nb": (8, 8, 8), "box": (1.0, 1.0, 1.0), **kw})
    with pytest.raises(cpl.CoupleError) as ei:
        cpl.Part(cfg, nparts)
    assert ei.value.code == cpl.COUPLE_EINVAL
    assert msg in str(ei.value)


def test_part_null_arguments():
    import ctypes as C
    import paper_1807_11834_amd as cpl
    L = cpl._lib
    assert L.couple_part_step(None, None, None, 0, None) == cpl.COUPLE_EINVAL
    assert L.couple_part_free(None) == cpl.COUPLE_OK
    assert L.couple_part_comm_matrix(None, None) == cpl.COUPLE_EINVAL
    c = cpl.Config().to_c()
    assert L.couple_part_init(C.byref(c), 2, None) == cpl.COUPLE_EINVAL


def test_hbmref_rejects_bad_calls_before_any_launch():
    """The streaming reference kernels' argument checks (no device work)."""
    import ctypes as C
    import paper_1807_11834_amd as cpl
    L = cpl._lib
    buf = C.create_string_buffer(64)
    p = C.cast(buf, C.c_void_p).value
    p16 = (p + 15) & ~15
    assert L.couple_hbmref(3, p16, p16, 1, 0.0, None) == cpl.COUPLE_EINVAL          # unknown kind
    assert L.couple_hbmref(-1, p16, p16, 1, 0.0, None) == cpl.COUPLE_EINVAL
    assert L.couple_hbmref(cpl.COUPLE_HBMREF_COPY, p16, p16, -1, 0.0, None) == cpl.COUPLE_EINVAL
    assert L.couple_hbmref(cpl.COUPLE_HBMREF_COPY, None, p16, 1, 0.0, None) == cpl.COUPLE_EINVAL
    assert L.couple_hbmref(cpl.COUPLE_HBMREF_READ, p16, None, 1, 0.0, None) == cpl.COUPLE_EINVAL
    assert L.couple_hbmref(cpl.COUPLE_HBMREF_WRITE, None, p16 + 4, 1, 0.0, None) == cpl.COUPLE_EINVAL  # misaligned
    assert L.couple_hbmref(cpl.COUPLE_HBMREF_COPY, p16 + 8, p16, 1, 0.0, None) == cpl.COUPLE_EINVAL
    for k in (0, 1, 2):
        assert L.couple_hbmref(k, None, None, 0, 0.0, None) == cpl.COUPLE_OK       # nothing to do
    assert L.couple_hbmref(cpl.COUPLE_HBMREF_READ, p16, p16 + 2, 1, 0.0, None) == cpl.COUPLE_EINVAL  # flag alignment
