"""CPU checks of the C ABI: the library loads, exports every entry point that
include/couple.h declares, its structs have the header's layout, and argument
validation rejects bad calls before any device work."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "couple.h")
LIB = os.path.join(ROOT, "paper_1807_11834_amd", "libcouple.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(couple_[a-z_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    assert declared_functions() == ["couple_free", "couple_init", "couple_last_error", "couple_step",
                                    "couple_timing_begin", "couple_timing_end"]


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
#include "couple.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu\\n", sizeof(couple_config), offsetof(couple_config, rho_f),
         offsetof(couple_config, deposit), offsetof(couple_config, dt), offsetof(couple_config, max_particles));
  printf("%zu %zu\\n", sizeof(couple_inputs), offsetof(couple_inputs, uf_given));
  printf("%zu %zu\\n", sizeof(couple_outputs), offsetof(couple_outputs, diag));
  return 0; }
""")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    lines = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    a = [int(x) for x in lines[0].split()]
    assert a == [C.sizeof(cpl._Config), cpl._Config.rho_f.offset, cpl._Config.deposit.offset,
                 cpl._Config.dt.offset, cpl._Config.max_particles.offset]
    b = [int(x) for x in lines[1].split()]
    assert b == [C.sizeof(cpl._Inputs), cpl._Inputs.uf_given.offset]
    c = [int(x) for x in lines[2].split()]
    assert c == [C.sizeof(cpl._Outputs), cpl._Outputs.diag.offset]


BAD = [
    dict(box=(0.0, 1.0, 1.0)), dict(box=(1.0, float("nan"), 1.0)), dict(nb=(0, 4, 4)), dict(ratio=3),
    dict(rho_f=-1.0), dict(mu_f=0.0), dict(eps_min=1.0), dict(deposit=2), dict(precision=7),
    dict(vel_source=9), dict(advect=2), dict(advect=1, dt=float("inf")), dict(max_particles=-5),
    dict(nb=(2048, 2048, 1024)), dict(nb=(40000, 2, 2)),
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
