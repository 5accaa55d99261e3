"""C-ABI checks that need no GPU: the library loads, exports every symbol include/imb.h declares,
the Python struct matches the C struct, and host-side validation rejects bad configurations."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_1809_07008_amd import imb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "imb.h")


def declared_symbols():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(imb_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = imb.load_library()
    decl = declared_symbols()
    assert len(decl) > 30
    missing = [s for s in decl if not hasattr(lib, s)]
    assert not missing, missing
    assert set(decl) <= set(imb.EXPORTED)


def test_config_struct_layout_matches_header(tmp_path):
    prog = tmp_path / "layout.c"
    prog.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "imb.h"
#define O(f) printf("%s %zu\n", #f, offsetof(imb_config, f));
int main(void) {
  printf("size %zu\n", sizeof(imb_config));
  O(nx) O(ny) O(storage) O(n_sub) O(tau0) O(smag_cs) O(gx) O(gy) O(rho0) O(kn)
  O(damping_ratio) O(rho_solid) O(max_particles) O(flags) O(tile_w) O(tile_rows)
  O(eps_subcells) O(reserved) O(wall_ux_bottom) O(wall_ux_top) O(kt) O(mu)
  O(contact_model) O(reserved2) O(young) O(poisson)
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split("\n")
    vals = dict(line.split() for line in out if line.strip())
    assert int(vals["size"]) == C.sizeof(imb.Config)
    for name, _ in imb.Config._fields_:
        assert int(vals[name]) == getattr(imb.Config, name).offset, name


def required(**kw):
    lib = imb.load_library()
    c = imb.make_config(**{**dict(nx=64, ny=32, tau0=0.6), **kw})
    n = C.c_size_t()
    return lib.imb_required_bytes(C.byref(c), C.byref(n)), n.value


def test_required_bytes_scales_with_storage():
    rc64, b64 = required(nx=2048, ny=1024, storage="f64", max_particles=500)
    rc32, b32 = required(nx=2048, ny=1024, storage="f32", max_particles=500)
    rc16, b16 = required(nx=2048, ny=1024, storage="f16", max_particles=500)
    assert rc64 == rc32 == rc16 == 0
    pop = 2 * 9 * 2048 * 1024
    assert b64 > 8 * pop and b32 > 4 * pop and b16 > 2 * pop
    assert b64 - b32 == pytest.approx(4 * pop, rel=1e-3)


@pytest.mark.parametrize("kw", [dict(tau0=0.5), dict(tau0=0.3), dict(nx=1), dict(ny=0),
                                dict(storage=7), dict(cs=-0.1), dict(n_sub=0),
                                dict(max_particles=5000), dict(tile_w=48), dict(tile_rows=3),
                                dict(rho0=0.0), dict(rho_s=0.0), dict(eps_subcells=-1),
                                dict(eps_subcells=65), dict(uw_top=0.4), dict(uw_bot=-0.31),
                                dict(walls=False, uw_top=0.01), dict(kt=-1.0),
                                dict(mu=float("nan")), dict(kt=float("inf"), mu=0.3)])
def test_invalid_configs_rejected(kw):
    rc, _ = required(**kw)
    assert rc == -1


def test_reserved_config_word_must_be_zero():
    lib = imb.load_library()
    c = imb.make_config(nx=64, ny=32, tau0=0.6, eps_subcells=5)
    n = C.c_size_t()
    assert lib.imb_required_bytes(C.byref(c), C.byref(n)) == 0
    c.reserved = 1
    assert lib.imb_required_bytes(C.byref(c), C.byref(n)) == -1


def test_strerror_and_version():
    lib = imb.load_library()
    assert lib.imb_strerror(0) == b"ok"
    for code in range(-1, -8, -1):
        assert lib.imb_strerror(code) not in (b"", b"unknown error")
    assert b"gfx950" in lib.imb_version()


def test_library_has_no_oracle_dependency():
    """The product library and binding never load the CPU oracle."""
    out = subprocess.check_output(["nm", "-D", "--defined-only", imb.LIB_PATH]).decode()
    assert "o_step" not in out and "o_collide_cell" not in out
    src = open(os.path.join(ROOT, "paper_1809_07008_amd", "imb.py")).read()
    assert "oracle" not in src.replace("Oracle", "")


def test_host_memory_is_refused_for_the_hip_library():
    """The binding never hands host memory to the GPU library as its workspace (the check runs
    before any device call, so it is a CPU test)."""
    from paper_1809_07008_amd import workloads
    case = workloads.single_disk_channel()
    with pytest.raises(ValueError):
        imb.Simulation(imb.config_from_case(case), device="cpu")


def test_config3_struct_layout_matches_header(tmp_path):
    prog = tmp_path / "layout3.c"
    names = [n for n, _ in imb.Config3._fields_]
    prog.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"imb.h\"\n"
                    "int main(void) {\n  printf(\"size %zu\\n\", sizeof(imb3_config));\n" +
                    "".join('  printf("%s %%zu\\n", offsetof(imb3_config, %s));\n' % (n, n)
                            for n in names) + "  return 0;\n}\n")
    exe = tmp_path / "layout3"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)])
    vals = dict(line.split() for line in subprocess.check_output([str(exe)]).decode().split("\n")
                if line.strip())
    assert int(vals["size"]) == C.sizeof(imb.Config3)
    for name in names:
        assert int(vals[name]) == getattr(imb.Config3, name).offset, name
