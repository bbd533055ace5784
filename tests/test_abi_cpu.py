"""Host-side checks of the C-ABI library that need no GPU: every symbol the
header declares is exported, and argument validation / footprint planning
(pure host logic) behave as documented."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("pt_mg.h", "pt_serve.h")]


def _declared():
    names = set()
    for hdr in HEADERS:
        src = open(hdr).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(pt_[a-z_0-9]+)\s*\(", src))
    return sorted(names)


@pytest.fixture(scope="module")
def L():
    from paper_2206_11294_amd import ptmg
    return ptmg.lib()


def test_every_declared_symbol_is_exported(L):
    names = _declared()
    assert "pt_mg_setup" in names and "pt_mg_solve" in names and "pt_mg_residual" in names
    for n in names:
        assert hasattr(L, n), n


def test_binding_covers_header(L):
    from paper_2206_11294_amd import ptmg, serve
    assert set(ptmg.exported_symbols()) | set(serve.exported_symbols()) == set(_declared())


def _prob(dim=2, n=(64, 64, 1), mode=0):
    from paper_2206_11294_amd import ptmg
    s = ptmg.pt_problem()
    s.dim = dim
    for a in range(3):
        s.n[a] = n[a]
    s.h = 1.0 / n[0]
    s.mode = mode
    s.alpha_p_const = 1.0
    s.alpha_T_const = 0.1
    s.B_const[0] = s.B_const[3] = 1000.0
    return s


def test_footprint_and_validation(L):
    from paper_2206_11294_amd import ptmg
    s = _prob()
    fp = ptmg.footprint_bytes(s, ptmg.PT_PREC_FP64)
    # finest FP64 operator + iterate + FP64 hierarchy
    assert fp > 64 * 64 * (16 + 32 + 16 + 32)
    bad = _prob(dim=4)
    assert ptmg.footprint_bytes(bad, 0) == 0
    odd = _prob(2, (4099, 4099, 1))    # does not coarsen to a small grid
    assert ptmg.footprint_bytes(odd, 0) == 0
    s3 = _prob(3, (512, 512, 512))
    big = ptmg.footprint_bytes(s3, ptmg.PT_PREC_MIXED)
    assert 10e9 < big < 20e9
    # validation happens before any device work
    h = ctypes.c_void_p()
    rc = L.pt_mg_setup(ctypes.byref(bad), 0, None, ctypes.byref(h))
    assert rc == ptmg.PT_ERR_ARG and not h.value
    assert b"dim" in L.pt_mg_last_error(None)
    ph = _prob(mode=1)          # phases mode without C
    rc = L.pt_mg_setup(ctypes.byref(ph), 0, None, ctypes.byref(h))
    assert rc == ptmg.PT_ERR_ARG


def test_serving_sizes_coarsen(L):
    """Every grid of the serving mix coarsens to a small dense grid."""
    from paper_2206_11294_amd import ptmg
    import workloads as W
    for n in W.SERVE_SIZES_2D:
        assert ptmg.footprint_bytes(_prob(2, (n, n, 1)), 1) > 0, n
    for n in W.SERVE_SIZES_3D:
        assert ptmg.footprint_bytes(_prob(3, (n, n, n)), 1) > 0, n


def test_struct_layouts_match_header(tmp_path):
    """Every structure the Python binding passes through the C ABI has the
    size and field offsets of the header's declaration (a host C program
    compiled against include/ prints them)."""
    import ctypes
    import shutil
    import subprocess
    from paper_2206_11294_amd import ptmg, serve
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = [ptmg.pt_phase, ptmg.pt_problem, ptmg.pt_state, ptmg.pt_downstream,
               ptmg.pt_solve_opts, ptmg.pt_solve_info, serve.pt_server_config,
               serve.pt_request_info]
    cname = {"async_": "async"}     # Python keyword on the binding side
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pt_mg.h"',
             '#include "pt_serve.h"', 'int main(void) {']
    want = []
    for st in structs:
        lines.append(f'  printf("%zu\\n", sizeof({st.__name__}));')
        want.append(ctypes.sizeof(st))
        for f in st._fields_:
            name = f[0]
            lines.append(f'  printf("%zu\\n", offsetof({st.__name__}, {cname.get(name, name)}));')
            want.append(getattr(st, name).offset)
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), "-o", str(exe),
                    str(src)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    assert got == want
