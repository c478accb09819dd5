"""The C ABI without a GPU: the library loads, exports every function declared in include/rte.h,
and rejects invalid arguments before touching the device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("rte.h", "rte_nn.h")]
LIB = os.path.join(ROOT, "paper_1802_03061_amd", "librte.so")


def declared_functions():
    src = "".join(open(h).read() for h in HEADERS)
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rte_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("librte.so is not built (python -m paper_1802_03061_amd.build)")
    from paper_1802_03061_amd import rte
    return rte.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("rte_setup", "rte_apply", "rte_solve", "rte_solve_batched", "rte_destroy",
                 "rte_last_error", "rte_pc_attach", "rte_nn_create", "rte_nn_loss_grad", "rte_nn_adam_step",
                 "rte_pc_make_pairs"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def _grid(rte, dim=2, n=(16, 16, 1), h=1 / 16):
    g = rte.Grid()
    g.dim = dim
    for a in range(3):
        g.n[a] = n[a]
    g.h = h
    return g


@pytest.mark.parametrize("case", [
    dict(dim=4), dict(n=(1, 16, 1)), dict(h=0.0), dict(h=-1.0), dict(mu_a=-0.1), dict(mu_s=-1.0),
    dict(mu_a=0.0, mu_s=0.0), dict(L=-1), dict(L=33), dict(prec=7), dict(sigma=[0.5, 0.2], L=1),
    dict(sigma=[1.0, 1.5], L=1), dict(sigma=None, L=2),
])
def test_setup_rejects_invalid_arguments(lib, case):
    from paper_1802_03061_amd import rte
    g = _grid(rte, dim=case.get("dim", 2), n=case.get("n", (16, 16, 1)), h=case.get("h", 1 / 16))
    L = case.get("L", 0)
    sigma = case.get("sigma", [1.0] * (max(L, 0) + 1))
    arr = None if sigma is None else (C.c_double * len(sigma))(*sigma)
    out = C.c_void_p(123)
    rc = lib.rte_setup(C.byref(out), C.byref(g), case.get("mu_a", 0.1), case.get("mu_s", 1.0),
                       C.cast(arr, C.POINTER(C.c_double)) if arr is not None else None, L,
                       case.get("prec", 1), None)
    assert rc == rte.RTE_EINVAL
    assert out.value is None
    assert len(lib.rte_last_error()) > 0


def test_setup_3d_beyond_its_limits_is_unsupported(lib):
    """3D keeps spherical harmonics to degree RTE_MAX_L3 = 3, on grids up to 128 per side when
    L > 0; both limits are refused before any device work."""
    from paper_1802_03061_amd import rte
    arr = (C.c_double * 5)(1.0, 0.3, 0.09, 0.027, 0.0081)
    out = C.c_void_p()
    g = _grid(rte, dim=3, n=(8, 8, 8), h=1 / 8)
    rc = lib.rte_setup(C.byref(out), C.byref(g), 0.1, 1.0, C.cast(arr, C.POINTER(C.c_double)), 4, 1, None)
    assert rc == rte.RTE_EUNSUPPORTED
    g = _grid(rte, dim=3, n=(129, 8, 8), h=1 / 129)
    rc = lib.rte_setup(C.byref(out), C.byref(g), 0.1, 1.0, C.cast(arr, C.POINTER(C.c_double)), 1, 1, None)
    assert rc == rte.RTE_EUNSUPPORTED


def test_setup_oversize_is_unsupported(lib):
    from paper_1802_03061_amd import rte
    g = _grid(rte, n=(1024, 16, 1))
    out = C.c_void_p()
    assert lib.rte_setup(C.byref(out), C.byref(g), 0.1, 1.0, None, 0, 1, None) == rte.RTE_EUNSUPPORTED


def test_null_context_calls_fail_cleanly(lib):
    from paper_1802_03061_amd import rte
    assert lib.rte_apply(None, 0, 0, 1, None, None) == rte.RTE_EINVAL
    assert lib.rte_solve(None, None, 1e-8, 10, None, None) == rte.RTE_EINVAL
    assert lib.rte_rhs(None, None, 0, None) == rte.RTE_EINVAL
    assert lib.rte_rhs_source(None, None, 0, None) == rte.RTE_EINVAL
    assert lib.rte_solve_source(None, None, 0, 1e-8, 10, None, None) == rte.RTE_EINVAL
    assert lib.rte_set_solve_opts(None, None) == rte.RTE_EINVAL
    assert lib.rte_query(None, None, None, None) == rte.RTE_EINVAL
    assert lib.rte_autotune(None, 5) == rte.RTE_EINVAL
    assert lib.rte_scattering_term(None, 0, None, 8, None) == rte.RTE_EINVAL
    assert lib.rte_set_variant(None, 0, 0, 0) == rte.RTE_EINVAL
    assert lib.rte_get_variant(None, 0, 0, None, None) == rte.RTE_EINVAL
    for pass_, var in ((2, 0), (-1, 0), (0, 4), (1, -2)):
        assert lib.rte_set_batched_variant(pass_, var) == rte.RTE_EINVAL
    assert lib.rte_set_batched_variant(0, -1) == rte.RTE_OK
    assert lib.rte_set_batched_variant(1, -1) == rte.RTE_OK
    lib.rte_destroy(None)
    assert b"gfx950" in lib.rte_version()


def test_nn_create_rejects_bad_shapes(lib):
    from paper_1802_03061_amd import rte
    out = C.c_void_p()
    for ch, hid, lay in ((2, 32, 5), (19, 32, 5), (9, 24, 5), (9, 32, 1), (9, 32, 9)):
        assert lib.rte_nn_create(C.byref(out), ch, hid, lay, 0, 1, None) == rte.RTE_EINVAL
        assert out.value is None
    assert lib.rte_nn_adam_step(None, C.c_float(1e-3)) == rte.RTE_EINVAL
    assert lib.rte_pc_attach(None, None, 32, 5, 4) == rte.RTE_EINVAL


def test_binding_structs_match_the_header(tmp_path):
    """The ctypes structures of the binding have the size and field offsets of the C structs in
    include/rte.h (compiled with the host C compiler)."""
    import shutil
    import subprocess
    from paper_1802_03061_amd import rte
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = {"rte_grid": rte.Grid, "rte_solve_info": rte.SolveInfo, "rte_solve_opts": rte.SolveOpts}
    lines = ['#include "rte.h"', "#include <stdio.h>", "#include <stddef.h>", "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'    printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'    printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            parts = line.split()
            got[(parts[0], parts[1])] = int(parts[2])
    for cname, py in structs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
