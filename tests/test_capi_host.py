"""Host-only checks of the C ABI: the library loads, exports every function
include/fsic.h declares, and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fsic.h")
LIB = os.path.join(ROOT, "paper_2108_01186_amd", "libfsic.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fsic_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libfsic.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("fsic_create", "fsic_forward", "fsic_backward", "fsic_destroy",
                     "fsic_status_string", "fsic_default_opts"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_names_match_header():
    from paper_2108_01186_amd import fsic
    assert sorted(fsic.EXPORTED) == declared_functions()


def test_default_opts_and_status_strings():
    from paper_2108_01186_amd import fsic
    o = fsic.default_opts()
    assert o.fd_order == 12 and o.lmax == 6 and o.tol == 1e-10 and o.max_iter == 20000
    assert o.vsic_scale == 1.0 and o.rho_floor == 1e-30 and o.flags == fsic.FSIC_WANT_VSIC
    for s in range(10):
        assert fsic.fsic_status_string(s)
    assert b"unknown" in fsic.fsic_status_string(99)


def test_struct_layout_matches_header(tmp_path):
    """Size and every field offset of the ABI structs in the binding equal what
    gcc lays out from include/fsic.h."""
    import subprocess
    from paper_2108_01186_amd import fsic
    structs = [fsic.fsic_grid, fsic.fsic_opts, fsic.fsic_system, fsic.fsic_stats]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "fsic.h"', 'int main(void) {']
    for st in structs:
        lines.append(f'printf("%zu\\n", sizeof({st.__name__}));')
        for name, _ in st._fields_:
            lines.append(f'printf("%zu\\n", offsetof({st.__name__}, {name}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    want = []
    for st in structs:
        want.append(ctypes.sizeof(st))
        want.extend(getattr(st, name).offset for name, _ in st._fields_)
    assert got == want


def test_invalid_arguments_rejected_on_host():
    from paper_2108_01186_amd import fsic
    n = (ctypes.c_int32 * 3)(16, 16, 16)
    # odd stencil order, zero count, null pointers: rejected before any HIP call
    assert fsic.fsic_op_laplacian(n, 0.3, 7, 1, ctypes.c_void_p(8), ctypes.c_void_p(8), None) == fsic.FSIC_EINVAL
    assert fsic.fsic_op_laplacian(n, 0.3, 12, 0, ctypes.c_void_p(8), ctypes.c_void_p(8), None) == fsic.FSIC_EINVAL
    assert fsic.fsic_op_laplacian(n, 0.3, 12, 1, None, ctypes.c_void_p(8), None) == fsic.FSIC_EINVAL
    bad = (ctypes.c_int32 * 3)(4, 16, 16)
    assert fsic.fsic_op_laplacian(bad, 0.3, 12, 1, ctypes.c_void_p(8), ctypes.c_void_p(8), None) == fsic.FSIC_EINVAL
    assert fsic.fsic_op_laplacian(n, -0.3, 12, 1, ctypes.c_void_p(8), ctypes.c_void_p(8), None) == fsic.FSIC_EINVAL
    assert fsic.fsic_op_invsqrt(0, 1, ctypes.c_void_p(8), ctypes.c_void_p(8), None, None) == fsic.FSIC_EINVAL
    assert fsic.fsic_op_invsqrt(200, 1, ctypes.c_void_p(8), ctypes.c_void_p(8), None, None) == fsic.FSIC_EINVAL
    o = fsic.default_opts(fd_order=13)
    h = ctypes.c_void_p()
    assert fsic.fsic_create(ctypes.byref(h), ctypes.byref(o), None) == fsic.FSIC_EINVAL
    o = fsic.default_opts(tol=0.0)
    assert fsic.fsic_create(ctypes.byref(h), ctypes.byref(o), None) == fsic.FSIC_EINVAL
    o = fsic.default_opts(lmax=9)
    assert fsic.fsic_create(ctypes.byref(h), ctypes.byref(o), None) == fsic.FSIC_EINVAL
    assert fsic.fsic_create(None, ctypes.byref(fsic.default_opts()), None) == fsic.FSIC_EINVAL
    # the context-bound calls reject a null context before anything else
    assert fsic.fsic_forward(None, 1, None, None, None, None, None) == fsic.FSIC_EINVAL
    assert fsic.fsic_backward(None, None, None, None) == fsic.FSIC_EINVAL
    assert fsic.fsic_forward_backward(None, 1, None, None, None, None, None, None, None, None) == fsic.FSIC_EINVAL


def test_flag_and_solver_constants_match_header():
    """Every FSIC_* flag and solver value of the header has the same value in
    the binding (the ABI passes them as plain integers)."""
    from paper_2108_01186_amd import fsic as F
    text = open(HEADER).read()
    flags = dict(re.findall(r"#define\s+(FSIC_[A-Z0-9_]+)\s+(\d+)u", text))
    assert {"FSIC_WANT_VSIC", "FSIC_KEEP_TAPE", "FSIC_PAPER_GRADIENT", "FSIC_EQ9_FORCES",
            "FSIC_GRAPHS", "FSIC_FP32_ORBITALS"} <= set(flags)
    for name, val in flags.items():
        assert getattr(F, name) == int(val), name
    enum = re.search(r"enum\s*\{\s*(FSIC_CG[^}]*)\}", text).group(1)
    for name, val in re.findall(r"(FSIC_[A-Z]+)\s*=\s*(\d+)", enum):
        assert getattr(F, name) == int(val), name


def test_stored_traffic_follows_kernel_sources(tmp_path, monkeypatch):
    """bench.py reads the committed HBM-traffic summary only while the kernel
    sources hash to the value stored with it."""
    import bench
    prof = tmp_path / "profiles"
    prof.mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    src = tmp_path / "paper_2108_01186_amd" / "csrc"
    src.mkdir(parents=True)
    for f in bench.KERNEL_SOURCES:
        (src / f).write_text("// " + f + "\n")
    good = bench.kernel_source_hash()
    path = prof / "precond_pcg_f32_toy_hbm_traffic.txt"
    path.write_text(f"traffic_bytes_per_launch: 123\nalgorithmic_bytes_per_launch: 100\n"
                    f"kernel_source_sha256: {good}\n")
    assert bench.stored_traffic("toy", "precond", "pcg") == (123.0, 100.0)
    (src / "dst.hip").write_text("// changed\n")
    assert bench.stored_traffic("toy", "precond", "pcg") is None
    assert bench.stored_traffic("other", "precond", "pcg") is None
