"""Host-side checks of the C ABI (no GPU needed): every symbol declared in
include/hmc.h is exported by libhmc.so, and argument validation reports
HMC_E_ARG / HMC_E_OOM with a message."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hmc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hmc_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def H():
    from paper_1212_0785_amd import hmc
    hmc.lib()
    return hmc


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("hmc_alloc_fields", "hmc_wilson_dslash", "hmc_cg_solve", "hmc_gauge_force", "hmc_fermion_force",
                 "hmc_md_leapfrog", "hmc_exp_update_reunit", "hmc_refresh", "hmc_plaquette", "hmc_trajectory",
                 "hmc_norm2", "hmc_inner", "hmc_sum_multi"):
        assert must in names


def test_every_declared_symbol_is_exported(H):
    lib = C.CDLL(H.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding wraps every one of them
    assert set(declared_functions()) <= set(H._SIGNATURES)


def test_version(H):
    a, b = C.c_int32(), C.c_int32()
    assert H.lib().hmc_get_version(C.byref(a), C.byref(b)) == 0 and a.value == 1


@pytest.mark.parametrize("L", [(3, 4, 4, 4), (4, 4, 4, 5), (4, 0, 4, 4), (4, 4, -2, 4)])
def test_bad_geometry_rejected(H, L):
    n = C.c_size_t()
    st = H.lib().hmc_fields_bytes(C.byref(H.geom(L)), 0, C.byref(n))
    assert st == H.HMC_E_ARG
    assert "even" in H.last_error()


def test_field_sizes(H):
    L = (4, 4, 4, 4)
    Vh = 128
    assert H.hmc_field_bytes(L, H.F64, H.KIND_HALF_SPINOR) == Vh * 192
    assert H.hmc_field_bytes(L, H.F32, H.KIND_FULL_SPINOR) == 2 * Vh * 96
    assert H.hmc_field_bytes(L, H.F16, H.KIND_HALF_SPINOR) == Vh * 52
    assert H.hmc_field_bytes(L, H.F64, H.KIND_GAUGE) == Vh * 8 * 144
    with pytest.raises(H.HmcError):
        H.hmc_field_bytes(L, H.F32, H.KIND_MOMENTA)
    assert H.hmc_fields_bytes(L, H.FIELDS_LOWPREC) > H.hmc_fields_bytes(L, 0)


def test_arena_too_small_is_oom(H):
    L = (4, 4, 4, 4)
    need = H.hmc_fields_bytes(L, 0)
    buf = C.create_string_buffer(need + 512)
    base = (C.addressof(buf) + 255) & ~255
    h = C.c_void_p()
    a = H.Action(5.6, 0.15)
    st = H.lib().hmc_alloc_fields(C.byref(H.geom(L)), C.byref(a), 0, base, need - 1, C.byref(h))
    assert st == H.HMC_E_OOM and "smaller" in H.last_error()
    st = H.lib().hmc_alloc_fields(C.byref(H.geom(L)), C.byref(a), 0, base + 8, need, C.byref(h))
    assert st == H.HMC_E_ARG


def test_null_arguments_rejected(H):
    assert H.lib().hmc_free_fields(None) == H.HMC_E_ARG
    assert H.lib().hmc_plaquette(None, None, None) == H.HMC_E_ARG


def test_triad_argument_errors(H):
    lib = H.lib()
    # checked before any device work: odd length, misaligned or null buffers
    assert lib.hmc_stream_triad(4096, 8192, 12288, 1.0, 3, 0, None) == H.HMC_E_ARG
    assert lib.hmc_stream_triad(4096, 8200, 12288, 1.0, 4, 0, None) == H.HMC_E_ARG
    assert lib.hmc_stream_triad(None, 8192, 12288, 1.0, 4, 0, None) == H.HMC_E_ARG
    assert "even" in H.last_error() or "null" in H.last_error()
    assert lib.hmc_stream_triad(4096, 8192, 12288, 1.0, 0, 1, None) == H.HMC_OK  # empty: no launch


def test_bench_refuses_more_than_one_gpu():
    """bench.py has no multi-GPU path: --gpus N > 1 exits 2 with a message
    (checked before anything touches a GPU)."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


# the boundary's entry points, each documented with the passage of the paper
# that defines (or motivates) the operation
BOUNDARY = ("hmc_field_bytes", "hmc_fields_bytes", "hmc_alloc_fields", "hmc_free_fields", "hmc_import_gauge",
            "hmc_export_gauge", "hmc_import_momenta", "hmc_export_momenta", "hmc_import_spinor",
            "hmc_export_spinor", "hmc_wilson_dslash", "hmc_mhat", "hmc_wilson_m", "hmc_norm2", "hmc_inner",
            "hmc_sum_multi", "hmc_plaquette", "hmc_gauge_action", "hmc_kinetic_energy", "hmc_gauge_force",
            "hmc_fermion_force", "hmc_exp_update_reunit", "hmc_refresh", "hmc_weak_field_start",
            "hmc_make_source", "hmc_cg_solve", "hmc_md_leapfrog", "hmc_trajectory", "hmc_request_bytes",
            "hmc_service_create", "hmc_service_submit", "hmc_service_poll", "hmc_service_wait",
            "hmc_service_step", "hmc_service_destroy")


def doc_block(name):
    """The last comment block standing on its own lines before the
    declaration of `name`."""
    text = open(HEADER).read()
    m = re.search(r"^hmc_status\s+%s\s*\(" % name, text, flags=re.M)
    assert m, name
    blocks = [b for b in re.finditer(r"^[ \t]*/\*.*?\*/[ \t]*$", text[:m.start()], flags=re.S | re.M)]
    assert blocks, name
    return blocks[-1].group(0)


@pytest.mark.parametrize("name", BOUNDARY)
def test_boundary_entry_cites_the_paper(name):
    assert re.search(r"Sec\. \d", doc_block(name)), name


def test_service_needs_caller_streams(H):
    """The service runs on streams the caller owns: zero streams is an
    argument error (checked before any device work)."""
    buf = C.create_string_buffer(1 << 16)
    base = (C.addressof(buf) + 255) & ~255
    p = H.ServiceParams(base, 1 << 15, 4, H.F32, 1e-10, 100, 1, 16, 0)
    h = C.c_void_p()
    assert H.lib().hmc_service_create(C.byref(p), C.byref(h)) == H.HMC_E_ARG
    assert "n_streams" in H.last_error()
    p.n_streams = 9
    assert H.lib().hmc_service_create(C.byref(p), C.byref(h)) == H.HMC_E_ARG


# ctypes mirrors of the header's structs: every field at the C offset
STRUCTS = {"hmc_geom": "Geom", "hmc_action": "Action", "hmc_cg_params": "CgParams", "hmc_cg_stats": "CgStats",
           "hmc_md_stats": "MdStats", "hmc_traj_params": "TrajParams", "hmc_traj_result": "TrajResult",
           "hmc_mts_params": "MtsParams", "hmc_mts_stats": "MtsStats", "hmc_service_params": "ServiceParams",
           "hmc_solve_request": "SolveRequest", "hmc_solve_result": "SolveResult",
           "hmc_timing_entry": "TimingEntry"}


def test_binding_structs_match_the_header(tmp_path):
    """The C compiler's sizeof and offsetof of every struct of include/hmc.h
    against the binding's ctypes layouts (a field added on one side only
    would shift every later field)."""
    import ctypes
    import subprocess

    from paper_1212_0785_amd import hmc as Hm
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "hmc.h"', "int main(void) {"]
    for cname, pyname in STRUCTS.items():
        cls = getattr(Hm, pyname)
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            cname, field, value = line.split()
            got[(cname, field)] = int(value)
    for cname, pyname in STRUCTS.items():
        cls = getattr(Hm, pyname)
        assert got[(cname, "sizeof")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)
