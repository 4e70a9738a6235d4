"""Host-only checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/pic.h declares, the ctypes mirrors of its structs
have the C layout, and configuration errors are rejected before any device
work."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

import pic_inputs as pin

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pic.h")


@pytest.fixture(scope="module")
def P():
    from paper_2404_10270_amd import pic
    if not os.path.exists(pic.LIB_PATH):
        from paper_2404_10270_amd import build
        build.build()
    pic.lib()
    return pic


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(pic_\w+)\s*\(", src, re.M)))


def test_exports_every_declared_symbol(P):
    names = _declared()
    assert set(names) == set(P.ABI_SYMBOLS)
    out = subprocess.run(["nm", "-D", "--defined-only", P.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r" T (pic_\w+)", out))
    for n in names:
        assert n in exported, n
        assert hasattr(P.lib(), n)


def test_struct_layout_matches_header(P, tmp_path):
    """Compile a C program against pic.h and compare sizes and offsets."""
    structs = {"pic_species": P.pic_species, "pic_config": P.pic_config,
               "pic_sizes": P.pic_sizes, "pic_buffers": P.pic_buffers, "pic_diag": P.pic_diag}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pic.h"', 'int main(void){']
    for name, T in structs.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f, _ in T._fields_:
            lines.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines.append("return 0;}")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(c), "-o",
                           str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = dict(l.split() for l in out if l.strip())
    for name, T in structs.items():
        assert int(got[name]) == C.sizeof(T), name
        for f, _ in T._fields_:
            assert int(got[f"{name}.{f}"]) == getattr(T, f).offset, f"{name}.{f}"


def _cfg(P, wl=None, precision=None, caps=None):
    wl = wl or pin.bounded_mcc(nc=256, ppc=10)
    precision = P.PIC_FP32 if precision is None else precision
    st = pin.initial_state(wl)
    caps = caps or [s.n + 100 for s in st]
    return P.make_config(wl, precision, caps, [s.n for s in st], sum(s.n for s in st))


def test_query_sizes_layout(P):
    c = _cfg(P)
    sizes, seg = P.pic_query_sizes([c])
    assert sizes.n_segments == 2
    assert sizes.n_nodes == 257
    assert seg[0] == 0 and seg[1] % 64 == 0 and seg[1] >= c.sp[0].capacity
    assert seg[2] - seg[1] >= c.sp[1].capacity and sizes.n_slots == seg[2]
    assert sizes.work_bytes > 0 and sizes.work_bytes % 256 == 0
    assert sizes.x_elem_bytes == 4
    c64 = _cfg(P, precision=P.PIC_FP64)
    s64, _ = P.pic_query_sizes([c64])
    assert s64.x_elem_bytes == 8 and s64.v_elem_bytes == 8
    # batched: instances are concatenated
    sb, segb = P.pic_query_sizes([c, c, c])
    assert sb.n_segments == 6 and sb.n_nodes == 3 * 257 and len(segb) == 7
    assert all(b % 64 == 0 for b in segb)


@pytest.mark.parametrize("mutate", [
    lambda c: setattr(c, "nc", 1),
    lambda c: setattr(c, "dt", 0.0),
    lambda c: setattr(c, "dx", float("nan")),
    lambda c: setattr(c, "eps0", -1.0),
    lambda c: setattr(c, "bc", 7),
    lambda c: setattr(c, "nsp", 5),
    lambda c: setattr(c, "precision", 3),
    lambda c: setattr(c.sp[0], "m", 0.0),
    lambda c: setattr(c.sp[0], "kind", 9),
    lambda c: setattr(c.sp[1], "kind", 0),          # MCC needs an ion species
    lambda c: setattr(c.sp[0], "n_init", c.sp[0].capacity + 1),
    lambda c: setattr(c.sp[0], "v_cap", 0.0),       # MCC needs a finite nu_max
    lambda c: setattr(c, "sig_el", -1.0),
    lambda c: setattr(c, "B0", float("inf")),
    lambda c: setattr(c, "next_id", 1 << 62),
])
def test_bad_config_rejected(P, mutate):
    c = _cfg(P)
    mutate(c)
    assert P.pic_query_sizes_rc([c]) == P.PIC_E_CONFIG


def test_mismatched_instances_rejected(P):
    a = _cfg(P)
    b = _cfg(P, precision=P.PIC_FP64)
    assert P.pic_query_sizes_rc([a, b]) == P.PIC_E_CONFIG
    assert P.pic_query_sizes_rc([]) == P.PIC_E_ARG


def test_init_argument_errors_before_device_work(P):
    c = _cfg(P)
    arr = (P.pic_config * 1)(c)
    ctx = C.c_void_p()
    L = P.lib()
    # null buffers
    assert L.pic_init(arr, 1, None, None, 0, C.byref(ctx)) == P.PIC_E_ARG
    # misaligned buffers
    b = P.pic_buffers()
    for i in range(2):
        b.x[i] = b.vx[i] = b.vy[i] = b.vz[i] = b.id_lo[i] = b.id_hi[i] = b.cell[i] = 0x1000 + 8
    b.work = 0x2000
    assert L.pic_init(arr, 1, C.byref(b), None, 0, C.byref(ctx)) == P.PIC_E_ARG
    assert ctx.value is None
    # calls on a null context
    assert L.pic_push(None, 0) == P.PIC_E_STATE
    assert L.pic_field_solve(None) == P.PIC_E_STATE
    assert L.pic_step(None, 1, 0) == P.PIC_E_STATE
    assert L.pic_step_graph(None, 1, 0) == P.PIC_E_STATE
    assert L.pic_autotune_sort(None, None, 0, 1, None, None) == P.PIC_E_STATE
    assert L.pic_destroy(None) == P.PIC_E_ARG


def test_init_static_refuses_before_device_work(P):
    """pic_init_static: a caller workspace, or a configuration whose workspace
    exceeds PIC_STATIC_WORK_MAX, is refused before any device call."""
    L = P.lib()
    ctx = C.c_void_p()
    small = _cfg(P)
    arr = (P.pic_config * 1)(small)
    b = P.pic_buffers()
    b.work = 0x100000
    assert L.pic_init_static(arr, 1, C.byref(b), None, 0, C.byref(ctx)) == P.PIC_E_ARG
    assert L.pic_init_static(arr, 1, None, None, 0, C.byref(ctx)) == P.PIC_E_ARG
    assert ctx.value is None
    wl = pin.bounded_mcc(nc=100_000, ppc=100, seed=3)
    n = [int(round(sp.ppc * wl.nc)) for sp in wl.species]
    big = P.make_config(wl, P.PIC_FP32, [m + 1024 for m in n], n, sum(n))
    sizes, _ = P.pic_query_sizes([big])
    assert sizes.work_bytes > P.PIC_STATIC_WORK_MAX
    b.work = None
    arr = (P.pic_config * 1)(big)
    assert L.pic_init_static(arr, 1, C.byref(b), None, 0, C.byref(ctx)) == P.PIC_E_SCRATCH
    bad = _cfg(P)
    bad.dt = 0.0
    arr = (P.pic_config * 1)(bad)
    assert L.pic_init_static(arr, 1, C.byref(b), None, 0, C.byref(ctx)) == P.PIC_E_CONFIG
    assert ctx.value is None


def test_strerror(P):
    for code in (0, -1, -2, -3, -4, -5, -6, -7, -8, -9, -99):
        s = P.pic_strerror(code)
        assert isinstance(s, str) and s


def test_layout_study_library_exports_and_layout(P, tmp_path):
    """libpic_layout (the mover in four particle layouts): every entry point
    include/pic_layout.h declares is exported, the ctypes mirrors have the C
    layout, and bad arguments are refused without device work."""
    from paper_2404_10270_amd import layout as Lb
    src = open(os.path.join(ROOT, "include", "pic_layout.h")).read()
    names = sorted(set(re.findall(r"^\s*int\s+(pls_\w+)\s*\(", src, re.M)))
    assert set(names) == set(Lb.ABI_SYMBOLS)
    out = subprocess.run(["nm", "-D", "--defined-only", Lb.LIB], capture_output=True, text=True,
                         check=True).stdout
    for n in names:
        assert re.search(rf" T {n}$", out, re.M), n
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pic_layout.h"', 'int main(void){']
    for name, T in {"pls_soa": Lb.pls_soa, "pls_params": Lb.pls_params}.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f, _ in T._fields_:
            lines.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines.append("return 0;}")
    c = tmp_path / "pls.c"
    c.write_text("\n".join(lines))
    exe = tmp_path / "pls"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)])
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                 check=True).stdout.split("\n") if l.strip())
    for name, T in {"pls_soa": Lb.pls_soa, "pls_params": Lb.pls_params}.items():
        assert int(got[name]) == C.sizeof(T), name
        for f, _ in T._fields_:
            assert int(got[f"{name}.{f}"]) == getattr(T, f).offset, f"{name}.{f}"
    L = Lb.lib()
    nb = C.c_uint64()
    assert L.pls_work_bytes(Lb.PLS_SOA, 1000, 100, 0, C.byref(nb)) == 0 and nb.value > 24000
    assert L.pls_work_bytes(7, 1000, 100, 0, C.byref(nb)) == -1          # no such layout
    assert L.pls_work_bytes(Lb.PLS_CELLPAD, 1000, 100, 100, C.byref(nb)) == -1  # slack not a multiple of 64
    assert L.pls_work_bytes(Lb.PLS_SOA, 1000, 1, 0, C.byref(nb)) == -1   # too few cells
    assert L.pls_step(Lb.PLS_SOA, None, 10, 0, 0, None, None) == -1
