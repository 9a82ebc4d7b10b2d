"""Host-side checks of the C-ABI library (no GPU needed).

The library loads, exports every entry point include/st.h declares, and
rejects bad mesh descriptors on the host before touching a device.
"""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "st.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    return sorted(set(re.findall(r"\b(st_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def N():
    from paper_2603_26691_amd import _native
    return _native


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["st_create_mesh", "st_inject", "st_step", "st_get_sources", "st_backward"]:
        assert required in names


def test_library_exports_every_declared_symbol(N):
    lib = N.lib()
    for name in declared_functions():
        assert hasattr(lib, name), f"missing export {name}"
    out = subprocess.run(["nm", "-D", "--defined-only", N.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (st_[a-z_]+)\b", out))
    assert set(declared_functions()) <= exported
    # and the binding knows every one of them
    assert set(declared_functions()) == set(N.SIGNATURES)


def test_mesh_desc_layout_matches_header(N, tmp_path):
    # ask the C compiler for the layout of st_mesh_desc
    fields = [f for f, _ in N.MeshDesc._fields_]
    prog = ["#include <stdio.h>", "#include <stddef.h>", '#include "st.h"', "int main(void){",
            'printf("%zu\\n", sizeof(st_mesh_desc));']
    prog += [f'printf("%zu\\n", offsetof(st_mesh_desc, {f}));' for f in fields]
    prog += ["return 0;}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(prog))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                           check=True).stdout.split()]
    assert vals[0] == ctypes.sizeof(N.MeshDesc)
    for f, off in zip(fields, vals[1:]):
        assert getattr(N.MeshDesc, f).offset == off, f


def _desc(N, **kw):
    d = N.MeshDesc()
    d.n[:] = kw.get("n", (16, 16, 16))
    d.chunk_edge = kw.get("chunk_edge", 8)
    d.L[:] = kw.get("L", (0.1, 0.1, 0.1))
    d.rho_f = kw.get("rho_f", 1.2)
    d.mu_f = kw.get("mu_f", 1.8e-5)
    d.g[:] = (0.0, 0.0, -9.81)
    d.rho_p = kw.get("rho_p", 1000.0)
    d.parcel_weight = kw.get("w", 1.0)
    d.form = kw.get("form", 1)
    d.interp = kw.get("interp", 0)
    d.drag = kw.get("drag", 0)
    d.reserved = kw.get("reserved", 0)
    d.capacity = kw.get("capacity", 1000)
    return d


@pytest.mark.parametrize("bad", [
    dict(chunk_edge=3), dict(chunk_edge=16), dict(n=(12, 16, 16)), dict(n=(16, 16, 0)),
    dict(L=(0.1, -1.0, 0.1)), dict(L=(0.1, float("nan"), 0.1)), dict(mu_f=0.0),
    dict(rho_p=-1.0), dict(w=0.0), dict(form=7), dict(interp=2), dict(capacity=0),
    dict(capacity=1 << 40), dict(drag=2), dict(drag=-1), dict(reserved=1),
    dict(drag=1, rho_f=-1.0), dict(drag=1, rho_f=float("nan")),
])
def test_create_rejects_bad_descriptor_on_host(N, bad):
    ctx = ctypes.c_void_p()
    st = N.lib().st_create_mesh(ctypes.byref(_desc(N, **bad)), 0, ctypes.byref(ctx))
    assert st == N.ST_ERR_INVALID
    assert not ctx.value
    msg = N.lib().st_last_error(None).decode()
    assert msg.startswith("st_create_mesh:")


def test_null_arguments(N):
    L = N.lib()
    assert L.st_create_mesh(None, 0, None) == N.ST_ERR_INVALID
    assert L.st_destroy(None) == N.ST_ERR_INVALID
    assert L.st_step(None, None, 1e-4, 1, 0, None) == N.ST_ERR_INVALID
    assert L.st_inject(None, 1, None, None, None, 0, None) == N.ST_ERR_INVALID
    assert L.st_get_sources(None, None, 0, 0, None) == N.ST_ERR_INVALID
    assert L.st_backward(None, None, None, None, None) == N.ST_ERR_INVALID
    assert L.st_tape_reserve(None, 20, 200) == N.ST_ERR_INVALID
    assert L.st_count(None, None) == N.ST_ERR_INVALID


def test_create_without_device_fails_cleanly(N):
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a device is present")
    ctx = ctypes.c_void_p()
    st = N.lib().st_create_mesh(ctypes.byref(_desc(N)), 0, ctypes.byref(ctx))
    assert st in (N.ST_ERR_DEVICE, N.ST_ERR_OOM)
    assert not ctx.value
