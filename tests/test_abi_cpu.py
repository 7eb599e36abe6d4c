"""C ABI checks that need no GPU: the library loads, exports every entry
point of include/sfr.h, and rejects invalid arguments on the host before
any device work."""
import ctypes
import os
import re

import pytest

import paper_1503_03004_amd as sfr
from paper_1503_03004_amd import _binding as B

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "sfr.h")


def declared():
    txt = open(HDR).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sfr_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_entry_points():
    names = declared()
    for want in ("sfr_create", "sfr_solve", "sfr_solve_nys", "sfr_tsvd", "sfr_create_batch", "sfr_solve_batch",
                 "sfr_tune_batch", "sfr_destroy", "sfr_status_string", "sfr_version", "sfr_workspace_bytes",
                 "sfr_solve_noalloc"):
        assert want in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(sfr.LIB_PATH)
    for name in declared():
        assert hasattr(lib, name), name


def test_struct_layouts_match_header(tmp_path):
    """The binding's ctypes structs have the C compiler's size and offsets."""
    import subprocess
    fields = {"sfr_options": [f for f, _ in B.sfr_options._fields_],
              "sfr_info": [f for f, _ in B.sfr_info._fields_],
              "sfr_batch_item": [f for f, _ in B.sfr_batch_item._fields_]}
    lines = ['#include "sfr.h"', "#include <stdio.h>", "#include <stddef.h>", "int main(void) {"]
    for st, fs in fields.items():
        lines.append(f'printf("%zu\\n", sizeof({st}));')
        for f in fs:
            cname = {"lam": "lambda"}.get(f, f)      # a Python keyword in the header
            lines.append(f'printf("%zu\\n", offsetof({st}, {cname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.dirname(HDR), str(src), "-o", str(exe)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    want = []
    for cls in (B.sfr_options, B.sfr_info, B.sfr_batch_item):
        want.append(ctypes.sizeof(cls))
        want += [getattr(cls, f).offset for f, _ in cls._fields_]
    assert got == want


def test_status_strings_and_version():
    L = sfr.lib()
    assert L.sfr_version().decode().count(".") == 2
    for code in (0, -1, -2, -3, -4, -5, -6, -7, -8, 1, 2):
        s = L.sfr_status_string(code).decode()
        assert s and s != "unknown status"
    assert L.sfr_status_string(99).decode() == "unknown status"


def _create(m, n, r, lam, mu, tol, **kw):
    o = B.sfr_options()
    o.struct_size = ctypes.sizeof(B.sfr_options)
    for k, v in kw.items():
        setattr(o, k, v)
    h = ctypes.c_void_p(None)
    rc = sfr.lib().sfr_create(ctypes.byref(h), m, n, r, lam, mu, tol, ctypes.byref(o))
    return rc, h


@pytest.mark.parametrize("args,kw", [
    ((0, 10, 1, 0.1, 1.0, 1e-7), {}),            # m < 1
    ((10, 0, 1, 0.1, 1.0, 1e-7), {}),            # n < 1
    ((10, 10, 0, 0.1, 1.0, 1e-7), {}),           # r < 1
    ((10, 5, 6, 0.1, 1.0, 1e-7), {}),            # r > min(m, n)
    ((100, 100, 33, 0.1, 1.0, 1e-7), {}),        # r above the supported 32
    ((10, 10, 2, 0.0, 1.0, 1e-7), {}),           # lambda <= 0
    ((10, 10, 2, float("nan"), 1.0, 1e-7), {}),  # lambda NaN
    ((10, 10, 2, 0.1, float("nan"), 1e-7), {}),  # mu NaN (mu <= 0 selects the default)
    ((10, 10, 2, 0.1, float("inf"), 1e-7), {}),  # mu infinite
    ((10, 10, 2, 0.1, float("inf"), 1e-7), {}),  # mu infinite
    ((10, 10, 2, 0.1, 1.0, -1.0), {}),           # tol < 0
    ((10, 10, 2, 0.1, 1.0, 1e-7), {"precision": 7}),
    ((10, 10, 2, 0.1, 1.0, 1e-7), {"rho": 0.9}),       # rho must exceed 1 (Alg. 1)
    ((10, 10, 2, 0.1, 1.0, 1e-7), {"max_iter": -3}),
    ((10, 10, 2, 0.1, 1.0, 1e-7), {"fixed_iters": -1}),
    ((10, 10, 2, 0.1, 1.0, 1e-7), {"nystrom_l": 1}),   # l < r
    ((10, 10, 2, 0.1, 1.0, 1e-7), {"nystrom_l": 11}),  # l > min(m, n)
    ((10, 10, 2, 0.1, 1.0, 1e-7), {"nystrom_l": 4}),   # missing mu_left / mu_top
    ((10, 10, 2, 0.1, 1.0, 1e-7), {"bf16": 1}),                          # BF16 needs FP32 storage
    ((10, 10, 2, 0.1, 1.0, 1e-7), {"bf16": 1, "precision": 1, "nystrom_l": 4, "mu_left": 1.0, "mu_top": 1.0}),
    ((10, 10, 2, 0.1, 1.0, 1e-7), {"bf16_iters": 3, "precision": 1}),   # BF16 fields without bf16
    ((10, 10, 2, 0.1, 1.0, 1e-7), {"bf16_tol": 1e-3, "precision": 1}),
    ((10, 10, 2, 0.1, 1.0, 1e-7), {"bf16": 1, "precision": 1, "bf16_iters": -1}),
    ((10, 10, 2, 0.1, 1.0, 1e-7), {"bf16": 1, "precision": 1, "bf16_tol": -1.0}),
])
def test_create_rejects_invalid_arguments(args, kw):
    rc, h = _create(*args, **kw)
    assert rc == B.SFR_ERR_ARG
    assert not h.value


def test_create_rejects_wrong_struct_size():
    o = B.sfr_options()
    o.struct_size = 12
    h = ctypes.c_void_p(None)
    assert sfr.lib().sfr_create(ctypes.byref(h), 10, 10, 2, 0.1, 1.0, 1e-7, ctypes.byref(o)) == B.SFR_ERR_ARG
    assert sfr.lib().sfr_create(None, 10, 10, 2, 0.1, 1.0, 1e-7, None) == B.SFR_ERR_ARG


@pytest.mark.parametrize("args,kw", [
    ((0, 100, 64, 4), {}),                # capacity < 1
    ((70000, 100, 64, 4), {}),            # capacity above 65536
    ((4, 0, 64, 4), {}),                  # max_m < 1
    ((4, 100, 0, 4), {}),                 # max_n < 1
    ((4, 100, 513, 4), {}),               # max_n above 512
    ((4, 100, 64, 0), {}),                # max_r < 1
    ((4, 100, 64, 17), {}),               # max_r above 16
    ((4, 100, 3, 4), {}),                 # max_r > max_n
    ((4, 100, 64, 4), {"precision": 0}),  # FP32 only
    ((4, 100, 64, 4), {"nystrom_l": 8}),
    ((4, 100, 64, 4), {"rho": 1.0}),
    ((4, 100, 64, 4), {"max_iter": -1}),
    ((4, 100, 64, 4), {"fixed_iters": -2}),
    ((4, 100, 64, 4), {"struct_size": 3}),
    ((4, 100, 64, 4), {"bf16_iters": 3}),                # BF16 fields without bf16
    ((4, 100, 64, 4), {"bf16": 1, "bf16_tol": -1.0}),
])
def test_create_batch_rejects_invalid_arguments(args, kw):
    o = B.sfr_options()
    o.struct_size = ctypes.sizeof(B.sfr_options)
    o.precision = B.SFR_F32
    for k, v in kw.items():
        setattr(o, k, v)
    h = ctypes.c_void_p(None)
    assert sfr.lib().sfr_create_batch(ctypes.byref(h), *args, ctypes.byref(o)) == B.SFR_ERR_ARG
    assert not h.value
    assert sfr.lib().sfr_create_batch(ctypes.byref(h), 4, 100, 64, 4, None) == B.SFR_ERR_ARG


def test_null_handle_paths():
    L = sfr.lib()
    info = B.sfr_info()
    assert L.sfr_solve(None, None, 0, None, None, None, None, 0, ctypes.byref(info), None) == B.SFR_ERR_HANDLE
    assert L.sfr_solve_nys(None, None, 0, None, None, None, None, None, 0, ctypes.byref(info),
                           None) == B.SFR_ERR_HANDLE
    assert L.sfr_tsvd(None, None, 0, None, None, None, ctypes.byref(info), None) == B.SFR_ERR_HANDLE
    items = (B.sfr_batch_item * 1)()
    assert L.sfr_solve_batch(None, items, 1, None, None, None) == B.SFR_ERR_HANDLE
    assert L.sfr_tune_batch(None, items, 1, None, None) == B.SFR_ERR_HANDLE
    assert L.sfr_destroy(None) == B.SFR_OK
    b = ctypes.c_uint64(0)
    assert L.sfr_workspace_bytes(None, ctypes.byref(b)) == B.SFR_ERR_HANDLE


def test_binding_refuses_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(B, "_lib", None)
    with pytest.raises(ImportError):
        B.lib()


def test_output_buffer_checks_on_host():
    """Caller-supplied outputs are checked (shape, dtype, device, layout)
    before any library call; CPU tensors stand in for device ones here."""
    import torch
    cpu = torch.device("cpu")
    m, n, r = 6, 5, 2
    U = torch.empty((m, r), dtype=torch.float32)
    Bm = torch.empty((r, r), dtype=torch.float64)
    V = torch.empty((n, r), dtype=torch.float32)
    S = torch.empty((m, n), dtype=torch.float32)
    B.check_outputs(U, Bm, V, S, m, n, r, torch.float32, cpu)
    B.check_outputs(U, Bm, V, None, m, n, r, torch.float32, cpu)
    B.check_outputs(U, Bm, V, torch.empty((m, n + 3), dtype=torch.float32)[:, :n], m, n, r, torch.float32, cpu)
    bad = [
        (torch.empty((m, r + 1), dtype=torch.float32), Bm, V, S),
        (U.double(), Bm, V, S),
        (U, Bm.float(), V, S),
        (U, Bm, torch.empty((r, n), dtype=torch.float32).t(), S),
        (U, Bm, V, torch.empty((n, m), dtype=torch.float32).t()),
        (U, Bm, V, torch.empty((m, n), dtype=torch.float64)),
        (U, Bm, V, torch.empty((m, 2 * n), dtype=torch.float32)[:, ::2]),
        (None, Bm, V, S),
    ]
    for args in bad:
        with pytest.raises(ValueError):
            B.check_outputs(*args, m, n, r, torch.float32, cpu)
    with pytest.raises(ValueError):
        B.check_outputs(U, Bm, V, S, m, n, r, torch.float32, torch.device("cuda", 0))


def test_noalloc_rejects_invalid_arguments_on_host():
    """sfr_solve_noalloc validates on the host before any device call: the
    checks of sfr_create, NULL buffers, ld < n, and the options it does not
    take (FR-Nys, profiling)."""
    L = sfr.lib()
    info = B.sfr_info()
    dummy = ctypes.c_void_p(16)

    def call(m=100, n=80, r=3, lam=0.1, mu=0.5, tol=1e-7, opt=None, M=dummy, ldm=80, U=dummy, Bp=dummy, V=dummy,
             S=None, lds=0):
        o = ctypes.byref(opt) if opt is not None else None
        return L.sfr_solve_noalloc(m, n, r, lam, mu, tol, o, M, ldm, U, Bp, V, S, lds, ctypes.byref(info), None)

    assert call(m=0) == B.SFR_ERR_ARG
    assert call(r=81) == B.SFR_ERR_ARG
    assert call(lam=0.0) == B.SFR_ERR_ARG
    assert call(mu=float("nan")) == B.SFR_ERR_ARG
    assert call(M=None) == B.SFR_ERR_ARG
    assert call(V=None) == B.SFR_ERR_ARG
    assert call(ldm=79) == B.SFR_ERR_ARG
    assert call(S=dummy, lds=10) == B.SFR_ERR_ARG
    o = B._options("f32", nystrom_l=10, mu_left=1.0, mu_top=1.0)
    assert call(opt=o) == B.SFR_ERR_ARG
    o = B._options("f32", profile=True)
    assert call(opt=o) == B.SFR_ERR_ARG
    o = B._options("f32")
    o.struct_size = 3
    assert call(opt=o) == B.SFR_ERR_ARG


def test_queue_entry_points_reject_bad_handles():
    """The queue form's entry points check the handle on the host."""
    L = sfr.lib()
    info = B.sfr_info()
    t = ctypes.c_int32(0)
    d = ctypes.c_int32(0)
    st = ctypes.c_int32(0)
    item = B.sfr_batch_item()
    assert L.sfr_queue_start(None, 0, 0) == B.SFR_ERR_HANDLE
    assert L.sfr_queue_submit(None, ctypes.byref(item), ctypes.byref(t)) == B.SFR_ERR_HANDLE
    assert L.sfr_queue_poll(None, 0, ctypes.byref(d), ctypes.byref(info), ctypes.byref(st)) == B.SFR_ERR_HANDLE
    assert L.sfr_queue_stop(None) == B.SFR_ERR_HANDLE


@pytest.mark.parametrize("argv, env", [(["--gpus", "2"], {}), (["--gpus", "8"], {}), ([], {"WORLD_SIZE": "2"})])
def test_bench_refuses_more_than_one_gpu(argv, env):
    # the bench is a one-GPU measurement: a multi-GPU request exits with a
    # message, before any device work
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    e = dict(os.environ, **env)
    p = subprocess.run([sys.executable, os.path.join(root, "bench.py"), *argv], cwd=root, env=e,
                       capture_output=True, text=True, timeout=60)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""
