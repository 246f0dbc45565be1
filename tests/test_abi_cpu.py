"""C ABI checks that need no GPU: exports, struct layout, host validation."""

import ctypes
import math
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2512_24840_amd import lasp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lasp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lasp_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = lasp.load()
    names = declared_functions()
    assert set(names) == set(lasp.EXPORTED)
    out = subprocess.run(["nm", "-D", "--defined-only", lasp.library_path()], capture_output=True,
                         text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    for n in names:
        assert n in exported, n
        assert hasattr(lib, n)


def test_opts_struct_layout_matches_c(tmp_path):
    fields = [f for f, _ in lasp.LaspOpts._fields_]
    prog = tmp_path / "layout.c"
    prog.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "lasp.h"\nint main(void){\n'
                    + "".join(f'printf("%zu\\n", offsetof(lasp_opts, {f}));\n' for f in fields)
                    + 'printf("%zu\\n", sizeof(lasp_opts));return 0;}\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)],
                   check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    want = [getattr(lasp.LaspOpts, f).offset for f in fields] + [ctypes.sizeof(lasp.LaspOpts)]
    assert got == want


def test_default_opts():
    o = lasp.LaspOpts()
    lasp.load().lasp_default_opts(ctypes.byref(o))
    assert (o.n_basis, o.margin, o.degree, o.precision) == (20, 64, 10, 0)
    assert o.box_lo[0] == pytest.approx(math.log10(4000.0))
    assert o.box_hi[3] == 300.0 and o.box_lo[4] == 50.0
    assert o.lr == pytest.approx(1e-2) and o.beta2 == pytest.approx(0.999)
    assert o.weight_quantile == pytest.approx(0.5)
    assert o.n_classes == 1 and list(o.class_edges) == [4000.0, 4550.0, 7000.0, 9000.0]
    assert o.step_graph == 1


def _call_fit(o, grid, null_obs=False):
    lib = lasp.load()
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first
    return lib.lasp_fit_group(None if null_obs else fake, fake,
                              grid.ctypes.data_as(ctypes.c_void_p), fake, fake, fake, None, 10,
                              ctypes.byref(o))


def _opts(**kw):
    o = lasp.LaspOpts()
    lasp.load().lasp_default_opts(ctypes.byref(o))
    o.n_spec, o.n_pix = 4, 64
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _grid(P=64, step=1e-4):
    return 4000.0 * 10.0 ** (step * np.arange(P))


@pytest.mark.parametrize("kw,code", [
    (dict(n_basis=19), -1),
    (dict(margin=0), -1),
    (dict(margin=81), -1),
    (dict(degree=5), -5),
    (dict(degree=12), -5),
    (dict(precision=7), -5),
    (dict(n_pix=16), -1),
    (dict(lr=0.0), -1),
    (dict(n_arms=5), -1),
    (dict(n_classes=2, n_basis=40), -1),
    (dict(n_classes=3), -1),                      # n_basis must be 60
    (dict(n_classes=3, n_basis=60, precision=1), -5),
])
def test_invalid_options_rejected_on_host(kw, code):
    o = _opts(**kw)
    assert _call_fit(o, _grid(o.n_pix)) == code
    assert lasp.load().lasp_last_error().decode() != ""


def test_class_edges_must_increase():
    o = _opts(n_classes=3, n_basis=60)
    o.class_edges[2] = 4000.0
    assert _call_fit(o, _grid()) == -1
    assert b"class_edges" in lasp.load().lasp_last_error()


def _resample(n_src=100, lam0=4000.0, dlam=0.2, n_out=10, lg0=None, d=1e-5, src=0x1000,
              out=0x100000):
    lib = lasp.load()
    if lg0 is None:
        lg0 = math.log10(lam0 + 5.0)
    return lib.lasp_resample(ctypes.c_void_p(src), 3, n_src, n_src, lam0, dlam,
                             ctypes.c_void_p(out), n_out, n_out, lg0, d, None)


def test_resample_validation_on_host():
    assert _resample(n_src=0) == -1
    assert _resample(dlam=0.0) == -1
    assert _resample(d=float("nan")) == -1
    assert _resample(src=0x1000, out=0x1010) == -1                  # out overlaps src
    assert b"overlap" in lasp.load().lasp_last_error()
    assert _resample(lg0=math.log10(3990.0)) == -2                  # starts below the source
    assert _resample(n_out=1000) == -2                              # runs past its end
    assert b"leave the source range" in lasp.load().lasp_last_error()


def test_nonuniform_grid_rejected():
    o = _opts()
    g = _grid()
    g[10] *= 1.00001
    assert _call_fit(o, g) == -2
    assert b"not uniform" in lasp.load().lasp_last_error()
    g = _grid()[::-1].copy()
    assert _call_fit(o, g) == -2


def test_null_pointer_rejected():
    o = _opts()
    assert _call_fit(o, _grid(), null_obs=True) == -1


def test_arms_validation():
    o = _opts(n_arms=2)
    o.arm_start[0], o.arm_start[1] = 0, 70
    assert _call_fit(o, _grid()) == -1
    o.arm_start[1] = 30
    o.arm_sigma_kms[0], o.arm_sigma_kms[1] = 10.0, float("nan")
    assert _call_fit(o, _grid()) == -1


def test_missing_library_fails_loudly(monkeypatch):
    monkeypatch.setattr(lasp, "_lib", None)
    monkeypatch.setattr(lasp, "_LIB_PATH", "/nonexistent/liblasp.so")
    with pytest.raises(ImportError):
        lasp.load()
