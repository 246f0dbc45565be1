"""The oracle and the HIP path share nothing.

The oracle (oracle/) is test infrastructure written from the paper; the
product (paper_2512_24840_amd/ and include/) is the HIP library and its
binding.  Neither includes, imports, loads or links the other, they have no
source lines in common, and only the seeded input generators (synth/, no
method arithmetic) serve both.
"""

import ast
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2512_24840_amd")
ORACLE = os.path.join(ROOT, "oracle")
SYNTH = os.path.join(ROOT, "synth")
INCLUDE = os.path.join(ROOT, "include")


def files(root, exts):
    out = []
    for d, _, fs in os.walk(root):
        if "__pycache__" in d or "_lib" in d:
            continue
        out += [os.path.join(d, f) for f in fs if f.endswith(exts)]
    return sorted(out)


def imported_modules(path):
    tree = ast.parse(open(path).read(), path)
    mods = set()
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            mods |= {a.name.split(".")[0] for a in node.names}
        elif isinstance(node, ast.ImportFrom) and node.level == 0 and node.module:
            mods.add(node.module.split(".")[0])
    return mods


def c_includes(path):
    return re.findall(r'^\s*#\s*include\s*([<"][^>"]+[>"])', open(path).read(), re.M)


def code_lines(path):
    """Non-trivial source lines with comments stripped (C/C++/HIP)."""
    text = re.sub(r"/\*.*?\*/", "", open(path).read(), flags=re.S)
    out = set()
    for ln in text.splitlines():
        ln = ln.split("//")[0].strip()
        if len(ln) >= 30:
            out.add(re.sub(r"\s+", " ", ln))
    return out


def test_package_never_imports_or_names_the_oracle():
    for path in files(PKG, (".py",)):
        mods = imported_modules(path)
        assert "oracle" not in mods, path
        assert "lasp_oracle" not in open(path).read(), path
    for path in files(PKG, (".hip", ".h", ".cpp", ".c")) + files(INCLUDE, (".h",)):
        text = open(path).read()
        assert "lasp_oracle" not in text and "orc_" not in text, path


def test_oracle_never_imports_the_package_or_the_generators():
    allowed = {"__future__", "ctypes", "os", "subprocess", "concurrent", "numpy"}
    for path in files(ORACLE, (".py",)):
        mods = imported_modules(path)
        assert mods <= allowed, (path, mods - allowed)


def test_generators_import_neither_side():
    for path in files(SYNTH, (".py",)):
        mods = imported_modules(path)
        assert "oracle" not in mods and "paper_2512_24840_amd" not in mods, path


def test_c_sources_include_only_their_own_side():
    for path in files(ORACLE, (".c", ".h")):
        for inc in c_includes(path):
            assert inc.startswith("<"), (path, inc)
            assert "hip" not in inc and "lasp" not in inc, (path, inc)
    own = {'"lasp.h"', '"lasp_internal.h"'}
    for path in files(os.path.join(PKG, "csrc"), (".hip", ".h")):
        for inc in c_includes(path):
            assert inc.startswith("<") or inc in own, (path, inc)


# Lines both sides write from the same definition in the interface: the
# left edge of the first source bin of the resampling (bins of width dlam
# centred on lam0 + i dlam, Eqs. 2-4).
SAME_DEFINITION = {"const double e0 = lam0 - 0.5 * dlam;"}


def test_no_source_line_in_common():
    orc = set()
    for path in files(ORACLE, (".c", ".h")):
        orc |= code_lines(path)
    for path in files(os.path.join(PKG, "csrc"), (".hip", ".h")) + files(INCLUDE, (".h",)):
        common = (orc & code_lines(path)) - SAME_DEFINITION
        assert not common, (path, sorted(common)[:5])


def test_built_libraries_do_not_link_each_other():
    lib = os.path.join(PKG, "_lib", "liblasp.so")
    olib = os.path.join(ORACLE, "liblasp_oracle.so")
    if not (os.path.exists(lib) and os.path.exists(olib)):
        pytest.skip("libraries not built")
    # both are built in this tree from the sources above
    lb, ob = open(lib, "rb").read(), open(olib, "rb").read()
    assert b"lasp_oracle" not in lb and b"orc_eval" not in lb
    assert b"lasp_fit_group" not in ob and b"liblasp.so" not in ob


def test_bench_calls_the_oracle_only_after_its_timed_gpu_work():
    """bench.py imports the oracle only inside functions, and main() names it
    only after its last timed GPU call (the baseline and the checks run after
    the measurements, never inside them)."""
    path = os.path.join(ROOT, "bench.py")
    tree = ast.parse(open(path).read(), path)
    for node in tree.body:
        if isinstance(node, (ast.Import, ast.ImportFrom)):
            names = [a.name for a in node.names] + [getattr(node, "module", None) or ""]
            assert not any(n.split(".")[0] == "oracle" for n in names), "module-level oracle import"
    main = next(n for n in tree.body if isinstance(n, ast.FunctionDef) and n.name == "main")
    gpu_calls = [n.lineno for n in ast.walk(main) if isinstance(n, ast.Call)
                 and isinstance(n.func, (ast.Attribute, ast.Name))
                 and getattr(n.func, "attr", getattr(n.func, "id", "")) in
                 ("fit_group", "forward", "resample", "timed", "once", "serving_leg")]
    oracle_refs = [n.lineno for n in ast.walk(main)
                   if (isinstance(n, ast.Name) and n.id == "oracle")
                   or (isinstance(n, ast.alias) and n.name == "oracle")]
    assert gpu_calls and oracle_refs
    assert min(oracle_refs) > max(gpu_calls), (min(oracle_refs), max(gpu_calls))
