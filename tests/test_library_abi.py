"""The C-ABI library loads and exports every entry point the header declares
(no device calls)."""
import ctypes
import os
import re
import subprocess

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "narrowsdc.h")
LIB = os.path.join(ROOT, "paper_1309_7327_amd", "libnarrowsdc.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^(?:int|void|const char\s*\*)\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("set_mechanism", "rhs_eval", "sdc_step", "sdc_step_batched", "prim_to_cons",
              "sdc_context_create", "sdc_context_destroy", "sdc_workspace_size", "last_status",
              "last_error_message"):
        assert n in names, n


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "library not built"
    lib = ctypes.CDLL(LIB)
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    for n in declared():
        assert n in exported, n
        assert getattr(lib, n) is not None


def test_binding_fails_loudly_without_library(tmp_path):
    import sys
    code = ("import sys, os; sys.path.insert(0, %r); import shutil\n"
            "import paper_1309_7327_amd.narrowsdc as n\n") % ROOT
    env = dict(os.environ)
    # a copy of the package without the shared library must refuse to import
    pkg = tmp_path / "paper_1309_7327_amd"
    pkg.mkdir()
    for f in ("__init__.py", "narrowsdc.py"):
        (pkg / f).write_text(open(os.path.join(ROOT, "paper_1309_7327_amd", f)).read())
    r = subprocess.run([sys.executable, "-c", "import sys; sys.path.insert(0, %r); import paper_1309_7327_amd.narrowsdc" % str(tmp_path)],
                       capture_output=True, text=True, env=env)
    assert r.returncode != 0 and "no CPU fallback" in r.stderr


def test_species_counts_of_the_build():
    """The kernels are specialised per species count; the query touches no
    device.  The default build covers 9, 12 and 21 species."""
    lib = ctypes.CDLL(LIB)
    lib.sdc_species_supported.argtypes = [ctypes.c_int]
    lib.sdc_species_supported.restype = ctypes.c_int
    assert [n for n in range(0, 30) if lib.sdc_species_supported(n)] == [9, 12, 21]
