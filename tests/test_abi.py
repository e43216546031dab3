"""The C-ABI library loads and exports every function include/*.h declares
(no compute call: this runs without a GPU)."""
import glob
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        names += re.findall(r"^(?:qap_status|void|const char\s*\*)\s+(qap_\w+)\s*\(", text, re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def libpath():
    from paper_1510_02065_amd import build
    if build.needs_build():
        build.build()
    return build.LIB


def test_every_declared_symbol_is_exported(libpath):
    names = _declared()
    assert len(names) >= 12
    out = subprocess.run(["nm", "-D", "--defined-only", libpath], capture_output=True, text=True, check=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    missing = [n for n in names if n not in exported]
    assert not missing, missing


def test_library_loads_and_binding_covers_header(libpath):
    import paper_1510_02065_amd as pkg
    from paper_1510_02065_amd import _binding
    L = pkg.lib()
    for n in _declared():
        getattr(L, n)
        assert n in _binding.SIGNATURES, n
