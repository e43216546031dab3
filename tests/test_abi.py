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


def _tool(name):
    p = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm", "bin", name)
    return p if os.path.exists(p) else None


def test_every_registered_kernel_has_device_code(libpath, tmp_path):
    """Every kernel whose host stub an object registers is defined, under the
    same name, in that object's gfx950 code.  A kernel whose template
    arguments involve a type with internal linkage (an unnamed enum) gets a
    translation-unit-local device name, and the runtime then fails to find
    it at its first launch."""
    from paper_1510_02065_amd import build
    bundler, readelf = _tool("clang-offload-bundler"), _tool("llvm-readelf")
    if not bundler or not readelf:
        pytest.skip("ROCm LLVM tools not found")
    checked = 0
    for src in build.SOURCES:
        if not src.endswith(".hip"):
            continue
        obj = os.path.join(build.OBJDIR, os.path.basename(src) + ".o")
        fat = str(tmp_path / (os.path.basename(src) + ".fatbin"))
        co = str(tmp_path / (os.path.basename(src) + ".co"))
        subprocess.run(["objcopy", "--dump-section", f".hip_fatbin={fat}", obj], capture_output=True)
        if not os.path.exists(fat):
            continue   # no device code in this object
        subprocess.run([bundler, "--type=o", "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", f"--input={fat}",
                        f"--output={co}", "--unbundle"], check=True)
        syms = subprocess.run([readelf, "-s", "--wide", co], capture_output=True, text=True, check=True).stdout
        dev = set(l.split()[7] for l in syms.splitlines() if len(l.split()) >= 8 and l.split()[3] == "FUNC")
        strs = subprocess.run(["strings", obj], capture_output=True, text=True, check=True).stdout.split()
        stubs = set(s for s in strs if "__device_stub__" in s and "." not in s)
        host = set(s.replace("__device_stub__", "", 1) for s in stubs)
        # the stub's name differs from the kernel's by the inserted prefix,
        # whose length is part of the mangled identifier: rebuild it
        names = set()
        for s in stubs:
            m = re.match(r"(_ZN(?:\d+\w+?)*?)(\d+)__device_stub__", s)
            assert m, f"unrecognised stub name {s}"
            k = int(m.group(2)) - len("__device_stub__")
            names.add(m.group(1) + str(k) + s[m.end():])
        internal = sorted(n for n in names if "_GLOBAL__N_" in n)
        assert not internal, ("kernels with internal linkage", internal[:3])
        assert names, f"no kernel stubs found in {obj}"
        missing = sorted(n for n in names if n not in dev)
        assert not missing, (os.path.basename(src), missing[:3])
        checked += len(names)
    assert checked > 0
