"""Build the qap_rlt2 HIP library for gfx950 in-tree (libqap_rlt2.so).

hipcc cross-compiles the device code without a GPU.  The sources compile in
parallel: the C ABI (api.hip, and lap_solve.hip for the batched assignment
solve), the launch code of each precision mode
(ops_f64.hip, ops_f32d.hip, ops_f32n.hip) and the host-only branch and bound
(bnb.cpp); then one link.  Flags:
  -ffp-contract=off   no fused multiply-add contraction, so the element-wise
                      kernels perform exactly the IEEE operations written;
  -fno-honor-nans     (device code only) NaN never occurs in the state, so
                      min/max need no NaN canonicalisation;
  -packed-fp32-ops    disabled: no packed FP32 instructions are emitted.
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libqap_rlt2.so")
OBJDIR = os.path.join(HERE, "_build")
SOURCES = [os.path.join(CSRC, f) for f in ("api.hip", "lap_solve.hip", "ops_f64.hip", "ops_f32d.hip", "ops_f32n.hip", "bnb.cpp")]
HEADERS = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))] + [
    os.path.join(ROOT, "include", "qap_rlt2.h")]
ARCH = os.environ.get("QAP_OFFLOAD_ARCH", "gfx950")
NOISE = "is not a recognized feature for this target"


def hipcc():
    for cand in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def compile_command(src, obj):
    common = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    if src.endswith(".cpp"):   # host-only C++
        return [hipcc(), "-x", "c++"] + common + ["-c", "-o", obj, src]
    return [hipcc(), f"--offload-arch={ARCH}", "-ffp-contract=off", "-Xarch_device", "-fno-honor-nans",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + common + ["-c", "-o", obj, src]


def link_command(objs, out):
    return [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", out] + objs


def _clean(text):
    return "\n".join(l for l in (text or "").splitlines() if NOISE not in l)


def build(verbose=False):
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = []
    for src in SOURCES:
        obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
        cmd = compile_command(src, obj)
        if verbose:
            print(" ".join(cmd), flush=True)
        jobs.append((src, obj, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
    objs, errors = [], []
    for src, obj, proc in jobs:
        out, err = proc.communicate()
        err = _clean(err)
        if proc.returncode != 0:
            errors.append(f"{os.path.basename(src)}:\n{err}")
        elif verbose and err.strip():
            print(err)
        objs.append(obj)
    if errors:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errors))
    tmp = LIB + ".tmp"
    cmd = link_command(objs, tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + _clean(res.stderr))
    os.replace(tmp, LIB)
    return LIB


def needs_build():
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(s) > t for s in SOURCES + HEADERS)


if __name__ == "__main__":
    print(build(verbose=True))
