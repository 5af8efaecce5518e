"""Build libsmc.so (HIP kernels for gfx950 + host runtime) in-tree with hipcc.

Device code: -O3, -ffp-contract=off (the numeric contract forbids fused
multiply-adds the source does not spell out), packed-FP32 instructions off.
Host code: amdclang++ with the same contraction rule (it computes eqs. 3-4).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libsmc.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = os.environ.get("SMC_OFFLOAD_ARCH", "gfx950")

DEVICE_SOURCES = ["ssa_kernel.hip", "surrogate.hip"]
HOST_SOURCES = ["smc_api.cpp", "formula.cpp", "surrogate_api.cpp", "hull.cpp", "spec.cpp"]
# device headers the runtime compiler needs for specialised kernels
EMBEDDED = [("kEmbeddedDeviceHeader", "smc_device.h"), ("kEmbeddedCoreHeader", "ssa_core.h")]


def _embedded_source(path, csrc=CSRC):
    """C++ file defining the device headers as strings (raw literals)."""
    out = ["namespace smc {"]
    for sym, name in EMBEDDED:
        text = open(os.path.join(csrc, name)).read()
        assert ")SMCSRC\"" not in text
        out.append(f'extern const char {sym}[] = R"SMCSRC({text})SMCSRC";')
    out.append("}")
    with open(path, "w") as f:
        f.write("\n".join(out) + "\n")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose: bool = False, jobs: int = 4, out: str | None = None, defines=(), csrc: str = CSRC) -> str:
    """Compile and link the library (default: in-tree).  `csrc` selects another
    source directory with the same file names (e.g. a modified copy)."""
    hipcc = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
    clang = os.path.join(ROCM, "bin", "amdclang++")
    if not os.path.exists(clang):
        clang = os.path.join(ROCM, "llvm", "bin", "clang++")
    inc = ["-I", INCLUDE, "-I", csrc] + [f"-D{d}" for d in defines]
    lib_path = out or LIB
    tmp = tempfile.mkdtemp(prefix="smc_build_")
    try:
        procs, objs = [], []
        for src in DEVICE_SOURCES:
            obj = os.path.join(tmp, src + ".o")
            cmd = [hipcc, "-c", "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
                   "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                   "-Wno-unused-command-line-argument", *inc, os.path.join(csrc, src), "-o", obj]
            procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
            objs.append(obj)
        emb = os.path.join(tmp, "embedded_headers.cpp")
        _embedded_source(emb, csrc)
        for src in HOST_SOURCES + [emb]:
            obj = os.path.join(tmp, os.path.basename(src) + ".o")
            cmd = [clang, "-c", "-O2", "-std=c++17", "-fPIC", "-ffp-contract=off",
                   "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include"), *inc,
                   os.path.join(csrc, src), "-o", obj]
            procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
            objs.append(obj)
        failed = []
        for cmd, p in procs:
            out, _ = p.communicate()
            if verbose or p.returncode:
                print(out.decode(errors="replace"), flush=True)
            if p.returncode:
                failed.append(" ".join(cmd))
        if failed:
            raise RuntimeError("compilation failed:\n" + "\n".join(failed))
        out_tmp = lib_path + ".tmp%d" % os.getpid()
        _run([hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-L", os.path.join(ROCM, "lib"),
              "-lhiprtc", "-o", out_tmp], verbose)
        os.replace(out_tmp, lib_path)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return lib_path


if __name__ == "__main__":
    print(build(verbose=True))
