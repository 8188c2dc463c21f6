"""Build libfpm.so (HIP for gfx950 + host C++) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfpm.so")
SOURCES = ["kernels.hip", "mfma.hip", "stitch.hip", "plan.cpp", "runtime.cpp", "capi.cpp", "serve.cpp",
           "defocus.cpp"]
ARCH = os.environ.get("FPM_OFFLOAD_ARCH", "gfx950")


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every source with hipcc (objects in parallel) and link."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    common = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-ffp-contract=off",
              "-I" + os.path.join(HERE, "..", "include")]
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        objs.append(obj)
        cmd = ["hipcc", "-c"]
        if not src.endswith(".hip"):
            cmd += ["-x", "c++"]
        cmd += [os.path.join(CSRC, src), "-o", obj] + common
        if src.endswith(".hip"):
            # kernels.hip writes its fused multiply-adds out (its rounding is
            # then fixed by the source); the other kernels let the compiler fuse
            contract = "off" if src == "kernels.hip" else "fast"
            cmd += ["--offload-arch=" + ARCH, "-ffp-contract=" + contract,
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-mcode-object-version=5"]
        else:  # host-only translation units: plain C++ against the HIP headers
            cmd += ["-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            failed.append((src, out.decode(errors="replace")))
        elif verbose and out:
            sys.stderr.write(out.decode(errors="replace"))
    if failed:
        msg = "\n".join(f"--- {s}\n{o}" for s, o in failed)
        raise RuntimeError("libfpm build failed:\n" + msg)
    tmp = LIB + ".tmp%d" % os.getpid()
    link = ["hipcc", "-shared", "-o", tmp] + objs + ["--offload-arch=" + ARCH]
    subprocess.check_call(link)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
