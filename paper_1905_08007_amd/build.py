"""Build libqedamm.so (HIP for gfx950) in-tree.

Usage: python -m paper_1905_08007_amd.build   (or build() from Python)
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libqedamm.so")
SOURCES = ["host.cpp", "tables.cpp", "capi.cpp", "kernels.hip"]
ARCH = os.environ.get("QA_OFFLOAD_ARCH", "gfx950")


def _newest_header():
    hdrs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    hdrs.append(os.path.join(HERE, "..", "include", "qedamm.h"))
    return max(os.path.getmtime(h) for h in hdrs)


def build(verbose=False, jobs=8, incremental=False):
    """Compile and link the library.  incremental=True (development only) skips
    objects newer than their source and every header."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = []
    procs = []
    common = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-result"]
    newest_h = _newest_header() if incremental else None
    for src in SOURCES:
        obj = os.path.join(CSRC, "_build", src + ".o")
        os.makedirs(os.path.dirname(obj), exist_ok=True)
        path = os.path.join(CSRC, src)
        if incremental and os.path.exists(obj) and os.path.getmtime(obj) > max(os.path.getmtime(path), newest_h):
            objs.append(obj)
            continue
        if src.endswith(".hip"):
            cmd = [hipcc, "-x", "hip", f"--offload-arch={ARCH}", "-ffp-contract=fast-honor-pragmas",
                   "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                   "-munsafe-fp-atomics"] + common + ["-c", path, "-o", obj]
        else:
            cmd = ["g++", "-O3", "-fPIC", "-std=c++17", "-pthread", "-D__HIP_PLATFORM_AMD__",
                   "-I/opt/rocm/include", "-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    ok = True
    for src, p in procs:
        out = p.communicate()[0].decode()
        if p.returncode != 0:
            ok = False
            sys.stderr.write(f"--- {src}\n{out}\n")
        elif verbose and out.strip():
            sys.stderr.write(out)
    if not ok:
        raise RuntimeError("libqedamm build failed")
    tmp = LIB + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-pthread", "-o", tmp] + objs
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout.decode())
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="-i" in sys.argv))
