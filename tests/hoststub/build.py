"""Build the sanitizer driver: the library's host code, compiled without its
device code, linked with the HIP stand-in (hip_stub.cpp) and the driver.

    python tests/hoststub/build.py address|thread
    python tests/hoststub/build.py device OUTDIR

Writes _build/hoststub_<sanitizer>/driver (or OUTDIR/driver for the build
against the real runtime) and prints its path.  The sanitizer
instruments host code only (hipcc gets it through -Xarch_host; no device code
is built).
"""
import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
REPO = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(REPO, "paper_1702_02241_amd", "csrc")
INCLUDE = os.path.join(REPO, "include")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = os.environ.get("HOSTSTUB_CXX", "/opt/rocm/llvm/bin/clang++")
ROCM_INCLUDE = "/opt/rocm/include"


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("command failed: " + " ".join(cmd) + "\n" + res.stdout + res.stderr)


def build(sanitizer):
    assert sanitizer in ("address", "thread"), sanitizer
    san = "-fsanitize=" + sanitizer
    out = os.path.join(REPO, "_build", "hoststub_" + sanitizer)
    os.makedirs(out, exist_ok=True)
    srcs = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))

    def host_object(f):
        obj = os.path.join(out, f.replace(".hip", ".o"))
        _run([HIPCC, "-x", "hip", "--cuda-host-only", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
              "-fno-omit-frame-pointer", "-I", INCLUDE, "-Xarch_host", san, "-c", os.path.join(CSRC, f),
              "-o", obj])
        return obj

    with ThreadPoolExecutor(max_workers=8) as ex:
        objs = list(ex.map(host_object, srcs))
    # each host object names its translation unit's (absent) device image
    names = set()
    for o in objs:
        res = subprocess.run(["nm", "-u", o], capture_output=True, text=True, check=True)
        names.update(re.findall(r"\b(__hip_fatbin_[0-9a-f]+)\b", res.stdout))
    fatbins = os.path.join(out, "fatbins.cpp")
    with open(fatbins, "w") as fh:
        for nme in sorted(names):
            fh.write(f'extern "C" {{ char {nme}[16]; }}\n')
    cxx = [CLANG, "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer", san, "-D__HIP_PLATFORM_AMD__",
           "-I", ROCM_INCLUDE, "-I", INCLUDE]
    extra = []
    for src in ("hip_stub.cpp", "driver.cpp"):
        obj = os.path.join(out, src.replace(".cpp", ".o"))
        _run(cxx + ["-c", os.path.join(HERE, src), "-o", obj])
        extra.append(obj)
    fobj = os.path.join(out, "fatbins.o")
    _run(cxx + ["-c", fatbins, "-o", fobj])
    exe = os.path.join(out, "driver")
    _run([CLANG, san, "-rdynamic", "-o", exe, *objs, *extra, fobj, "-lpthread"])
    return exe


def build_device(out):
    """The same driver against the real HIP runtime: the library built whole
    (device code as in the product build), AddressSanitizer on its host side."""
    os.makedirs(out, exist_ok=True)
    srcs = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    san = "-fsanitize=address"

    def obj(f):
        o = os.path.join(out, f.replace(".hip", ".o"))
        _run([HIPCC, "--offload-arch=gfx950", "-O3", "-g", "-std=c++17", "-fno-omit-frame-pointer",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", INCLUDE,
              "-Xarch_host", san, "-c", os.path.join(CSRC, f), "-o", o])
        return o

    with ThreadPoolExecutor(max_workers=8) as ex:
        objs = list(ex.map(obj, srcs))
    drv = os.path.join(out, "driver.o")
    _run([CLANG, "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer", san, "-D__HIP_PLATFORM_AMD__",
          "-I", ROCM_INCLUDE, "-I", INCLUDE, "-c", os.path.join(HERE, "driver.cpp"), "-o", drv])
    exe = os.path.join(out, "driver")
    _run([CLANG, san, "-o", exe, *objs, drv, "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64",
          "-lpthread"])
    return exe


if __name__ == "__main__":
    if len(sys.argv) > 2 and sys.argv[1] == "device":
        print(build_device(sys.argv[2]))
    else:
        print(build(sys.argv[1] if len(sys.argv) > 1 else "address"))
