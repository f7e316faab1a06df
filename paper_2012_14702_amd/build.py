"""Builds libipt.so (the HIP library behind include/ipt.h) for gfx950 with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libipt.so")
SOURCES = ["ipt_api.hip", "ipt_setup.hip", "ipt_gemm.hip", "ipt_spmm.hip", "ipt_batched.hip", "ipt_mlp.hip",
           "ipt_acx.hip", "ipt_pairs.hip", "ipt_complex.hip", "ipt_zcsr.hip", "ipt_rs.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
         # packed FP32 instructions are kept out of every kernel
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(jobs: int = 4) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        objs.append(obj)
        cmd = [HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _wait(procs.pop(0))
    for p in procs:
        _wait(p)
    tmp = LIB + ".tmp"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


# Host sanitizer variant: the library's host code (argument checks, workspace layout,
# sweep loops, polling) built with the address and undefined-behaviour sanitizers, the
# kernels as above, and a driver that calls every entry point through the C ABI.
SAN = ["-g", "-fno-omit-frame-pointer", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined"]
SAN_DIR = os.path.join(HERE, "_build_hostsan")
SAN_LIB = os.path.join(SAN_DIR, "libipt_hostsan.so")
SAN_DRIVER = os.path.join(SAN_DIR, "abi_sanitize_driver")
DRIVER_SRC = os.path.join(os.path.dirname(HERE), "tests", "abi_sanitize_driver.cpp")


def build_hostsan(jobs: int = 4) -> str:
    os.makedirs(SAN_DIR, exist_ok=True)
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(SAN_DIR, src.replace(".hip", ".o"))
        objs.append(obj)
        cmd = [HIPCC] + FLAGS + SAN + ["-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _wait(procs.pop(0))
    for p in procs:
        _wait(p)
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", SAN_LIB + ".tmp"] + SAN + objs)
    os.replace(SAN_LIB + ".tmp", SAN_LIB)
    include = os.path.join(os.path.dirname(HERE), "include")
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-std=c++17", "-O1"] + SAN +
                          ["-I", include, DRIVER_SRC, "-o", SAN_DRIVER + ".tmp", "-L", SAN_DIR, "-lipt_hostsan",
                           "-Wl,-rpath," + SAN_DIR])
    os.replace(SAN_DRIVER + ".tmp", SAN_DRIVER)
    return SAN_DRIVER


def _wait(item):
    src, p = item
    out, _ = p.communicate()
    text = out.decode(errors="replace")
    lines = [l for l in text.splitlines() if "packed-fp32-ops" not in l]
    if p.returncode != 0:
        sys.stderr.write("\n".join(lines) + "\n")
        raise RuntimeError("hipcc failed on " + src)
    if any("warning" in l for l in lines):
        sys.stderr.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    print(build())
    if len(sys.argv) > 1 and sys.argv[1] == "hostsan":
        print(build_hostsan())
