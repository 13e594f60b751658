"""Build the HIP library libjk.so for gfx950, in-tree.

Steps: generate the per-class recurrences (csrc/gen_eri.py -> eri_gen.inc,
eri_cost.inc, eri_counts.json); compile the per-class kernels (one
translation unit per canonical class, in parallel), the small kernels and the
host side of the C-ABI; link one shared library next to this file.  The
compiler's per-kernel resource report (VGPRs, AGPRs, scratch, occupancy) is
kept in _build/resource_usage.txt.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libjk.so")
OBJ = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
NCLASS = 21
HOST_SOURCES = ["jk_host", "jk_laplace", "jk_remez", "jk_cd"]
DEVICE_SOURCES = ["jk_kernels", "jk_gemm", "jk_cd"]

# no packed FP32 instructions anywhere in device code
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-variable", "-Wno-unused-but-set-variable",
          f"-I{INCLUDE}", f"-I{CSRC}"]


def generate() -> None:
    subprocess.check_call([sys.executable, os.path.join(CSRC, "gen_eri.py"),
                           os.path.join(CSRC, "eri_gen.inc"),
                           "--counts", os.path.join(CSRC, "eri_counts.json"),
                           "--cost", os.path.join(CSRC, "eri_cost.inc")],
                          stdout=subprocess.DEVNULL)


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + r.stdout)
    return r.stdout


def build(verbose: bool = False, jobs: int | None = None) -> str:
    generate()
    os.makedirs(OBJ, exist_ok=True)
    dev = [HIPCC, f"--offload-arch={ARCH}", *COMMON, *DEVICE_FLAGS, "-Rpass-analysis=kernel-resource-usage"]
    steps = []
    for n in range(NCLASS):
        steps.append(dev + [f"-DJK_CLASS_INDEX={n}", "-c", os.path.join(CSRC, "jk_class.hip"),
                            "-o", os.path.join(OBJ, f"jk_class_{n}.o")])
    for src in DEVICE_SOURCES:
        steps.append(dev + ["-c", os.path.join(CSRC, src + ".hip"), "-o", os.path.join(OBJ, src + "_dev.o")])
    for host in HOST_SOURCES:
        steps.append([HIPCC, *COMMON, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-x", "c++", "-c",
                      os.path.join(CSRC, host + ".cpp"), "-o", os.path.join(OBJ, host + ".o")])
    jobs = jobs or min(16, os.cpu_count() or 4)
    with ThreadPoolExecutor(jobs) as ex:
        logs = list(ex.map(_run, steps))
    with open(os.path.join(OBJ, "resource_usage.txt"), "w") as fh:
        for lg in logs:
            fh.write("\n".join(l for l in lg.splitlines() if "remark" in l) + "\n")
    summarize_resources(os.path.join(OBJ, "resource_usage.txt"), os.path.join(OBJ, "resource_summary.txt"))
    objs = [os.path.join(OBJ, f"jk_class_{n}.o") for n in range(NCLASS)]
    objs += [os.path.join(OBJ, src + "_dev.o") for src in DEVICE_SOURCES]
    objs += [os.path.join(OBJ, host + ".o") for host in HOST_SOURCES]
    tmp = LIB + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def summarize_resources(src: str, dst: str) -> list:
    """One line per kernel: VGPRs, AGPRs, spills, scratch, occupancy."""
    import re
    rows, cur = [], None
    keys = {"VGPRs": "vgpr", "AGPRs": "agpr", "VGPRs Spill": "spill",
            "ScratchSize [bytes/lane]": "scratch", "Occupancy [waves/SIMD]": "occ",
            "LDS Size [bytes/block]": "lds"}
    with open(src) as fh:
        for line in fh:
            m = re.search(r"Function Name: (\S+)", line)
            if m:
                cur = {"name": m.group(1)}
                rows.append(cur)
                continue
            m = re.search(r"remark:\s+([A-Za-z ]+(?:\[[^\]]*\])?):\s+(\d+)", line)
            if m and cur is not None and m.group(1).strip() in keys:
                cur[keys[m.group(1).strip()]] = int(m.group(2))
    with open(dst, "w") as fh:
        fh.write("%-58s %5s %5s %6s %7s %3s\n" % ("kernel", "vgpr", "agpr", "spill", "scratch", "occ"))
        for r in rows:
            fh.write("%-58s %5s %5s %6s %7s %3s\n" % (r["name"][:58], r.get("vgpr"), r.get("agpr"),
                                                     r.get("spill"), r.get("scratch"), r.get("occ")))
    return rows


if __name__ == "__main__":
    build(verbose=True)
