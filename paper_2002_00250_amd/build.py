"""Build libfgs.so for gfx950 with hipcc (in-tree, no JIT cache).

    python -m paper_2002_00250_amd.build          # compile every source, link the library
    python -m paper_2002_00250_amd.build --resource-usage [FILE]   # the compiler's register,
                                                  # LDS, scratch and occupancy report of the
                                                  # step, serving and evaluation kernels (with
                                                  # FILE: written there as a summary)

Every HIP source is compiled with -ffp-contract=off (no multiply-add fusion: the
per-pixel recursions must round each operation separately), default IEEE
division and square root, and packed-FP32 instruction selection disabled.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libfgs.so")
SOURCES = ["gmm_kernels.hip", "gmm_window.hip", "pbas_kernels.hip", "pbas_grad_kernels.hip", "serve_kernels.hip", "diag_kernels.hip", "eval_kernels.hip", "postfilter_kernels.hip", "static_kernels.hip",
           "runtime.cpp", "server.cpp"]
ARCH = os.environ.get("FGS_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP toolchain is required to build libfgs")


def common_flags():
    return ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-ffp-contract=off",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", f"-I{INCLUDE}", f"-I{CSRC}"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    lang = ["-x", "hip"]
    cmd = [hipcc()] + common_flags() + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking libfgs.so failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


# Kernels whose resources the report lists: (source, mangled-name fragment, readable name).
REPORT_KERNELS = [
    ("gmm_kernels.hip", "gmm_step_kernelILi8ELi5ELi5ELb1ELb0ELi1E", "gmm_step_kernel<8,5,5,NT,0,1>"),
    ("gmm_kernels.hip", "gmm_step_kernelILi1ELi5ELi5ELb1ELb0ELi1E", "gmm_step_kernel<1,5,5,NT,0,1>"),
    ("gmm_kernels.hip", "gmm_step_kernelILi8ELi7ELi3ELb1ELb0ELi1E", "gmm_step_kernel<8,7,3,NT,0,1>"),
    ("pbas_kernels.hip", "pbas_step_kernelILi8ELi36ELb1E", "pbas_step_kernel<8,36,NT>"),
    ("pbas_kernels.hip", "pbas_step_kernelILi1ELi20ELb0E", "pbas_step_kernel<1,20,cached>"),
    ("serve_kernels.hip", "serve_kernelILi5ELi24ELb0E", "serve_kernel<5,24,cached>"),
    ("serve_kernels.hip", "serve_kernelILi5ELi24ELb1E", "serve_kernel<5,24,NT>"),
    ("eval_kernels.hip", "eval_count_kernel", "eval_count_kernel"),
    ("postfilter_kernels.hip", "median_mask_kernelILi4ELi16E", "median_mask_kernel<4,16>"),
]
FIELDS = ["VGPRs", "AGPRs", "TotalSGPRs", "ScratchSize [bytes/lane]", "Occupancy [waves/SIMD]",
          "LDS Size [bytes/block]", "VGPRs Spill", "SGPRs Spill"]


def resource_usage() -> str:
    """The compiler's resource-usage remarks (-Rpass-analysis=kernel-resource-usage) for the
    kernels in REPORT_KERNELS, compiled with the library's own flags, as a text table."""
    import re
    import tempfile
    out = {}
    with tempfile.TemporaryDirectory() as td:
        for src in sorted({k[0] for k in REPORT_KERNELS}):
            cmd = [hipcc()] + common_flags() + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o",
                                                os.path.join(td, "x.o"), "-Rpass-analysis=kernel-resource-usage"]
            r = subprocess.run(cmd, capture_output=True, text=True)
            if r.returncode != 0:
                raise RuntimeError(f"compiling {src} failed:\n{r.stderr}")
            cur = None
            for line in r.stderr.splitlines():
                m = re.search(r"remark:\s+Function Name: (\S+)", line)
                if m:
                    cur = m.group(1)
                    out.setdefault(cur, {})
                    continue
                m = re.search(r"remark:\s+([^:]+): (\S+) \[-Rpass", line)
                if m and cur:
                    out[cur][m.group(1).strip()] = m.group(2)
    rows = ["kernel | " + " | ".join(FIELDS)]
    for src, frag, name in REPORT_KERNELS:
        hits = [k for k in out if frag in k]
        if not hits:
            raise RuntimeError(f"no remarks for {name} ({frag}) in {src}")
        f = out[hits[0]]
        rows.append(name + " | " + " | ".join(f.get(x, "?") for x in FIELDS))
    return "\n".join(rows)


def resource_report() -> str:
    """resource_usage() as a summary: the sources it covers with their hash, the compiler
    version and the command."""
    import hashlib
    heads = ["device_common.h", "fgs_internal.h", "gmm_device.h", "pbas_device.h", "postfilter.h"]
    paths = [os.path.join("paper_2002_00250_amd", "csrc", s) for s in sorted({k[0] for k in REPORT_KERNELS}) + heads]
    h = hashlib.sha256()
    for p in paths:
        h.update(open(os.path.join(ROOT, p), "rb").read())
    ver = subprocess.run([hipcc(), "--version"], capture_output=True, text=True).stdout.splitlines()
    ver = "; ".join(v.strip() for v in ver if "HIP version" in v or "clang version" in v)
    return "\n".join([
        "# Compiler resource usage of the step, serving, evaluation and median kernels (gfx950)", "",
        "sources: " + " ".join(paths),
        "sources_sha256_16: " + h.hexdigest()[:16],
        "compiler: " + ver, "",
        "The compiler's -Rpass-analysis=kernel-resource-usage remarks, with the library's own flags",
        "(-O3, -ffp-contract=off, packed-FP32 selection off).  Occupancy is waves per SIMD as the",
        "compiler bounds it from VGPRs, SGPRs and LDS (the hardware maximum is 8).", "",
        resource_usage(), "",
        "command:",
        "  python -m paper_2002_00250_amd.build --resource-usage profiles/compiler_resources_gfx950.txt", ""])


if __name__ == "__main__":
    if "--resource-usage" in sys.argv[1:]:
        rest = [a for a in sys.argv[1:] if a != "--resource-usage"]
        if rest:
            with open(rest[0], "w") as fh:
                fh.write(resource_report())
        else:
            print(resource_usage())
    else:
        build()
    sys.exit(0)
