"""Build the HIP library libtk.so in-tree for gfx950 with hipcc.

Every call recompiles.  Sources: csrc/tk_host.cpp (planner + C-ABI) and
csrc/tk_kernels.hip (device kernels); public header: include/tk.h.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libtk.so")
ARCH = os.environ.get("TK_OFFLOAD_ARCH", "gfx950")

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
COMMON = ["-O3", "-fPIC", "-std=c++17", f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]
# packed fp32 instructions are kept out of every device code object
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(ln for ln in r.stdout.splitlines() if "packed-fp32-ops" not in ln)
    if r.returncode != 0:
        raise RuntimeError(f"build failed: {' '.join(cmd)}\n{out}")
    if verbose and out.strip():
        print(out)


# host-side sanitizers for the planner (tk_host.cpp): every flag applies to
# the host compilation only, device code is built as usual
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host",
            "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
LIB_SANITIZED = os.path.join(HERE, "libtk_asan.so")


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """Compiles libtk.so; with sanitize=True, libtk_asan.so instead, whose
    planner is built with AddressSanitizer and UndefinedBehaviorSanitizer
    (load it with TK_LIBRARY=<path> and the sanitizer runtime preloaded, see
    the design doc)."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(BUILD, exist_ok=True)
    objs, cmds = [], []
    tag = ".asan" if sanitize else ""
    for src in ("tk_host.cpp", "tk_kernels.hip"):
        obj = os.path.join(BUILD, src + tag + ".o")
        cmd = [HIPCC] + COMMON + DEVICE + ["-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd = [HIPCC] + COMMON + ["-x", "hip"] + DEVICE + (SANITIZE + ["-g"] if sanitize else []) + \
                  ["-c", os.path.join(CSRC, src), "-o", obj]
        cmds.append(cmd)
        objs.append(obj)
    # the two translation units compile side by side
    with ThreadPoolExecutor(len(cmds)) as pool:
        for f in [pool.submit(_run, c, verbose) for c in cmds]:
            f.result()
    lib = LIB_SANITIZED if sanitize else LIB
    tmp = lib + ".tmp"
    _run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp] + objs + (SANITIZE if sanitize else []), verbose)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv))
