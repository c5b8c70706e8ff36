"""Build the solver's shared library (HIP for gfx950 + host C++) in-tree."""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libbddmma.so")
# (source, object name, extra defines); sweep_reg.hip is built once per
# (precision, direction, update) so its unrolled kernels compile in parallel
UNITS = [("kernels.hip", "kernels", []), ("problem.cpp", "problem", []), ("capi.cpp", "capi", []), ("pool.cpp", "pool", []),
         ("assemble.hip", "assemble", []), ("serial.hip", "serial", []),
         ("termination.hip", "termination", []), ("static_workspace.hip", "static_workspace", []),
         ("stream_probe.hip", "stream_probe", [])] + [
    ("persist.hip", f"persist_{t}", [f"-DBDDMMA_PERSIST_T={t}"]) for t in ("float", "double")] + [
    ("sweep_reg.hip", f"sweep_reg_{t}_{d}_{u}",
     [f"-DBDDMMA_REG_T={t}", f"-DBDDMMA_REG_DIR={d}", f"-DBDDMMA_REG_UPD={u}"])
    for t in ("float", "double") for d in (0, 1) for u in ("true", "false")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-I", CSRC, "-I", INCLUDE]


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every source (always; the call is the build check) and link libbddmma.so."""
    from concurrent.futures import ThreadPoolExecutor

    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    cmds, objs = [], []
    for src, name, defs in UNITS:
        obj = os.path.join(objdir, name + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmds.append([HIPCC] + FLAGS + defs + lang + ["-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, stderr=subprocess.PIPE, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stderr}")
        return r.stderr

    jobs = jobs or min(len(cmds), max(1, min(8, os.cpu_count() or 1)))
    with ThreadPoolExecutor(jobs) as ex:
        for err in ex.map(run, cmds):
            if verbose and err:
                print(err, flush=True)
    tmp = LIB + ".tmp"
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs +
                   ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"], check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
