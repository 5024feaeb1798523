"""Builds the gfx950 library `_libgf.so` in-tree with hipcc."""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "_libgf.so")
SOURCES = [os.path.join(HERE, "csrc", name)
           for name in ("gf_host.cpp", "gf_server.cpp", "gf_kernels.hip", "gf_diag_kernels.hip",
                         "gf_noalloc.hip", "gf_fit.cpp")]
ARCH = "gfx950"

# Device code is built without packed FP32 instructions (the compiler would
# otherwise form them by itself), and with multiply-add contraction decided per
# source expression rather than by the backend: a point's arithmetic is then
# the same in every kernel that computes it (one-grid scan, serving launch),
# so results are reproducible bit for bit across them.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-ffp-contract=on"]


def build(verbose: bool = False, extra: list[str] | None = None, out: str | None = None) -> str:
    """Compiles every source (in parallel, one object each) and links them into
    one shared library; always recompiles."""
    out = out or LIB
    common = ["hipcc", "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-Wall",
              *DEVICE_FLAGS, *(extra or [])]
    with tempfile.TemporaryDirectory() as tmp:
        objs = [os.path.join(tmp, os.path.basename(src) + ".o") for src in SOURCES]
        cmds = [[*common, "-c", src, "-o", obj] for src, obj in zip(SOURCES, objs)]
        if verbose:
            for c in cmds:
                print(" ".join(c), flush=True)
        with concurrent.futures.ThreadPoolExecutor(len(cmds)) as pool:
            results = list(pool.map(lambda c: subprocess.run(c, capture_output=True, text=True), cmds))
        for r in results:
            if r.returncode != 0:
                raise RuntimeError(f"hipcc failed ({r.returncode}):\n{r.stderr}")
            if verbose and r.stderr.strip():
                print(r.stderr)
        link = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", out + ".tmp", *objs]
        if verbose:
            print(" ".join(link), flush=True)
        r = subprocess.run(link, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc link failed ({r.returncode}):\n{r.stderr}")
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
