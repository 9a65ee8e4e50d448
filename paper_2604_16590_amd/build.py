"""Build the gfx950 libraries in-tree with hipcc.

liblinattn.so  -- the attention library behind include/la.h
liblagen.so    -- the synthetic-input generator behind include/la_gen.h
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
ARCH = os.environ.get("LA_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed FP32 instructions are disabled for all device code.
COMMON = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-result"]

# liblagen.so first: liblinattn.so links it (the serving loop generates
# inputs for requests that ask for them).
LIBS = {
    "liblagen.so": ["gen.hip"],
    "liblinattn.so": ["la_api.cpp", "la_forward.hip", "la_backward.hip", "la_serve.cpp",
                      "la_profile.cpp", "la_tiles.hip", "la_probe.hip", "la_noalloc.hip", "la_tiled.hip"],
}


# The input generator follows a definition written as separate FP32
# operations (mirrored on the host with numpy); fusing a product and a sum
# into one rounding would move its grid phase by up to half an ulp of a
# ~70-valued intermediate, so contraction is off for that file.
PER_FILE = {"gen.hip": ["-ffp-contract=off"]}


def _compile(src: str) -> str:
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    lang = ["-x", "hip"] if src.endswith(".cpp") else []
    cmd = [HIPCC] + COMMON + PER_FILE.get(src, []) + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stderr))
    return obj


def build(verbose: bool = False) -> dict:
    os.makedirs(OBJ, exist_ok=True)
    srcs = sorted({s for v in LIBS.values() for s in v if os.path.exists(os.path.join(CSRC, s))})
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = dict(zip(srcs, ex.map(_compile, srcs)))
    out = {}
    for lib, parts in LIBS.items():
        present = [objs[p] for p in parts if p in objs]
        path = os.path.join(HERE, lib)
        tmp = path + ".tmp%d" % os.getpid()
        cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + present
        if lib == "liblinattn.so":
            cmd += ["-L" + HERE, "-llagen", "-Wl,-rpath,$ORIGIN", "-lpthread"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("link failed for %s:\n%s" % (lib, r.stderr))
        os.replace(tmp, path)
        out[lib] = path
        if verbose:
            print("built", path)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
