"""Build libwl.so (the HIP library behind include/wl.h) for gfx950, in-tree."""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")

SOURCES = ["wl_kernels.hip", "wl_api.hip", "wl_server.hip", "wl_thermo.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # every a*b+c in the walk must round twice, as the definition prescribes
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def write_tune_header() -> str:
    """csrc/wl_tune_table.h from tune_table.json (the autotuner's table)."""
    from paper_1302_2320_amd import autotune
    path = os.path.join(CSRC, "wl_tune_table.h")
    text = autotune.c_header(autotune.load_table())
    old = open(path).read() if os.path.exists(path) else None
    if old != text:
        with open(path, "w") as f:
            f.write(text)
    return path


def build(verbose: bool = False) -> str:
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    write_tune_header()
    out = os.path.join(PKG, "libwl.so")
    cmd = ["hipcc", *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           *[os.path.join(CSRC, s) for s in SOURCES], "-o", out + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
