"""Builds libsvdphat.so (HIP, gfx950) in place with hipcc."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libsvdphat.so")
BUILD = os.path.join(os.path.dirname(HERE), "_build")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

HIPFLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-Wno-unused-result",
]


def _compile(src: str, build_dir: str = BUILD, extra=()) -> str:
    obj = os.path.join(build_dir, os.path.basename(src) + ".o")
    cmd = [os.path.join(ROCM, "bin", "hipcc"), *HIPFLAGS, *extra, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False, out: str = OUT, bdir: str = BUILD, extra=(), link_extra=()) -> str:
    """Compiles every source and links the library (in place by default;
    `extra` hipcc flags for every step, `link_extra` for the link only)."""
    extra = list(extra)
    os.makedirs(bdir, exist_ok=True)
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, bdir, extra), srcs))
    tmp = out + ".tmp"
    cmd = [os.path.join(ROCM, "bin", "hipcc"), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs,
           *extra, f"-L{ROCM}/lib", "-lrocsolver", "-lrocblas", "-lamdhip64", f"-Wl,-rpath,{ROCM}/lib"]
    cmd += list(link_extra)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, out)
    if verbose:
        print("built", out)
    return out


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
