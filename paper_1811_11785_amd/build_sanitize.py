"""Builds a host-sanitized variant of the library at
_build/asan/libsvdphat.so: the host code with AddressSanitizer and
UndefinedBehaviorSanitizer, the device code as usual.  It is for CPU runs
only (argument checks, the file parsers, error paths); load it with the
sanitizer runtime preloaded, e.g.

  LD_PRELOAD=$(ls /opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so) \
  ASAN_OPTIONS=detect_leaks=0 SVDPHAT_LIB=_build/asan/libsvdphat.so \
  python -m pytest tests -m "not gpu" -k "abi or persist"
"""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from paper_1811_11785_amd import build as b  # noqa: E402

# every sanitizer flag applies to the host compilation only
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]

if __name__ == "__main__":
    bdir = os.path.join(b.BUILD, "asan")
    b.build(verbose=True, out=os.path.join(bdir, "libsvdphat.so"), bdir=bdir, extra=HOST_SAN,
            link_extra=["-Xarch_host", "-shared-libsan"])
