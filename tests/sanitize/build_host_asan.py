"""Build tests/bin/rift_host_asan: the library's host code (rift_ile.hip)
compiled with AddressSanitizer and UndefinedBehaviorSanitizer on the host
side only (the device code is built as usual), linked with the kernel
objects of the normal build and the driver tests/sanitize/host_driver.cpp.
Needs the normal build's objects (paper_2210_07912_amd.build.build()).

    python tests/sanitize/build_host_asan.py
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(ROOT, "tests", "bin", "rift_host_asan")


def build(verbose=False):
    sys.path.insert(0, ROOT)
    from paper_2210_07912_amd import build as b
    hipcc = b._hipcc()
    bdir = os.path.join(ROOT, "_build")
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    host_obj = os.path.join(bdir, "rift_ile_asan.o")
    drv_obj = os.path.join(bdir, "host_driver_asan.o")
    cmds = [
        [hipcc, "-O1", "-g", "-std=c++17", "-fPIC", f"--offload-arch={b.ARCH}", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), *san, "-c",
         os.path.join(ROOT, "paper_2210_07912_amd", "csrc", "rift_ile.hip"), "-o", host_obj],
        [hipcc, "-O1", "-g", "-std=c++17", f"--offload-arch={b.ARCH}", "-I", os.path.join(ROOT, "include"), *san,
         "-x", "hip", "-c", os.path.join(HERE, "host_driver.cpp"), "-o", drv_obj],
    ]
    kern = [os.path.join(bdir, os.path.splitext(s)[0] + ".o") for s in b.SOURCES if s != "rift_ile.hip"]
    link = [hipcc, f"--offload-arch={b.ARCH}", *san, host_obj, drv_obj, *kern, "-L/opt/rocm/lib", "-lhipfft",
            "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib", "-o", OUT]
    for c in cmds + [link]:
        r = subprocess.run(c, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("host sanitizer build failed:\n" + " ".join(c) + "\n" + r.stdout + r.stderr)
    if verbose:
        print(f"built {OUT}")
    return OUT


if __name__ == "__main__":
    build(verbose=True)
