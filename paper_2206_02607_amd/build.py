"""Builds libcrom.so (the HIP kernels and the C interface in include/crom.h)
for gfx950 with hipcc, in place next to this file."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["csrc/step.hip", "csrc/decode.hip", "csrc/fd.hip", "csrc/train.hip", "csrc/sampling.hip", "csrc/stencil.hip", "csrc/guess.hip", "csrc/standardize.hip", "csrc/step_static.hip", "csrc/fallback.hip"]
LIB = os.path.join(HERE, "libcrom.so")
ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # keep the compiler from forming packed FP32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{os.path.join(ROOT, 'include')}",
]


# Host AddressSanitizer build of the library (CPU-side checking of the
# interface layer: argument validation, layouts, the stencil builder); the
# device code is built as usual.  Loaded with the sanitizer runtime
# preloaded, e.g. by tests/test_abi_asan.py.
ASAN_LIB = os.path.join(HERE, "libcrom_asan.so")
ASAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer", "-shared-libasan"]


def asan_runtime() -> str:
    """Path of the compiler's shared AddressSanitizer runtime."""
    r = subprocess.run([os.path.join(os.path.dirname(HIPCC), "amdclang++"),
                        "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if not os.path.isabs(path):
        raise RuntimeError("the AddressSanitizer runtime was not found")
    return path


def asan_runtime_dir() -> str:
    return os.path.dirname(asan_runtime())


def _compile(src: str, obj: str, extra=()) -> None:
    cmd = [HIPCC, *FLAGS, *extra, "-c", os.path.join(HERE, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")


def build(jobs: int = 4, asan: bool = False) -> str:
    out = os.path.join(ROOT, "_build", "asan" if asan else "")
    os.makedirs(out, exist_ok=True)
    objs = [os.path.join(out, os.path.basename(s).replace(".hip", ".o")) for s in SOURCES]
    extra = ASAN_FLAGS if asan else ()
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(lambda so: _compile(*so, extra), zip(SOURCES, objs)))
    lib = ASAN_LIB if asan else LIB
    tmp = lib + ".tmp"
    link_extra = ["-fsanitize=address", "-shared-libasan", f"-Wl,-rpath,{asan_runtime_dir()}"] if asan else []
    r = subprocess.run([HIPCC, f"--offload-arch={ARCH}", "-shared", *link_extra, "-o", tmp, *objs],
                       capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(asan="--asan" in sys.argv))
