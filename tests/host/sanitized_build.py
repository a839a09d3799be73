"""Host builds for the CPU test suite, with the address and
undefined-behaviour sanitizers on the host code:

* rules_check  -- the scalar rules header (csrc/rules.h) under g++;
* abi_check    -- the whole library, host parts instrumented (device code
  compiled as usual but never run), linked into tests/host/abi_check.cpp,
  which drives the C ABI in a planning context on a machine without a GPU.

Objects are cached under _build/sanitized/<hash of sources and flags>.
"""

from __future__ import annotations

import hashlib
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
PKG = os.path.join(ROOT, "paper_2601_16734_amd")
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
CACHE = os.path.join(ROOT, "_build", "sanitized")
ROCM = "/opt/rocm"

# host-side instrumentation only: each sanitizer flag is scoped to the host
# pass, the device pass is the library's usual gfx950 build at -O1
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
HIP_FLAGS = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", "-Wno-unused-result", "-Wno-unused-value", "-I", INCLUDE, "-I", CSRC]
LINK_SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def _sources():
    import importlib.util
    spec = importlib.util.spec_from_file_location("_smps_build", os.path.join(PKG, "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return list(mod.SOURCES)


def _digest(paths, flags) -> str:
    h = hashlib.sha256(" ".join(flags).encode())
    for p in sorted(paths):
        with open(p, "rb") as f:
            h.update(os.path.basename(p).encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def build_rules_check(out: str) -> str:
    cxx = shutil.which("g++")
    if cxx is None:
        raise RuntimeError("no host C++ compiler")
    cmd = [cxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", CSRC, "-I", INCLUDE, os.path.join(HERE, "rules_check.cpp"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(r.stderr)
    return out


def build_abi_check() -> str:
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    clang = os.path.join(ROCM, "lib", "llvm", "bin", "clang++")
    srcs = [os.path.join(CSRC, s) for s in _sources()]
    headers = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    headers.append(os.path.join(INCLUDE, "seemps_hip.h"))
    driver = os.path.join(HERE, "abi_check.cpp")
    key = _digest(srcs + headers + [driver], HIP_FLAGS + HOST_SAN + LINK_SAN)
    out_dir = os.path.join(CACHE, key)
    exe = os.path.join(out_dir, "abi_check")
    if os.path.exists(exe):
        return exe
    os.makedirs(out_dir, exist_ok=True)

    def compile_one(src):
        obj = os.path.join(out_dir, os.path.basename(src) + ".o")
        r = subprocess.run([hipcc, *HIP_FLAGS, *HOST_SAN, "-c", src, "-o", obj], capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"{src}:\n{r.stderr}")
        return obj

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, srcs))
    drv = os.path.join(out_dir, "abi_check.o")
    r = subprocess.run([clang, "-O1", "-g", "-std=c++17", *LINK_SAN, "-I", INCLUDE, "-c", driver, "-o", drv],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(r.stderr)
    tmp = exe + ".tmp"
    r = subprocess.run([clang, "--hip-link", "--offload-arch=gfx950", *LINK_SAN, drv, *objs,
                        "-L", os.path.join(ROCM, "lib"), "-lamdhip64", f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}",
                        "-o", tmp], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(r.stderr)
    os.replace(tmp, exe)
    return exe


def run_abi_check(exe: str, script: str, timeout: float = 600.0) -> list[str]:
    env = {**os.environ, "ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0:exitcode=23",
           "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1:exitcode=24"}
    r = subprocess.run([exe], input=script, capture_output=True, text=True, timeout=timeout, env=env)
    if r.returncode != 0:
        raise AssertionError(f"abi_check exited {r.returncode}\n{r.stderr[-6000:]}")
    return r.stdout.splitlines()
