"""Builds libgg.so (the HIP library behind include/gg.h) in-tree for gfx950.

Usage: python -m paper_2511_10353_amd.build   (or build() from Python).
Every .hip file under csrc/ is compiled with hipcc into _build/, in parallel,
and linked into paper_2511_10353_amd/libgg.so; probe/issue_probe.hip becomes the
stand-alone issue-rate probe paper_2511_10353_amd/probe/issue_probe.
"""
import concurrent.futures
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libgg.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

ARCH = "gfx950"
CFLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-ffp-contract=fast-honor-pragmas",
    # packed FP32 instructions are kept out of the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{os.path.join(ROOT, 'include')}",
]


def _compile(src, build_dir=BUILD, defines=()):
    obj = os.path.join(build_dir, os.path.basename(src) + ".o")
    cmd = [HIPCC, *CFLAGS, *[f"-D{d}" for d in defines], "-c", src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{res.stdout}\n{res.stderr}")
    return obj


def build(verbose=True, lib=LIB, build_dir=BUILD, defines=()):
    """Compile and link; ``defines`` are extra -D macros (tuning variants)."""
    os.makedirs(build_dir, exist_ok=True)
    sources = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    if not sources:
        raise RuntimeError("no HIP sources found")
    jobs = min(len(sources), int(os.environ.get("MAX_JOBS", "8")))
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, build_dir, defines), sources))
    tmp = lib + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs,
           "-Wl,-rpath,/opt/rocm/lib"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print(f"built {lib} from {len(sources)} sources", flush=True)
    if lib == LIB:
        build_probe(verbose)
    return lib


PROBE_SRC = os.path.join(PKG, "probe", "issue_probe.hip")
PROBE = os.path.join(PKG, "probe", "issue_probe")


def build_probe(verbose=True):
    """The issue-rate probe (probe/issue_probe.hip), a stand-alone program
    that measures the throughput of single vector-ALU instruction classes."""
    tmp = PROBE + ".tmp"
    res = subprocess.run([HIPCC, *CFLAGS, PROBE_SRC, "-o", tmp], capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {PROBE_SRC}:\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, PROBE)
    if verbose:
        print(f"built {PROBE}", flush=True)
    return PROBE


def build_host_sanitized(build_dir=os.path.join(ROOT, "_build_san")):
    """libgg with its host code (gg_api.hip: validation, plans, dispatch)
    built under AddressSanitizer and UndefinedBehaviorSanitizer; the device
    code is built as usual (GPU sanitizers are not used).  The kernel-only
    sources are taken from the regular build.  Returns the library's path;
    load it with the clang ASan runtime preloaded (see
    tests/test_abi_sanitized.py)."""
    os.makedirs(build_dir, exist_ok=True)
    if not all(os.path.exists(os.path.join(BUILD, os.path.basename(s) + ".o"))
               for s in glob.glob(os.path.join(CSRC, "*.hip"))):
        build(verbose=False)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
    api = os.path.join(CSRC, "gg_api.hip")
    obj = os.path.join(build_dir, "gg_api.hip.o")
    flags = [f for f in CFLAGS if f != "-O3"] + ["-O1", "-g"]
    res = subprocess.run([HIPCC, *flags, *san, "-c", api, "-o", obj], capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc (host sanitizers) failed:\n{res.stdout}\n{res.stderr}")
    objs = [obj] + [os.path.join(BUILD, os.path.basename(s) + ".o")
                    for s in sorted(glob.glob(os.path.join(CSRC, "*.hip"))) if os.path.basename(s) != "gg_api.hip"]
    lib = os.path.join(build_dir, "libgg_san.so")
    res = subprocess.run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", lib, *objs, *san, "-shared-libasan",
                          "-Wl,-rpath,/opt/rocm/lib"], capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link (host sanitizers) failed:\n{res.stdout}\n{res.stderr}")
    return lib


if __name__ == "__main__":
    build()
    sys.exit(0)
