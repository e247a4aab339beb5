"""Build the ads HIP library (libads.so) for gfx950 with hipcc.

Usage: python -m paper_2201_02250_amd.build   (or build() from Python)
Every translation unit is compiled to an object in parallel (objects in a
scratch folder), then linked; the shared library is written next to this
file, in-tree."""
import concurrent.futures as cf
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libads.so")
SOURCES = ["ads_api.hip", "k_maps.hip", "k_extract.hip", "k_factor.hip", "k_eig.hip",
           "k_coarse.hip", "k_apply.hip", "k_krylov.hip", "k_gnn.hip", "tune.hip"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result", "-Wno-unused-command-line-argument"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed: " + " ".join(cmd[-3:]))


# host-code sanitizers (AddressSanitizer and UndefinedBehaviorSanitizer on
# the host pass only; the device code is built as usual)
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-sanitize-recover=undefined",
                 "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-O1"]


def build(verbose=False, jobs=None, sanitize=False, out=None):
    """Build libads.so in-tree; sanitize=True builds the host code with ASan
    and UBSan into out (for the host-sanitizer test), linked against the
    shared sanitizer runtimes."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = ["-I", os.path.join(HERE, "..", "include")]
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 1, 16)
    out = out or OUT
    extra = HOST_SANITIZE if sanitize else []
    with tempfile.TemporaryDirectory(prefix="ads_build_") as tmpd:
        objs = [os.path.join(tmpd, s.replace(".hip", ".o")) for s in SOURCES]
        cmds = [[hipcc, *FLAGS, *extra, *inc, "-c", os.path.join(CSRC, s), "-o", o]
                for s, o in zip(SOURCES, objs)]
        with cf.ThreadPoolExecutor(jobs) as ex:
            for f in [ex.submit(_run, c, verbose) for c in cmds]:
                f.result()
        tmp = out + ".tmp"
        if sanitize:
            # the objects carry their device code; the LLVM driver links them
            # with the HIP runtime and the shared sanitizer runtimes
            rocm = os.path.dirname(os.path.dirname(os.path.realpath(hipcc)))
            clangxx = os.path.join(rocm, "llvm", "bin", "clang++")
            rt = os.path.dirname(subprocess.run(
                [clangxx, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                text=True).stdout.strip())
            _run([clangxx, "-shared", "-fPIC", "-fsanitize=address,undefined", "-shared-libsan",
                  *objs, "-L" + os.path.join(rocm, "lib"), "-lamdhip64",
                  "-Wl,-rpath," + os.path.join(rocm, "lib"), "-Wl,-rpath," + rt, "-o", tmp], verbose)
        else:
            _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp], verbose)
        os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
