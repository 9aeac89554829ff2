"""Builds libshapegrad.so (the C-ABI library) from csrc/ with hipcc for gfx950.

    python -m paper_2311_05646_amd.build
    python -m paper_2311_05646_amd.build --sanitize address|thread   (host code instrumented, CPU runs)
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libshapegrad.so")
SOURCES = ["sg_api.hip", "sg_kernels.hip", "sg_serve.hip", "sg_mode_eps.hip", "sg_mode_vjp.hip", "sg_mode_geps.hip",
           "sg_mode_fd.hip", "sg_mode_sparse.hip", "sg_mode_fdsparse.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-munsafe-fp-atomics",
    # never let the compiler form packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-variable", "-Wno-unused-function", "-pthread",
]


def build(verbose=False, jobs=None):
    """Compiles every translation unit (in parallel: the column kernel's modes
    are separate units) and links the shared library."""
    import concurrent.futures
    import tempfile
    tmp = LIB + ".tmp"
    with tempfile.TemporaryDirectory(prefix="sg_build_") as od:
        objs = [os.path.join(od, os.path.splitext(s)[0] + ".o") for s in SOURCES]
        cmds = [[HIPCC] + FLAGS + ["-c", os.path.join(CSRC, s), "-o", o] for s, o in zip(SOURCES, objs)]
        jobs = jobs or min(len(cmds), max(1, os.cpu_count() or 1))
        with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
            for cmd, r in zip(cmds, ex.map(lambda c: subprocess.run(c, capture_output=True, text=True), cmds)):
                if verbose:
                    print(" ".join(cmd), flush=True)
                if r.returncode != 0:
                    sys.stderr.write(r.stdout + r.stderr)
                    raise RuntimeError("hipcc failed building libshapegrad.so")
        link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread"] + objs + ["-o", tmp]
        if verbose:
            print(" ".join(link), flush=True)
        r = subprocess.run(link, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("linking libshapegrad.so failed")
    os.replace(tmp, LIB)
    return LIB


SANITIZERS = {"address": "asan", "thread": "tsan"}
SAN_DIR = os.path.join(os.path.dirname(HERE), "_build")     # sanitizer builds (not part of the package)


def sanitizer_runtime(kind):
    """Path of the compiler's shared sanitizer runtime (to preload into a
    Python that loads the instrumented library)."""
    clang = os.path.join(os.path.dirname(os.path.realpath(HIPCC)), "..", "llvm", "bin", "clang")
    out = subprocess.run([clang, f"-print-file-name=libclang_rt.{SANITIZERS[kind]}-x86_64.so"], capture_output=True,
                         text=True).stdout.strip()
    return out


def build_host_sanitized(kind, out_dir=None, verbose=False):
    """A build whose host code is instrumented with AddressSanitizer or
    ThreadSanitizer (device code at -O1, uninstrumented), for running the C++
    runtime on the CPU: the C-ABI argument checks and the serving scheduler
    with its fake executor.  Returns the library's path."""
    import concurrent.futures
    import tempfile
    tag = SANITIZERS[kind]
    out_dir = out_dir or SAN_DIR
    os.makedirs(out_dir, exist_ok=True)
    lib = os.path.join(out_dir, f"libshapegrad_{tag}.so")
    san = ["-Xarch_host", "-fsanitize=" + kind, "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-pthread",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-result"] + san
    with tempfile.TemporaryDirectory(prefix="sg_san_") as od:
        objs = [os.path.join(od, os.path.splitext(s)[0] + ".o") for s in SOURCES]
        cmds = [[HIPCC] + flags + ["-c", os.path.join(CSRC, s), "-o", o] for s, o in zip(SOURCES, objs)]
        with concurrent.futures.ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 1)) as ex:
            for cmd, r in zip(cmds, ex.map(lambda c: subprocess.run(c, capture_output=True, text=True), cmds)):
                if verbose:
                    print(" ".join(cmd), flush=True)
                if r.returncode != 0:
                    sys.stderr.write(r.stdout + r.stderr)
                    raise RuntimeError(f"hipcc failed building the {kind}-sanitized library")
        link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread",
                "-shared-libsan"] + san + objs + ["-o", lib]
        r = subprocess.run(link, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError(f"linking the {kind}-sanitized library failed")
    return lib


if __name__ == "__main__":
    if len(sys.argv) > 2 and sys.argv[1] == "--sanitize":
        print(build_host_sanitized(sys.argv[2], verbose=True))
    else:
        print(build(verbose=True))
