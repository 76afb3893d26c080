"""Build libhufield.so for gfx950 in-tree with hipcc.

Every .hip source under csrc/ is compiled to an object in parallel, then linked into
paper_2509_08675_amd/libhufield.so.  Run ``python -m paper_2509_08675_amd.build``.
"""

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libhufield.so")

ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         # packed FP32 instructions stay off: the compiler must not form v_pk_* FP32 ops
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # no automatic multiply-add contraction: a formula rounds the same way in every
         # instantiation (tile widths, batch layouts); the kernels write their fmaf explicitly
         "-ffp-contract=off",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found: the HIP library cannot be built")
    return exe


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src, verbose):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [hipcc()] + FLAGS + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed on %s:\n%s" % (src, r.stderr[-4000:]))
    if verbose:
        print("compiled", os.path.basename(src), flush=True)
    return obj


def build(verbose=False, jobs=None):
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, os.cpu_count() or 1), 8)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr[-4000:])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB, flush=True)
    return LIB


ASAN_DIR = os.path.join(BUILD, "host_asan")
ASAN_LIB = os.path.join(ASAN_DIR, "libhufield_host_asan.so")


def asan_runtime():
    """Path of the compiler's AddressSanitizer runtime (to preload into an uninstrumented python)."""
    r = subprocess.run([hipcc(), "--print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


def build_host_asan(verbose=False):
    """The library's host code only (argument validation, tables, layouts, plans), built with
    AddressSanitizer and UndefinedBehaviorSanitizer for the CPU tests of the C-ABI.  No device code
    is compiled: its kernels cannot run, which the host-only tests never need."""
    os.makedirs(ASAN_DIR, exist_ok=True)
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "--cuda-host-only",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
             "-ffp-contract=off", "-I", os.path.join(ROOT, "include"), "-I", CSRC]

    def one(src):
        obj = os.path.join(ASAN_DIR, os.path.basename(src) + ".o")
        r = subprocess.run([hipcc()] + flags + ["-c", src, "-o", obj], capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("hipcc (host sanitizer build) failed on %s:\n%s" % (src, r.stderr[-4000:]))
        return obj

    with cf.ThreadPoolExecutor(8) as ex:
        objs = list(ex.map(one, sources()))
    # the host-only objects name their device code as an external symbol: define it with the code
    # objects of the regular build (section .hip_fatbin of the same source's object)
    clang = os.path.join(os.path.dirname(os.path.realpath(hipcc())), "..", "llvm", "bin", "clang")
    if not os.path.exists(clang):
        clang = shutil.which("clang") or "/opt/rocm/llvm/bin/clang"
    for src, obj in zip(sources(), list(objs)):
        names = subprocess.run(["nm", obj], capture_output=True, text=True).stdout.split()
        sym = next((n for n in names if n.startswith("__hip_fatbin_") and n != "__hip_fatbin_wrapper"
                    and "." not in n and not n.endswith("_global")), None)
        if sym is None:
            continue
        reg = os.path.join(BUILD, os.path.basename(src) + ".o")
        if not os.path.exists(reg):
            raise RuntimeError("the regular build's %s is missing: run build() first" % reg)
        blob = os.path.join(ASAN_DIR, os.path.basename(src) + ".fatbin")
        subprocess.run(["objcopy", "--dump-section", ".hip_fatbin=" + blob, reg], check=True, capture_output=True)
        asm = os.path.join(ASAN_DIR, os.path.basename(src) + ".fatbin.s")
        with open(asm, "w") as fh:
            fh.write('  .section .hip_fatbin,"a",@progbits\n  .p2align 12\n  .globl %s\n%s:\n  .incbin "%s"\n'
                     % (sym, sym, blob))
        fo = asm + ".o"
        subprocess.run([clang, "-c", asm, "-o", fo], check=True, capture_output=True)
        objs.append(fo)
    r = subprocess.run([hipcc(), "-shared", "-fPIC", "-fsanitize=address", "-fsanitize=undefined", "-shared-libsan",
                        "-o", ASAN_LIB] + objs, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link (host sanitizer build) failed:\n" + r.stderr[-4000:])
    if verbose:
        print("built", ASAN_LIB, flush=True)
    return ASAN_LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
