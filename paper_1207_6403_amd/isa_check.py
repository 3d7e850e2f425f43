"""Development-tree check of the built gfx950 code objects: fail the build if the
compiler emitted any scalar-cache write (scalar stores, scalar atomics, scalar
cache write-back or discard).  Takes the object files of the build (one device
code bundle each).  Reads only code built here from source."""
import os
import re
import subprocess
import sys
import tempfile

LLVM = "/opt/rocm/llvm/bin"
BAD = re.compile(r"\b(s_store_\w+|s_buffer_store\w*|s_atomic_\w+|s_buffer_atomic_\w+|s_scratch_store\w*|"
                 r"s_dcache_wb\w*|s_dcache_discard\w*)\b")


def check(lib):
    heads = subprocess.run([os.path.join(LLVM, "llvm-objdump"), "-h", lib], stdout=subprocess.PIPE, text=True,
                           check=True).stdout
    if ".hip_fatbin" not in heads:
        return 0   # host code only
    with tempfile.TemporaryDirectory() as d:
        fat = os.path.join(d, "fatbin")
        subprocess.check_call([os.path.join(LLVM, "llvm-objcopy"), "--dump-section", ".hip_fatbin=" + fat, lib,
                               os.path.join(d, "copy.o")])
        co = os.path.join(d, "gfx950.co")
        subprocess.check_call([os.path.join(LLVM, "clang-offload-bundler"), "--unbundle", "--type=o",
                               "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", "--input=" + fat, "--output=" + co])
        dis = subprocess.run([os.path.join(LLVM, "llvm-objdump"), "-d", co], stdout=subprocess.PIPE, text=True,
                             check=True).stdout
    hits = sorted(set(BAD.findall(dis)))
    n = sum(1 for l in dis.splitlines() if l.startswith("\t") or l.startswith("  "))
    if hits:
        raise SystemExit("forbidden scalar-cache writes in %s: %s" % (lib, ", ".join(hits)))
    if n < 100:
        raise SystemExit("isa_check: disassembly of %s looks empty" % lib)
    return n


if __name__ == "__main__":
    print("isa_check ok: %s instructions" % ", ".join(
        "%s %d" % (os.path.basename(f), check(f)) for f in sys.argv[1:]))
