"""Build the HIP library libkg.so in-tree for gfx950 with hipcc.

Flags: binary64 without FMA contraction (the variates must match the
reference bit for bit), packed fp32 instructions disabled."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libkg.so")
SOURCES = [os.path.join(HERE, "csrc", "kg_lib.hip")]
DEPS = SOURCES + [os.path.join(HERE, "csrc", f) for f in ("kg_device.hpp", "kg_kernels.hpp", "kg_tile.hpp", "kg_skip.hpp",
                                                                   "kg_rgg.hpp", "kg_rgg3.hpp", "kg_hash.hpp")] + \
    [os.path.join(ROOT, "include", "kg.h")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("KG_OFFLOAD_ARCH", "gfx950")

FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
         "-fno-fast-math", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall"]


def up_to_date():
    if not os.path.exists(LIB):
        return False
    t = os.path.getmtime(LIB)
    return all(os.path.getmtime(d) <= t for d in DEPS)


def build(force=True, verbose=False):
    if not force and up_to_date():
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + ["-o", tmp] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    out = r.stdout.decode(errors="replace")
    # hipcc's host pass does not know the packed-fp32 feature: harmless
    lines = [ln for ln in out.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
    if r.returncode != 0:
        sys.stderr.write("\n".join(lines) + "\n")
        raise RuntimeError("hipcc failed (%d)" % r.returncode)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True, verbose=True))
