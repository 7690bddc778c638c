"""Build the CPU emulation of libekm (the test-only host build of the
library's own kernel sources, see hip/hip_runtime.h) with AddressSanitizer.

The sources under paper_2412_02244_amd/csrc are copied unchanged except for
two mechanical rewrites the shim header cannot express:
  * ``extern __shared__ T name[];`` (dynamic LDS) becomes a pointer to the
    launch's dynamic shared buffer;
  * the relative include of include/ekm.h points at the repository's
    include directory.
"""

from __future__ import annotations

import hashlib
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2412_02244_amd", "csrc")
CXX = os.environ.get("EMU_CXX", "/opt/rocm/llvm/bin/clang++")
# -O0: a wave operation's call site is identified by its return address, and
# an optimiser may duplicate code so that one source-level operation gets
# two addresses (reported as a divergent wave operation that is not one).
FLAGS = ["-std=c++17", "-O0", "-g", "-fsanitize=address", "-fno-omit-frame-pointer", "-ffp-contract=off",
         "-Wno-unknown-pragmas", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-parameter",
         "-Wno-pass-failed"]

_DYN = re.compile(r"extern\s+__shared__\s+([A-Za-z_][\w\s]*?)\s+(\w+)\s*\[\s*\]\s*;")


def rewrite(src: str) -> str:
    src = _DYN.sub(lambda m: f"{m.group(1)} *{m.group(2)} = ({m.group(1)} *)emu::dyn_shared();", src)
    return src.replace('#include "../../include/ekm.h"', '#include "ekm.h"')


def sources() -> list[str]:
    return sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".hpp")))


def build(out_dir: str) -> str:
    os.makedirs(out_dir, exist_ok=True)
    h = hashlib.sha256()
    for name in sources() + ["hip/hip_runtime.h", "emu_runtime.cpp", "driver.cpp"]:
        path = os.path.join(CSRC, name) if name in sources() else os.path.join(HERE, name)
        h.update(name.encode())
        h.update(open(path, "rb").read())
    h.update(" ".join([CXX] + FLAGS).encode())
    exe = os.path.join(out_dir, "driver_" + h.hexdigest()[:16])
    if os.path.exists(exe):
        return exe
    src_dir = os.path.join(out_dir, "src")
    os.makedirs(src_dir, exist_ok=True)
    units = []
    for name in sources():
        text = rewrite(open(os.path.join(CSRC, name)).read())
        dst = os.path.join(src_dir, name.replace(".hip", ".cpp"))
        with open(dst, "w") as f:
            f.write(text)
        if name.endswith(".hip"):
            units.append(dst)
    units += [os.path.join(HERE, "emu_runtime.cpp"), os.path.join(HERE, "driver.cpp")]
    inc = ["-I", HERE, "-I", os.path.join(ROOT, "include"), "-I", src_dir]
    objs = []
    procs = []
    for u in units:
        obj = os.path.join(out_dir, os.path.basename(u) + ".o")
        procs.append(subprocess.Popen([CXX, *FLAGS, *inc, "-c", u, "-o", obj], stdout=subprocess.PIPE,
                                      stderr=subprocess.STDOUT, text=True))
        objs.append(obj)
    errs = []
    for p, u in zip(procs, units):
        out, _ = p.communicate()
        if p.returncode != 0:
            errs.append(f"{u}:\n{out}")
    if errs:
        raise RuntimeError("cpu emulation build failed:\n" + "\n".join(errs))
    tmp = exe + ".tmp"
    r = subprocess.run([CXX, "-fsanitize=address", "-o", tmp, *objs], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("cpu emulation link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, exe)
    return exe


if __name__ == "__main__":
    print(build(sys.argv[1] if len(sys.argv) > 1 else os.path.join(ROOT, "_work", "emu")))
