"""Build libbrillouin.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1701_00726_amd.build

Every HIP source under csrc/ is compiled for gfx950 with packed-FP32
instructions disabled, then linked into one shared library next to this file.
"""

from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbrillouin.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    "-O3",
    "-std=c++17",
    "-fPIC",
    f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


# host code instrumented with AddressSanitizer and UndefinedBehaviorSanitizer (CPU checks of the
# argument validation, planning and host bookkeeping); -Xarch_host keeps the sanitizer off the
# device pass (the CPU job launches no kernel)
SANITIZE_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer",
                  "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-sanitize-recover=undefined"]


def build(verbose: bool = False, jobs: int = 8, sanitize_to: str | None = None) -> str:
    """Compile every csrc/*.hip for gfx950 and link libbrillouin.so next to this file; with
    sanitize_to, link a copy whose host code is sanitized at that path instead."""
    srcs = sources()
    flags = [f for f in FLAGS if f != "-O3"] + SANITIZE_FLAGS if sanitize_to else FLAGS
    out_lib = sanitize_to or LIB
    tmpdir = tempfile.mkdtemp(prefix="bri_build_")
    try:
        objs, procs = [], []
        for src in srcs:
            obj = os.path.join(tmpdir, os.path.basename(src) + ".o")
            cmd = [HIPCC, *flags, "-c", src, "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
            objs.append(obj)
            running = [p for _, p in procs if p.poll() is None]
            if len(running) >= jobs:
                running[0].wait()  # at most `jobs` compilers at a time
        failed = []
        for src, p in procs:
            out, _ = p.communicate()
            text = out.decode(errors="replace")
            # hipcc's host pass does not know the packed-fp32 feature; that warning is harmless
            lines = [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
            if p.returncode != 0:
                failed.append((src, text))
            elif verbose and lines:
                print("\n".join(lines))
        if failed:
            for src, text in failed:
                sys.stderr.write(f"--- hipcc failed on {src}\n{text}\n")
            raise RuntimeError("HIP build failed")
        tmp_lib = os.path.join(tmpdir, "libbrillouin.so")
        link = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp_lib, *objs]
        if sanitize_to:
            link += ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-shared-libsan"]
        subprocess.check_call(link)
        shutil.copyfile(tmp_lib, out_lib + ".tmp")
        os.replace(out_lib + ".tmp", out_lib)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    return out_lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
