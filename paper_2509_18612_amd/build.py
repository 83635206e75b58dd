"""Build the gfx950 HIP library libdeco.so in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = [os.path.join(HERE, "csrc", f)
           for f in ("kernels.hip", "step_momentum.hip", "step_wide.hip", "step_wide_momentum.hip", "resident.hip",
                     "api.hip", "mpnn.hip")]
LIB = os.path.join(HERE, "libdeco.so")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-munsafe-fp-atomics",
    # keep the compiler from forming packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    """Compile every source to an object in parallel (one hipcc each), then link."""
    from concurrent.futures import ThreadPoolExecutor
    tmp = out + f".tmp{os.getpid()}"
    objs = [f"{tmp}.{os.path.basename(src)}.o" for src in SOURCES]
    cflags = [f for f in FLAGS if f != "-shared"]

    def compile_one(src_obj):
        src, obj = src_obj
        cmd = ["hipcc", *cflags, *[f"-D{d}" for d in defines], "-I", os.path.join(ROOT, "include"), "-c",
               "-o", obj, src]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if verbose:
            print(" ".join(cmd))
        return res, cmd

    try:
        with ThreadPoolExecutor(len(SOURCES)) as ex:
            for res, cmd in ex.map(compile_one, zip(SOURCES, objs)):
                if res.returncode != 0:
                    raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + res.stdout + res.stderr)
        cmd = ["hipcc", *FLAGS, "-o", tmp, *objs]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError("hipcc link failed:\n" + res.stdout + res.stderr)
        if verbose:
            print(" ".join(cmd))
        os.replace(tmp, out)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
