"""Compile the CPU oracle (plain C, gcc) into oracle/liboracle.so.

Flags: no fused multiply-add contraction and no fast-math, so the *_f32 build
rounds every operation to binary32 and the *_f64 build to binary64.
"""
import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
CFLAGS = ["-O2", "-std=c99", "-fPIC", "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
          "-Wno-unused-parameter"]


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB):
        return LIB
    with tempfile.TemporaryDirectory() as tmp:
        objs = []
        units = [("tracker.c", ["-DORACLE_F32"], "tracker_f32.o"),
                 ("tracker.c", [], "tracker_f64.o"),
                 ("links.c", [], "links.o"),
                 ("refit_mixed.c", [], "refit_mixed.o"),
                 ("select.c", [], "select.o"),
                 ("fullfit.c", ["-DORACLE_F32"], "fullfit_f32.o"),
                 ("fullfit.c", [], "fullfit_f64.o"),
                 ("merge.c", [], "merge.o")]
        for src, defs, obj in units:
            o = os.path.join(tmp, obj)
            subprocess.run(["gcc", *CFLAGS, *defs, "-c", os.path.join(HERE, src), "-o", o], check=True)
            objs.append(o)
        out = LIB + ".tmp"
        subprocess.run(["gcc", "-shared", *objs, "-o", out, "-lm"], check=True)
        os.replace(out, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
