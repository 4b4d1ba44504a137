"""Build libddlpb.so for gfx950 with hipcc (in-tree, next to this file)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libddlpb.so")
SOURCES = [os.path.join(CSRC, f) for f in
           ("ddlpb.hip", "near_lane.hip", "m2l_lane_yf.hip", "m2l_lane_yt.hip", "m2l_lane_lf.hip", "m2l_lane_lt.hip",
            "m2l_lane_yf32.hip", "m2l_lane_yt32.hip",
            "level_lane_ym2m.hip", "level_lane_yl2l.hip", "level_lane_ym2mT.hip", "level_lane_yl2lT.hip",
            "level_lane_ym2m32.hip", "level_lane_yl2l32.hip", "level_lane_ym2mT32.hip", "level_lane_yl2lT32.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-Wno-unused-result", "-pthread"]


def build(verbose: bool = False) -> str:
    """Compile every source to an object (in parallel: the order-12 translation kernels
    take minutes each) and link the shared library next to this file."""
    if os.path.exists(os.path.join(CSRC, "gen_lebedev.py")) and not os.path.exists(
            os.path.join(CSRC, "lebedev_data.h")):
        subprocess.run([sys.executable, os.path.join(CSRC, "gen_lebedev.py")], check=True)
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(os.path.basename(src))[0] + ".o")
        objs.append(obj)
        procs.append((src, subprocess.Popen([HIPCC] + FLAGS + ["-c", "-o", obj, src], stdout=subprocess.PIPE,
                                            stderr=subprocess.STDOUT, text=True)))
    errors = []
    for src, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            errors.append(f"{src}:\n{out}")
        elif verbose:
            print(out)
    if errors:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errors))
    tmp = LIB + ".tmp"
    cmd = [HIPCC] + FLAGS + ["-shared", "-o", tmp] + objs
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
