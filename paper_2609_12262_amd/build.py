"""Builds libpsb.so (HIP, gfx950) in-tree with hipcc."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libpsb.so")
REPLAY = os.path.join(HERE, "libpsb_replay.so")
SRCS = [os.path.join(HERE, "csrc", f) for f in ("psb_lib.hip", "psb_lane.hip", "psb_server.hip", "psb_tune.hip", "psb_window.hip", "psb_complementary.hip", "psb_slots.hip", "psb_stream.hip")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # never emit packed fp32 instructions (none of this code is floating point)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose: bool = False) -> str:
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = ["hipcc", *HIPCC_FLAGS, "-o", tmp, *SRCS]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stderr[-4000:])
    if verbose:
        print(r.stderr)
    os.replace(tmp, LIB)
    # load replay tool for the serving benchmark (links against libpsb.so)
    rtmp = REPLAY + f".tmp{os.getpid()}"
    cmd = ["hipcc", "-O2", "-std=c++17", "-fPIC", "-shared", "-o", rtmp,
           os.path.join(HERE, "csrc", "serve_replay.cpp"), "-L" + HERE, "-lpsb", "-Wl,-rpath,$ORIGIN", "-pthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc (replay tool) failed:\n" + r.stderr[-4000:])
    os.replace(rtmp, REPLAY)
    return LIB


if __name__ == "__main__":
    print(build(verbose=False))
