"""Builds and runs the CPU build of the decoder engine (engine_host.cpp) for
tests: g++ with the address and undefined-behaviour sanitizers and the
invariant checks, one shot at a time through the engine's single-lane code."""
import os
import subprocess
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "engine_host.cpp")
CSRC = os.path.join(os.path.dirname(os.path.dirname(HERE)), "paper_2609_12262_amd", "csrc")


def build(out_dir, sanitize=True, nb_table=False):
    exe = os.path.join(out_dir, "engine_host" + ("_nb" if nb_table else ""))
    cmd = ["g++", "-std=c++17", "-g", "-Wall", "-Wno-unknown-pragmas", "-DPSB_CHECK_INVARIANTS", "-o", exe, SRC]
    cmd[2:2] = (["-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]
                if sanitize else ["-O2"])
    if nb_table:
        cmd.insert(2, "-DPSB_NB_TABLE=1")
    subprocess.check_call(cmd)
    return exe


def run(exe, g, syndromes, seed=0x5EED, mode=0, reading=0, caps=(1024, 768, 512), force_hash=False, log=None,
        direct1=True, walk=False):
    """Decodes every row of `syndromes`; returns dict of arrays (status, n_edges, weight, obs, stats, edges).
    `log`: file name that receives the program's standard error; `walk`: the clustering search walks its
    paths at every level (else levels of at most two edges read the ball tables)."""
    with tempfile.TemporaryDirectory() as d:
        with open(os.path.join(d, "graph.bin"), "wb") as f:
            f.write(np.int32(g.num_detectors).tobytes()); f.write(np.int64(g.num_edges).tobytes())
            for a, t in ((g.u, np.int32), (g.v, np.int32), (g.w, np.int32), (g.obs_mask, np.uint64)):
                f.write(np.ascontiguousarray(a, t).tobytes())
        with open(os.path.join(d, "synd.bin"), "wb") as f:
            f.write(np.int64(syndromes.shape[0]).tobytes()); f.write(np.int32(syndromes.shape[1]).tobytes())
            f.write(np.ascontiguousarray(syndromes, np.uint8).tobytes())
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        r = subprocess.run([exe, d, str(seed), str(mode), str(reading), *[str(x) for x in caps],
                            "1" if force_hash else "0", "1" if direct1 else "0", "1" if walk else "0"],
                           capture_output=True, text=True,
                           env=env)
        if log:
            with open(log, "w") as fh:
                fh.write(r.stderr)
        if r.returncode != 0:
            raise RuntimeError(f"engine_host exited {r.returncode}:\n{r.stderr[-6000:]}")
        raw = open(os.path.join(d, "out.bin"), "rb").read()
    stride = int(np.frombuffer(raw[:4], np.int32)[0])
    rec = np.dtype([("status", np.int32), ("n_edges", np.int32), ("weight", np.int64), ("obs", np.uint64),
                    ("stats", np.int32, 12), ("edges", np.int32, stride)])
    a = np.frombuffer(raw[4:], rec)
    return {k: a[k].copy() for k in ("status", "n_edges", "weight", "obs", "stats", "edges")}
