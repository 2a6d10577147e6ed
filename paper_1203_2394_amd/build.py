"""Build libdpf.so for gfx950 with hipcc (in-tree, next to this file).

The library is several translation units (the C entry points, and one per
built-in model holding that model's step kernels); they compile in parallel
and are linked into one shared library.
"""
import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdpf.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["dpf_lib.hip", "dpf_eng_lingauss.hip", "dpf_eng_nonlin.hip", "dpf_eng_highdim.hip",
           "dpf_eng_twodim.hip", "dpf_eng_fourdim.hip", "dpf_eng_twodimz.hip", "dpf_data.hip"]
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed-FP32 instructions (v_pk_*_f32) in generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose: bool = False, jobs: int = 0) -> str:
    jobs = jobs or min(len(SOURCES), max(1, os.cpu_count() or 1))
    tmpdir = tempfile.mkdtemp(prefix="dpf_build_")
    try:
        objs, pending = [], []
        for s in SOURCES:
            obj = os.path.join(tmpdir, os.path.splitext(s)[0] + ".o")
            objs.append(obj)
            cmd = [HIPCC] + FLAGS + ["-c", "-o", obj, os.path.join(CSRC, s)]
            if verbose:
                print(" ".join(cmd), flush=True)
            pending.append(cmd)
        running = []
        failed = []
        while pending or running:
            while pending and len(running) < jobs:
                cmd = pending.pop(0)
                running.append((cmd, subprocess.Popen(cmd, cwd=CSRC, stdout=subprocess.PIPE,
                                                      stderr=subprocess.STDOUT, text=True)))
            cmd, proc = running.pop(0)
            out, _ = proc.communicate()
            if proc.returncode != 0:
                failed.append((cmd[-1], out))
        if failed:
            for name, out in failed:
                sys.stderr.write("== %s\n%s\n" % (name, out))
            raise RuntimeError("hipcc failed building libdpf.so")
        tmp = LIB + ".tmp%d" % os.getpid()
        link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
        if verbose:
            print(" ".join(link), flush=True)
        res = subprocess.run(link, cwd=CSRC, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("hipcc failed linking libdpf.so")
        os.replace(tmp, LIB)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
