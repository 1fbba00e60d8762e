"""Build libtc.so (HIP for gfx950) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libtc.so")
SOURCES = ["tc_api.hip", "tc_scan.hip", "tc_csr.hip", "tc_sample.hip", "tc_count.hip", "tc_rp.hip", "tc_tune.hip", "tc_serve.hip", "tc_triple.hip", "tc_noalloc.hip", "tc_stream.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result"]


def build(jobs=8, verbose=False):
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        objs.append(obj)
        cmd = [HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        text = "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l)
        if p.returncode != 0:
            failed.append((src, text))
        elif verbose and text.strip():
            print(text)
    if failed:
        for src, text in failed:
            sys.stderr.write("---- %s ----\n%s\n" % (src, text))
        raise RuntimeError("hipcc failed for " + ", ".join(s for s, _ in failed))
    tmp = OUT + ".tmp"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, OUT)
    build_torch_alloc()
    return OUT


TORCH_ALLOC = os.path.join(HERE, "libtc_torch_alloc.so")


def build_torch_alloc():
    """The allocator shim (host code): tc_torch_alloc / tc_torch_free over
    PyTorch's caching allocator, installed by the binding with tc_set_allocator."""
    import torch
    tdir = os.path.dirname(torch.__file__)
    tmp = TORCH_ALLOC + ".tmp"
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(HIPCC)))
    subprocess.check_call([HIPCC, "-O2", "-std=c++17", "-fPIC", "-shared", "-x", "c++", "-D__HIP_PLATFORM_AMD__",
                           "-I" + os.path.join(tdir, "include"), "-I" + os.path.join(rocm, "include"),
                           os.path.join(CSRC, "torch_alloc.cpp"),
                           "-L" + os.path.join(tdir, "lib"), "-lc10_hip", "-lc10",
                           "-Wl,-rpath," + os.path.join(tdir, "lib"), "-o", tmp])
    os.replace(tmp, TORCH_ALLOC)
    return TORCH_ALLOC


if __name__ == "__main__":
    print(build(verbose=True))
