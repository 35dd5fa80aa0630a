"""Builds libfdd.so (HIP kernels for gfx950 + host orchestration + C ABI) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libfdd.so")

SOURCES = ["kernels_mg.hip", "kernels_iface.hip", "kernels_batch.hip", "kernels_cnn.hip", "kernels_3d.hip",
           "kernels_full.hip", "kernels_model.hip", "ra_build.cpp", "api.cpp", "api_batch.cpp", "api_cnn.cpp", "api_3d.cpp",
           "api_full.cpp", "api_model.cpp", "kernels_hdiv.hip", "hdiv_setup.cpp", "api_hdiv.cpp",
           "ell_host.cpp", "ell_mg.cpp", "kernels_ds.hip", "ds_setup.cpp", "api_ds.cpp"]

# Packed FP32 instructions are disabled in device code (see the project notes on gfx950).
HIP_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose=False, jobs=4):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    common = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-I", os.path.join(ROOT, "include"),
              "-I", SRC, "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        objs.append(obj)
        lang = ["-x", "hip"] if src.endswith(".hip") else ["-x", "hip"]
        cmd = [hipcc] + common + HIP_FLAGS + lang + ["-c", os.path.join(SRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = False
    for src, p in procs:
        out, _ = p.communicate()
        text = "\n".join(l for l in out.decode(errors="replace").splitlines()
                         if "packed-fp32-ops" not in l and "is not a recognized feature" not in l)
        if p.returncode != 0:
            failed = True
            sys.stderr.write(f"--- {src} failed ---\n{text}\n")
        elif verbose and text.strip():
            sys.stderr.write(text + "\n")
    if failed:
        raise RuntimeError("libfdd build failed")
    tmp = OUT + ".tmp"
    cmd = [hipcc, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    subprocess.check_call(cmd)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
