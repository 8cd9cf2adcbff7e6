"""Compiles the HIP library for gfx950 in-tree (``libhfz.so`` beside this file)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libhfz.so")
SOURCES = [os.path.join(HERE, "csrc", "hfz.hip"), os.path.join(HERE, "csrc", "hfz3.hip")]
DEPS = [os.path.join(HERE, "csrc", f) for f in os.listdir(os.path.join(HERE, "csrc"))]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed FP32 instructions (v_pk_add/mul/fma_f32) in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def build(verbose=False):
    """Compiles each source to an object in its own hipcc process (in
    parallel), then links the shared library."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = [os.path.join(HERE, os.path.basename(src) + ".o") for src in SOURCES]
    compile_flags = [f for f in FLAGS if f != "-shared"]
    procs = []
    for src, obj in zip(SOURCES, objs):
        cmd = [hipcc] + compile_flags + ["-c", "-I", os.path.join(ROOT, "include"), "-o", obj, src]
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
    errs, failed = [], False
    for p in procs:
        _, err = p.communicate()
        errs.append("\n".join(l for l in err.splitlines() if "packed-fp32-ops" not in l))
        failed |= p.returncode != 0
    err = "\n".join(e for e in errs if e.strip())
    if failed:
        raise RuntimeError("hipcc failed:\n" + err)
    res = subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs,
                         capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + res.stderr)
    for obj in objs:
        os.remove(obj)
    if verbose and err.strip():
        print(err)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
