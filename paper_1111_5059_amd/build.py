"""Build libdwf.so (HIP for gfx950) in-tree with hipcc.

Every translation unit under csrc/ is compiled in parallel, then linked into
paper_1111_5059_amd/libdwf.so.  Run as ``python -m paper_1111_5059_amd.build``.
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libdwf.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# Packed-FP32 instructions are disabled: hipcc would otherwise pair FP32 work into
# v_pk_* forms.
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result", "-I", os.path.join(HERE, "..", "include")]


# the hop kernels are compiled once per compile-time fifth-dimension extent
HOP_LS = (0, 8, 12, 16, 32)


def sources():
    units = []
    for f in sorted(os.listdir(CSRC)):
        if not f.endswith((".hip", ".cpp")):
            continue
        if f.startswith("hop_"):
            units += [(f, f"-DDWF_HOP_LS={ls}") for ls in HOP_LS]
        units.append((f, None))
    return units


def _up_to_date(obj):
    """The object exists and is newer than every file its dependency list (-MMD) names."""
    dep = obj + ".d"
    if not (os.path.exists(obj) and os.path.exists(dep)):
        return False
    with open(dep) as fh:
        text = fh.read().replace("\\\n", " ")
    files = text.split(":", 1)[1].split() if ":" in text else []
    t = os.path.getmtime(obj)
    return bool(files) and all(os.path.exists(f) and os.path.getmtime(f) < t for f in files)


def _compile(unit, incremental=False):
    src, define = unit
    tag = "" if define is None else "." + define.split("=")[1]
    obj = os.path.join(OBJ, src + tag + ".o")
    if incremental and _up_to_date(obj):
        return src, obj, 0, ""
    extra = [] if define is None else [define]
    cmd = [HIPCC] + FLAGS + extra + ["-MMD", "-MF", obj + ".d", "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    return src, obj, r.returncode, r.stdout + r.stderr


def build(verbose=False, jobs=None, incremental=False):
    """Compile every translation unit and link libdwf.so.  incremental=True (development only)
    skips units whose object is newer than every file it depends on."""
    os.makedirs(OBJ, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 4)))
    objs = []
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        for src, obj, rc, out in ex.map(lambda u: _compile(u, incremental), srcs):
            if rc != 0:
                sys.stderr.write(out)
                raise RuntimeError(f"hipcc failed on {src}")
            if verbose and out.strip():
                sys.stderr.write(out)
            objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link of libdwf.so failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="--incremental" in sys.argv))
