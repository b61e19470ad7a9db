"""Build the gfx950 shared libraries in-tree with hipcc.

* paper_1605_01020_amd/libiedg.so  -- the solver (csrc/*.hip, include/iedg.h)
* synth/libsynth.so                 -- the device-side input generator
"""
import concurrent.futures as cf
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1605_01020_amd")
BUILD = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-result"]

# Longest compiles first: they start at once on the worker pool.
IEDG_SOURCES = ["condense_f32.hip", "condense_bf16.hip", "condense_f32_single.hip", "condense_bf16_single.hip",
                "condense_f64.hip", "condense_f64_single.hip", "sparse.hip", "context.hip", "condense.hip",
                "mdf.hip", "ras.hip", "krylov.hip", "local.hip", "mr.hip", "probe.hip"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout)
    return r.stdout


def build_iedg(jobs=8):
    os.makedirs(BUILD, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc")]
    objs = []
    cmds = []
    for src in IEDG_SOURCES:
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        objs.append(obj)
        cmds.append([HIPCC] + COMMON + inc + ["-c", os.path.join(PKG, "csrc", src), "-o", obj])
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(_run, cmds))
    out = os.path.join(PKG, "libiedg.so")
    tmp = out + ".tmp"
    _run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp] + objs)
    os.replace(tmp, out)
    return out


def build_synth():
    os.makedirs(BUILD, exist_ok=True)
    src = os.path.join(ROOT, "synth", "csrc", "synth_gen.hip")
    out = os.path.join(ROOT, "synth", "libsynth.so")
    tmp = out + ".tmp"
    _run([HIPCC] + COMMON + ["-ffp-contract=off", "-shared", src, "-o", tmp])
    os.replace(tmp, out)
    return out


def build_all():
    with cf.ThreadPoolExecutor(max_workers=2) as ex:
        f1 = ex.submit(build_iedg)
        f2 = ex.submit(build_synth)
        return [f1.result(), f2.result()]


if __name__ == "__main__":
    for p in build_all():
        print(p)
