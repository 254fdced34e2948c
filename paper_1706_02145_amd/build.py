"""Build the HIP library libceles_amd.so in-tree (gfx950).

Compiles every translation unit with hipcc in parallel (one per multipole
cut-off for the coupling kernels) and links the shared library next to this
file.  Usage: python -m paper_1706_02145_amd.build [--lmax-compiled 6] [-j N]
"""
import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libceles_amd.so")
BUILD = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-mllvm", "-disable-machine-licm", "-fopenmp", "-Wno-unused-value", "-Wno-unused-result", "-I", os.path.join(HERE, "..", "include")]


def _run(cmd):
    p = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in (p.stderr or "").splitlines() if "packed-fp32-ops" not in l)
    if p.returncode != 0:
        raise RuntimeError("command failed: " + " ".join(cmd) + "\n" + err)
    return err


def build(lmax_compiled=6, jobs=None, verbose=False, force=False):
    """Compile (objects newer than their sources and headers are reused unless
    force=True) and link libceles_amd.so."""
    os.makedirs(BUILD, exist_ok=True)
    units = []
    for L in range(1, lmax_compiled + 1):
        units.append((os.path.join(CSRC, "wx_kernels.hip"), os.path.join(BUILD, f"wx_L{L}.o"), [f"-DCELES_WX_L={L}"]))
        units.append((os.path.join(CSRC, "wx_rtr.hip"), os.path.join(BUILD, f"wx_rtr_L{L}.o"), [f"-DCELES_WX_L={L}"]))
    for f in ("wx_mfma.hip", "wx_dispatch.hip", "vec_kernels.hip", "batch_kernels.hip", "precond.hip", "nn.hip", "farfield.hip", "nearfield.hip", "noalloc.hip",
              "host_math.cpp",
              "celes_lib.cpp"):
        units.append((os.path.join(CSRC, f), os.path.join(BUILD, os.path.splitext(f)[0] + ".o"), []))
    # the largest cut-offs take longest: start them first
    units.sort(key=lambda u: -int(u[2][0].split("=")[1]) if u[2] else 0)
    jobs = jobs or min(8, os.cpu_count() or 1)

    def deps(path, seen=None):
        # local #include "..." files, recursively
        seen = set() if seen is None else seen
        if path in seen or not os.path.exists(path):
            return seen
        seen.add(path)
        for line in open(path, encoding="utf-8", errors="replace"):
            line = line.strip()
            if line.startswith("#include \""):
                inc = os.path.normpath(os.path.join(os.path.dirname(path), line.split('"')[1]))
                deps(inc, seen)
        return seen

    def compile_one(u):
        src, obj, extra = u
        newest = max(os.path.getmtime(f) for f in deps(src) | {__file__})
        if not force and os.path.exists(obj) and os.path.getmtime(obj) >= newest:
            return ""
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        return _run([HIPCC] + COMMON + extra + lang + ["-c", src, "-o", obj])

    with cf.ThreadPoolExecutor(jobs) as ex:
        for u, msg in zip(units, ex.map(compile_one, units)):
            if verbose and msg.strip():
                print(msg, file=sys.stderr)
    objs = [u[1] for u in units]
    if lmax_compiled < 6:
        # provide empty launchers for the cut-offs that were not compiled
        stub = os.path.join(BUILD, "wx_stub.hip")
        with open(stub, "w") as f:
            f.write('#include "%s"\nnamespace celes {\n' % os.path.join(CSRC, "wx_launch.hpp"))
            for L in range(lmax_compiled + 1, 7):
                for T in ("double", "float"):
                    f.write(f"template <> void wx_run_L<{T}, {L}>(const WxArgs<{T}>&, int, int, hipStream_t) {{}}\n")
                    f.write(f"template <> void wx_rtr_run_L<{T}, {L}>(const WxArgs<{T}>&, int, int, hipStream_t) {{}}\n")
                    f.write(f"template <> void wx_rtr_batch_run_L<{T}, {L}>(const WxArgs<{T}>*, const int*, const int*, "
                            f"const int*, int, int*, int, int, hipStream_t) {{}}\n")
                f.write(f"template <> int wx_num_groups_L<{L}>() {{ return 1; }}\n")
                for T in ("double", "float"):
                    f.write(f"template <> int wx_max_kb_L<{T}, {L}>() {{ return 1; }}\n")
                    f.write(f"template <> void wx_batch_run_L<{T}, {L}>(const WxArgs<{T}>*, const int*, const int*, "
                            f"const int*, int, int*, int, int, int, hipStream_t) {{}}\n")
            f.write("}\n")
        _run([HIPCC] + COMMON + ["-c", stub, "-o", os.path.join(BUILD, "wx_stub.o")])
        objs.append(os.path.join(BUILD, "wx_stub.o"))
    tmp = OUT + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-fopenmp", "-o", tmp] + objs +
         ["-L/opt/rocm/lib", "-lrocsolver", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--lmax-compiled", type=int, default=int(os.environ.get("CELES_LMAX_COMPILED", "6")))
    ap.add_argument("-j", type=int, default=None)
    ap.add_argument("-v", action="store_true")
    ap.add_argument("--force", action="store_true")
    a = ap.parse_args()
    print(build(a.lmax_compiled, a.j, a.v, a.force))
