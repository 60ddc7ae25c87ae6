"""Build libcpm.so (HIP kernels + C ABI) in-tree for gfx950 with hipcc."""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "libcpm.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

SOURCES = ["cpm_sweep.hip", "cpm_sweep_inst.hip", "cpm_serial.hip", "cpm_kernels.hip", "cpm_stats.hip",
           "emu_kernels.hip", "cpm_api.cpp", "emu_api.cpp"]
# the activation kernels are instantiated in groups, one compilation each
SWEEP_PARTS = 7
HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES]


def units():
    """(source, extra flags, object) of every compilation."""
    out = []
    for src in sources():
        base = os.path.join(OUT_DIR, os.path.basename(src))
        if src.endswith("cpm_sweep_inst.hip"):
            out += [(src, [f"-DCPM_SWEEP_PART={i}"], f"{base}.{i}.o") for i in range(SWEEP_PARTS)]
        else:
            out.append((src, [], base + ".o"))
    return out


def build(verbose: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    jobs = []
    for src, extra, obj in units():
        cmd = ["hipcc", *HIPCC_FLAGS, *extra, "-I", INCLUDE, "-I", CSRC, "-x", "hip", "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd))
        jobs.append((cmd, obj))
    # one compiler process per compilation, at most eight at a time
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 4)) as pool:
        for f in [pool.submit(subprocess.run, cmd, check=True) for cmd, _ in jobs]:
            f.result()
    objs = [obj for _, obj in jobs]
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = sources() + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))]
    deps += [os.path.join(INCLUDE, f) for f in os.listdir(INCLUDE) if f.endswith(".h")]
    return any(os.path.getmtime(d) > t for d in deps)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
