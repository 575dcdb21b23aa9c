"""Build the HIP library ``libapsp.so`` (gfx950) in the package directory.

Every call recompiles (no staleness check): ``python paper_1902_04446_amd/build.py``.
Run it as a file: importing the package itself loads the built library.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["apsp_plain.hip", "apsp_pair.hip", "apsp_small.hip", "apsp_runtime.hip", "apsp_batched.hip",
           "apsp_batch_plan.hip", "apsp_autotune.hip", "apsp_minplus.hip", "apsp_symmetric.hip",
           "apsp_copy.hip", "apsp_api.hip"]
LIB = os.path.join(HERE, "libapsp.so")
# diagnostic: VALU issue-rate probe used by the benchmark to state its ceiling
PROBE_SOURCES = ["valu_probe.hip"]
PROBE_LIB = os.path.join(HERE, "libapsp_probe.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # no packed fp32 instructions anywhere
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-command-line-argument",
]


def _run(cmd, verbose, what):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed building {what}")


def _compile(sources, out, extra, verbose):
    """Compile each source to an object in parallel (each translation unit
    launches only its own kernels), then link the shared library."""
    from concurrent.futures import ThreadPoolExecutor

    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    flags = [f for f in FLAGS if f != "-shared"]
    objs = []
    jobs = []
    for src in sources:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        jobs.append(([HIPCC, *flags, *extra, "-c", os.path.join(CSRC, src), "-o", obj], src))
    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with ThreadPoolExecutor(workers) as pool:
        for f in [pool.submit(_run, cmd, verbose, what) for cmd, what in jobs]:
            f.result()
    tmp = out + ".tmp"
    _run([HIPCC, *FLAGS, *extra, *objs, "-o", tmp], verbose, os.path.basename(out))
    os.replace(tmp, out)
    return out


def build(extra=(), out=LIB, verbose=False) -> str:
    _compile(PROBE_SOURCES, PROBE_LIB, extra, verbose)
    return _compile(SOURCES, out, extra, verbose)


if __name__ == "__main__":
    print(build(verbose=True))
