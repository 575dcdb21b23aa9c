"""Build the HIP library ``libapsp.so`` (gfx950) in the package directory.

Every call recompiles (no staleness check): ``python paper_1902_04446_amd/build.py``.
Run it as a file: importing the package itself loads the built library.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["apsp_plain.hip", "apsp_pair.hip", "apsp_runtime.hip", "apsp_batched.hip",
           "apsp_batch_plan.hip", "apsp_autotune.hip", "apsp_minplus.hip", "apsp_symmetric.hip",
           "apsp_api.hip"]
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


def _compile(sources, out, extra, verbose):
    srcs = [os.path.join(CSRC, s) for s in sources]
    tmp = out + ".tmp"
    cmd = [HIPCC, *FLAGS, *extra, *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed building {os.path.basename(out)}")
    os.replace(tmp, out)
    return out


def build(extra=(), out=LIB, verbose=False) -> str:
    _compile(PROBE_SOURCES, PROBE_LIB, extra, verbose)
    return _compile(SOURCES, out, extra, verbose)


if __name__ == "__main__":
    print(build(verbose=True))
