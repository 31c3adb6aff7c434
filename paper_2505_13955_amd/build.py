"""Build libxct.so (all HIP sources, gfx950) next to this file.

    python -m paper_2505_13955_amd.build
"""

from __future__ import annotations

import glob
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libxct.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def sources() -> list[str]:
    return sorted(glob.glob(os.path.join(_HERE, "csrc", "*.hip")))


# The packed-FP32 feature switch is a device-code option, but hipcc hands
# -Xclang options to the host pass as well (-Xarch_device cannot carry them),
# and the x86 host target reports it does not know the feature.  That one
# message is dropped from the build output; everything else is shown.
_HOST_FEATURE_NOTE = "'-packed-fp32-ops' is not a recognized feature for this target"


def build(verbose: bool = False, extra: list[str] | None = None) -> str:
    tmp = LIB_PATH + ".tmp"
    cmd = [HIPCC, *FLAGS, *(extra or []), "-o", tmp, *sources()]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(line for line in r.stdout.splitlines() if _HOST_FEATURE_NOTE not in line)
    if out.strip():
        print(out, flush=True)
    if r.returncode != 0:
        raise subprocess.CalledProcessError(r.returncode, cmd, output=out)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose=True))
