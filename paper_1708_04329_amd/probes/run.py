"""Build and run the gfx950 microbenchmarks behind the scan's ceilings.

    python -m paper_1708_04329_amd.probes.run [--build-only]

Compiles issue_lds_mix.hip with hipcc into ``_build/issue_lds_mix`` and runs
it on the current GPU; see the source for what each line measures.
"""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(os.path.dirname(HERE), "_build", "issue_lds_mix")


def build() -> str:
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    subprocess.check_call([os.environ.get("HIPCC", "/opt/rocm/bin/hipcc"), "--offload-arch=gfx950", "-O3",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           os.path.join(HERE, "issue_lds_mix.hip"), "-o", OUT])
    return OUT


if __name__ == "__main__":
    exe = build()
    if "--build-only" not in sys.argv:
        sys.exit(subprocess.call([exe]))
