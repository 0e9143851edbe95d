"""Build libomm.so (HIP, gfx950) in-tree: ``python -m paper_1312_1549_amd.build``.

Each ``.hip`` translation unit is compiled to an object in ``_build/`` (in parallel), then linked
into ``paper_1312_1549_amd/libomm.so``. Objects are rebuilt only when their source, the shared
headers or the flags changed, unless ``force=True``.
"""

from __future__ import annotations

import concurrent.futures as cf
import hashlib
import os
import subprocess
import sys
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
BUILD = ROOT / "_build"
LIB = PKG / "libomm.so"
SOURCES = ["omm_gemm_bf16x3.hip", "omm_gemm_bf16x2.hip", "omm_gemm_f32.hip", "omm_gemm_f64.hip", "omm_gemm.hip",
           "omm_kernels.hip", "omm_precon.hip", "omm_context.hip", "omm_batch.hip"]
HEADERS = [CSRC / "omm_internal.h", CSRC / "omm_gemm_impl.h", ROOT / "include" / "omm.h"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("OMM_OFFLOAD_ARCH", "gfx950")
FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{ROOT / 'include'}",
]


def _stamp(src: Path) -> str:
    h = hashlib.sha256()
    for p in [src, *HEADERS]:
        h.update(p.read_bytes())
    h.update(" ".join(FLAGS).encode())
    return h.hexdigest()


def _compile(src: Path, force: bool) -> Path:
    obj = BUILD / (src.stem + ".o")
    stamp = BUILD / (src.stem + ".stamp")
    key = _stamp(src)
    if not force and obj.exists() and stamp.exists() and stamp.read_text() == key:
        return obj
    cmd = [HIPCC, *FLAGS, "-c", str(src), "-o", str(obj)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src.name}:\n{r.stderr}")
    stamp.write_text(key)
    return obj


def build(force: bool = False, verbose: bool = True) -> Path:
    BUILD.mkdir(exist_ok=True)
    srcs = [CSRC / s for s in SOURCES]
    with cf.ThreadPoolExecutor(max_workers=min(len(srcs), os.cpu_count() or 4)) as ex:
        objs = list(ex.map(lambda s: _compile(s, force), srcs))
    tmp = LIB.with_suffix(".so.tmp")
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", str(tmp), *map(str, objs)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build(force="--force" in sys.argv)
