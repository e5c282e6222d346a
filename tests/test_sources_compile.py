"""Every source of the library and of the benchmark library passes hipcc's
front end for gfx950 (host and device), with the flags of the real build.
The CPU suite otherwise runs against whatever library was built last, so a
source that no longer compiles would go unnoticed until the next build."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

from paper_2504_07264_amd import build


def _hipcc():
    try:
        return build.hipcc()
    except RuntimeError:
        return None


@pytest.mark.skipif(_hipcc() is None, reason="hipcc is not installed")
def test_every_source_compiles():
    cc = _hipcc()
    flags = [f for f in build.HIPCC_FLAGS if f not in ("-O3", "-fPIC")]

    def check(src):
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [cc, *flags, "-fsyntax-only", *lang, os.path.join(build.CSRC, src)]
        res = subprocess.run(cmd, capture_output=True, text=True)
        return src, res.returncode, res.stderr[-3000:]

    srcs = build.SOURCES + build.BENCH_SOURCES
    with ThreadPoolExecutor(max_workers=min(4, os.cpu_count() or 1)) as ex:
        results = list(ex.map(check, srcs))
    failed = [(s, err) for s, rc, err in results if rc != 0]
    assert not failed, "\n".join("%s:\n%s" % f for f in failed)
    assert shutil.which(cc) or os.path.exists(cc)
