"""Every kernel of the library compiles for gfx950 without spilling registers
to scratch memory (a spill in a hot kernel shows up as extra HBM traffic and
time, not as a wrong result, so the GPU parity tests cannot catch it).  CPU
only: it compiles the sources with the compiler's resource-usage report."""
import concurrent.futures as cf
import os
import re
import subprocess
import tempfile

import pytest

from paper_2408_14070_amd import build as B


def _usage(src):
    with tempfile.TemporaryDirectory() as d:
        r = subprocess.run([B.hipcc(), *B.FLAGS, "-c", src, "-o", os.path.join(d, "k.o"),
                            "-Rpass-analysis=kernel-resource-usage"],
                           capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    names = re.findall(r"Function Name: (\S+)", r.stderr)
    scratch = [int(x) for x in re.findall(r"ScratchSize \[bytes/lane\]: (\d+)", r.stderr)]
    return names, scratch


def test_no_kernel_spills_to_scratch():
    try:
        B.hipcc()
    except RuntimeError:
        pytest.skip("hipcc not available")
    srcs = B.sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        res = list(ex.map(_usage, srcs))
    bad, total = [], 0
    for src, (names, scratch) in zip(srcs, res):
        assert len(names) == len(scratch), src
        total += len(names)
        bad += [(os.path.basename(src), n, sc) for n, sc in zip(names, scratch) if sc]
    assert total > 100
    assert not bad, bad
