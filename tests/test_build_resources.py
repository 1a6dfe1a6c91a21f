"""The hot kernels compile without scratch (private) memory for every
reduced-precision codec (CPU only: hipcc cross-compiles for gfx950).

Scratch in these kernels has come from two sources, each costing a multiple
of the step time: a private array the compiler could not keep in registers,
and a runtime index into an array of the by-value grid descriptor, which
makes the compiler copy the whole descriptor into scratch in every thread."""
import concurrent.futures as cf
import os
import re
import subprocess
import tempfile

import pytest

from paper_2607_04516_amd import build_lib

pytestmark = pytest.mark.skipif(not os.path.exists(build_lib.HIPCC), reason="hipcc not available")

# (source, kernel-name pattern); codecs 1..3 (FP32, binary16, bfloat16)
HOT = [("lbm_step.hip", r"k_(even|odd|push)ILi[123]E"),
       ("lbm_adjoint.hip", r"k_adjointILi[123]E"),
       ("lbm_kernels.hip", r"k_(step|outflow_ghost|outflow_copy)ILi[123]E")]


def _resources(src):
    with tempfile.TemporaryDirectory() as d:
        cmd = [build_lib.HIPCC, *build_lib.FLAGS, "-c", os.path.join(build_lib.CSRC, src), "-o",
               os.path.join(d, "k.o"), "-Rpass-analysis=kernel-resource-usage"]
        r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    out, cur = {}, None
    for line in r.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            out[cur] = {}
            continue
        m = re.search(r"remark: (.*?): (\S+) \[-Rpass", line)
        if m and cur:
            out[cur][m.group(1).strip()] = m.group(2)
    return out


def test_hot_kernels_use_no_scratch():
    with cf.ThreadPoolExecutor(max_workers=len(HOT)) as ex:
        res = list(ex.map(_resources, [s for s, _ in HOT]))
    checked = 0
    for (src, pat), kernels in zip(HOT, res):
        for name, v in kernels.items():
            if not re.search(pat, name):
                continue
            checked += 1
            assert int(v["ScratchSize [bytes/lane]"]) == 0, (src, name, v)
    assert checked >= 12
