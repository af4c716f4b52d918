"""Every GEMM kernel the autotuner may choose, forced one at a time, against
the oracle.  The tuner keeps only the fastest candidate's output, so the
others are checked here: each case runs `tests/variant_child.py` in a child
process whose environment forces one FP64 LDS kernel (HOTRG_GEMM_VARIANT)
or one reduced-precision tile configuration (HOTRG_RP_CFG with the tuner
off); the variables are read once per process."""

import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# FP64: 0 = 128 x 128 tile with 32-deep slabs, 1 = 256 x 128 with two LDS stages,
# 3 = three stages (software-pipelined), 4 = 128 x 128 tile, 5 = 512 x 64 tile
# (forced, it also runs the wide products, and C3 with N = 32 half-masked);
# reduced precision: 0 = 256 x 256, 1 = 256 x 128 two stages,
# 2 = 256 x 128 three stages (software-pipelined)
CASES = ([("fp64", {"HOTRG_GEMM_VARIANT": v}) for v in ("0", "1", "3", "4", "5")]
         + [(p, {"HOTRG_AUTOTUNE": "0", "HOTRG_RP_CFG": c})
            for p in ("fp32", "bf16x3") for c in ("0", "1", "2")])


@pytest.mark.parametrize("prec,env", CASES, ids=["%s-%s" % (p, "-".join(e.values()))
                                                 for p, e in CASES])
def test_forced_kernel_variant(prec, env):
    print("forced", prec, env, flush=True)
    full = dict(os.environ)
    full.update(env)
    r = subprocess.run([sys.executable, "-m", "tests.variant_child", prec], cwd=ROOT, env=full,
                       capture_output=True, text=True, timeout=600)
    print(r.stdout, r.stderr[-2000:], flush=True)
    assert r.returncode == 0, r.stderr[-2000:]
