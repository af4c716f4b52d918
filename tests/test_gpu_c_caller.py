"""The boundary from plain C: a C99 program built with gcc against
include/hotrg.h and libhotrg.so runs one problem on the GPU; its ln Z/N
must equal the FP64 oracle's."""

import os
import shutil
import subprocess
import sys

import pytest

from oracle import hotrg, tensors

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SRC = r"""
#include <stdio.h>
#include "hotrg.h"
int main(void) {
  hotrg_ctx* ctx;
  if (hotrg_ctx_create(0, NULL, 0, &ctx) != HOTRG_OK) { puts(hotrg_last_error()); return 1; }
  hotrg_model_params p = {0};
  p.model = HOTRG_ISING; p.beta = 0.4406867935097715; p.J = 1.0;
  hotrg_opts o = {0};
  o.d_cut = 16; o.n_steps = 20; o.prec = HOTRG_FP64;
  hotrg_step_info info[20];
  hotrg_result r = {0};
  r.steps = info;
  if (hotrg_run(ctx, &p, &o, &r) != HOTRG_OK) { puts(hotrg_last_error()); return 1; }
  printf("%.17g %d %d\n", r.lnz_per_site, r.n_steps, info[19].kept);
  hotrg_ctx_destroy(ctx);
  return 0;
}
"""


def test_c_program_runs_on_the_gpu(tmp_path):
    from paper_2306_00358_amd import _lib

    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    (tmp_path / "caller.c").write_text(SRC)
    libdir = os.path.dirname(_lib.LIB_PATH)
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"),
                    str(tmp_path / "caller.c"), "-o", str(tmp_path / "caller"), "-L", libdir,
                    "-lhotrg", "-Wl,-rpath," + libdir], check=True)
    print("running the C caller", flush=True)
    sys.stdout.flush()
    out = subprocess.run([str(tmp_path / "caller")], check=True, capture_output=True, text=True,
                         timeout=120).stdout.split()
    lnz, n_steps, kept = float(out[0]), int(out[1]), int(out[2])
    want = hotrg.run(tensors.ising(0.4406867935097715), 16, 20)
    assert n_steps == 20 and kept == 16
    assert abs(lnz - want.lnz_per_site) <= 1e-12 * abs(want.lnz_per_site)
