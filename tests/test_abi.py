"""The C-ABI library loads and exports every function include/hotrg.h
declares (no compute call: this runs without a GPU)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hotrg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hotrg_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("hotrg_init_tensor", "hotrg_step", "hotrg_run", "hotrg_finish"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2306_00358_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libhotrg.so is not built (run python -m paper_2306_00358_amd.build)")
    L = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_names_match_header():
    from paper_2306_00358_amd import _lib

    assert sorted(_lib.EXPORTS) == sorted(n for n in declared_functions() if n in _lib.EXPORTS)
    assert set(_lib.EXPORTS) <= set(declared_functions())


def test_struct_layouts_match_header():
    # field order and sizes of the ctypes mirrors against the C declarations
    from paper_2306_00358_amd import _lib

    assert ctypes.sizeof(_lib.StepInfo) == 4 * 4 + 4 * 8 + 8  # side, padded
    assert ctypes.sizeof(_lib.Opts) == 4 * 4 + 8 + 3 * 4 + 4 + 8  # 4 ints, double, 3 ints, pad, tol
    assert [f for f, _ in _lib.ModelParams._fields_] == [
        "model", "beta", "J", "n_max", "q", "raw", "raw_dx", "raw_dy", "delta"]


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2306_00358_amd import _lib

    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(RuntimeError, match="not built"):
        _lib.lib()


def test_flop_model_matches_oracle_bookkeeping():
    from oracle import hotrg
    from paper_2306_00358_amd import flops

    for d0, dc, K in [(2, 8, 20), (2, 64, 30), (7, 24, 25)]:
        assert flops.dims_schedule(d0, dc, K) == hotrg.dims_schedule(d0, dc, K)
        for d in flops.dims_schedule(d0, dc, K):
            # the oracle counts each Gram half as a full square product too
            assert flops.step_flops(*d)["total"] == hotrg.step_flops(*d)


def test_footprint_host_estimate():
    # pure host arithmetic on the dimension schedule (no device call)
    from paper_2306_00358_amd import hotrg_footprint, make_opts, model_params

    p = model_params("ising", beta=0.44)
    f32 = hotrg_footprint(p, make_opts(32, 30))
    f64 = hotrg_footprint(p, make_opts(64, 30))
    assert 0 < f32 < f64
    # the two D^5 intermediates dominate: 2 * 64^5 * 8 bytes at D = 64
    assert 2 * 64**5 * 8 < f64 < 4 * 64**5 * 8
    assert hotrg_footprint(p, make_opts(64, 30, prec="fp32")) < f64


def test_struct_offsets_match_the_c_compiler(tmp_path):
    # offsetof / sizeof of every field as gcc lays out include/hotrg.h,
    # against the ctypes mirrors of the binding
    import shutil
    import subprocess

    from paper_2306_00358_amd import _lib

    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    structs = {"hotrg_model_params": _lib.ModelParams, "hotrg_opts": _lib.Opts,
               "hotrg_step_info": _lib.StepInfo, "hotrg_result": _lib.Result}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "hotrg.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append('printf("%s sizeof %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in py._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(line.split()[:2]): int(line.split()[2]) for line in out if line}
    for cname, py in structs.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_c_program_compiles_and_links(tmp_path):
    # a plain C99 caller of the boundary builds and links against libhotrg.so
    # (it is not run here: running needs a GPU)
    import shutil
    import subprocess

    from paper_2306_00358_amd import _lib

    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    src = tmp_path / "caller.c"
    src.write_text("""
#include <stdio.h>
#include "hotrg.h"
int main(void) {
  hotrg_ctx* ctx;
  if (hotrg_ctx_create(0, NULL, 0, &ctx) != HOTRG_OK) { puts(hotrg_last_error()); return 1; }
  hotrg_model_params p = {0};
  p.model = HOTRG_ISING; p.beta = 0.4406867935097715; p.J = 1.0;
  hotrg_opts o = {0};
  o.d_cut = 16; o.n_steps = 20; o.prec = HOTRG_FP64;
  hotrg_result r = {0};
  if (hotrg_run(ctx, &p, &o, &r) != HOTRG_OK) { puts(hotrg_last_error()); return 1; }
  printf("%.15f\\n", r.lnz_per_site);
  hotrg_ctx_destroy(ctx);
  return 0;
}
""")
    libdir = os.path.dirname(_lib.LIB_PATH)
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(tmp_path / "caller"), "-L", libdir, "-lhotrg", "-Wl,-rpath," + libdir],
                   check=True)


def test_footprint_properties():
    # admission arithmetic (host only): more steps or a larger cut never need
    # less memory, the two-sided isometry never less than one-sided; an
    # unknown model is rejected.  (Reduced precision is not always smaller:
    # its early steps run in FP64 and both sets of buffers stay allocated.)
    import pytest

    from paper_2306_00358_amd import HotrgError, hotrg_footprint, make_opts, model_params

    for p in (model_params("ising", beta=0.44), model_params("xy", beta=1.0, n_max=3),
              model_params("potts", beta=1.0, q=3)):
        prev_cut = 0
        for d_cut in (8, 16, 24, 32, 48):
            prev_steps = 0
            for n_steps in (1, 2, 4, 8, 16, 30):
                f = hotrg_footprint(p, make_opts(d_cut, n_steps))
                assert f >= prev_steps
                prev_steps = f
                two = hotrg_footprint(p, make_opts(d_cut, n_steps, isometry="two"))
                assert two >= f
            assert prev_steps >= prev_cut
            prev_cut = prev_steps
    bad = model_params("ising", beta=0.44)
    bad.model = 99
    with pytest.raises(HotrgError):
        hotrg_footprint(bad, make_opts(8, 4))
