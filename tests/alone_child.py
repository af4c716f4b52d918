"""Child process of `test_gpu_batch_serve.test_batch_equals_alone`: the
problems of the mix, each run alone in this fresh process (its GEMM tuner
measures without other work on the GPU).  Prints the ln Z / N values as one
JSON line."""

import json

from paper_2306_00358_amd import Context, hotrg_run
from tests.test_gpu_batch_serve import _mix


def main():
    with Context(0) as ctx:
        vals = [hotrg_run(ctx, p, o)["lnz_per_site"] for p, o in _mix()]
    print(json.dumps(vals), flush=True)


if __name__ == "__main__":
    main()
