"""Write stored oracle results for the parity tests.

Calls only ``oracle/`` (never the HIP library).  Each output file records the
command that made it.  Usage, from the repository root:

    python tests/golden/make_golden.py ising_d32      # ~1.5 min on 8 cores
    python tests/golden/make_golden.py ising_d64      # ~35 min on 8 cores
    python tests/golden/make_golden.py xy_batch       # XY problems of the batch workload
"""

import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import hotrg, tensors, exact  # noqa: E402
from tests.sensitivity import oracle_drift, spectra_drift  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
BETA_C = math.log(1.0 + math.sqrt(2.0)) / 2.0


def _dump(name, payload):
    payload["command"] = "python tests/golden/make_golden.py " + name
    path = os.path.join(HERE, name + ".json")
    with open(path, "w") as f:
        json.dump(payload, f, indent=1)
    print("wrote", path)


def _record(res, spec_len):
    return {
        "lnz_per_site": res.lnz_per_site,
        "steps": [s.__dict__ for s in res.steps],
        "spectra": [list(map(float, sp[:spec_len])) for sp in res.spectra],
    }


def ising_run(beta, d_cut, n_steps, spec_len):
    t = time.time()
    res = hotrg.run(tensors.ising(beta), d_cut, n_steps, spec_len=spec_len)
    rec = _record(res, spec_len)
    rec.update(beta=beta, d_cut=d_cut, n_steps=n_steps, seconds=time.time() - t)
    drift, _ = spectra_drift(tensors.ising(beta), d_cut, n_steps, spec_len, base=res)
    rec["spectra_drift"] = drift
    return rec


def ising_d32():
    # Ising at T in {2.0, Tc, 2.5}, D_cut = 32, 30 directional steps
    runs = []
    for beta in (1.0 / 2.0, BETA_C, 1.0 / 2.5):
        rec = ising_run(beta, 32, 30, 33)
        rec["onsager"] = exact.onsager_hyper(beta)
        runs.append(rec)
        print(beta, rec["lnz_per_site"], rec["seconds"])
    _dump("ising_d32", {"model": "ising", "runs": runs})


def ising_d64():
    # Ising at Tc, D_cut = 64, 40 directional steps (2^20 x 2^20 sites);
    # the result after 30 steps is steps[29]["lnz_torus"].
    rec = ising_run(BETA_C, 64, 40, 65)
    rec["onsager"] = exact.onsager_tc()
    _dump("ising_d64", {"model": "ising", "runs": [rec]})


def xy_batch():
    # XY problems: beta on an inclusive grid in [0.8, 1.4], n_max in 3..6,
    # D_cut in {24, 32, 40, 48}, 25 steps, multiplet-safe truncation.
    # Only a subset of the 64-problem batch (the cheap D_cut values) is
    # stored; it is enough to check each problem inside the batch.
    runs = []
    for i in range(64):
        beta = 0.8 + 0.6 * i / 63.0
        n_max = 3 + (i % 4)
        d_cut = (24, 32, 40, 48)[(i // 4) % 4]
        if d_cut > 32 or i % 3:
            continue
        t = time.time()
        res = hotrg.run(tensors.xy(beta, n_max), d_cut, 25, trunc="multiplet",
                        tau=1e-10, spec_len=d_cut + 1)
        rec = _record(res, d_cut + 1)
        drift, lnz_drift, kept_pert, _ = oracle_drift(tensors.xy(beta, n_max), d_cut, 25,
                                                      d_cut + 1, trunc="multiplet", base=res)
        rec.update(spectra_drift=drift, lnz_drift=lnz_drift, kept_perturbed=kept_pert)
        rec.update(index=i, beta=beta, n_max=n_max, d_cut=d_cut, n_steps=25,
                   trunc="multiplet", tau=1e-10, seconds=time.time() - t)
        runs.append(rec)
        print(i, beta, n_max, d_cut, rec["lnz_per_site"], rec["seconds"])
    _dump("xy_batch", {"model": "xy", "runs": runs})


if __name__ == "__main__":
    for name in sys.argv[1:]:
        globals()[name]()
