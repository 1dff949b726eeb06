"""Writes pass_fractions.json: the pass fraction of the FP32 dose criterion
(tests/parity.py) between two runs of the oracle with independent seeds, at
the history and batch counts of each GPU parity case.  The reference run is
the one the GPU is compared with (the workload's seed, the same batches);
the second run takes each of several other seeds.  Only oracle/ computes
anything here.

    python tests/golden/make_pass_fractions.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
from paper_1809_03927_amd import workloads as W  # noqa: E402
from parity import dose_parity, oracle_with_sigma  # noqa: E402

SEEDS = (1001, 1002, 1003, 1004, 1005, 1006)


def thorax128():
    ph = W.make_thorax((128, 128, 80), 0)
    plan = W.plan_thorax(3)
    plan.spots["phase"] = 0
    return W.Workload("thorax128", [ph], plan, 200_000, seed=3)


CASES = {
    "tiny_1e5": (W.workload_tiny, 100_000, 100),
    "slabs_3e5": (W.workload_slabs, 300_000, 100),
    "thorax128_2e5": (thorax128, 200_000, 100),
}


def main(names):
    path = os.path.join(HERE, "pass_fractions.json")
    out = json.load(open(path)) if os.path.exists(path) else {}
    for name in names:
        make, n, nb = CASES[name]
        wl = make()
        ref, sig, _ = oracle_with_sigma(oracle, wl, n, n_batches=nb)
        fr = []
        for s in SEEDS:
            t, _, _ = oracle.dose(wl.phases, wl.plan, n, s, with_dose=False)
            f, e_rel, zm, zr, nv = dose_parity(t[0], ref, sig)
            fr.append(f)
            print(name, s, f"pass {f:.5f} dE {e_rel:.2e} mean z {zm:+.3f} rms z {zr:.3f} voxels {nv}", flush=True)
        out[name] = {"histories": n, "batches": nb, "reference_seed": wl.seed, "seeds": list(SEEDS),
                     "fractions": fr, "mean": float(np.mean(fr)), "sd": float(np.std(fr, ddof=1)),
                     "voxels": nv}
        with open(path, "w") as f:
            json.dump(out, f, indent=1)


if __name__ == "__main__":
    main(sys.argv[1:] or list(CASES))
