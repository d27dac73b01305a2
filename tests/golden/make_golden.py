"""Write the oracle regression fixture ``oracle_tiny.json``.

Calls only ``oracle`` (and the seeded input generator ``synth``): the stored
values are the oracle's FP64 render of the 4,096-Gaussian, 128x128,
16-state workload at 64 fixed pixels, plus per-state composited-pair totals.
Re-run only when a reading of the paper changes the oracle's arithmetic.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402

BG = (0.25, 0.5, 0.75)


def main():
    w = synth.make_workload("g4k_128px_16states", background=BG)
    rng = np.random.default_rng(2606)
    pix = rng.integers(0, 128, size=(64, 2))
    r = oracle.render(w.scene, w.camera, w.basis, w.codes, w.background, pixels=pix)
    full = oracle.render(w.scene, w.camera, w.basis, w.codes, w.background)
    out = dict(workload=w.name, background=list(BG), pixels=pix.tolist(),
               image=r["image"].tolist(), tfinal=r["tfinal"].tolist(),
               ncomp_total=[int(x) for x in full["ncomp"].reshape(16, -1).sum(1)])
    with open(os.path.join(HERE, "oracle_tiny.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
