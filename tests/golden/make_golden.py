"""Writes the stored expected values under tests/golden/.

Inputs come from the seeded generators in paper_1807_11830_amd.synth;
every expected value of the method comes from the FP64 oracle (oracle/),
never from the GPU path.  Re-run with:  python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_1807_11830_amd import synth  # noqa: E402


def main():
    hashes = {
        "phantom2d_64_s11": synth.sha256(synth.phantom2d(64, seed=11)),
        "maps2d_64_c4": synth.sha256(synth.coil_maps2d(64, 4)),
        "mask_regular_64": synth.sha256(synth.mask_regular(64, 2, 8)),
        "mask_vd_256_r4": synth.sha256(synth.mask_variable_density(256, 4.0, 24)),
        "noise_4x64x64": synth.sha256(synth.complex_noise((4, 64, 64))),
    }
    with open(os.path.join(HERE, "synth_hashes.json"), "w") as f:
        json.dump(hashes, f, indent=1, sort_keys=True)

    # 64x64, 4 coils, R=2 regular + 8 centre lines, sigma 1e-3, 20 iterations
    w = synth.SMALL_64
    imgs, maps, mask = synth.slice_inputs(w, 1)
    y = oracle.E(imgs, maps, mask) + synth.complex_noise((1, w.ncoils, w.n, w.n)) * mask[None, None, :, None]
    x, iters, status, hist = oracle.cg(y, maps, mask, w.iters)
    out = {
        "workload": w.name,
        "source": "oracle.cg (FP64) on synth.slice_inputs(SMALL_64) + synth.complex_noise",
        "iters": int(iters[0]), "status": int(status[0]),
        "rho_hist": [float(v) for v in hist[0]],
        "x_norm": float(np.linalg.norm(x)),
        "x_sum": [float(x.sum().real), float(x.sum().imag)],
        "x_true_rel_err": float(np.linalg.norm(x - imgs) / np.linalg.norm(imgs)),
    }
    with open(os.path.join(HERE, "small64_cg_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
