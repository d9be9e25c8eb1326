"""Writes model_scaling.json: the per-component descriptor scaler of each
seeded model, s_nu = 1 / (max q_nu - min q_nu) over the atoms of the
model's reference frame(s), computed with the FP64 oracle only.

The scaler is a model parameter (the descriptor-scaling step of the NEP
network input, Sec. 2.1); it keeps the random-weight tanh layer out of
saturation.  Run from the repository root:  python tests/golden/make_model_scaling.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402


def reference_frames(name):
    if name in ("water_dipole_small", "water_dipole_5b", "water_polarizability_5b", "water_pes_5b"):
        return synth.water_small(1), [0]
    if name in ("water_dipole", "water_polarizability", "water_pes"):
        pos, spc, cell = synth.water_large_reference()
        fr = synth.Frames(np.array([0, len(spc)], np.int64), pos, spc, cell[None], np.ones((1, 3), np.uint8))
        return fr, [0]
    if name == "perovskite_susceptibility":
        return synth.perovskite(1), [0]
    if name.startswith("molecule_"):
        fr = synth.molecules(64)
        return fr, list(range(64))
    raise KeyError(name)


def main():
    out = {}
    for name in synth.MODEL_SPECS:
        m = synth.model_raw(name)
        fr, idx = reference_frames(name)
        q = np.concatenate([oracle.frame_descriptors(m, fr, f)[0] for f in idx])
        span = q.max(0) - q.min(0)
        out[name] = {"q_scaler": (1.0 / span).tolist()}
        print(name, q.shape, "span min/max", span.min(), span.max(), flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "model_scaling.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
