"""Writes synth_manifest.json: SHA-256 of the seeded generator's arrays.

Calls only the input generator (no method arithmetic).  Re-run after an
intentional change to the generator's draw order.
"""
import hashlib
import json
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
import numpy as np  # noqa: E402

import synth  # noqa: E402


def digest(a):
    a = np.ascontiguousarray(a)
    return hashlib.sha256(a.tobytes() + str(a.dtype).encode() + str(a.shape).encode()).hexdigest()


def manifest():
    out = {}
    for name, t in [("arm7", synth.arm7(0)), ("tree34", synth.tree34(5)), ("hand16", synth.hand16(8))]:
        for f in ["parent", "mount_quat", "offset", "axis", "lower", "upper", "ee_joint",
                  "ee_offset", "ee_quat", "ee_kind"]:
            out[f"{name}.{f}"] = digest(getattr(t, f))
    for wl, tg in [("arm16", None), ("arm131k", 64), ("tree4k", 16), ("mixed84k", 8),
                   ("beam", 10), ("mobile", 10)]:
        w = synth.workload(wl, targets=tg)
        for i, g in enumerate(w["groups"]):
            out[f"{wl}.{i}.q_star"] = digest(g["q_star"])
            out[f"{wl}.{i}.seeds"] = digest(g["seeds"])
    tr = synth.workload("traj", targets=4)
    out["traj.init"] = digest(tr["init"])
    out["mlp_init.small"] = digest(np.concatenate([np.r_[W.ravel(), b] for W, b in
                                                   synth.mlp_init([7, 16, 16, 14], 18)]))
    out["perm.100.e0"] = digest(synth.epoch_permutation(100, 19, 0))
    return out


if __name__ == "__main__":
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "synth_manifest.json")
    with open(path, "w") as f:
        json.dump(manifest(), f, indent=1, sort_keys=True)
    print("wrote", path)
