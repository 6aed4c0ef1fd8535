"""Writes qem_noise4_L8.json: the FP64 oracle's round schedule on the 1.31M-face
simplification workload (noise4 icosphere L8) to the two target sizes of
Sec. 6.1's comparison (10k and 5k faces): SHA-256 of the output faces (int32)
and of the vertices rounded to float32, the counts and the per-round stats.
Calls only oracle/ and synth/ (about a minute per target on one core).

    python tests/golden/make_qem_golden.py
"""
import hashlib
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synth import shapes as S  # noqa: E402


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def main():
    out = {"workload": None, "rho": 0.25, "targets": {}}
    for cfg in (2, 3):
        V, F, target, name = S.simplify_input(cfg)
        out["workload"] = name.split(" -> ")[0]
        r = oracle.qem_simplify(V, F, target, method="rounds", rho=0.25)
        out["targets"][str(target)] = {
            "faces": int(r.F.shape[0]), "vertices": int(r.V.shape[0]), "rounds": int(r.rounds),
            "sha256_F_int32": digest(r.F.astype(np.int32)),
            "sha256_V_float32": digest(r.V.astype(np.float32)),
            "stats": r.stats.tolist(),
        }
        print(name, r.rounds, r.F.shape, flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "qem_noise4_L8.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
