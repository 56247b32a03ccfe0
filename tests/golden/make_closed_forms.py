"""Write tests/golden/closed_forms.json.

Every value is either derived by hand from geometry (stated in the entry's
"source") or computed here through the oracle package only.  Run from the
repository root:  python -m tests.golden.make_closed_forms
"""
import json
import os

import numpy as np

from oracle import cpu

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "closed_forms.json")


def lattice_sums(h_over_dx: float, reach: int = 3):
    r = np.arange(-reach, reach + 1)
    X, Y, Z = np.meshgrid(r, r, r, indexing="ij")
    d = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1).astype(float)
    sw = 0.0
    M = np.zeros((3, 3))
    for dd in d:
        rr = float(np.linalg.norm(dd))
        sw += cpu.kernel_W(rr, h_over_dx)
        if rr > 0:
            M += np.outer(dd, cpu.kernel_F(rr, h_over_dx) * dd / rr)
    return sw, M


def main():
    sw, M = lattice_sums(1.3)
    shells = {}
    r = np.arange(-3, 4)
    for a in r:
        for b in r:
            for c in r:
                k = int(a * a + b * b + c * c)
                if 0 < k < (2 * 1.3) ** 2:
                    shells[k] = shells.get(k, 0) + 1
    out = {
        "lattice_sums_h1.3": {
            "sum_W": sw,
            "sum_xgradW_diag": float(M[0, 0]),
            "offdiag_max": float(np.abs(M - np.diag(np.diag(M))).max()),
            "source": "oracle kernel W and F summed over the infinite unit lattice (|offset| <= 3), "
                      "h = 1.3 dx; continuum limits are 1 and the identity",
        },
        "lattice_neighbours_h1.3": {
            "count": int(sum(shells.values())),
            "shells": {str(k): v for k, v in sorted(shells.items())},
            "source": "integer enumeration of lattice offsets with 0 < r^2 < (2.6)^2",
        },
        "share_slab_boundary_count": {
            "n_B": 2 * 200 * 200,
            "source": "lattice 250x200x200, dx = 1e-3, jitter +-0.05 dx, remote = columns >= 200; "
                      "bucket side 2.6 dx: remote bucket 77 = [200.2, 202.8) dx, local bucket 76 = "
                      "[197.6, 200.2) dx holds columns 198 and 199 (column 197 tops out at 197.55 dx)",
        },
        "cylinder_count": {
            "n": 3987920,
            "source": "12620 lattice sites of spacing 1.5777e-4 m within r <= 10 mm, times 316 layers",
        },
    }
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
