"""TEST INFRASTRUCTURE: algorithmic operation counts of the HARM step, from
the oracle's counting build (every +, -, *, /, sqrt counts one flop).

Counts one face flux (per direction) and one zone update on a sample of
zones of the 32^3 torus, and prints the mean per unit and per zone-cycle.
Usage: python -m oracle.count_flops
"""

import json

import numpy as np

import oracle
from workloads import fm_torus, RECON_MC, RECON_WENO5


def main():
    grid, P, _ = fm_torus(32, 32, 32)
    rng = np.random.default_rng(0)
    sample = [(int(rng.integers(0, 32)), int(rng.integers(0, 32)), int(rng.integers(0, 32)))
              for _ in range(48)]
    res = {}
    for name, recon in (("mc", RECON_MC), ("weno5", RECON_WENO5)):
        c = oracle.cfg(grid, gam=13 / 9, recon=recon, nthreads=1)
        face = []
        for (i, j, k) in sample:
            for d in (1, 2, 3):
                if d == 2 and j == 0:
                    continue
                face.append(oracle.count_face(c, P, d, i, j, k))
        face = np.array(face, dtype=float)
        upd = np.array([oracle.count_zone_update(c, P, i, j, k, 1e-3) for (i, j, k) in sample[:12]],
                       dtype=float)
        f_face = face[:, :4].sum(1).mean()
        f_upd = upd[:, :4].sum(1).mean()
        res[name] = {"flops_per_face": f_face, "face_breakdown_add_mul_div_sqrt": face[:, :4].mean(0).tolist(),
                     "flops_per_zone_update": f_upd,
                     "update_breakdown_add_mul_div_sqrt": upd[:, :4].mean(0).tolist(),
                     # per zone-cycle: two stages x (3 faces + update + 3 EMFs (4 flops each) +
                     # 6 rebuilt B fluxes (2 flops each))
                     "flops_per_zone_cycle": 2 * (3 * f_face + f_upd + 3 * 4 + 6 * 2)}
    print(json.dumps(res, indent=1))


if __name__ == "__main__":
    main()
