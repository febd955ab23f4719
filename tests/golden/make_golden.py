"""Writes the stored expected values under tests/golden/ by calling only the oracle.

    python tests/golden/make_golden.py

coupled_counts.json : per-source coupled-set sizes for the three single-system
    workloads and a few edge shapes (closed form of Eq. 4's construction; the
    tests re-derive them by brute force and by the closed form).
tiny_oracle.json    : the tiny workload's oracle results (energy, a digest of
    the dense coupled output), a regression pin of the oracle itself.
"""
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import sci_inputs as si  # noqa: E402


def main():
    cases = []
    for name, wl in si.WORKLOADS.items():
        cases.append(dict(name=name, n_orb=wl.n_orb, n_alpha=wl.n_alpha, n_beta=wl.n_beta,
                          per_source=oracle.n_coupled(wl.n_orb, wl.n_alpha, wl.n_beta)))
    for n, na, nb in [(2, 1, 1), (4, 0, 2), (5, 5, 5), (6, 3, 2), (40, 20, 20), (128, 10, 10)]:
        cases.append(dict(name=f"edge_{n}_{na}_{nb}", n_orb=n, n_alpha=na, n_beta=nb,
                          per_source=oracle.n_coupled(n, na, nb)))
    with open(os.path.join(HERE, "coupled_counts.json"), "w") as f:
        json.dump({"source": "oracle.n_coupled (closed form of the single+double construction)",
                   "cases": cases}, f, indent=1)

    wl = si.WORKLOADS["tiny"]
    s = si.make_system(wl)
    keys, hij, _ = oracle.gen_coupled(wl.n_orb, wl.n_alpha, wl.n_beta, s.h1, s.eri, s.dets)
    e, hp, g = oracle.energy(wl.n_orb, wl.n_alpha, wl.n_beta, s.h1, s.eri, s.dets, s.psi)
    u, nov = oracle.dedup_merge(wl.W, keys, s.dets)
    out = dict(
        workload="tiny", n_candidates=int(keys.shape[0]),
        keys_sha256=hashlib.sha256(np.ascontiguousarray(keys).tobytes()).hexdigest(),
        hij_first=[float(x) for x in hij[:8]], hij_abs_sum=float(np.abs(hij).sum()),
        n_unique_with_sel=int(u.shape[0]), n_novel=int(nov.shape[0]),
        energy=e, hpsi_first=[float(x) for x in hp[:4]], grad_first=[float(x) for x in g[:4]],
    )
    with open(os.path.join(HERE, "tiny_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
