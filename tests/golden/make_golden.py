"""Write tests/golden/oracle_energies.json from the CPU oracle alone.

Each case runs the oracle's two-site DMRG (oracle/dmrg.py) on a seeded
workload with a fixed sweep schedule and options, and records the sweep
energies (and, for the measuring cases, the orbital entropies, the mutual
information and the correlations they come from).  The GPU parity tests run the library with the same workload,
schedule, ordering and options and compare energies (relative 1e-8 in FP64,
1e-6 in the mixed modes).  Nothing here touches the GPU library.

    python tests/golden/make_golden.py
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import dmrg, ed  # noqa: E402
from workloads import WORKLOADS, make_hamiltonian, make_space, random_ordering  # noqa: E402

OPTS = dict(davidson_tol=1e-9, noise=1e-4, noise_sweeps=2, seed=7)

CASES = [
    # name, workload (or (space, seed, n_p, n_n, 2M)), ordering seed, D schedule
    ("p_2p2n_D64", "p_2p2n", None, [64, 64]),
    ("p_2p2n_M2_D16", ("p", 11, 2, 2, 4), None, [16, 16]),
    ("sd_4p4n_D32", "sd_4p4n", None, [32, 32, 32]),
    ("sd_3p2n_M1_rand_D24", ("sd", 13, 3, 2, 1), 5, [24, 24]),
    ("pf_8p8n_D32", "pf_8p8n", None, [32, 32]),
    # pf + g9/2 (60 sites, 12p + 12n, the 64Ge-sized space), J_z = 0 and J_z = 2
    ("pfg9_12p12n_D16", "pfg9_12p12n", None, [16, 16]),
    ("pfg9_12p12n_M2_D16", "pfg9_12p12n_M2", None, [16]),
    # dynamic block-state selection: the kept count follows the truncation error
    ("p_2p2n_dbss", "p_2p2n", None, [64, 64, 64], {"trunc_eps": 1e-6, "d_min": 4}),
    ("sd_4p4n_dbss", "sd_4p4n", None, [128, 128, 128], {"trunc_eps": 1e-3, "d_min": 8}),
    # the two lowest states targeted at once (averaged density matrix)
    ("p_2p2n_two", "p_2p2n", None, [64, 64], {"n_states": 2}),
    ("sd_4p4n_two", "sd_4p4n", None, [32, 32], {"n_states": 2}),
    # orbital correlations, entropies and mutual information (last sweep)
    ("p_2p2n_ent", "p_2p2n", None, [16, 16], {"measure": True}),
    ("sd_4p4n_ent", "sd_4p4n", None, [32, 32], {"measure": True}),
    ("sd_3p2n_M1_rand_ent", ("sd", 13, 3, 2, 1), 5, [24, 24], {"measure": True}),
    ("pf_8p8n_ent", "pf_8p8n", None, [32, 32], {"measure": True}),
    ("sd_4p4n_two_ent", "sd_4p4n", None, [32, 32], {"measure": True, "n_states": 2}),
    ("sd_4p4n_dbss_ent", "sd_4p4n", None, [128, 128], {"measure": True, "trunc_eps": 1e-3, "d_min": 8}),
]


def hamiltonian(spec):
    if isinstance(spec, str):
        return WORKLOADS[spec].hamiltonian()
    space, seed, n_p, n_n, two_M = spec
    return make_hamiltonian(make_space(space), seed, n_p, n_n, two_M)


def main():
    out = {"options": OPTS, "cases": {}}
    for name, spec, oseed, sched, *extra in CASES:
        extra = extra[0] if extra else {}
        h = hamiltonian(spec)
        sp = h.space
        order = None if oseed is None else random_ordering(sp.n_sites, oseed)
        t = time.time()
        o = dmrg.DMRG(h.eps, h.V, sp.species, sp.two_m, h.n_p, h.n_n, h.two_M, order,
                      dmrg.Options(**OPTS, **extra))
        res = [o.sweep(D) for D in sched]
        energies = [r["energy"] for r in res]
        case = {"workload": spec, "ordering_seed": oseed, "D": sched, "energies": energies,
                "kept_max": [r["kept_max"] for r in res], "options": extra,
                "energies_excited": [r.get("energy_excited") for r in res],
                "target": [h.n_p, h.n_n, h.two_M]}
        if extra.get("measure"):
            s1, mutual, m = o.entropies()
            case["s1"] = s1.tolist()
            case["mutual"] = mutual.tolist()
            case["correlations"] = {k: v.tolist() for k, v in m.items()}
        if sp.n_sites <= 24:
            case["exact"] = float(ed.ground_energy(h.eps, h.V, sp.species, sp.two_m,
                                                   h.n_p, h.n_n, h.two_M)[0])
        out["cases"][name] = case
        print(f"{name}: {energies} ({time.time() - t:.1f} s)", flush=True)
    with open(os.path.join(HERE, "oracle_energies.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
