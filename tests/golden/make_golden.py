"""Write the golden files under tests/golden/ from the CPU oracle alone.

Each case runs the oracle's two-site DMRG (oracle/dmrg.py) on a seeded
workload with a fixed sweep schedule and options, and records the sweep
energies (and, for the measuring cases, the orbital entropies, the mutual
information and the correlations they come from).  The GPU parity tests run the library with the same workload,
schedule, ordering and options and compare energies (relative 1e-8 in FP64,
1e-6 in the mixed modes).  Nothing here touches the GPU library.

    python tests/golden/make_golden.py                 all cases of CASES
    python tests/golden/make_golden.py NAME ...        only those cases (merged into the file)
    python tests/golden/make_golden.py --bench-schedule
    python tests/golden/make_golden.py --batched 64

--bench-schedule writes oracle_bench_schedule.json: the benchmark's own
workload (pf 8p+8n), options and D schedule (512, 512, 1024, 1024, then
2048), one entry per sweep, the file rewritten after every sweep.
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
    ("pfg9_12p12n_D64", "pfg9_12p12n", None, [32, 64]),
    ("pfg9_12p12n_M2_D64", "pfg9_12p12n_M2", None, [32, 64]),
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
    # CI-DEAS start: entropies and occupations from a measuring run (2 sweeps at D = 16)
    ("p_2p2n_cideas", "p_2p2n", 3, [16, 16], {"cideas": 16}),
    ("sd_4p4n_cideas", "sd_4p4n", None, [32, 32], {"cideas": 16}),
    ("pf_8p8n_cideas", "pf_8p8n", None, [32, 32], {"cideas": 16}),
]


def cideas_profile(h, order, D):
    """(s1, n1) in site indices from two measuring sweeps of the oracle at D."""
    sp = h.space
    m = dmrg.DMRG(h.eps, h.V, sp.species, sp.two_m, h.n_p, h.n_n, h.two_M, order,
                  dmrg.Options(**OPTS, measure=True))
    for _ in range(2):
        m.sweep(D)
    s1, _, raw = m.entropies()
    n1 = [0.0] * sp.n_sites
    for pos, site in enumerate(m.order):
        n1[int(site)] = float(raw["n1"][pos])
    return [float(x) for x in s1], n1


def hamiltonian(spec):
    if isinstance(spec, str):
        return WORKLOADS[spec].hamiltonian()
    space, seed, n_p, n_n, two_M = spec
    return make_hamiltonian(make_space(space), seed, n_p, n_n, two_M)


# the benchmark's schedule and options (bench.py: the D ramp, then D = 2048)
BENCH_OPTS = dict(davidson_tol=1e-7, noise=1e-4, noise_sweeps=2, seed=1507)
BENCH_SCHEDULE = [512, 512, 1024, 1024, 2048, 2048, 2048]


def bench_schedule():
    h = WORKLOADS["pf_8p8n"].hamiltonian()
    sp = h.space
    o = dmrg.DMRG(h.eps, h.V, sp.species, sp.two_m, h.n_p, h.n_n, h.two_M, None, dmrg.Options(**BENCH_OPTS))
    out = {"workload": "pf_8p8n", "options": BENCH_OPTS, "D": [], "energies": [], "kept_max": [],
           "products": [], "seconds": []}
    path = os.path.join(HERE, "oracle_bench_schedule.json")
    for D in BENCH_SCHEDULE:
        t = time.time()
        r = o.sweep(D)
        out["D"].append(D)
        out["energies"].append(r["energy"])
        out["kept_max"].append(r["kept_max"])
        out["products"].append(r["nprod"])
        out["seconds"].append(time.time() - t)
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
        print(f"bench schedule D={D}: {r['energy']} ({time.time() - t:.0f} s)", flush=True)


# the independent small solves advanced together by dmrg_sweep_many (one
# sweep each at the instance's D, mixed-mode options of bench.py --batched)
BATCH_OPTS = dict(davidson_tol=1e-7, noise=1e-4, noise_sweeps=1, seed=1507)


def batched(count):
    """oracle_batched.json: the first sweep energy of each of the first
    `count` seeded instances whose oracle sweep is cheap (p and sd spaces at
    every D, pf at D <= 128)."""
    from workloads import batched_instances
    out = {"options": BATCH_OPTS, "count": count, "instances": {}}
    path = os.path.join(HERE, "oracle_batched.json")
    for i, w in enumerate(batched_instances(count)):
        D = w.D_schedule[0]
        if w.space == "pf" and D > 128:
            continue
        h = w.hamiltonian()
        sp = h.space
        t = time.time()
        o = dmrg.DMRG(h.eps, h.V, sp.species, sp.two_m, h.n_p, h.n_n, h.two_M, None, dmrg.Options(**BATCH_OPTS))
        r = o.sweep(D)
        out["instances"][str(i)] = {"space": w.space, "n_p": h.n_p, "n_n": h.n_n, "D": D, "energy": r["energy"]}
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
        print(f"instance {i} {w.space} {h.n_p}p{h.n_n}n D={D}: {r['energy']} ({time.time() - t:.1f} s)", flush=True)


def main():
    if sys.argv[1:] == ["--bench-schedule"]:
        bench_schedule()
        return
    if sys.argv[1:2] == ["--batched"]:
        batched(int(sys.argv[2]))
        return
    only = set(sys.argv[1:])
    path = os.path.join(HERE, "oracle_energies.json")
    out = {"options": OPTS, "cases": {}}
    if only:
        with open(path) as f:
            out = json.load(f)
    for name, spec, oseed, sched, *extra in CASES:
        if only and name not in only:
            continue
        extra = extra[0] if extra else {}
        h = hamiltonian(spec)
        sp = h.space
        order = None if oseed is None else random_ordering(sp.n_sites, oseed)
        t = time.time()
        opts = dict(extra)
        prof = None
        if "cideas" in opts:
            prof = cideas_profile(h, order, opts.pop("cideas"))
            opts.update(cideas_entropy=prof[0], cideas_occupation=prof[1])
        o = dmrg.DMRG(h.eps, h.V, sp.species, sp.two_m, h.n_p, h.n_n, h.two_M, order,
                      dmrg.Options(**OPTS, **opts))
        res = [o.sweep(D) for D in sched]
        energies = [r["energy"] for r in res]
        case = {"workload": spec, "ordering_seed": oseed, "D": sched, "energies": energies,
                "kept_max": [r["kept_max"] for r in res], "options": extra,
                "energies_excited": [r.get("energy_excited") for r in res],
                "target": [h.n_p, h.n_n, h.two_M]}
        if prof is not None:
            case["cideas_s1"], case["cideas_n1"] = prof
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
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
