"""Write tests/golden/<workload>_reference.json: the closed-form minimum of the OMM functional.

Calls only the oracle (its LAPACK-based closed form) and the seeded input generator:
E_min = 2 sum_{i<=M} min(eps_i - eta, 0) over the lowest generalized eigenvalues of (H, S).
A name of the form <workload>@k<value> (for example c5@k0.3) takes the complex Hermitian
H(k), S(k) of that workload made periodic along x (synth.bloch_system). The name c4 takes the
64 batched systems (synth.batched_systems, seeds 100..163) and, for the warm start, each one's
H perturbed by synth.perturb_hamiltonian with seed 200 + i.
Usage: python tests/golden/make_golden.py c3 [c2 c5 c5@k0.3 c4 ...]
"""

import json
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parents[2]
sys.path.insert(0, str(ROOT))

from oracle import brute  # noqa: E402
from synth import batched_systems, bloch_system, config_system, perturb_hamiltonian  # noqa: E402


def batch_reference():
    """Closed forms of the 64 batched systems, cold and after the warm-start perturbation."""
    t0 = time.time()
    systems = batched_systems(count=64)
    t_gen = time.time() - t0
    rows = []
    for i, x in enumerate(systems):
        w = brute.generalized_eigh_lapack(x.H, x.S, count=x.M + 1)[0]
        Hp = perturb_hamiltonian(x.H, 200 + i)
        wp = brute.generalized_eigh_lapack(Hp, x.S, count=x.M + 1)[0]
        rows.append({"seed": x.seed, "N": x.N, "M": x.M, "eta": x.eta, "tau": x.tau,
                     "E_min": brute.closed_form_energy(w, x.M, x.eta),
                     "E_min_warm": brute.closed_form_energy(wp, x.M, x.eta),
                     "gap": float(w[x.M] - w[x.M - 1]),
                     "trace_H": float(np.trace(x.H)), "sum_S": float(np.sum(x.S))})
    out = {"workload": "c4", "count": len(rows), "systems": rows,
           "source": "oracle.brute.closed_form_energy over LAPACK generalized eigenvalues; "
                     "warm: H + 1e-3 sym(N(0,1)) from synth.perturb_hamiltonian(seed 200 + i)"}
    (Path(__file__).parent / "c4_reference.json").write_text(json.dumps(out, indent=1) + "\n")
    print("c4", f"generation {t_gen:.1f}s, total {time.time() - t0:.1f}s", flush=True)


def main(names):
    for name in names:
        if name == "c4":
            batch_reference()
            continue
        t0 = time.time()
        if "@k" in name:
            base, k = name.split("@k")
            s = bloch_system(base, float(k), 0)
        else:
            s = config_system(name, 0)
        w = brute.generalized_eigh_lapack(s.H, s.S, count=s.M + 1)[0]
        E = brute.closed_form_energy(w, s.M, s.eta)
        out = {
            "workload": name, "N": s.N, "M": s.M, "eta": s.eta, "tau": s.tau, "seed": 0,
            "E_min": E,
            # the same closed form at both shifts of the eta grid (below and above eps_M)
            "E_min_by_eta": {str(e): brute.closed_form_energy(w, s.M, e) for e in (0.0, 0.5)},
            "eps_M": float(w[s.M - 1]), "eps_M1": float(w[s.M]),
            "gap": float(w[s.M] - w[s.M - 1]), "eps_1": float(w[0]),
            "trace_H": float(np.real(np.trace(s.H))), "sum_S": float(np.real(np.sum(s.S))),
            "shift": s.shift,
            "source": "oracle.brute.closed_form_energy over LAPACK generalized eigenvalues",
        }
        fname = name.replace("@", "_")
        (Path(__file__).parent / f"{fname}_reference.json").write_text(json.dumps(out, indent=1) + "\n")
        print(name, E, f"{time.time() - t0:.1f}s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c2", "c5", "c3"])
