"""Write tests/golden/config4_adjoint.json from the CPU oracle only.

Config 4: the 24-qubit hardware-efficient ansatz (10 layers, 480 angles) and
its 200-term Pauli sum.  Stored: <H> and the parameter-shift gradient (exact
for exp(-i theta P / 2) gates) for a sample of parameters.  Takes several
minutes of CPU; run from the repository root:

    python tests/golden/make_config4_golden.py
"""
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

PARAMS = [0, 1, 47, 240, 478, 479]


def _energy(theta_list):
    import numpy as np
    import oracle
    import workloads as W
    circ, ham = W.config4()
    return oracle.energy(circ.with_theta(np.array(theta_list)), ham)


def main():
    import math
    import numpy as np
    import workloads as W
    circ, ham = W.config4()
    theta = circ.theta
    jobs = [theta.tolist()]
    for p in PARAMS:
        for sgn in (+1, -1):
            t = theta.copy()
            t[p] += sgn * math.pi / 2
            jobs.append(t.tolist())
    t0 = time.time()
    with ProcessPoolExecutor(max_workers=min(6, os.cpu_count() or 1)) as ex:
        vals = list(ex.map(_energy, jobs))
    grads = [0.5 * (vals[1 + 2 * i] - vals[2 + 2 * i]) for i in range(len(PARAMS))]
    out = {
        "source": "CPU oracle (oracle/), parameter-shift rule; written by "
                  "tests/golden/make_config4_golden.py",
        "workload": "config 4: 24-qubit HEA, 10 layers of RY,RZ per qubit + CZ ladder, "
                    "200-term Pauli sum of weight <= 4",
        "energy": vals[0],
        "params": PARAMS,
        "grad": grads,
        "cpu_seconds": time.time() - t0,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config4_adjoint.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
